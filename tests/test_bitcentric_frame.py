"""The bit-centric machine in the frame of its current error (CPU).

On a chain (the repetition code of the SM's analysis) the machine's state can
be carried in the frame of the current error x = e0 ^ z: with
M_{c->v} = (-1)^{x_v} m_{c->v} and Y_{v->c} = (-1)^{x_v} m_{v->c}, the syndrome
sign of a check (s_c = x_v ^ x_w on a check of degree 2) and the LLR switch
cancel, and each step becomes a shift and an add:

    Y^i_{v->c} = (-1)^{e0_v} pi0 + M^{i-1}_{c'->v}   (c' the other check of v)
    M^i_{c->v} = Y^{i-1}_{w->c}                      (w the other bit of c)
    L^i_v      = (-1)^{x^{i-1}_v} ((-1)^{e0_v} pi0 + sum_c M^{i-1}_{c->v})

and x^i_v is 1 where that bracket is positive, 0 where it is negative and
x^{i-1}_v where it is zero. Negation commutes with round-to-nearest, so the
doubles are the machine's up to the sign of a zero, which no decision reads;
the machine's beliefs are never -0 (the prior is never zero's negative
counterpart in a sum that cancels), so a zero belief is +0.

The GPU's chain form runs exactly this recursion. This test runs it in numpy
(float64, the same additions in the same order) and requires the oracle's
traces -- errors, clearing iteration and the bits of every belief -- on
periodic and open chains, over priors and noise levels, and with the checks
labelled so that other bits sum their two messages in the other order."""
import math

import numpy as np
import pytest

from paper_2609_38139_amd import codes


def chain_checks(H, d):
    """For a code whose checks are the edges of a path or cycle over bits
    0..d-1 in index order: (periodic, left check, right check) per bit (-1
    where the bit has no such check)."""
    rp, col = H.rowptr, H.col
    left = np.full(d, -1, dtype=np.int64)
    right = np.full(d, -1, dtype=np.int64)
    m = H.rows
    for c in range(m):
        a, b = sorted(int(x) for x in col[rp[c]:rp[c + 1]])
        if b == a + 1:
            right[a], left[b] = c, c
        else:
            assert (a, b) == (0, d - 1)
            left[0], right[d - 1] = c, c
    return m == d, left, right


def error_frame_machine(H, d, q, e0, iters):
    periodic, left, right = chain_checks(H, d)
    # the bit sums its messages in ascending check order: left first unless
    # its left check has the larger index
    swap = (left >= 0) & (right >= 0) & (left > right)
    pi0 = math.log(q / (1.0 - q))
    e0 = np.asarray(e0, dtype=np.uint8)
    P = np.where(e0 == 1, -pi0, pi0)
    Y = {p: (np.zeros(d), np.zeros(d)) for p in (0, 1)}  # (Y to the right check, Y to the left check)
    x = e0.astype(np.uint8).copy()
    xs, Ls = [], []
    iclr = 0 if (x == x[0]).all() else -1
    for it in range(1, iters + 1):
        yr_old, yl_old = Y[it & 1]
        # M^{it-1}: from the neighbours' Y^{it-2} (nothing past an open end)
        ML = np.roll(yr_old, 1)
        MR = np.roll(yl_old, -1)
        if not periodic:
            ML[0] = 0.0
            MR[d - 1] = 0.0
        yr = P + ML
        yl = P + MR
        Lg = np.where(swap, yl + ML, yr + MR)
        L = np.where(x == 1, -Lg, Lg) + 0.0
        x = np.where(Lg > 0, 1, np.where(Lg < 0, 0, x)).astype(np.uint8)
        Y[it & 1] = (yr, yl)
        xs.append(x.copy())
        Ls.append(L)
        if iclr < 0 and (x == x[0]).all():
            iclr = it
    return np.array(xs).reshape(iters, d), np.array(Ls).reshape(iters, d), iclr


def relabel_checks(code, perm):
    """The same code with its checks listed in the order perm."""
    H = code.H
    rows = [list(H.col[H.rowptr[c]:H.rowptr[c + 1]]) for c in perm]
    return codes.Code(code.name + "_relabelled", codes.CSR.from_rows(H.rows, H.cols, rows),
                      code.G, dict(code.meta))


CASES = [(d, per, q, p) for d in (3, 4, 9, 31) for per in (True, False) for q in (0.1, 0.3)
         for p in (0.2, 0.45)] + [(101, True, 0.1, 0.3), (64, False, 0.02, 0.4), (5, True, 0.5, 0.4)]


@pytest.mark.parametrize("d,periodic,q,p", CASES)
def test_error_frame_equals_machine(orc, d, periodic, q, p):
    code = codes.repetition(d, periodic=periodic)
    e0 = orc.sample_noise(code, p, 11, 0, 24)
    iters = d + 5
    for i in range(e0.shape[0]):
        et, Lt, ic = orc.bitcentric_machine(code, q, e0[i], iters)
        xs, Ls, ic2 = error_frame_machine(code.H, d, q, e0[i], iters)
        assert np.array_equal(xs, et), (i, "errors")
        assert ic2 == ic, (i, "clearing iteration")
        assert np.array_equal(Ls.view(np.uint64), Lt.view(np.uint64)), (i, "belief bits")


def test_error_frame_with_relabelled_checks(orc):
    """Check orders where other bits (not bit 0) sum their right message
    first: the recursion still matches once each bit keeps its own order."""
    rng = np.random.default_rng(5)
    for d, periodic in ((12, True), (12, False), (33, True)):
        base = codes.repetition(d, periodic=periodic)
        perm = rng.permutation(base.H.rows)
        code = relabel_checks(base, perm)
        e0 = orc.sample_noise(code, 0.35, 2, 0, 16)
        for i in range(e0.shape[0]):
            et, Lt, ic = orc.bitcentric_machine(code, 0.2, e0[i], d + 2)
            xs, Ls, ic2 = error_frame_machine(code.H, d, 0.2, e0[i], d + 2)
            assert np.array_equal(xs, et) and ic2 == ic
            assert np.array_equal(Ls.view(np.uint64), Lt.view(np.uint64))


def test_error_frame_catches_a_wrong_sum_order(orc):
    """The order of the two additions matters in the last bit: summing every
    bit left first (ignoring the wrap check's index) changes some belief of
    the periodic chain, so the comparison above can see an order mistake."""
    d, q = 31, 0.1
    code = codes.repetition(d, periodic=True)
    e0 = orc.sample_noise(code, 0.3, 4, 0, 64)
    differs = False
    for i in range(e0.shape[0]):
        _, Lt, _ = orc.bitcentric_machine(code, q, e0[i], d)
        periodic, left, right = chain_checks(code.H, d)
        pi0 = math.log(q / (1.0 - q))
        P = np.where(e0[i] == 1, -pi0, pi0)
        Y = {p: (np.zeros(d), np.zeros(d)) for p in (0, 1)}
        x = e0[i].astype(np.uint8).copy()
        for it in range(1, d + 1):
            yr_old, yl_old = Y[it & 1]
            ML, MR = np.roll(yr_old, 1), np.roll(yl_old, -1)
            yr, yl = P + ML, P + MR
            Lg = yr + MR
            L = np.where(x == 1, -Lg, Lg) + 0.0
            x = np.where(Lg > 0, 1, np.where(Lg < 0, 0, x)).astype(np.uint8)
            Y[it & 1] = (yr, yl)
            if not np.array_equal(L.view(np.uint64), Lt[it - 1].view(np.uint64)):
                differs = True
    assert differs
