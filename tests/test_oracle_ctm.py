"""Pins of the oracle's continuous-time machine (Algorithm 1 as stated, with
the simulation of SM "Numerical details"): its FP64 logarithm, the Euler-
damped Jacobi BP, and the clock-event process, each against something the
oracle does not compute itself."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2609_38139_amd import codes
from test_oracle_pins import exact_llr, random_tree_code


def CP(**kw):
    from oracle import oracle as O
    return O.ContinuousParams(**kw)


def test_ln_unit_matches_libm(orc):
    """The waiting times' logarithm against the C library's log, over the
    whole range the event sampler feeds it ((w + 1) 2^-32) and the branch
    point sqrt(1/2)."""
    rng = np.random.default_rng(3)
    w = rng.integers(0, 2**32, size=20000, dtype=np.uint64)
    u = (w.astype(np.float64) + 1.0) / 2.0**32
    extra = np.array([2.0**-32, 1.0, 0.5, 0.25, math.sqrt(0.5), np.nextafter(math.sqrt(0.5), 1),
                      np.nextafter(math.sqrt(0.5), 0), np.nextafter(1.0, 0), 1e-9])
    u = np.concatenate([u, extra])
    got = orc.ln_unit(u)
    ref = np.log(u)
    err = np.abs(got - ref)
    assert np.all(err <= 4.5e-16 * np.maximum(np.abs(ref), 1e-300) + 2.5e-16), float(err.max())
    assert got[np.where(u == 1.0)[0][0]] == 0.0


def _rep_cycle(d):
    H = np.zeros((d, d), dtype=np.uint8)
    for j in range(d):
        H[j, j] = 1
        H[j, (j + 1) % d] = 1
    return H


@pytest.mark.parametrize("bp,alpha", [("minsum", 0.75), ("sumproduct", 1.0)])
@pytest.mark.parametrize("dt,tau,K", [(0.001, 0.1, 400), (0.1, 0.1, 7), (0.03, 0.1, 60)])
def test_euler_bp_on_a_cycle_is_the_affine_recursion(orc, bp, alpha, dt, tau, K):
    """With check degree 2 the BP map is affine: a check passes its other
    input times (-1)^{s_c} alpha (sum-product: alpha = 1), a qubit adds its
    prior to its other check's message. The oracle's K Euler steps must
    equal x <- x + lambda (A x + b - x) iterated in float64 from x = 0, with
    A and b written here from the cycle's structure; this fixes lambda, the
    Jacobi order (both directions from the old state), zero start and signs."""
    d = 9
    H = _rep_cycle(d)
    code = codes.from_dense(H)
    q = 0.05
    rng = np.random.default_rng(5)
    e0 = (rng.random(d) < 0.3).astype(np.uint8)
    s = (H @ e0) % 2
    mcv, mvc = orc.ctm_bp_steps(code, CP(bp=bp, alpha=alpha, q=q, dt=dt, tau=tau), s, K)
    # message index: cv[(c, v)] and vc[(v, c)] over the 2d edges
    edges = [(c, v) for c in range(d) for v in np.nonzero(H[c])[0]]
    ix = {e: i for i, e in enumerate(edges)}
    E = len(edges)
    A = np.zeros((2 * E, 2 * E))
    b = np.zeros(2 * E)
    pi = math.log(q / (1 - q))
    for (c, v), i in ix.items():
        other_v = [w for w in np.nonzero(H[c])[0] if w != v][0]
        sign = -1.0 if s[c] else 1.0
        A[i, E + ix[(c, other_v)]] = sign * alpha        # m_{c->v} from m_{v'->c}
        other_c = [k for k in np.nonzero(H[:, v])[0] if k != c][0]
        A[E + i, ix[(other_c, v)]] = 1.0                 # m_{v->c} from m_{c'->v}
        b[E + i] = pi
    lam = float(np.float32(dt / tau))
    x = np.zeros(2 * E)
    for _ in range(K):
        x = x + lam * (A @ x + b - x)
    got = np.concatenate([mcv, mvc]).astype(np.float64)
    assert np.allclose(got, x, rtol=2e-4, atol=2e-4), np.abs(got - x).max()


def test_damped_bp_reaches_exact_marginals_on_trees(orc):
    """On a tree the damped dynamics has the BP fixed point, which is exact:
    after enough Euler steps the beliefs pi + sum m_{c->v} equal brute-force
    posterior log-odds (random trees, odd and even check degrees)."""
    rng = np.random.default_rng(17)
    for trial in range(8):
        H = random_tree_code(rng, nmax=10)
        n = H.shape[1]
        q = float(rng.uniform(0.1, 0.35))
        e0 = (rng.random(n) < 0.3).astype(np.uint8)
        s = (H @ e0) % 2
        code = codes.from_dense(H)
        mcv, _ = orc.ctm_bp_steps(code, CP(bp="sumproduct", q=q, dt=0.05, tau=0.1), s, 600)
        pi = np.float32(math.log(q / (1 - q)))
        L = np.full(n, pi, dtype=np.float64)
        k = 0
        for c in range(H.shape[0]):
            for v in np.nonzero(H[c])[0]:
                L[v] += mcv[k]
                k += 1
        with np.errstate(divide="ignore"):
            ex = exact_llr(H, q, s)
        pinned = ~np.isfinite(ex)
        assert np.all(np.sign(L[pinned]) == np.sign(ex[pinned])) and np.all(np.abs(L[pinned]) > 900)
        assert np.allclose(L[~pinned], ex[~pinned], rtol=1e-4, atol=1e-4), (trial, L, ex)


def _replay(orc, code, params, e0, shot, trace, out):
    """Re-derive the event times and ringing checks from the Philox words with
    numpy's log, applying the traced flips."""
    H = code.H.to_dense()
    s = (H @ e0) % 2
    z = np.zeros_like(e0)
    nS = int(s.sum())
    T = 0.0
    for j, (t_ev, n_before, c, v) in enumerate(trace):
        w = orc.philox([shot & 0xFFFFFFFF, shot >> 32, j, 2],
                       [params.seed & 0xFFFFFFFF, params.seed >> 32])[0]
        u = (float(w[0]) + 1.0) / 2.0**32
        T = T + (-math.log(u)) / nS
        assert n_before == nS
        assert abs(t_ev - T) <= 1e-12 * max(T, 1.0), (j, t_ev, T)
        T = t_ev  # carry the oracle's own value forward (each step checked alone)
        active = np.nonzero(s)[0]
        idx = (int(w[1]) * nS) >> 32
        assert int(c) == int(active[idx]), (j, c, active[idx])
        if v >= 0:
            v = int(v)
            assert H[int(c), v] == 1
            z[v] ^= 1
            s = (s + H[:, v]) % 2
            nS = int(s.sum())
    assert np.array_equal(s, out["s"][0]) and np.array_equal(z, out["z"][0])
    if nS == 0:
        assert out["tclr"][0] == trace[-1][0]
    assert out["events"][0] == len(trace)


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_event_process_replays_from_the_random_words(orc, bp):
    """Gillespie bookkeeping: waiting time -ln((w0 + 1) 2^-32) / |S| with |S|
    after the previous event, ringing check = active check number
    floor(w1 |S| / 2^32), one Philox counter per event; the flipped qubit is
    a neighbour of the ringing check; t_clr is the clearing event's time."""
    for name, p in (("toric2d:6", 0.06), ("toric3d_point:3", 0.05), ("bb:6x6", 0.03)):
        code = codes.by_name(name)
        params = CP(bp=bp, dt=0.01, t_max=40, seed=7)
        for shot in (3, 11):
            e0 = orc.sample_noise(code, p, 0, shot, 1)
            out = orc.ctm_decode(code, params, e0, shot0=shot, trace_cap=100000)
            if out["events"][0] == 0:
                continue
            _replay(orc, code, params, e0[0], shot, out["trace"], out)


def test_first_waiting_time_is_exponential(orc):
    """The oracle's first event time T_0, times |S(0)|, is Exp(1) over many
    shots (Kolmogorov-Smirnov)."""
    from scipy import stats
    code = codes.by_name("toric2d:3")
    params = CP(dt=0.05, t_max=2.0, evidence=False)
    e0 = orc.sample_noise(code, 0.2, 0, 0, 1500)
    x = []
    for i in range(e0.shape[0]):
        out = orc.ctm_decode(code, params, e0[i:i + 1], shot0=i, trace_cap=1)
        if out["events"][0] > 0:
            x.append(out["trace"][0][0] * out["trace"][0][1])
    assert len(x) > 1000
    assert stats.kstest(x, "expon").pvalue > 1e-3


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_continuous_machine_invariants(orc, bp):
    """s = H (e0 ^ z) at the end; t_clr >= 0 exactly when s = 0; moves never
    exceed events; a clear start needs no event."""
    for name, p in (("toric2d:8", 0.05), ("toric3d_membrane:3", 0.05), ("rep:7", 0.2)):
        code = codes.by_name(name)
        e0 = orc.sample_noise(code, p, 0, 0, 48)
        e0[0] = 0
        out = orc.ctm_decode(code, CP(bp=bp, dt=0.01, t_max=30), e0, nthreads=4)
        s = orc.syndrome(code, e0 ^ out["z"])
        assert np.array_equal(s, out["s"])
        assert np.array_equal(out["tclr"] >= 0, s.sum(axis=1) == 0)
        assert np.all(out["moves"] <= out["events"])
        assert out["tclr"][0] == 0.0 and out["events"][0] == 0


def test_threads_do_not_change_results(orc):
    code = codes.by_name("toric2d:6")
    e0 = orc.sample_noise(code, 0.05, 0, 100, 24)
    params = CP(dt=0.01, t_max=20)
    a = orc.ctm_decode(code, params, e0, shot0=100, nthreads=1)
    b = orc.ctm_decode(code, params, e0, shot0=100, nthreads=6)
    for k in ("z", "s", "tclr", "events", "moves"):
        assert np.array_equal(a[k], b[k])
    one = orc.ctm_decode(code, params, e0[5:6], shot0=105)
    assert one["tclr"][0] == a["tclr"][5] and np.array_equal(one["z"][0], a["z"][5])


def test_sum_product_clears_every_2d_toric_shot(orc):
    """The paper reports that every 2D toric code syndrome clears under the
    continuous machine (SM, clearing-time histograms); below threshold the
    sum-product machine clears all of these shots, at two sizes."""
    for L in (8, 12):
        code = codes.toric_2d(L)
        e0 = orc.sample_noise(code, 0.03, 0, 0, 96)
        out = orc.ctm_decode(code, CP(bp="sumproduct", t_max=50), e0, nthreads=8)
        assert np.all(out["tclr"] >= 0)
        assert orc.logical_failure(code, e0, out["z"]).mean() <= 0.05


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_clock_decisions_follow_the_pinned_euler_state(orc, bp):
    """Until the first flip the syndrome is the initial one, so the BP state
    that event j sees is that of k Euler steps from zero, k the first step
    count with k dt >= T_j; the affine-recursion and tree pins above fix
    those steps. From that state, written out here: beliefs pi + sum of
    m_{c->v} (ascending c, clamped), Evidence max_{v in N(c)} L_v >=
    -log(d_c - 1), LocalMove the arg-max with ties split by word w2. Every
    traced decision up to and including the first flip must agree, which
    pins the decode path's own damping, step count and Evidence test."""
    checked = ev_yes = ev_no = 0
    for name, p in (("toric2d:6", 0.06), ("toric3d_point:3", 0.05), ("bb:6x6", 0.03)):
        code = codes.by_name(name)
        H = code.H.to_dense()
        rp, cl = code.H.rowptr, code.H.col
        params = CP(bp=bp, dt=0.01, tau=0.1, t_max=40, seed=3)
        thr = orc.evidence_thresholds(int(np.diff(rp).max()))
        pi = np.float32(math.log(params.q / (1 - params.q)))
        for shot in range(6):
            e0 = orc.sample_noise(code, p, 0, shot, 1)
            out = orc.ctm_decode(code, params, e0, shot0=shot, trace_cap=100000)
            s0 = (H @ e0[0]) % 2
            for j, (t_ev, _, c, v) in enumerate(out["trace"]):
                k = 0
                while k * params.dt < t_ev:
                    k += 1
                mcv, _ = orc.ctm_bp_steps(code, params, s0, k)
                c = int(c)
                nb = cl[rp[c]:rp[c + 1]]
                L = []
                for u in nb:
                    acc = pi
                    for c2 in np.nonzero(H[:, u])[0]:
                        e = rp[c2] + int(np.nonzero(cl[rp[c2]:rp[c2 + 1]] == u)[0][0])
                        acc = np.float32(acc + mcv[e])
                    L.append(np.float32(min(max(acc, -params.clamp), params.clamp)))
                Lmax = max(L)
                if Lmax >= thr[len(nb)]:
                    ev_yes += 1
                    ties = [u for u, x in zip(nb, L) if x == Lmax]
                    w2 = int(orc.philox([shot & 0xFFFFFFFF, shot >> 32, j, 2],
                                        [params.seed & 0xFFFFFFFF, params.seed >> 32])[0][2])
                    want = int(ties[(w2 * len(ties)) >> 32])
                else:
                    ev_no += 1
                    want = -1
                assert int(v) == want, (name, shot, j, k, L)
                checked += 1
                if want >= 0:
                    break
    assert checked >= 20 and ev_yes >= 5 and ev_no >= 5, (checked, ev_yes, ev_no)
