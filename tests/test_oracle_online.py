"""Pins of the oracle's online decoder (Discussion: new faults and syndrome
rounds keep arriving; the Tanner graph becomes a spacetime decoding graph,
and the local dynamics runs inside overlapping spacetime windows).

The reading pinned here: N syndrome rounds, new data errors before every
round and measurement errors on every round but the last; detectors
D_t = m_t ^ m_{t-1}; windows of W rounds of which the first C are
committed, the committed measurement corrections of a window's last
committed round carried into the next window's first detectors. Each part
is checked against something computed here without the oracle's online
code: the Philox words, a numpy construction of the spacetime graph, the
telescoping identity of the detectors, a numpy replay of the window and
commit bookkeeping, the reduction to the offline machine for one round, and
single faults that the machine must fix in place."""
import numpy as np
import pytest

from paper_2609_38139_amd import codes


def P(**kw):
    from oracle import oracle as O
    return O.DecodeParams(**kw)


def OP(**kw):
    from oracle import oracle as O
    return O.OnlineParams(**kw)


def spacetime_dense(H, w, w_eps):
    """The window's parity-check matrix built from H by blocks: rows are
    the detectors (tau, c); columns the data errors (tau, v) and then the
    measurement errors (tau, c) for tau < w_eps."""
    m, n = H.shape
    A = np.zeros((w * m, w * n + w_eps * m), dtype=np.uint8)
    for tau in range(w):
        A[tau * m:(tau + 1) * m, tau * n:(tau + 1) * n] = H
        if tau < w_eps:
            A[tau * m:(tau + 1) * m, w * n + tau * m: w * n + (tau + 1) * m] = np.eye(m, dtype=np.uint8)
        if tau >= 1 and tau - 1 < w_eps:
            A[tau * m:(tau + 1) * m, w * n + (tau - 1) * m: w * n + tau * m] = np.eye(m, dtype=np.uint8)
    return A


def detectors(H, e, eps):
    """D_t = H e_t ^ eps_t ^ eps_{t-1} for one shot (e [N, n], eps [N, m])."""
    D = (e.astype(np.int64) @ H.T.astype(np.int64)) % 2
    D ^= eps
    D[1:] ^= eps[:-1]
    return D.astype(np.uint8)


def test_noise_words_rates_and_perfect_last_round(orc):
    c = codes.toric_2d(6)
    n, m = c.n, c.m
    op = OP(rounds_total=5, window=3, commit=2, p=0.07, p_meas=0.11)
    e, eps = orc.online_noise(c, op, 9, 100, 400)
    assert not eps[:, -1].any()  # the last round is perfect
    # rates
    for a, rate in ((e, 0.07), (eps[:, :-1], 0.11)):
        assert abs(a.mean() - rate) < 5 * np.sqrt(rate * (1 - rate) / a.size)
    # words: e_t[v] is word v mod 4 of Philox(seed, (shot, v/4, 16 t + 3)),
    # eps_t[c] word c mod 4 of Philox(seed, (shot, c/4, 16 t + 4))
    bd, bm = orc.bernoulli_bound(0.07), orc.bernoulli_bound(0.11)
    for shot, t, v in ((100, 1, 5), (101, 3, 17), (499, 5, n - 1)):
        w = orc.philox([shot, 0, v // 4, 16 * t + 3], [9, 0])[0]
        assert e[shot - 100, t - 1, v] == int(int(w[v % 4]) < bd)
    for shot, t, ch in ((100, 1, 2), (250, 4, m - 1)):
        w = orc.philox([shot, 0, ch // 4, 16 * t + 4], [9, 0])[0]
        assert eps[shot - 100, t - 1, ch] == int(int(w[ch % 4]) < bm)
    # shot ids address the streams
    e2, eps2 = orc.online_noise(c, op, 9, 117, 3)
    assert np.array_equal(e2, e[17:20]) and np.array_equal(eps2, eps[17:20])


@pytest.mark.parametrize("name", ["toric2d:4", "bb:6x6", "toric3d_point:3"])
@pytest.mark.parametrize("w,w_eps", [(1, 0), (3, 3), (3, 2), (4, 4)])
def test_window_code_is_the_spacetime_graph(orc, name, w, w_eps):
    """The oracle's window CSR equals the block construction from H: each
    detector holds its round's data errors and the measurement errors of
    its own and the previous round."""
    c = codes.by_name(name)
    H = c.H.to_dense()
    rp, cl, nv = orc.window_code(c, w, w_eps)
    A = spacetime_dense(H, w, w_eps)
    assert nv == A.shape[1]
    B = np.zeros_like(A)
    for r in range(A.shape[0]):
        cols = cl[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cols) > 0)
        B[r, cols] = 1
    assert np.array_equal(A, B)


def test_detectors_telescope_to_the_final_syndrome():
    """Sum over t of D_t = H E_N with a perfect last round (the identity the
    windows rely on to explain every detector by a final correction)."""
    from oracle import oracle as O
    c = codes.bivariate_bicycle(6, 6)
    H = c.H.to_dense()
    op = OP(rounds_total=6, window=3, commit=1, p=0.05, p_meas=0.08)
    e, eps = O.online_noise(c, op, 1, 0, 50)
    for i in range(50):
        D = detectors(H, e[i], eps[i])
        E = np.bitwise_xor.reduce(e[i], axis=0)
        assert np.array_equal(np.bitwise_xor.reduce(D, axis=0), (H.astype(np.int64) @ E) % 2)


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
@pytest.mark.parametrize("name,N,W,C", [("toric2d:4", 7, 3, 2), ("toric2d:5", 6, 4, 1), ("bb:6x6", 5, 2, 2),
                                        ("toric3d_point:3", 4, 3, 3)])
def test_windows_and_commits_replay(orc, bp, name, N, W, C):
    """Every window of a run re-derived here: its syndrome from the detectors
    (computed from the sampled errors) with the carried measurement
    correction on its first round, its correction from the round machine on
    that window's graph (built here by blocks) with rounds numbered from
    k R, the commit of its first C rounds (all rounds in the last window),
    the carried correction, the final z, E_N and the failure flag."""
    c = codes.by_name(name)
    H = c.H.to_dense()
    n, m = c.n, c.m
    R = 6
    prm = P(bp=bp, rounds=R, iters=5, seed=3)
    op = OP(rounds_total=N, window=W, commit=C, p=0.04, p_meas=0.06)
    nwin, w_last = op.layout()
    e, eps = orc.online_noise(c, op, 3, 0, 6)
    for shot in range(6):
        out = orc.online_decode(c, prm, op, shot0=shot, nshots=1, trace=True)
        D = detectors(H, e[shot], eps[shot])
        bnd = np.zeros(m, dtype=np.uint8)
        z = np.zeros(n, dtype=np.uint8)
        cleared = 0
        for k in range(nwin):
            last = k == nwin - 1
            w = w_last if last else W
            w_eps = w - 1 if last else w
            sw = D[k * C:k * C + w].copy()
            sw[0] ^= bnd
            sw = sw.ravel()
            assert np.array_equal(out["trace_s"][k][:w * m], sw), (shot, k)
            A = spacetime_dense(H, w, w_eps)
            Hw = codes.CSR.from_dense(A)
            r = orc.decode_syndrome(Hw, prm, sw, shot0=shot, r0=k * R)
            zw = r["z"][0]
            assert np.array_equal(out["trace_z"][k][:A.shape[1]], zw), (shot, k)
            cleared += int(r["tclr"][0] >= 0)
            cr = w if last else C
            for tau in range(cr):
                z ^= zw[tau * n:(tau + 1) * n]
            if not last:
                bnd = zw[w * n + (cr - 1) * m: w * n + cr * m].copy()
        assert np.array_equal(out["z"][0], z), shot
        assert np.array_equal(out["E"][0], np.bitwise_xor.reduce(e[shot], axis=0)), shot
        assert out["cleared"][0] == cleared
        assert out["fail"][0] == orc.logical_failure(c, out["E"], out["z"])[0]
        if cleared == nwin:  # every detector explained: the residual has no syndrome
            resid = out["E"][0] ^ out["z"][0]
            assert not ((H.astype(np.int64) @ resid) % 2).any(), shot


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_one_round_is_the_offline_machine(orc, bp):
    """With one (perfect) round there are no measurement errors and one
    window: the online decoder is the offline machine on e_1."""
    c = codes.toric_2d(6)
    op = OP(rounds_total=1, window=3, commit=2, p=0.06, p_meas=0.2)
    prm = P(bp=bp, rounds=24, seed=5)
    out = orc.online_decode(c, prm, op, shot0=10, nshots=80, nthreads=4)
    e, _ = orc.online_noise(c, op, 5, 10, 80)
    ref = orc.decode(c, prm, e[:, 0], shot0=10, nthreads=4)
    assert np.array_equal(out["z"], ref["z"])
    assert np.array_equal(out["cleared"], (ref["tclr"] >= 0).astype(np.int32))
    assert np.array_equal(out["fail"], orc.logical_failure(c, e[:, 0], ref["z"]))


def test_one_window_is_one_spacetime_decode(orc):
    """A window covering every round: the online correction is the data part
    of the offline machine run on the spacetime graph (built here by blocks)
    with the spacetime error as its initial error, summed over rounds."""
    c = codes.toric_2d(4)
    H = c.H.to_dense()
    n, m = c.n, c.m
    N = 4
    op = OP(rounds_total=N, window=N, commit=2, p=0.05, p_meas=0.05)
    prm = P(bp="sumproduct", rounds=20, seed=2)
    out = orc.online_decode(c, prm, op, shot0=0, nshots=40, nthreads=4)
    e, eps = orc.online_noise(c, op, 2, 0, 40)
    A = spacetime_dense(H, N, N - 1)
    spec = codes.Code(name="spacetime", H=codes.CSR.from_dense(A), G=codes.CSR.from_rows(0, A.shape[1], []))
    x = np.concatenate([e.reshape(40, N * n), eps[:, :N - 1].reshape(40, (N - 1) * m)], axis=1)
    ref = orc.decode(spec, prm, x, shot0=0, nthreads=4)
    zd = np.bitwise_xor.reduce(ref["z"][:, :N * n].reshape(40, N, n), axis=1)
    assert np.array_equal(out["z"], zd)


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5])
def test_single_measurement_error_is_fixed_in_time(orc, t):
    """One measurement error and nothing else lights two detectors of one
    check at rounds t and t + 1; with every clock ringing, both checks pick
    the measurement variable they share -- or, at the top of a window, the
    lone measurement variable there -- so nothing is flipped on the data and
    the shot does not fail."""
    c = codes.toric_2d(5)
    n, m = c.n, c.m
    N = 6
    op = OP(rounds_total=N, window=3, commit=2, p=0.0, p_meas=0.0)
    prm = P(bp="sumproduct", rounds=8, mask_density=1.0)
    e = np.zeros((1, N, n), dtype=np.uint8)
    eps = np.zeros((1, N, m), dtype=np.uint8)
    eps[0, t - 1, 7] = 1
    out = orc.online_decode(c, prm, op, nshots=1, e_in=e, eps_in=eps)
    assert not out["z"].any() and not out["E"].any() and out["fail"][0] == 0
    assert out["cleared"][0] == out["windows"]


@pytest.mark.parametrize("t", [1, 3, 6])
def test_single_data_error_is_corrected(orc, t):
    """One data error in round t: two detectors of that round; the machine
    flips the shared qubit, which z records, and the shot succeeds."""
    c = codes.toric_2d(5)
    n, m = c.n, c.m
    N = 6
    op = OP(rounds_total=N, window=3, commit=2, p=0.0, p_meas=0.0)
    prm = P(bp="sumproduct", rounds=8, mask_density=1.0)
    e = np.zeros((1, N, n), dtype=np.uint8)
    e[0, t - 1, 11] = 1
    eps = np.zeros((1, N, m), dtype=np.uint8)
    out = orc.online_decode(c, prm, op, nshots=1, e_in=e, eps_in=eps)
    assert np.array_equal(out["z"][0], e[0, t - 1]) and out["fail"][0] == 0


def test_windows_cover_every_round(orc):
    """The layout: window k starts at round k C + 1, the last is the first
    to reach round N, and every round is committed exactly once."""
    for N in range(1, 12):
        for W in range(1, 6):
            for C in range(1, W + 1):
                op = OP(rounds_total=N, window=W, commit=C)
                nwin, w_last = op.layout()
                starts = [k * C for k in range(nwin)]
                assert starts[-1] + w_last == N and 1 <= w_last <= W
                assert all(s + W < N for s in starts[:-1])
                committed = [r for k, s in enumerate(starts) for r in range(s, s + (w_last if k == nwin - 1 else C))]
                assert committed == list(range(N)), (N, W, C)
