"""Pins of the oracle's method against what the paper and the mathematics fix.

Every test here runs on the CPU and checks the oracle against something other
than its own code: closed forms (the repetition-code window lemma, the exact
posterior of an open chain), brute-force marginals (BP is exact on trees),
exact symmetries (gauge covariance), the code parameters the paper states,
invariants of the dynamics (syndrome identity, defect-parity conservation,
homology classes, early exit), and special cases of Algorithm 1.
"""
import itertools

import numpy as np
import pytest

from paper_2609_38139_amd import codes


def P(**kw):
    from oracle import oracle as O
    return O.DecodeParams(**kw)


# ----------------------------------------------------------------- helpers
def gf2_nullspace(A):
    """Basis of {x : A x = 0 mod 2} (rows), by plain Gaussian elimination."""
    A = (np.array(A, dtype=np.uint8) & 1).copy()
    m, n = A.shape
    piv_cols, r = [], 0
    for c in range(n):
        rows = np.nonzero(A[r:, c])[0]
        if len(rows) == 0:
            continue
        p = r + rows[0]
        A[[r, p]] = A[[p, r]]
        for i in range(m):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        piv_cols.append(c)
        r += 1
        if r == m:
            break
    free = [c for c in range(n) if c not in piv_cols]
    basis = []
    for f in free:
        x = np.zeros(n, dtype=np.uint8)
        x[f] = 1
        for i, c in enumerate(piv_cols):
            x[c] = A[i, f]
        basis.append(x)
    return np.array(basis, dtype=np.uint8).reshape(-1, n)


def exact_llr(H, q, s):
    """log Pr(e_v=1|s)/Pr(e_v=0|s) by enumerating every error with H e = s."""
    m, n = H.shape
    allE = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint8)
    ok = ((allE @ H.T) % 2 == s).all(1)
    E = allE[ok].astype(np.float64)
    w = E.sum(1)
    logw = w * np.log(q) + (n - w) * np.log(1 - q)
    mx = logw.max()
    pw = np.exp(logw - mx)
    p1 = (pw[:, None] * E).sum(0)
    p0 = (pw[:, None] * (1 - E)).sum(0)
    return np.log(p1) - np.log(p0)


def random_tree_code(rng, nmax=13):
    """A random tree-shaped Tanner graph with check degrees 2..6 (and the
    occasional degree-1 check), qubits of varying degree."""
    n = 1
    rows = []
    while n < nmax:
        d = int(rng.integers(1, 6))  # new qubits attached by this check
        d = min(d, nmax - n)
        anchor = int(rng.integers(0, n))
        rows.append([anchor] + list(range(n, n + d)))
        n += d
    if rng.random() < 0.3:
        rows.append([int(rng.integers(0, n))])  # a degree-1 check
    H = np.zeros((len(rows), n), dtype=np.uint8)
    for i, r in enumerate(rows):
        H[i, r] = 1
    return H


# ------------------------------------------------------------ BP closed forms
@pytest.mark.parametrize("bp,alpha", [("minsum", 0.75), ("minsum", 1.0), ("minsum", 0.5), ("sumproduct", 0.75)])
def test_rep_code_window_beliefs(orc, bp, alpha):
    """Periodic odd-d repetition code at a fixed syndrome (SM, window lemma):
    after t two-phase sweeps from m = 0, L_v = pi sigma_v sum_{|u-v|<=t-1}
    w^{|u-v|} sigma_u with sigma = (-1)^{e0} and w = alpha (min-sum) or 1
    (sum-product: a degree-2 check copies its other input), while the window
    does not wrap."""
    d = 21
    c = codes.repetition(d)
    q = 0.1
    pi = np.log(q / (1 - q))
    rng = np.random.default_rng(3)
    w = 1.0 if bp == "sumproduct" else alpha
    for t in range(1, (d + 1) // 2 + 1):
        e0 = (rng.random((4, d)) < 0.3).astype(np.uint8)
        r = orc.decode(c, P(bp=bp, alpha=alpha, q=q, iters=t, rounds=1, retire=False, mask_density=0.0),
                       e0, want_beliefs=True)
        sig = 1 - 2 * e0.astype(np.float64)
        for k in range(4):
            exp = np.array([pi * sig[k, v] * sum(w ** abs(o) * sig[k, (v + o) % d] for o in range(-(t - 1), t))
                            for v in range(d)])
            assert np.allclose(r["L"][k], exp, rtol=2e-6, atol=1e-6), (t, k)


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_open_chain_exact_posterior(orc, bp):
    """Open chain (a tree): the two consistent errors are e0 and its
    complement, so L_v = pi sigma_v (n - 2|E|); BP reaches it (min-sum with
    alpha = 1 coincides with sum-product on degree-2 checks)."""
    n = 15
    c = codes.repetition(n, periodic=False)
    q = 0.05
    pi = np.log(q / (1 - q))
    rng = np.random.default_rng(4)
    e0 = (rng.random((20, n)) < 0.3).astype(np.uint8)
    r = orc.decode(c, P(bp=bp, alpha=1.0, q=q, iters=n, rounds=1, retire=False, mask_density=0.0),
                   e0, want_beliefs=True)
    sig = 1 - 2 * e0.astype(np.float64)
    exp = pi * sig * (n - 2 * e0.sum(1, keepdims=True))
    assert np.allclose(r["L"], exp, rtol=1e-5, atol=1e-5)


def test_sum_product_exact_on_trees(orc):
    """BP is exact on trees (Preliminaries): sum-product beliefs after enough
    sweeps equal brute-force posterior log-odds, on random trees with odd and
    even check degrees (which exercises the (-1)^{s_c + d_c} sign)."""
    from paper_2609_38139_amd.codes import from_dense
    rng = np.random.default_rng(11)
    for trial in range(12):
        H = random_tree_code(rng)
        n = H.shape[1]
        q = float(rng.uniform(0.1, 0.35))
        e0 = (rng.random(n) < 0.3).astype(np.uint8)
        s = (H @ e0) % 2
        code = from_dense(H)
        r = orc.decode(code, P(bp="sumproduct", q=q, iters=2 * n + 2, rounds=1, retire=False,
                               mask_density=0.0), e0[None], want_beliefs=True)
        with np.errstate(divide="ignore"):
            ex = exact_llr(H, q, s)
        # a degree-1 check fixes its qubit, and parity checks carry that
        # certainty on (exact LLR +-inf); clamped BP sends +-CLAMP and each
        # hop adds a prior: compare sign and size there
        pinned = ~np.isfinite(ex)
        got = r["L"][0]
        assert np.all(np.sign(got[pinned]) == np.sign(ex[pinned])) and np.all(np.abs(got[pinned]) > 900)
        assert np.allclose(got[~pinned], ex[~pinned], rtol=1e-5, atol=1e-5), (trial, got, ex)


def test_min_sum_is_not_exact_but_sign_correct_on_star(orc):
    """A single degree-4 check with s = 1 (a star, so a tree): sum-product gives
    the exact posterior; normalised min-sum gives alpha * min |m| with the
    same signs. Pins the min-sum rule's scale and sign separately."""
    from paper_2609_38139_amd.codes import from_dense
    H = np.ones((1, 4), dtype=np.uint8)
    q = 0.05
    pi = np.float32(np.log(q / (1 - q)))
    e0 = np.array([[1, 0, 0, 0]], dtype=np.uint8)
    rm = orc.decode(from_dense(H), P(bp="minsum", alpha=0.75, q=q, iters=2, rounds=1, retire=False,
                                     mask_density=0.0), e0, want_beliefs=True)
    # inputs pi (negative) x3; sigma = (-1)^{1+4} = -1; product of signs -1 -> +alpha |pi|
    assert np.all(rm["L"][0] == np.float32(pi + np.float32(np.float32(0.75) * np.float32(-pi))))
    rs = orc.decode(from_dense(H), P(bp="sumproduct", q=q, iters=2, rounds=1, retire=False,
                                     mask_density=0.0), e0, want_beliefs=True)
    assert np.allclose(rs["L"][0], exact_llr(H, q, np.array([1])), rtol=1e-6)


# -------------------------------------------------- bit-centric machine (SM)
def test_bitcentric_window_majority_and_threshold(orc):
    """Discrete machine on the periodic odd-d repetition code (SM, window
    lemma and theorem): after iteration i, e_v = 1 iff |E n W_v^(i)| > k_i/2
    with r_i = floor((i-1)/2), k_i = 2 r_i + 1; the run fails exactly when
    |E| > d/2; beliefs are pi sigma_v M_v times (-1)^{z}."""
    rng = np.random.default_rng(5)
    q = 0.1
    for d in (11, 21, 31):
        c = codes.repetition(d)
        for shot in range(60):
            p = rng.uniform(0.05, 0.45)
            e0 = (rng.random(d) < p).astype(np.uint8)
            et, Lt, iclr = orc.bitcentric_machine(c, q, e0, d)
            for i in range(1, d + 1):
                ri = (i - 1) // 2
                ki = 2 * ri + 1
                cnt = np.array([sum(e0[(v + o) % d] for o in range(-ri, ri + 1)) for v in range(d)])
                assert np.array_equal(et[i - 1], (cnt > ki / 2).astype(np.uint8)), (d, shot, i)
            final = et[d - 1]
            fails = bool(final.any())
            assert fails == (e0.sum() > d / 2)
            if not fails and e0.any():
                assert iclr >= 1 and not et[iclr - 1].any()


def test_bitcentric_ler_is_binomial_tail(orc):
    """Failure iff |E| > d/2, so over shots the LER is the binomial tail."""
    from scipy.stats import binom
    d, p, S = 11, 0.35, 400
    c = codes.repetition(d)
    e0 = orc.sample_noise(c, p, 1, 0, S)
    fails = 0
    for k in range(S):
        et, _, _ = orc.bitcentric_machine(c, 0.1, e0[k], d)
        fails += int(et[-1].any())
    assert fails == int((e0.sum(1) > d / 2).sum())
    tail = binom.sf(d // 2, d, p)
    assert abs(fails / S - tail) < 5 * np.sqrt(tail * (1 - tail) / S)


# ----------------------------------------------------------- symmetries
@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
@pytest.mark.parametrize("name", ["toric2d:4", "bb:6x6", "toric3d_membrane:2"])
def test_gauge_covariance(orc, bp, name):
    """F_BP(G_g m; s + H g; G_g pi) = G_g F_BP(m; s; pi) (SM, proposition on
    gauge covariance), exactly in FP32 for one full sweep."""
    c = codes.by_name(name)
    H = c.H.to_dense()
    rng = np.random.default_rng(12)
    E = c.H.nnz
    edge_v = c.H.col
    for trial in range(5):
        pi = np.full(c.n, np.log(0.05 / 0.95), dtype=np.float32)
        mvc = (rng.standard_normal(E) * 5).astype(np.float32)
        s = rng.integers(0, 2, c.m).astype(np.uint8)
        g = rng.integers(0, 2, c.n).astype(np.uint8)
        sign_v = np.where(g == 1, -1.0, 1.0).astype(np.float32)
        prm = P(bp=bp)
        mcv1, mvc1 = orc.bp_sweep(c, prm, pi, s, mvc)
        s2 = (s + H @ g) % 2
        mcv2, mvc2 = orc.bp_sweep(c, prm, pi * sign_v, s2.astype(np.uint8), mvc * sign_v[edge_v])
        assert np.array_equal(mcv2, mcv1 * sign_v[edge_v])
        assert np.array_equal(mvc2, mvc1 * sign_v[edge_v])


def test_evidence_union_bound_exact_marginals(orc):
    """For an active check, sum_{v in N(c)} Pr(e_v = 1 | s) >= 1, so the
    largest exact marginal is >= 1/d_c (Evidence); the FP32 thresholds
    decide sigmoid(L) >= 1/d_c correctly on the exact LLRs."""
    c = codes.toric_2d(3)
    H = c.H.to_dense()
    q = 0.05
    thr = orc.evidence_thresholds(4)
    rng = np.random.default_rng(9)
    for trial in range(6):
        e0 = (rng.random(c.n) < 0.15).astype(np.uint8)
        s = (H @ e0) % 2
        L = exact_llr(H, q, s)
        pr = 1 / (1 + np.exp(-L))
        for ch in np.nonzero(s)[0]:
            nb = np.nonzero(H[ch])[0]
            assert pr[nb].sum() >= 1 - 1e-12
            assert pr[nb].max() >= 1 / 4 - 1e-12
            Lmax = L[nb].max()
            if abs(1 / (1 + np.exp(-Lmax)) - 0.25) > 1e-6:
                assert (np.float32(Lmax) >= thr[4]) == (1 / (1 + np.exp(-Lmax)) >= 0.25)


def test_tensor_network_contraction_equals_partition_function():
    """Z_TN(s) = Pr(s) (SM, proposition), and sum_s Pr(s) = 1, on a tiny code:
    contracts the check and data tensors over the virtual edge indices."""
    c = codes.toric_2d(2)
    H = c.H.to_dense()
    m, n = H.shape
    q = 0.13
    edges = [(ci, v) for ci in range(m) for v in np.nonzero(H[ci])[0]]
    allE = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint8)
    synd = (allE @ H.T) % 2
    w = allE.sum(1)
    prob = q ** w * (1 - q) ** (n - w)
    total = 0.0
    for s in {tuple(x) for x in synd}:
        s = np.array(s)
        direct = prob[(synd == s).all(1)].sum()
        # contraction: sum over virtual indices x_e of prod_c T * prod_v D
        Z = 0.0
        for x in itertools.product([0, 1], repeat=len(edges)):
            x = np.array(x)
            okc = all((x[[k for k, (ci, _) in enumerate(edges) if ci == cc]].sum() % 2) == s[cc] for cc in range(m))
            if not okc:
                continue
            term = 1.0
            for v in range(n):
                xs = x[[k for k, (_, vv) in enumerate(edges) if vv == v]]
                term *= (1 - q) * float(np.all(xs == 0)) + q * float(np.all(xs == 1))
            Z += term
        assert abs(Z - direct) < 1e-12
        total += direct
    assert abs(total - 1.0) < 1e-12


# -------------------------------------------------------- code parameters
@pytest.mark.parametrize("name,k,rank_h", [
    ("toric2d:3", 2, 8), ("toric2d:8", 2, 63), ("toric3d_point:3", 3, 26),
    ("toric3d_membrane:3", 3, None), ("bb:6x6", 12, 30), ("bb:12x6", 12, 66), ("rep:9", 1, 8)])
def test_code_parameters(orc, name, k, rank_h):
    """H G^T = 0 and k = n - rank H - rank G: the [[72,12,6]] and [[144,12,12]]
    bivariate-bicycle codes, k = 2 (2D toric), k = 3 (3D toric), k = 1 (rep)."""
    c = codes.by_name(name)
    if c.G.rows:
        assert not ((c.H.to_dense().astype(np.int64) @ c.G.to_dense().T) % 2).any()
    rh, rg = orc.gf2_rank(c.H), orc.gf2_rank(c.G)
    assert c.n - rh - rg == k
    if rank_h is not None:
        assert rh == rank_h


def test_generators_match_lattice_construction():
    """The group-algebra 2D toric code equals the lattice picture: vertex
    checks, plaquette stabilisers, A-block edge (a, b) joining vertices
    (a-1, b) and (a, b), B-block edge joining (a, b-1) and (a, b)."""
    for L in (3, 5, 8):
        c = codes.toric_2d(L)
        n = 2 * L * L
        A = lambda a, b: (a % L) * L + (b % L)
        B = lambda a, b: L * L + (a % L) * L + (b % L)
        H = np.zeros((L * L, n), dtype=np.uint8)
        G = np.zeros((L * L, n), dtype=np.uint8)
        for a in range(L):
            for b in range(L):
                for e in (A(a, b), A(a + 1, b), B(a, b), B(a, b + 1)):
                    H[a * L + b, e] ^= 1
                for e in (A(a, b), A(a, b - 1), B(a, b), B(a - 1, b)):
                    G[a * L + b, e] ^= 1
        assert np.array_equal(c.H.to_dense(), H)
        assert np.array_equal(c.G.to_dense(), G)


def test_3d_membrane_meta_checks():
    """Membrane sector: the six faces of every cube sum to zero (the cube
    meta-checks), so any syndrome has even parity on every cube."""
    L = 3
    c = codes.toric_3d_membrane(L)
    H = c.H.to_dense()
    L3 = L ** 3
    for z in range(L):
        for y in range(L):
            for x in range(L):
                v = x + L * (y + L * z)
                nx = (x + 1) % L + L * (y + L * z)
                ny = x + L * ((y + 1) % L + L * z)
                nz = x + L * (y + L * ((z + 1) % L))
                faces = [0 * L3 + v, 0 * L3 + nz, 1 * L3 + v, 1 * L3 + ny, 2 * L3 + v, 2 * L3 + nx]
                assert not (H[faces].sum(0) % 2).any()


# ------------------------------------------------------ dynamics invariants
@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
@pytest.mark.parametrize("name,p", [("toric2d:6", 0.08), ("bb:6x6", 0.03), ("toric3d_membrane:3", 0.06),
                                    ("toric3d_point:3", 0.03)])
def test_syndrome_identity_and_defect_parity(orc, bp, name, p):
    """After every round s = H (e0 + z) (the syndrome update of Algorithm 1),
    so s stays orthogonal to the left kernel of H (defect-parity
    conservation; e.g. an even number of defects on the 2D toric code)."""
    c = codes.by_name(name)
    H = c.H.to_dense()
    meta = gf2_nullspace(H.T)
    prm = P(bp=bp, rounds=12, retire=False, q=0.125 if "membrane" in name else 0.05)
    e0 = orc.sample_noise(c, p, 2, 0, 6)
    for k in range(6):
        r = orc.decode(c, prm, e0[k:k + 1], shot0=k, trace=True)
        for rr in range(prm.rounds):
            s = r["s_trace"][rr]
            assert np.array_equal(s, (H @ (e0[k] ^ r["z_trace"][rr])) % 2)
            assert not ((meta @ s) % 2).any()


def test_homology_classes_2d_toric_l3(orc):
    """On the L = 3 toric code the 2^10 vectors of ker H split into 2^k = 4
    classes of 2^rank(G) = 256 (Preliminaries, condition (2)); the oracle's
    success test accepts exactly the trivial class."""
    c = codes.toric_2d(3)
    H = c.H.to_dense()
    K = gf2_nullspace(H)
    assert K.shape[0] == 10
    vecs = np.array([(np.array(bits) @ K) % 2 for bits in itertools.product([0, 1], repeat=10)], dtype=np.uint8)
    zeros = np.zeros_like(vecs)
    fail = orc.logical_failure(c, vecs, zeros)
    assert int((fail == 0).sum()) == 256
    # a class is a coset of row(G): pick one vector per class and count
    G = c.G.to_dense()
    classes = {}
    for v, f in zip(vecs, fail):
        key = None
        for rep in classes:
            if orc.logical_failure(c, (v ^ np.array(rep))[None], zeros[:1])[0] == 0:
                key = rep
                break
        if key is None:
            classes[tuple(v)] = 1
        else:
            classes[key] += 1
    assert sorted(classes.values()) == [256, 256, 256, 256]
    assert G.shape == (9, 18)


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_special_cases(orc, bp):
    """No error: t_clr = 0, no flips, success. A non-contractible loop:
    s = 0, t_clr = 0, failure. A single error with every clock ringing:
    both endpoint checks pick the shared qubit, one flip, cleared in round 1."""
    L = 8
    c = codes.toric_2d(L)
    prm = P(bp=bp, rounds=8, mask_density=1.0)
    e = np.zeros((1, c.n), dtype=np.uint8)
    r = orc.decode(c, prm, e)
    assert r["tclr"][0] == 0 and not r["z"].any() and orc.logical_failure(c, e, r["z"])[0] == 0
    loop = np.zeros((1, c.n), dtype=np.uint8)
    loop[0, [a * L + 3 for a in range(L)]] = 1  # A-block edges (a, 3), a = 0..L-1
    r = orc.decode(c, prm, loop)
    assert r["tclr"][0] == 0 and not r["s"].any() and orc.logical_failure(c, loop, r["z"])[0] == 1
    for q in (5, 77, 100):
        one = np.zeros((1, c.n), dtype=np.uint8)
        one[0, q] = 1
        r = orc.decode(c, prm, one)
        assert r["tclr"][0] == 1 and np.array_equal(r["z"], one)


@pytest.mark.parametrize("move", ["single", "multi"])
@pytest.mark.parametrize("conflict", ["or", "xor"])
@pytest.mark.parametrize("bp,rho", [("minsum", 0.5), ("sumproduct", 1.0), ("minsum", 0.125)])
def test_feedback_replays_from_beliefs_and_random_words(orc, bp, rho, conflict, move):
    """The feedback step of every round, re-derived here (Algorithm 1 with one
    Philox draw per check and round): check c rings when word 0 of
    Philox(seed, (shot_lo, shot_hi, c, 16 r + 1)) is below floor(rho 2^32);
    an active ringing check has Evidence when max_{v in N(c)} L_v >=
    -log(d_c - 1) and then asks for the arg-max qubit, ties split by word 1;
    the requests combine by OR or XOR. The beliefs L of round r come from a
    run stopped after r + 1 rounds (without the gauge option the state is
    not touched after the feedback), the window and tree pins above fix BP
    itself, and the traced z of successive rounds give the flips f.
    With multi-qubit moves an acting check asks instead for every qubit of
    N(c) with L_v > 0 (Pr_BP(e_v = 1 | s) > 1/2), or for the arg-max qubit
    when there is none."""
    checked = asked = multi = 0
    for name, p in (("toric2d:6", 0.08), ("bb:6x6", 0.04), ("toric3d_point:3", 0.04)):
        c = codes.by_name(name)
        H = c.H.to_dense()
        rp, cl = c.H.rowptr, c.H.col
        thr = orc.evidence_thresholds(int(np.diff(rp).max()))
        bound = orc.bernoulli_bound(rho)
        prm = dict(bp=bp, mask_density=rho, conflict=conflict, retire=False, seed=11, iters=6, move=move)
        R = 6
        for shot in range(3):
            e0 = orc.sample_noise(c, p, 0, shot, 1)
            tr = orc.decode(c, P(rounds=R, **prm), e0, shot0=shot, trace=True)
            s_r = (H @ e0[0]) % 2
            z_prev = np.zeros(c.n, dtype=np.uint8)
            for r in range(R):
                L = orc.decode(c, P(rounds=r + 1, **prm), e0, shot0=shot, want_beliefs=True)["L"][0]
                cnt = np.zeros(c.n, dtype=np.int64)
                for ch in np.nonzero(s_r)[0]:
                    w = orc.philox([shot, 0, int(ch), 16 * r + 1], [prm["seed"], 0])[0]
                    if int(w[0]) >= bound:
                        continue
                    nb = cl[rp[ch]:rp[ch + 1]]
                    Lmax = L[nb].max()
                    if not Lmax >= thr[len(nb)]:
                        continue
                    pos = nb[L[nb] > 0]
                    if move == "multi" and len(pos):
                        cnt[pos] += 1
                        multi += len(pos) > 1
                    else:
                        ties = nb[L[nb] == Lmax]
                        cnt[ties[(int(w[1]) * len(ties)) >> 32]] += 1
                    asked += 1
                f = (cnt > 0) if conflict == "or" else (cnt % 2 == 1)
                assert np.array_equal(tr["z_trace"][r] ^ z_prev, f.astype(np.uint8)), (name, shot, r)
                z_prev = tr["z_trace"][r]
                s_r = tr["s_trace"][r]
                checked += 1
    assert checked == 3 * 3 * 6 and asked >= 20, asked
    if move == "multi" and bp == "sumproduct":  # min-sum beliefs are rarely positive here
        assert multi >= 1, "no check asked for more than one qubit"


@pytest.mark.parametrize("name", ["toric2d:6", "bb:6x6", "toric3d_point:3"])
def test_multi_qubit_move_without_positive_beliefs_is_localmove(orc, name):
    """A multi-qubit move asks for the qubits of N(c) with L_v > 0 and falls
    back to LocalMove when there is none. With prior q = 1/2 (pi = 0) and no
    BP sweep every belief is exactly +0, so every move is the LocalMove:
    the two kinds of move give identical runs, which still correct."""
    c = codes.by_name(name)
    e0 = orc.sample_noise(c, 0.05, 0, 0, 60)
    kw = dict(q=0.5, iters=0, rounds=12, retire=False)
    a = orc.decode(c, P(move="single", **kw), e0, nthreads=4, want_beliefs=True)
    b = orc.decode(c, P(move="multi", **kw), e0, nthreads=4)
    assert not a["L"].any() and not np.signbit(a["L"]).any()
    for k in ("z", "s", "tclr"):
        assert np.array_equal(a[k], b[k]), k
    assert a["z"].any()


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_retire_equals_fixed_rounds(orc, bp):
    """Once s = 0 no check is active, so stopping a shot early changes none
    of z, s, t_clr (Algorithm 1 acts only on checks in S(t))."""
    c = codes.toric_2d(8)
    e0 = orc.sample_noise(c, 0.06, 0, 0, 200)
    a = orc.decode(c, P(bp=bp, rounds=32, retire=True), e0, nthreads=4)
    b = orc.decode(c, P(bp=bp, rounds=32, retire=False), e0, nthreads=4)
    for k in ("z", "s", "tclr"):
        assert np.array_equal(a[k], b[k])


def test_threads_and_batching_do_not_change_results(orc):
    c = codes.bivariate_bicycle(6, 6)
    e0 = orc.sample_noise(c, 0.04, 0, 100, 64)
    prm = P(rounds=16)
    a = orc.decode(c, prm, e0, shot0=100, nthreads=1)
    b = orc.decode(c, prm, e0, shot0=100, nthreads=8)
    d = orc.decode(c, prm, e0[10:20], shot0=110, nthreads=2)
    for k in ("z", "s", "tclr"):
        assert np.array_equal(a[k], b[k])
        assert np.array_equal(a[k][10:20], d[k])


def test_sum_product_ler_falls_with_size(orc):
    """Loose statistical sanity (sum-product): below threshold the failure
    rate drops from L = 8 to L = 16 (the round machine's rates have no
    published counterpart; this only checks the trend)."""
    rates = {}
    for L in (8, 16):
        c = codes.toric_2d(L)
        e0 = orc.sample_noise(c, 0.04, 0, 0, 600)
        r = orc.decode(c, P(bp="sumproduct", rounds=4 * L), e0, nthreads=8)
        rates[L] = orc.logical_failure(c, e0, r["z"]).mean()
    assert rates[16] < rates[8]
