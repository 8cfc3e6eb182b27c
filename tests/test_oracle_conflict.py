"""Pins of the oracle's conflict rules for one round's move requests
(Algorithm 1 has one clock ring at a time; a round of the discretised
machine gathers several requests, which combine by OR, XOR, or sequentially
in ring-time order with a request applying only while its check is active).

Each rule is pinned against a computation other than the oracle's:
brute force over every act/skip assignment (the sequential rule's history is
the unique self-consistent one), request counts, the cases where the rules
must coincide, and the single-edge error of the 2D toric code at clock
density 1, where both endpoint checks ask for the shared edge."""
import itertools

import numpy as np
import pytest

from paper_2609_38139_amd import codes


def random_code(rng, m, n, dmin=2, dmax=3):
    H = np.zeros((m, n), dtype=np.uint8)
    for r in range(m):
        H[r, rng.choice(n, size=int(rng.integers(dmin, dmax + 1)), replace=False)] = 1
    return codes.from_dense(H, name="random")


def random_requests(rng, H, s, key_range):
    """At most one request per check, for a qubit of the check."""
    req_c, req_v, req_key = [], [], []
    for c in range(H.shape[0]):
        if rng.random() < 0.7:
            nb = np.nonzero(H[c])[0]
            req_c.append(c)
            req_v.append(int(rng.choice(nb)))
            req_key.append(int(rng.integers(0, key_range)))
    return req_c, req_v, req_key


def consistent_histories(H, s, req_c, req_v, req_key):
    """Every act/skip assignment in which each request acts exactly when its
    check's syndrome, changed by the acting requests that precede it in
    (ring time, check index) order, is 1; with the flip vector of each."""
    K = len(req_c)
    before = [[(req_key[j], req_c[j]) < (req_key[i], req_c[i]) for j in range(K)] for i in range(K)]
    out = []
    for act in itertools.product((0, 1), repeat=K):
        ok = True
        for i in range(K):
            x = int(s[req_c[i]])
            for j in range(K):
                if act[j] and before[i][j] and H[req_c[i], req_v[j]]:
                    x ^= 1
            if x != act[i]:
                ok = False
                break
        if ok:
            f = np.zeros(H.shape[1], dtype=np.uint8)
            for i in range(K):
                if act[i]:
                    f[req_v[i]] ^= 1
            out.append(f)
    return out


@pytest.mark.parametrize("seed", range(40))
def test_sequential_is_the_unique_consistent_history(orc, seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(3, 8)), int(rng.integers(4, 9))
    code = random_code(rng, m, n)
    H = code.H.to_dense()
    s = rng.integers(0, 2, size=m).astype(np.uint8)
    if seed % 3 == 0:
        s[:] = 1  # every check active: the longest chains
    req_c, req_v, req_key = random_requests(rng, H, s, key_range=3 if seed % 2 else 2**32)
    hist = consistent_histories(H, s, req_c, req_v, req_key)
    assert len(hist) == 1
    f = orc.resolve_moves(code, "sequential", s, req_c, req_v, req_key)
    assert np.array_equal(f, hist[0])


def consistent_group_histories(H, s, groups):
    """As consistent_histories, for multi-qubit moves: groups[i] = (check,
    ring time, qubits); a group acts as a whole, exactly when its check's
    syndrome, changed by the acting groups before it in (ring time, check)
    order, is 1."""
    K = len(groups)
    out = []
    for act in itertools.product((0, 1), repeat=K):
        ok = True
        for i, (ci, ki, _) in enumerate(groups):
            x = int(s[ci])
            for j, (cj, kj, vj) in enumerate(groups):
                if act[j] and (kj, cj) < (ki, ci):
                    x ^= int(H[ci, vj].sum() % 2)
            if x != act[i]:
                ok = False
                break
        if ok:
            f = np.zeros(H.shape[1], dtype=np.uint8)
            for i, (_, _, vi) in enumerate(groups):
                if act[i]:
                    f[vi] ^= 1
            out.append(f)
    return out


@pytest.mark.parametrize("seed", range(30))
def test_sequential_multi_qubit_moves_apply_as_a_whole(orc, seed):
    """A multi-qubit move is one request per qubit, all with the check's
    ring time; under the sequential rule they apply together, exactly when
    the check is active before the first of them (brute force over every
    act/skip assignment of the moves: the history is unique)."""
    rng = np.random.default_rng(500 + seed)
    m, n = int(rng.integers(3, 7)), int(rng.integers(5, 9))
    code = random_code(rng, m, n, 2, 4)
    H = code.H.to_dense()
    s = rng.integers(0, 2, size=m).astype(np.uint8)
    if seed % 3 == 0:
        s[:] = 1
    groups, req_c, req_v, req_key = [], [], [], []
    for c in range(m):
        if rng.random() < 0.8:
            nb = np.nonzero(H[c])[0]
            vs = np.sort(rng.choice(nb, size=int(rng.integers(1, len(nb) + 1)), replace=False))
            key = int(rng.integers(0, 3 if seed % 2 else 2**32))
            groups.append((c, key, vs))
            for v in vs:
                req_c.append(c)
                req_v.append(int(v))
                req_key.append(key)
    hist = consistent_group_histories(H, s, groups)
    assert len(hist) == 1
    order = rng.permutation(len(req_c))  # the input order of the requests does not matter
    f = orc.resolve_moves(code, "sequential", s, [req_c[i] for i in order], [req_v[i] for i in order],
                          [req_key[i] for i in order])
    assert np.array_equal(f, hist[0])


@pytest.mark.parametrize("seed", range(10))
def test_or_and_xor_count_requests(orc, seed):
    rng = np.random.default_rng(100 + seed)
    code = random_code(rng, 12, 10, 2, 5)
    H = code.H.to_dense()
    s = rng.integers(0, 2, size=12).astype(np.uint8)
    req_c, req_v, req_key = random_requests(rng, H, s, 2**32)
    cnt = np.bincount(np.asarray(req_v, dtype=np.int64), minlength=10)
    assert np.array_equal(orc.resolve_moves(code, "or", s, req_c, req_v, req_key), (cnt > 0).astype(np.uint8))
    assert np.array_equal(orc.resolve_moves(code, "xor", s, req_c, req_v, req_key), (cnt % 2).astype(np.uint8))


@pytest.mark.parametrize("seed", range(10))
def test_rules_coincide_without_interaction(orc, seed):
    """No requested qubit belongs to another requesting check: every
    request of an active check applies under every rule."""
    rng = np.random.default_rng(200 + seed)
    code = codes.toric_2d(8)
    H = code.H.to_dense()
    s = np.ones(H.shape[0], dtype=np.uint8)
    req_c, req_v, req_key, used = [], [], [], np.zeros(H.shape[0], dtype=bool)
    for c in rng.permutation(H.shape[0]):
        v = int(rng.choice(np.nonzero(H[c])[0]))
        touched = np.nonzero(H[:, v])[0]
        if used[touched].any() or any(H[c, u] for u in req_v):
            continue
        req_c.append(int(c))
        req_v.append(v)
        req_key.append(int(rng.integers(0, 2**32)))
        used[touched] = True
    assert len(req_c) >= 5
    ref = np.zeros(H.shape[1], dtype=np.uint8)
    ref[req_v] = 1
    for rule in ("or", "xor", "sequential"):
        assert np.array_equal(orc.resolve_moves(code, rule, s, req_c, req_v, req_key), ref), rule


def test_empty_and_inactive_requests(orc):
    code = codes.toric_2d(3)
    m, n = code.H.rows, code.H.cols
    for rule in ("or", "xor", "sequential"):
        assert not orc.resolve_moves(code, rule, np.ones(m, np.uint8), [], [], []).any()
    # a sequential request of a check that is not active does not apply
    H = code.H.to_dense()
    v = int(np.nonzero(H[0])[0][0])
    assert not orc.resolve_moves(code, "sequential", np.zeros(m, np.uint8), [0], [v], [5]).any()
    assert orc.resolve_moves(code, "or", np.zeros(m, np.uint8), [0], [v], [5])[v] == 1


def test_unknown_rule_is_an_error(orc):
    code = codes.toric_2d(3)
    with pytest.raises(RuntimeError):
        orc.lib()
        import ctypes as C
        rp, cl = orc._csr(code.H)
        f = np.zeros(code.H.cols, np.uint8)
        s = np.zeros(code.H.rows, np.uint8)
        z = np.zeros(1, np.int32)
        rc = orc.lib().orc_resolve_moves(code.H.rows, code.H.cols, orc._p(rp, C.c_int32), orc._p(cl, C.c_int32),
                                         7, orc._p(s, C.c_uint8), 0, orc._p(z, C.c_int32),
                                         orc._p(z, C.c_int32), orc._p(z.view(np.uint32), C.c_uint32),
                                         orc._p(f, C.c_uint8))
        if rc != 0:
            raise RuntimeError(rc)


@pytest.mark.parametrize("L", [4, 5])
def test_single_edge_error_at_density_one(orc, L):
    """Both checks at the ends of an erroneous edge are active, ring every
    round and ask for that edge. OR and the sequential rule flip it once and
    clear in round 1; under XOR the two requests cancel in every round, so
    the shot never clears and z stays 0."""
    code = codes.toric_2d(L)
    n = code.H.cols
    e0 = np.zeros((n, n), dtype=np.uint8)
    e0[np.arange(n), np.arange(n)] = 1
    P = dict(mask_density=1.0, rounds=5)
    for rule in ("or", "sequential"):
        r = orc.decode(code, orc.DecodeParams(conflict=rule, **P), e0)
        assert (r["tclr"] == 1).all(), rule
        assert np.array_equal(r["z"], e0), rule
    r = orc.decode(code, orc.DecodeParams(conflict="xor", retire=False, **P), e0)
    assert (r["tclr"] == -1).all()
    assert not r["z"].any()


@pytest.mark.parametrize("rule,move", [("xor", "single"), ("sequential", "single"), ("or", "multi"),
                                       ("xor", "multi"), ("sequential", "multi")])
@pytest.mark.parametrize("name,p", [("toric2d:6", 0.08), ("bb:6x6", 0.04), ("toric3d_membrane:3", 0.06)])
def test_round_invariants_hold_under_every_rule(orc, rule, move, name, p):
    """Per round s == H (e0 ^ z) (the oracle also asserts s_new == s ^ H f
    and fails otherwise) and every left-kernel vector y of H keeps
    y^T s = 0, under every conflict rule and both kinds of move."""
    code = codes.by_name(name)
    H = code.H.to_dense().astype(np.int64)
    e0 = orc.sample_noise(code, p, 0, 0, 12)
    P = orc.DecodeParams(conflict=rule, rounds=12, retire=False, q=0.125 if "membrane" in name else 0.05,
                         bp="sumproduct" if move == "multi" else "minsum", move=move)
    # left kernel of H over GF(2) from a reduced basis of H^T
    Y = _left_kernel(H)
    for i in range(e0.shape[0]):
        r = orc.decode(code, P, e0[i:i + 1], shot0=i, trace=True)
        for k in range(P.rounds):
            s_k = (H @ (e0[i] ^ r["z_trace"][k]).astype(np.int64)) % 2
            assert np.array_equal(s_k, r["s_trace"][k])
            assert not ((Y @ s_k) % 2).any()


def _left_kernel(H):
    A = (H.T % 2).astype(np.uint8)  # y^T H = 0  <=>  H^T y = 0
    rows, cols = A.shape
    A = A.copy()
    piv, r = [], 0
    for c in range(cols):
        k = next((i for i in range(r, rows) if A[i, c]), None)
        if k is None:
            continue
        A[[r, k]] = A[[k, r]]
        for i in range(rows):
            if i != r and A[i, c]:
                A[i] ^= A[r]
        piv.append(c)
        r += 1
    free = [c for c in range(cols) if c not in piv]
    basis = []
    for fcol in free:
        y = np.zeros(cols, dtype=np.uint8)
        y[fcol] = 1
        for i, pc in enumerate(piv):
            y[pc] = A[i, fcol]
        basis.append(y)
    return np.array(basis, dtype=np.int64).reshape(len(basis), cols)


def test_rules_differ_on_the_paper_workload(orc):
    """The rules are distinct dynamics: on 2D toric L=8 at p=0.06 they give
    different corrections on some shots (and all keep the invariants)."""
    code = codes.toric_2d(8)
    e0 = orc.sample_noise(code, 0.06, 0, 0, 200)
    out = {rule: orc.decode(code, orc.DecodeParams(conflict=rule, rounds=32), e0, nthreads=4)
           for rule in ("or", "xor", "sequential")}
    assert (out["or"]["z"] != out["xor"]["z"]).any(axis=1).sum() > 0
    assert (out["or"]["z"] != out["sequential"]["z"]).any(axis=1).sum() > 0


def test_multi_qubit_moves_change_the_dynamics(orc):
    """Multi-qubit moves are a different dynamics from LocalMove on the 2D
    toric workload (sum-product, where positive beliefs are common): some
    shots end differently, and every shot still satisfies s = H (e0 ^ z)."""
    code = codes.toric_2d(8)
    e0 = orc.sample_noise(code, 0.06, 0, 0, 200)
    a = orc.decode(code, orc.DecodeParams(bp="sumproduct", rounds=32), e0, nthreads=4)
    b = orc.decode(code, orc.DecodeParams(bp="sumproduct", rounds=32, move="multi"), e0, nthreads=4)
    assert (a["z"] != b["z"]).any(axis=1).sum() > 0
    assert np.array_equal(b["s"], orc.syndrome(code, e0 ^ b["z"]))
