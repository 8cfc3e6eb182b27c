"""Parity of online decoding in overlapping spacetime windows on the GPU
with the oracle, through the C ABI: the committed correction z, the final
error E_N, the failure flag and the number of windows that cleared, bit for
bit, for sampled and for given errors, several window layouts, both BP
rules, the resident and the stream form of the window decodes, and a
full-size launch on sampled shots."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2609_38139_amd import codes

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2609_38139_amd import laim
    laim.lib()
    return laim


def oracle_params(orc, P):
    return orc.DecodeParams(bp=P.bp, alpha=P.alpha, q=P.q, clamp=P.clamp, iters=P.iters,
                            rounds=P.rounds, mask_density=P.mask_density, gauge=P.gauge,
                            evidence=P.evidence, retire=P.retire, seed=P.seed, conflict=P.conflict,
                            move=P.move)


def run_both(L, orc, name, P, op_kw, nshots, shot0=0, e_in=None, eps_in=None, tag=""):
    import torch
    spec = codes.by_name(name)
    code = L.Code(spec, 0)
    op = L.OnlineParams(**op_kw)
    plan = L.OnlinePlan(code, op)
    print(f"[online] {tag} {name} {op_kw} bp={P.bp} shots={nshots} shot0={shot0}", flush=True)
    g = plan.decode(P, nshots, shot0=shot0,
                    e_in=torch.from_numpy(e_in).cuda() if e_in is not None else None,
                    eps_in=torch.from_numpy(eps_in).cuda() if eps_in is not None else None)
    torch.cuda.synchronize()
    o = orc.online_decode(spec, oracle_params(orc, P), orc.OnlineParams(**op_kw), shot0=shot0, nshots=nshots,
                          e_in=e_in, eps_in=eps_in, nthreads=NTHREADS)
    for k in ("z", "E", "fail", "cleared"):
        got = g[k].cpu().numpy()
        bad = np.nonzero(got != o[k])[0] if got.ndim == 1 else np.nonzero((got != o[k]).any(1))[0]
        assert bad.size == 0, f"{k} differs in shots {bad[:8]} ({tag})"
    return g, o


LAYOUTS = [dict(rounds_total=6, window=3, commit=2, p=0.02, p_meas=0.02),
           dict(rounds_total=5, window=5, commit=5, p=0.03, p_meas=0.01),
           dict(rounds_total=7, window=2, commit=1, p=0.015, p_meas=0.03),
           dict(rounds_total=1, window=3, commit=2, p=0.05, p_meas=0.05)]


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
@pytest.mark.parametrize("op_kw", LAYOUTS, ids=["N6W3C2", "N5W5C5", "N7W2C1", "N1"])
@pytest.mark.parametrize("name", ["toric2d:5", "bb:6x6", "toric3d_point:3"])
def test_online_matches_oracle(L, orc, name, op_kw, bp):
    P = L.DecodeParams(bp=bp, rounds=12, iters=10, seed=4)
    run_both(L, orc, name, P, op_kw, 150, shot0=20, tag="layout")


def test_online_stream_form_and_multi_moves(L, orc):
    """Min-sum with alpha > 1 runs the window decodes in the stream form;
    multi-qubit moves and XOR work inside the windows as well."""
    op_kw = dict(rounds_total=6, window=3, commit=2, p=0.02, p_meas=0.02)
    run_both(L, orc, "toric2d:5", L.DecodeParams(alpha=1.25, rounds=10, iters=8), op_kw, 100, tag="stream")
    run_both(L, orc, "toric2d:5", L.DecodeParams(bp="sumproduct", rounds=10, iters=8, move="multi",
                                                 conflict="xor"), op_kw, 100, tag="multi xor")


def test_online_stream_form_many_tiles(L, orc):
    """Window decodes in the stream form over several 256-shot tiles, where
    the shots still running after most have stopped are moved to the first
    tiles (start syndromes, round offsets and per-window outputs included)."""
    op_kw = dict(rounds_total=8, window=3, commit=2, p=0.015, p_meas=0.015)
    run_both(L, orc, "toric2d:6", L.DecodeParams(alpha=1.25, rounds=12, iters=8), op_kw, 900, shot0=3,
             tag="stream tiles")
    run_both(L, orc, "toric2d:6", L.DecodeParams(alpha=1.25, rounds=12, iters=8, conflict="sequential"),
             op_kw, 600, tag="stream tiles sequential")


def test_online_given_errors(L, orc):
    """Given errors instead of sampled ones: a single measurement error, a
    single data error, and random histories (the last round's measurement
    errors are ignored: that round is perfect)."""
    spec = codes.toric_2d(5)
    n, m, N = spec.n, spec.m, 6
    S = 40
    rng = np.random.default_rng(3)
    e = (rng.random((S, N, n)) < 0.02).astype(np.uint8)
    eps = (rng.random((S, N, m)) < 0.03).astype(np.uint8)
    e[0] = 0
    eps[0] = 0
    eps[0, 2, 7] = 1
    e[1] = 0
    eps[1] = 0
    e[1, 3, 11] = 1
    P = L.DecodeParams(bp="sumproduct", rounds=8, mask_density=1.0)
    g, o = run_both(L, orc, "toric2d:5", P, dict(rounds_total=N, window=3, commit=2, p=0.0, p_meas=0.0), S,
                    e_in=e, eps_in=eps, tag="given")
    z = g["z"].cpu().numpy()
    assert not z[0].any() and np.array_equal(z[1], e[1, 3])
    assert g["fail"][0].item() == 0 and g["fail"][1].item() == 0


def test_online_one_round_equals_offline_decode(L, orc):
    """One perfect round: the online decode is decode_rounds on e_1."""
    import torch
    spec = codes.toric_2d(8)
    code = L.Code(spec, 0)
    op = L.OnlineParams(rounds_total=1, window=2, commit=1, p=0.06, p_meas=0.5)
    P = L.DecodeParams(rounds=24, seed=8)
    g = L.OnlinePlan(code, op).decode(P, 300, shot0=5)
    e, _ = orc.online_noise(spec, orc.OnlineParams(rounds_total=1, window=2, commit=1, p=0.06, p_meas=0.5),
                            8, 5, 300)
    r = L.decode_rounds(code, P, torch.from_numpy(np.ascontiguousarray(e[:, 0])).cuda(), shot0=5, want_fail=True)
    assert np.array_equal(g["z"].cpu().numpy(), r["z"].cpu().numpy())
    assert np.array_equal(g["E"].cpu().numpy(), e[:, 0])
    assert torch.equal(g["fail"], r["fail"])


def test_online_empty_and_single_shot(L, orc):
    spec = codes.toric_2d(4)
    code = L.Code(spec, 0)
    plan = L.OnlinePlan(code, L.OnlineParams(rounds_total=4, window=2, commit=1))
    out = plan.decode(L.DecodeParams(rounds=4), 0)
    assert out["z"].shape == (0, code.n)
    run_both(L, orc, "toric2d:4", L.DecodeParams(rounds=6), dict(rounds_total=4, window=2, commit=1, p=0.05,
                                                                 p_meas=0.05), 1, shot0=2**33 + 1, tag="single")


def test_online_invalid_arguments(L):
    code = L.Code(codes.toric_2d(4), 0)
    for kw in (dict(rounds_total=0), dict(window=2, commit=3), dict(commit=0)):
        with pytest.raises(L.LaimError) as ei:
            L.OnlinePlan(code, L.OnlineParams(**kw))
        assert ei.value.status == L.EINVAL


@pytest.mark.timeout(900)
@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_online_full_launch_sampled(L, orc, bp):
    """2D toric L = 16, 16 rounds (the last perfect), windows of 4 rounds
    committing 2, p = p_meas = 0.01, 65536 shots in one call; 32 shots
    recomputed by the oracle (those whose windows did not all clear first),
    and every shot with all windows cleared has no residual syndrome."""
    import torch
    spec = codes.toric_2d(16)
    code = L.Code(spec, 0)
    op_kw = dict(rounds_total=16, window=4, commit=2, p=0.01, p_meas=0.01)
    op = L.OnlineParams(**op_kw)
    P = L.DecodeParams(bp=bp, rounds=16)
    S = 65536
    plan = L.OnlinePlan(code, op)
    print(f"[online] full launch toric2d:16 {bp} {S} shots", flush=True)
    g = plan.decode(P, S)
    torch.cuda.synchronize()
    nwin = 7
    cl = g["cleared"].cpu().numpy()
    z = g["z"].cpu().numpy()
    E = g["E"].cpu().numpy()
    f = g["fail"].cpu().numpy()
    rng = np.random.default_rng(1)
    partial = np.nonzero(cl < nwin)[0]
    idx = set([0, S - 1])
    idx.update(int(i) for i in rng.choice(partial, size=min(8, len(partial)), replace=False))
    idx.update(int(i) for i in rng.choice(np.nonzero(f)[0], size=min(8, int(f.sum())), replace=False))
    while len(idx) < 32:
        idx.add(int(rng.integers(0, S)))
    idx = np.array(sorted(idx))
    po = oracle_params(orc, P)
    oo = orc.OnlineParams(**op_kw)
    with ThreadPoolExecutor(NTHREADS) as ex:
        refs = list(ex.map(lambda i: orc.online_decode(spec, po, oo, shot0=int(i), nshots=1), idx))
    for i, r in zip(idx, refs):
        assert np.array_equal(z[i], r["z"][0]) and np.array_equal(E[i], r["E"][0]), int(i)
        assert f[i] == r["fail"][0] and cl[i] == r["cleared"][0], int(i)
    full = cl == nwin
    resid = L.syndrome(code, torch.from_numpy(E ^ z).cuda()).cpu().numpy()
    assert not resid[full].any()
    print(f"[online] {bp}: failure rate {f.mean():.5f}, all windows cleared {full.mean():.4f}", flush=True)
