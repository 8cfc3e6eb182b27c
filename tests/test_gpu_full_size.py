"""Full-size launches of the benchmark configurations, with at least 32
shots of every launch recomputed one by one by the oracle.

The shots are chosen from the GPU's own outcome so that every kind of shot
is covered where the launch has it: shots that cleared early and late,
shots that never cleared (stuck), and shots that cleared into the wrong
homology class, plus the first and last shot and random ones. The oracle
then recomputes each from its e0 and shot id alone, and z, s, t_clr and the
failure flag must agree bit for bit. Every shot of the launch is also
checked against s = H (e0 ^ z) and t_clr >= 0 <=> s = 0.

Configurations (benchmark specification): 2D toric L = 32 and 64 at
65536 shots, p in {0.01, 0.05, 0.10}, 4L rounds, both BP rules; both 3D
toric sectors at L = 8, 16, 24 in one batched launch of 16384 shots each
(point sector p in {0.01, 0.08}, membrane sector p in {0.01, 0.05}); the
bivariate-bicycle codes (6,6) and (12,6) at 262144 shots with 2D toric
codes in one launch, p in {0.001, 0.01}; and the continuous-time machine
with sum-product at L = 32 in the launch shape the benchmark times (two
checks per thread)."""
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


def pick_shots(tclr, fail, k=36, seed=0):
    """At least k shot indices: first, second and last, then up to 6 that
    cleared earliest, 4 that cleared latest, 8 stuck, 8 in the wrong class,
    and random ones to fill. Returns (sorted indices, counts per kind)."""
    rng = np.random.default_rng(seed)
    S = tclr.shape[0]
    chosen = {0, 1 % S, S - 1}
    kinds = {}
    ok = np.nonzero((tclr >= 0) & (fail == 0))[0]
    stuck = np.nonzero(tclr < 0)[0]
    wrong = np.nonzero((tclr >= 0) & (fail == 1))[0]
    order = ok[np.argsort(tclr[ok], kind="stable")]
    for name, pool, n in (("early", order[: max(1, len(order) // 10)], 6),
                          ("late", order[-max(1, len(order) // 10):], 4),
                          ("stuck", stuck, 8), ("wrong_class", wrong, 8)):
        take = rng.choice(pool, size=min(n, len(pool)), replace=False) if len(pool) else []
        kinds[name] = len(take)
        chosen.update(int(i) for i in take)
    while len(chosen) < min(k, S):
        chosen.add(int(rng.integers(0, S)))
    return np.array(sorted(chosen)), kinds


def oracle_params(orc, P):
    return orc.DecodeParams(bp=P.bp, alpha=P.alpha, q=P.q, clamp=P.clamp, iters=P.iters,
                            rounds=P.rounds, mask_density=P.mask_density, gauge=P.gauge,
                            evidence=P.evidence, retire=P.retire, seed=P.seed, conflict=P.conflict,
                            move=P.move)


def check_sampled(L, orc, spec, dc, P, e0, out, tag, shot0=0):
    """Oracle recomputation of the sampled shots and the whole-launch
    properties. out holds device z, s, tclr, fail."""
    z, s, t, f = (out[k].cpu().numpy() for k in ("z", "s", "tclr", "fail"))
    idx, kinds = pick_shots(t, f)
    print(f"[full] {tag}: {len(idx)} oracle shots {kinds}; launch: cleared {(t >= 0).mean():.4f}, "
          f"failures {f.mean():.4f}", flush=True)
    e0s = e0[idx].cpu().numpy()
    assert np.array_equal(e0s, np.vstack([orc.sample_noise(spec, out["p"], out["seed"], shot0 + int(i), 1)
                                          for i in idx])), tag
    op = oracle_params(orc, P)
    with ThreadPoolExecutor(NTHREADS) as ex:  # the oracle call releases the GIL
        refs = list(ex.map(lambda j: orc.decode(spec, op, e0s[j:j + 1], shot0=shot0 + int(idx[j])),
                           range(len(idx))))
    for j, i in enumerate(idx):
        r = refs[j]
        assert np.array_equal(z[i], r["z"][0]), (tag, int(i), "z")
        assert np.array_equal(s[i], r["s"][0]), (tag, int(i), "s")
        assert int(t[i]) == int(r["tclr"][0]), (tag, int(i), int(t[i]), int(r["tclr"][0]))
    fo = orc.logical_failure(spec, e0s, np.vstack([r["z"] for r in refs]))
    assert np.array_equal(f[idx], fo), tag
    sfull = L.syndrome(dc, e0 ^ out["z"]).cpu().numpy()
    assert np.array_equal(sfull, s), tag
    assert np.array_equal(sfull.any(1), t < 0), tag
    return kinds


C2 = [(Lsz, p, bp) for Lsz in (32, 64) for p in (0.01, 0.05, 0.10) for bp in ("minsum", "sumproduct")]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("Lsz,p,bp", C2, ids=[f"L{a}-p{b}-{c}" for a, b, c in C2])
def test_2d_toric_full_launch(L, orc, Lsz, p, bp):
    """2D toric L = 32 and 64, 65536 shots in one resident launch, 4L rounds
    of 20 sweeps, retiring at clear; the failure test inside the launch."""
    import torch
    spec = codes.toric_2d(Lsz)
    dc = L.Code(spec, 0)
    S = 65536
    print(f"[full] toric2d:{Lsz} p={p} {bp}: decoding {S} shots", flush=True)
    e0 = L.sample_noise(dc, p, 0, 0, S)
    P = L.DecodeParams(bp=bp, rounds=4 * Lsz)
    g = L.decode_rounds(dc, P, e0, want_fail=True)
    torch.cuda.synchronize()
    g.update(p=p, seed=0)
    kinds = check_sampled(L, orc, spec, dc, P, e0, g, f"toric2d:{Lsz} p={p} {bp}")
    assert torch.equal(g["fail"], L.logical_failure(dc, e0, g["z"]))
    # below threshold the launch has early-cleared shots; above it, stuck ones
    if p <= 0.05:
        assert kinds["early"] > 0
    if p >= 0.10:
        assert kinds["stuck"] > 0


def _plan_full(L, orc, items_spec, tag, seed=1):
    import torch
    items = []
    for name, p, q, R, S in items_spec:
        spec = codes.by_name(name)
        code = L.Code(spec, 0)
        P = L.DecodeParams(q=q, rounds=R)
        e0 = L.sample_noise(code, p, seed, 0, S)
        items.append({"spec": spec, "code": code, "params": P, "e0": e0, "shot0": 0, "p": p})
    torch.cuda.synchronize()
    print(f"[full] {tag}: one plan of {len(items)} items", flush=True)
    plan = L.BatchPlan(items)
    outs = plan.launch()
    torch.cuda.synchronize()
    for it, o in zip(items, outs):
        o = dict(o, p=it["p"], seed=seed)
        check_sampled(L, orc, it["spec"], it["code"], it["params"], it["e0"], o,
                      f"{tag} {it['spec'].name} p={it['p']}")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("p_point,p_mem", [(0.01, 0.01), (0.08, 0.05)])
def test_3d_toric_mixed_sizes_full_launch(L, orc, p_point, p_mem):
    """Both 3D toric sectors at L = 8, 16, 24 in one batched launch of 16384
    shots each, 4L rounds, min-sum (prior q = 0.05 for the point sector and
    0.125 for the membrane sector). The codes whose shot does not fit the
    LDS run in the stream form inside the same graph."""
    spec = [(f"toric3d_point:{n}", p_point, 0.05, 4 * n, 16384) for n in (8, 16, 24)]
    spec += [(f"toric3d_membrane:{n}", p_mem, 0.125, 4 * n, 16384) for n in (8, 16, 24)]
    _plan_full(L, orc, spec, f"3D toric p_point={p_point} p_membrane={p_mem}")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("p", [0.001, 0.01])
def test_bivariate_bicycle_with_toric_full_launch(L, orc, p):
    """Bivariate-bicycle (6,6) and (12,6) at 262144 shots each, batched with
    2D toric L = 16 and 32 (p = 0.05) in one launch; 64 rounds for the BB
    codes, 4L for the toric codes, min-sum."""
    _plan_full(L, orc, [("bb:6x6", p, 0.05, 64, 262144), ("bb:12x6", p, 0.05, 64, 262144),
                        ("toric2d:16", 0.05, 0.05, 64, 16384), ("toric2d:32", 0.05, 0.05, 128, 16384)],
               f"BB p={p} with toric")


@pytest.mark.timeout(900)
def test_continuous_sum_product_benchmarked_instance(L, orc):
    """The continuous-time machine as the benchmark times it with sum-product:
    2D toric L = 32, p = 0.05, Table S1's dt = 0.001 and tau = 0.1, t_max = 30,
    2048 shots in one launch with two checks per thread (the kernel instance
    for check degree 4, qubit degree 2, 2 checks per thread, sum-product).
    Sampled shots -- cleared early and late, not cleared by t_max -- are
    recomputed by the oracle: z, s, t_clr (as doubles), event and move
    counts, and the failure flag."""
    import torch
    spec = codes.toric_2d(32)
    dc = L.Code(spec, 0)
    kw = dict(bp="sumproduct", dt=0.001, tau=0.1, t_max=30.0)
    S, shot0 = 2048, 7 * 10**9
    e0 = L.sample_noise(dc, 0.05, 0, shot0, S)
    print("[full] continuous machine, sum-product, toric2d:32, 2048 shots, 2 checks per thread", flush=True)
    g = L.decode_continuous(dc, L.ContinuousParams(**kw), e0, shot0=shot0, checks_per_thread=2,
                            want_fail=True, want_steps=True)
    torch.cuda.synchronize()
    t = g["tclr"].cpu().numpy()
    f = g["fail"].cpu().numpy()
    rng = np.random.default_rng(5)
    cleared = np.nonzero(t >= 0)[0]
    order = cleared[np.argsort(t[cleared], kind="stable")]
    stuck = np.nonzero(t < 0)[0]
    idx = set([0, S - 1])
    idx.update(int(i) for i in order[:4])
    idx.update(int(i) for i in order[-4:])
    idx.update(int(i) for i in rng.choice(stuck, size=min(4, len(stuck)), replace=False))
    while len(idx) < 16:
        idx.add(int(rng.integers(0, S)))
    idx = np.array(sorted(idx))
    print(f"[full] continuous machine: {len(idx)} oracle shots, {len(stuck)} of {S} not cleared", flush=True)
    e0s = e0[idx].cpu().numpy()
    P_or = orc.ContinuousParams(**kw)
    with ThreadPoolExecutor(NTHREADS) as ex:
        refs = list(ex.map(lambda j: orc.ctm_decode(spec, P_or, e0s[j:j + 1], shot0=shot0 + int(idx[j])),
                           range(len(idx))))
    z = g["z"].cpu().numpy()
    s = g["s"].cpu().numpy()
    cnt = g["counts"].cpu().numpy()
    for j, i in enumerate(idx):
        r = refs[j]
        assert np.array_equal(z[i], r["z"][0]) and np.array_equal(s[i], r["s"][0]), int(i)
        assert t[i] == r["tclr"][0], (int(i), t[i], r["tclr"][0])
        assert cnt[i, 0] == r["events"][0] and cnt[i, 1] == r["moves"][0], int(i)
    fo = orc.logical_failure(spec, e0s, np.vstack([r["z"] for r in refs]))
    assert np.array_equal(f[idx], fo)
    # the same launch with one check per thread and without the skip: identical outputs
    g1 = L.decode_continuous(dc, L.ContinuousParams(skip_fixed=False, **kw), e0, shot0=shot0,
                             checks_per_thread=1, want_fail=True)
    for k in ("z", "s", "tclr", "counts", "fail"):
        assert torch.equal(g1[k], g[k]), k
    sfull = L.syndrome(dc, e0 ^ g["z"]).cpu().numpy()
    assert np.array_equal(sfull, s)
    assert np.array_equal(sfull.any(1), t < 0)
