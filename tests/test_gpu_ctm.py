"""Parity of the continuous-time machine on the GPU with the oracle, through
the C ABI: corrections z, final syndromes s, event and move counts and
logical failures bit for bit, and clearing times t_clr equal as doubles
(both sides evaluate the same FP32 Euler steps and the same FP64 event
times). Codes of every family, both BP rules, the paper's dt values, ragged
shot counts, several launch shapes, and the degenerate cases."""
import os

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


_cache = {}


def dcode(L, name):
    key = name if isinstance(name, str) else id(name)
    if key not in _cache:
        c = codes.by_name(name) if isinstance(name, str) else name
        _cache[key] = (c, L.Code(c, 0))
    return _cache[key]


def run_both(L, orc, name, p, nshots, shot0=0, cpt=0, tag="", **kw):
    import torch
    code, dc = dcode(L, name)
    print(f"[ctm] {tag} code={name} p={p} n={nshots} shot0={shot0} cpt={cpt} {kw}", flush=True)
    e0 = orc.sample_noise(code, p, 0, shot0, nshots)
    P = L.ContinuousParams(**kw)
    g = L.decode_continuous(dc, P, torch.from_numpy(e0).cuda(), shot0=shot0, checks_per_thread=cpt,
                            want_fail=True)
    torch.cuda.synchronize()
    o = orc.ctm_decode(code, orc.ContinuousParams(**kw), e0, shot0=shot0, nthreads=NTHREADS)
    got = {k: g[k].cpu().numpy() for k in ("z", "s", "tclr", "counts", "fail")}
    for k in ("z", "s"):
        bad = np.nonzero(np.any(got[k] != o[k], axis=1))[0]
        assert bad.size == 0, f"{k} differs in shots {bad[:8]} ({tag})"
    bad = np.nonzero(got["tclr"] != o["tclr"])[0]
    assert bad.size == 0, (f"t_clr differs in shots {bad[:8]}: gpu {got['tclr'][bad[:4]]} "
                           f"oracle {o['tclr'][bad[:4]]} ({tag})")
    assert np.array_equal(got["counts"][:, 0], o["events"]) and np.array_equal(got["counts"][:, 1], o["moves"])
    assert np.array_equal(got["fail"], orc.logical_failure(code, e0, o["z"]))
    return got, o


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
@pytest.mark.parametrize("p", [0.03, 0.07])
def test_toric_2d_paper_parameters(L, orc, bp, p):
    """2D toric code with Table S1's row (dt = 0.001, tau = 0.1, q = 0.05)."""
    run_both(L, orc, "toric2d:8", p, 200, bp=bp, dt=0.001, tau=0.1, t_max=30.0, tag="2d")


@pytest.mark.parametrize("name,p,q,dt", [
    ("toric3d_point:4", 0.03, 0.05, 0.001),
    ("toric3d_membrane:3", 0.06, 0.125, 0.01),
    ("bb:6x6", 0.02, 0.05, 0.01),
    ("bb:12x6", 0.02, 0.05, 0.01),
    ("rep:9", 0.15, 0.05, 0.01),
    ("toric2d:5", 0.05, 0.05, 0.005),
])
@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_families(L, orc, name, p, q, dt, bp):
    run_both(L, orc, name, p, 150, shot0=17, bp=bp, q=q, dt=dt, tau=0.1, t_max=40.0, tag="family")


def test_irregular_graphs(L, orc):
    """The open chain (qubit degrees 1 and 2) and a code mixing check degrees
    1..6 and qubit degrees 1..4 (the padded kernel variant)."""
    rng = np.random.default_rng(5)
    H = np.zeros((20, 30), dtype=np.uint8)
    for r in range(20):
        H[r, rng.choice(30, size=int(rng.integers(1, 7)), replace=False)] = 1
    for v in range(30):
        if not H[:, v].any():
            H[rng.integers(0, 20), v] = 1
    for v in range(30):
        for r in np.nonzero(H[:, v])[0][4:]:
            H[r, v] = 0
    mixed = codes.from_dense(H, name="mixed")
    chain = codes.repetition(12, periodic=False)
    for code in (chain, mixed):
        for bp in ("minsum", "sumproduct"):
            run_both(L, orc, code, 0.15, 97, bp=bp, q=0.1, dt=0.01, t_max=20.0, tag="irregular")


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
@pytest.mark.parametrize("cpt", [1, 2, 4])
def test_launch_shapes_agree(L, orc, cpt, bp):
    """Results do not depend on checks per thread (toric L=12: 144 checks,
    several 64-check tiles and a ragged one), for both BP rules."""
    run_both(L, orc, "toric2d:12", 0.05, 64, shot0=1000, cpt=cpt, bp=bp, dt=0.005, t_max=20.0,
             tag="shape")


def test_min_sum_scale_above_one(L, orc):
    """alpha > 1 lets check outputs reach the clamp; such runs use the padded
    kernel variant, which clamps them."""
    run_both(L, orc, "toric2d:6", 0.06, 96, bp="minsum", alpha=1.25, dt=0.01, t_max=15.0, tag="alpha")


def test_evidence_off_and_other_seed(L, orc):
    run_both(L, orc, "toric2d:6", 0.08, 96, evidence=False, seed=99, dt=0.01, t_max=10.0, tag="ablation")


def test_degenerate_cases(L, orc):
    import torch
    code, dc = dcode(L, "toric2d:6")
    P = L.ContinuousParams(dt=0.01, t_max=5.0)
    # no shots
    e0 = torch.zeros((0, code.H.cols), dtype=torch.uint8, device="cuda")
    out = L.decode_continuous(dc, P, e0)
    assert out["z"].shape[0] == 0
    # a clear start: no event, t_clr = 0; t_max = 0: no Euler step at all
    e0 = np.zeros((3, code.H.cols), dtype=np.uint8)
    e0[1, 5] = 1
    e0[2, [0, 7, 30]] = 1
    for t_max in (0.0, 5.0):
        g = L.decode_continuous(dc, L.ContinuousParams(dt=0.01, t_max=t_max), torch.from_numpy(e0).cuda())
        o = orc.ctm_decode(code, orc.ContinuousParams(dt=0.01, t_max=t_max), e0)
        assert np.array_equal(g["tclr"].cpu().numpy(), o["tclr"])
        assert np.array_equal(g["z"].cpu().numpy(), o["z"])
        assert g["tclr"][0].item() == 0.0
    # a single shot with a late shot id
    run_both(L, orc, "toric2d:6", 0.1, 1, shot0=2**33 + 5, dt=0.01, t_max=10.0, tag="single")


def test_invalid_arguments(L):
    import torch
    code, dc = dcode(L, "toric2d:4")
    e0 = torch.zeros((2, code.H.cols), dtype=torch.uint8, device="cuda")
    for kw in ({"dt": 0.0}, {"tau": -1.0}, {"q": 1.5}, {"t_max": -1.0}):
        with pytest.raises(L.LaimError):
            L.decode_continuous(dc, L.ContinuousParams(**kw), e0)
    with pytest.raises(L.LaimError):
        L.decode_continuous(dc, L.ContinuousParams(), e0, checks_per_thread=3)
    with pytest.raises(ValueError):
        L.decode_continuous(dc, L.ContinuousParams(bp="other"), e0)


def test_full_size_sampled_shots(L, orc):
    """The bench's configuration (2D toric L=32, p=0.05, Table S1's dt and tau)
    at a full launch of 4096 shots; the oracle recomputes a sample of them."""
    import torch
    code, dc = dcode(L, "toric2d:32")
    kw = dict(bp="minsum", dt=0.001, tau=0.1, t_max=20.0)
    e0 = orc.sample_noise(code, 0.05, 0, 0, 4096)
    print("[ctm] full size toric2d:32 4096 shots", flush=True)
    g = L.decode_continuous(dc, L.ContinuousParams(**kw), torch.from_numpy(e0).cuda(), want_fail=True)
    torch.cuda.synchronize()
    idx = np.array([0, 1, 2, 511, 1000, 2047, 4095])
    for i in idx:
        o = orc.ctm_decode(code, orc.ContinuousParams(**kw), e0[i:i + 1], shot0=int(i))
        assert g["tclr"][i].item() == o["tclr"][0]
        assert np.array_equal(g["z"][i].cpu().numpy(), o["z"][0])
        assert np.array_equal(g["counts"][i].cpu().numpy(), [o["events"][0], o["moves"][0]])
    # properties that hold for every shot
    s = orc.syndrome(code, e0 ^ g["z"].cpu().numpy())
    assert np.array_equal(s, g["s"].cpu().numpy())
    assert np.array_equal(g["tclr"].cpu().numpy() >= 0, s.sum(axis=1) == 0)


def test_clamp_binding_settings(L, orc):
    """Settings where a clamp of the degree-2 min-sum dynamics can bind (a
    small CLAMP, or an Euler factor dt/tau > 1 that overshoots) run in the
    padded kernel variant, which clamps every message; both match the
    oracle, as does the default setting next to them."""
    for kw in ({"clamp": 3.0}, {"dt": 0.2, "tau": 0.1}, {}):
        run_both(L, orc, "toric2d:6", 0.08, 80, bp="minsum", t_max=12.0,
                 **({"dt": 0.01} | kw), tag=f"clamp {kw}")


@pytest.mark.parametrize("bp,name,p,t_max", [("minsum", "toric2d:8", 0.06, 20.0), ("sumproduct", "toric2d:8", 0.06, 20.0),
                                             ("minsum", "bb:6x6", 0.04, 10.0), ("minsum", "toric3d_point:3", 0.05, 10.0),
                                             ("minsum", "toric2d:16", 0.05, 30.0)])
def test_skipping_fixed_steps_is_exact(L, orc, bp, name, p, t_max):
    """Steps at a fixed point of the messages are skipped up to the next
    event (skip_fixed, the default): every output -- corrections,
    syndromes, clearing times, event and move counts, failures -- equals
    the same launch computing every step, and the oracle."""
    import torch
    kw = dict(bp=bp, dt=0.001, t_max=t_max)
    got, _ = run_both(L, orc, name, p, 77, tag="skip", **kw)
    code, dc = dcode(L, name)
    e0 = orc.sample_noise(code, p, 0, 0, 77)
    e0d = torch.from_numpy(e0).cuda()
    g = L.decode_continuous(dc, L.ContinuousParams(skip_fixed=False, **kw), e0d, want_fail=True,
                            want_steps=True)
    for k in ("z", "s", "tclr", "counts", "fail"):
        assert np.array_equal(g[k].cpu().numpy(), got[k]), k
    # steps computed: without the skip, those up to the step at which the
    # clearing event acts (the first k with k dt >= t_clr), or all K
    K = int(np.floor(t_max / 0.001 + 0.5))
    want = []
    for T in got["tclr"]:
        if T < 0:
            want.append(K)
        else:
            k = 0
            while k * 0.001 < T:
                k += 1
            want.append(min(k, K))
    assert np.array_equal(g["steps"].cpu().numpy(), np.array(want))
    on = L.decode_continuous(dc, L.ContinuousParams(**kw), e0d, want_steps=True)["steps"].cpu().numpy()
    assert np.all(on <= np.array(want))


@pytest.mark.parametrize("name,cpt", [("toric3d_point:3", 2), ("toric3d_point:3", 4), ("toric2d:5", 8)])
def test_padding_checks_continuous(L, orc, name, cpt):
    """Launch shapes whose last tile is padded (more checks per block than
    the code has): results equal the oracle, with and without the skip."""
    import torch
    got, _ = run_both(L, orc, name, 0.05, 41, cpt=cpt, tag="padding", dt=0.01, t_max=10.0)
    code, dc = dcode(L, name)
    e0 = orc.sample_noise(code, 0.05, 0, 0, 41)
    g = L.decode_continuous(dc, L.ContinuousParams(dt=0.01, t_max=10.0, skip_fixed=False),
                            torch.from_numpy(e0).cuda(), checks_per_thread=cpt, want_fail=True)
    for k in ("z", "s", "tclr", "counts", "fail"):
        assert np.array_equal(g[k].cpu().numpy(), got[k]), k
