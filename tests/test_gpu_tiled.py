"""The tiled resident variant changes no result.

On the 2D toric layout with min-sum and 8 checks per thread, each thread's
checks form a 2 x 4 tile of the lattice and the messages on the qubits inside
the tile stay in registers through a round's sweeps (written to LDS once per
round that swept, for the feedback). These tests check that the library
picks it exactly where it applies, and that z, s, t_clr, the beliefs, the
failure flags and the sweep counts are bit-identical to the plain variant and
equal to the oracle, over lattice sizes, decode parameters and launch shapes,
and at the full size of the measured workload."""
import numpy as np
import pytest

from test_gpu_parity import compare_decode, dcode, gpu_e0, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2609_38139_amd import laim
    laim.lib()
    return laim


TILE = {"checks_per_thread": 8}
PLAIN = {"checks_per_thread": 4}


def run(L, dc, P, e0, cfg):
    g = L.decode_rounds(dc, P, e0, form="resident", want_beliefs=True, want_fail=True, want_sweeps=True,
                        cfg=cfg)
    return {k: to_np(g[k]) for k in ("z", "s", "tclr", "L", "fail", "sweeps")}


def same(a, b):
    for k in ("z", "s", "tclr", "fail", "sweeps"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["L"].view(np.uint32), b["L"].view(np.uint32)), "beliefs"


def test_variant_choice(L):
    """Tiled exactly for min-sum (exact degree-2 kernels) with 8 checks per
    thread and m / 8 threads on toric layouts with L a multiple of 4."""
    for name, expect in (("toric2d:4", True), ("toric2d:8", True), ("toric2d:12", True),
                         ("toric2d:32", True), ("toric2d:6", False), ("toric2d:10", False),
                         ("bb:6x6", False), ("toric3d_point:4", False)):
        code, dc = dcode(L, name)
        try:
            v = dc.resident_variant(L.DecodeParams(), TILE)
        except L.LaimError:
            v = {"tiled": False}
        assert v["tiled"] == expect, name
    code, dc = dcode(L, "toric2d:16")
    assert not dc.resident_variant(L.DecodeParams(bp="sumproduct"), TILE)["tiled"]
    assert not dc.resident_variant(L.DecodeParams(conflict="sequential"), TILE)["tiled"]
    assert not dc.resident_variant(L.DecodeParams(alpha=1.0), TILE)["tiled"]  # padded variant
    assert not dc.resident_variant(L.DecodeParams(), PLAIN)["tiled"]
    assert not dc.resident_variant(L.DecodeParams(), {"checks_per_thread": 8, "threads_per_shot": 40})["tiled"]
    assert dc.resident_variant(L.DecodeParams(), {"checks_per_thread": 8, "shots_per_block": 4})["tiled"]


CASES = [
    ("toric2d:4", dict(rounds=24), 0.08, 300),
    ("toric2d:8", dict(rounds=32), 0.06, 600),
    ("toric2d:8", dict(rounds=32, skip_fixed=False), 0.06, 300),
    ("toric2d:8", dict(rounds=32, conflict="xor"), 0.06, 300),
    ("toric2d:8", dict(rounds=32, move="multi"), 0.06, 300),
    ("toric2d:8", dict(rounds=32, retire=False), 0.06, 300),
    ("toric2d:8", dict(rounds=24, evidence=False, mask_density=0.25), 0.05, 300),
    ("toric2d:8", dict(rounds=16, iters=1), 0.06, 300),
    ("toric2d:8", dict(rounds=16, iters=9), 0.06, 300),
    ("toric2d:12", dict(rounds=48, alpha=0.5), 0.05, 400),
    ("toric2d:16", dict(rounds=64), 0.05, 400),
    ("toric2d:16", dict(rounds=64, skip_fixed=False), 0.03, 200),
    ("toric2d:32", dict(rounds=40), 0.05, 128),
]


@pytest.mark.parametrize("name,kw,p,S", CASES,
                         ids=[f"{c[0]}-{'-'.join(f'{k}={v}' for k, v in c[1].items())}" for c in CASES])
def test_tiled_equals_oracle_and_plain(L, orc, name, kw, p, S):
    code, dc = dcode(L, name)
    P = L.DecodeParams(**kw)
    assert dc.resident_variant(P, TILE)["tiled"]
    e0_np = orc.sample_noise(code, p, 7, 0, S)
    compare_decode(L, orc, name, P, e0_np, form="resident", cfg=TILE, tag="tiled")
    e0 = gpu_e0(L, dc, e0_np)
    same(run(L, dc, P, e0, TILE), run(L, dc, P, e0, PLAIN))


def test_tiled_several_shots_per_block(L, orc):
    """Two and four shots per block (each shot's group its own LDS region)."""
    code, dc = dcode(L, "toric2d:8")
    P = L.DecodeParams(rounds=32)
    e0_np = orc.sample_noise(code, 0.06, 3, 0, 500)
    e0 = gpu_e0(L, dc, e0_np)
    ref = run(L, dc, P, e0, PLAIN)
    for spb in (2, 4):
        cfg = {"checks_per_thread": 8, "shots_per_block": spb}
        assert dc.resident_variant(P, cfg)["tiled"]
        same(run(L, dc, P, e0, cfg), ref)
    compare_decode(L, orc, "toric2d:8", P, e0_np, form="resident", cfg={"checks_per_thread": 8,
                                                                        "shots_per_block": 4})


@pytest.mark.timeout(600)
def test_tiled_full_launch(L, orc):
    """65,536 shots of 2D toric L = 32 at p = 0.05, R = 128, T = 20 (the
    measured workload): every output bit-identical to the plain variant,
    sampled shots equal to the oracle (the two launch times are printed)."""
    import torch
    code, dc = dcode(L, "toric2d:32")
    S = 65536
    P = L.DecodeParams(rounds=128)
    e0 = L.sample_noise(dc, 0.05, 0, 0, S)
    outs, times = {}, {}
    for tag, cfg in (("tiled", TILE), ("plain", PLAIN)):
        L.decode_rounds(dc, P, e0[:1024], form="resident", cfg=cfg)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g = L.decode_rounds(dc, P, e0, form="resident", want_fail=True, want_sweeps=True, cfg=cfg)
        b.record()
        torch.cuda.synchronize()
        times[tag] = a.elapsed_time(b)
        outs[tag] = {k: to_np(g[k]) for k in ("z", "s", "tclr", "fail", "sweeps")}
    for k in ("z", "s", "tclr", "fail", "sweeps"):
        assert np.array_equal(outs["tiled"][k], outs["plain"][k]), k
    rng = np.random.default_rng(17)
    idx = np.unique(np.concatenate([[0, S - 1], rng.integers(0, S, 24)]))
    e0_np = to_np(e0)
    from test_gpu_parity import oracle_params
    for i in idx:
        o = orc.decode(code, oracle_params(orc, P), e0_np[i:i + 1], shot0=int(i))
        assert np.array_equal(outs["tiled"]["z"][i], o["z"][0]), int(i)
        assert int(outs["tiled"]["tclr"][i]) == int(o["tclr"][0]), int(i)
    print(f"[tiled] L=32 p=0.05: {times['tiled']:.2f} ms tiled, {times['plain']:.2f} ms plain (4 checks "
          f"per thread)", flush=True)
