"""The stream form's exact shortcuts change no result.

With skip_fixed the stream form compares sweeps 7, 15, ... and the last of
each round against the messages they replace, marks the shots whose
messages are a fixed point of the sweep, skips the sweep of a 256-shot tile
whose shots are all retired or at a fixed point, stops a shot at a fixed
point whose active checks all fail Evidence (its later rounds would repeat
the last one exactly), and moves the shots still running to the first
tiles once most have stopped. These tests check that z, s, t_clr, the
beliefs and the failure flags are bit-identical with and without the
shortcuts, and equal to the oracle (which runs every sweep of every round),
on workloads where many shots get stuck, so that whole tiles stop, and on
many tiles whose shots mostly stop early, so that the running shots are
moved to the first tiles."""
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


def run(L, dc, P, e0):
    g = L.decode_rounds(dc, P, e0, form="stream", want_beliefs=True, want_fail=True)
    return {k: to_np(g[k]) for k in ("z", "s", "tclr", "L", "fail")}


def same(a, b):
    for k in ("z", "s", "tclr", "fail"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["L"].view(np.uint32), b["L"].view(np.uint32)), "beliefs"


CASES = [
    ("toric2d:16", dict(rounds=64), 0.05, 700),
    ("toric2d:16", dict(rounds=64, retire=False), 0.05, 300),
    ("toric2d:16", dict(rounds=64, conflict="xor"), 0.05, 300),
    ("toric2d:16", dict(rounds=64, conflict="sequential"), 0.05, 300),
    ("toric2d:16", dict(rounds=64, move="multi"), 0.05, 300),
    ("toric2d:12", dict(bp="sumproduct", rounds=48), 0.07, 300),
    ("toric2d:12", dict(rounds=48, evidence=False, mask_density=0.25), 0.04, 300),
    ("toric2d:12", dict(rounds=48, alpha=1.25), 0.05, 300),
    ("toric2d:8", dict(rounds=40, iters=1), 0.06, 300),
    ("toric2d:8", dict(rounds=24, iters=9), 0.06, 300),
    ("bb:6x6", dict(rounds=32), 0.05, 300),
    ("toric3d_point:6", dict(rounds=24), 0.05, 520),
    ("toric3d_membrane:4", dict(rounds=24, q=0.125), 0.06, 300),
    # many tiles, most shots stopping early: the running shots are compacted
    ("toric2d:12", dict(rounds=40), 0.03, 2000),
    ("toric2d:12", dict(rounds=40, conflict="sequential", retire=False), 0.04, 1100),
    ("toric2d:12", dict(bp="sumproduct", rounds=30, move="multi", conflict="xor"), 0.05, 1300),
]


@pytest.mark.parametrize("name,kw,p,S", CASES,
                         ids=[f"{c[0]}-{'-'.join(f'{k}={v}' for k, v in c[1].items())}" for c in CASES])
def test_stream_skip_is_exact(L, orc, name, kw, p, S):
    code, dc = dcode(L, name)
    e0_np = orc.sample_noise(code, p, 3, 0, S)
    P = L.DecodeParams(skip_fixed=True, **kw)
    # against the oracle, which runs every sweep and round ...
    compare_decode(L, orc, name, P, e0_np, form="stream", tag="stream-skip")
    # ... and against the stream form without the shortcuts, bit for bit
    e0 = gpu_e0(L, dc, e0_np)
    same(run(L, dc, P, e0), run(L, dc, L.DecodeParams(skip_fixed=False, **kw), e0))


@pytest.mark.timeout(600)
def test_stream_skip_full_launch(L, orc):
    """65536 shots of 2D toric L = 32 at p = 0.05 (most shots get stuck, so
    most tiles stop): every shot equals the launch without the shortcuts,
    the resident form's launch, and, on sampled shots, the oracle (the two
    launch times are printed)."""
    import torch
    code, dc = dcode(L, "toric2d:32")
    S = 65536
    e0 = L.sample_noise(dc, 0.05, 0, 0, S)
    P = L.DecodeParams(rounds=128)
    ws = torch.empty((L.workspace_bytes(dc, P, S, form="stream"),), dtype=torch.uint8, device="cuda")
    times = {}
    outs = {}
    for skip in (True, False):
        Pk = L.DecodeParams(rounds=128, skip_fixed=skip)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g = L.decode_rounds(dc, Pk, e0, form="stream", want_fail=True, workspace=ws)
        b.record()
        torch.cuda.synchronize()
        times[skip] = a.elapsed_time(b)
        outs[skip] = {k: g[k].clone() for k in ("z", "s", "tclr", "fail")}
    r = L.decode_rounds(dc, P, e0, form="resident", want_fail=True)
    for k in ("z", "s", "tclr", "fail"):
        assert torch.equal(outs[True][k], outs[False][k]), k
        assert torch.equal(outs[True][k], r[k]), k
    rng = np.random.default_rng(31)
    idx = np.unique(np.concatenate([[0, S - 1], rng.integers(0, S, 30)]))
    e0_np = to_np(e0)
    for i in idx:
        o = orc.decode(code, orc.DecodeParams(rounds=128), e0_np[i:i + 1], shot0=int(i))
        assert np.array_equal(to_np(outs[True]["z"][i]), o["z"][0]), int(i)
        assert int(outs[True]["tclr"][i]) == int(o["tclr"][0]), int(i)
    print(f"[stream-skip] L=32 p=0.05: {times[True]:.1f} ms with the shortcuts, {times[False]:.1f} ms without",
          flush=True)
