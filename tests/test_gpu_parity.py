"""Parity of the HIP path with the CPU oracle, through the C ABI.

Every output of the decoder is compared element by element with the oracle
on the same seeded inputs: noise, syndromes and failure flags bit for bit;
corrections z, final syndromes s and clearing rounds t_clr bit for bit;
beliefs L bit for bit for min-sum and within |dL| <= 1e-5 max(1, |L|) for
sum-product (both sides evaluate the same FP32 operations, so they are in
fact expected to agree exactly). Sizes span several tiles and a ragged
tail; the metric configuration is checked at full size on sampled shots.
"""
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


_code_cache = {}


def dcode(L, name):
    if name not in _code_cache:
        c = codes.by_name(name) if isinstance(name, str) else name
        _code_cache[name] = (c, L.Code(c, 0))
    return _code_cache[name]


def to_np(t):
    return t.cpu().numpy()


def gpu_e0(L, dc, e0_np):
    import torch
    return torch.from_numpy(np.ascontiguousarray(e0_np)).cuda()


def oracle_params(orc, P):
    return orc.DecodeParams(bp=P.bp, alpha=P.alpha, q=P.q, clamp=P.clamp, iters=P.iters,
                            rounds=P.rounds, mask_density=P.mask_density, gauge=P.gauge,
                            evidence=P.evidence, retire=P.retire, seed=P.seed, conflict=P.conflict,
                            move=P.move)


def compare_decode(L, orc, name, P, e0_np, shot0=0, form="auto", cfg=None, beliefs=True, tag=""):
    code, dc = dcode(L, name)
    print(f"[parity] {tag} code={getattr(code, 'name', name)} form={form} cfg={cfg} bp={P.bp} "
          f"shots={e0_np.shape[0]} shot0={shot0} rounds={P.rounds} iters={P.iters}", flush=True)
    g = L.decode_rounds(dc, P, gpu_e0(L, dc, e0_np), shot0=shot0, form=form, want_beliefs=beliefs,
                        cfg=cfg)
    o = orc.decode(code, oracle_params(orc, P), e0_np, shot0=shot0, nthreads=NTHREADS,
                   want_beliefs=beliefs)
    z, s, t = to_np(g["z"]), to_np(g["s"]), to_np(g["tclr"])
    bad = np.nonzero((z != o["z"]).any(1) | (s != o["s"]).any(1) | (t != o["tclr"]))[0]
    assert bad.size == 0, f"{bad.size} shots differ, first {bad[:8]} (tclr gpu {t[bad[:4]]} oracle {o['tclr'][bad[:4]]})"
    if beliefs:
        Lg = to_np(g["L"])
        if P.bp == "minsum":
            assert np.array_equal(Lg.view(np.uint32), o["L"].view(np.uint32)), "beliefs differ"
        else:
            assert np.all(np.abs(Lg - o["L"]) <= 1e-5 * np.maximum(1.0, np.abs(o["L"])))
    return g, o


# ------------------------------------------------------------ primitives
@pytest.mark.parametrize("name", ["toric2d:8", "toric3d_point:3", "bb:6x6", "rep:7", "toric2d:32",
                                  "toric3d_point:7"])
def test_noise_parity(L, orc, name):
    """Rows of 4k qubits are written a word at a time, others bytewise;
    rows over 1024 qubits span two blocks of the launch."""
    code, dc = dcode(L, name)
    for p in (0.0, 0.02, 0.37, 1.0):
        for seed in (0, 123456789012345):
            for shot0 in (0, (1 << 33) + 5):
                e = to_np(L.sample_noise(dc, p, seed, shot0, 257))
                assert np.array_equal(e, orc.sample_noise(code, p, seed, shot0, 257)), (p, seed, shot0)


def test_noise_into_a_misaligned_buffer(L, orc):
    import torch
    code, dc = dcode(L, "toric2d:8")
    S = 100
    flat = torch.full((S * code.n + 1,), 7, dtype=torch.uint8, device="cuda")
    out = flat[1:].view(S, code.n)
    L.sample_noise(dc, 0.1, 5, 9, S, out=out)
    assert np.array_equal(to_np(out), orc.sample_noise(code, 0.1, 5, 9, S))
    assert int(flat[0].item()) == 7


@pytest.mark.parametrize("name", ["toric2d:8", "toric3d_membrane:3", "bb:12x6", "rep:7"])
def test_syndrome_parity(L, orc, name):
    code, dc = dcode(L, name)
    rng = np.random.default_rng(1)
    e = (rng.random((301, code.n)) < 0.2).astype(np.uint8)
    s = to_np(L.syndrome(dc, gpu_e0(L, dc, e)))
    assert np.array_equal(s, orc.syndrome(code, e))


@pytest.mark.parametrize("name", ["toric2d:3", "toric2d:8", "bb:6x6", "bb:12x6", "toric3d_point:3",
                                  "toric3d_membrane:3", "rep:9", "toric2d:16", "toric2d:32",
                                  "toric3d_point:4"])
def test_failure_parity(L, orc, name):
    """Homology test by logicals (GPU) against the oracle's rank test, on
    random residuals and on residuals in ker H (mostly trivial or logical)."""
    code, dc = dcode(L, name)
    rng = np.random.default_rng(2)
    e0 = (rng.random((400, code.n)) < 0.1).astype(np.uint8)
    z = (rng.random((400, code.n)) < 0.1).astype(np.uint8)
    # residuals in ker H: stabilisers (rows of G) plus, half the time, a logical
    G = code.G.to_dense() if code.G.rows else np.zeros((0, code.n), dtype=np.uint8)
    kerH = []
    for i in range(200):
        r = np.zeros(code.n, dtype=np.uint8)
        if G.shape[0]:
            sel = rng.random(G.shape[0]) < 0.3
            r = (G[sel].sum(0) % 2).astype(np.uint8)
        if i % 2:
            lg = dc.logical_matrix()
            r ^= lg[rng.integers(0, lg.shape[0])]
        kerH.append(r)
    e0 = np.vstack([e0, np.array(kerH)])
    z = np.vstack([z, np.zeros((200, code.n), dtype=np.uint8)])
    f = to_np(L.logical_failure(dc, gpu_e0(L, dc, e0), gpu_e0(L, dc, z)))
    assert np.array_equal(f, orc.logical_failure(code, e0, z))
    assert f[400:].sum() > 0 and f[400:].sum() < 200


@pytest.mark.parametrize("form", ["resident", "stream"])
@pytest.mark.parametrize("name,p", [("toric2d:16", 0.06), ("bb:12x6", 0.06), ("toric3d_point:3", 0.05)])
def test_decode_reports_failures(L, orc, name, p, form):
    """fail_out of the decode call (inside the resident launch, after it in
    the stream form) equals the standalone failure test and the oracle."""
    code, dc = dcode(L, name)
    e0_np = orc.sample_noise(code, p, 3, 0, 211)
    e0 = gpu_e0(L, dc, e0_np)
    g = L.decode_rounds(dc, L.DecodeParams(rounds=24), e0, form=form, want_fail=True)
    f = to_np(g["fail"])
    assert np.array_equal(f, to_np(L.logical_failure(dc, e0, g["z"])))
    assert np.array_equal(f, orc.logical_failure(code, e0_np, to_np(g["z"])))
    assert 0 < f.sum() < len(f)


def test_failure_packed_and_direct_paths_agree(L, orc):
    """Rows whose length is a multiple of 32 on 16-byte aligned buffers take
    the bit-packed kernel; the same rows seen through buffers one byte off
    take the direct one. Both equal the oracle."""
    import torch
    code, dc = dcode(L, "toric2d:16")
    rng = np.random.default_rng(8)
    S = 333
    e0 = (rng.random((S, code.n)) < 0.08).astype(np.uint8)
    z = (rng.random((S, code.n)) < 0.08).astype(np.uint8)
    z[::3] = e0[::3]  # residual 0: success
    want = orc.logical_failure(code, e0, z)
    fa = to_np(L.logical_failure(dc, gpu_e0(L, dc, e0), gpu_e0(L, dc, z)))
    flat_e = torch.zeros(S * code.n + 1, dtype=torch.uint8, device="cuda")
    flat_z = torch.zeros(S * code.n + 1, dtype=torch.uint8, device="cuda")
    flat_e[1:] = torch.from_numpy(e0.ravel()).cuda()
    flat_z[1:] = torch.from_numpy(z.ravel()).cuda()
    fb = to_np(L.logical_failure(dc, flat_e[1:].view(S, code.n), flat_z[1:].view(S, code.n)))
    assert np.array_equal(fa, want) and np.array_equal(fb, want)
    assert 0 < want.sum() < S


# -------------------------------------------------------------- decode
@pytest.mark.parametrize("form", ["resident", "stream"])
@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_decode_2d_toric_l8(L, orc, form, bp):
    """2D toric L = 8, p in {0.02, 0.04, 0.06, 0.08}, seed 0, 1000 shots each,
    20 sweeps per round, 64 rounds, clocks at density 0.5."""
    code, dc = dcode(L, "toric2d:8")
    for p in (0.02, 0.04, 0.06, 0.08):
        e0 = orc.sample_noise(code, p, 0, 0, 1000)
        P = L.DecodeParams(bp=bp, rounds=64)
        compare_decode(L, orc, "toric2d:8", P, e0, form=form, tag=f"p={p}")


FAMILY_CASES = [
    ("toric2d:16", "minsum", 0.05, 0.05, 24),
    ("toric2d:16", "sumproduct", 0.06, 0.05, 24),
    ("toric3d_point:4", "minsum", 0.03, 0.05, 16),
    ("toric3d_point:4", "sumproduct", 0.03, 0.05, 16),
    ("toric3d_membrane:4", "minsum", 0.05, 0.125, 16),
    ("toric3d_membrane:4", "sumproduct", 0.05, 0.125, 16),
    ("bb:6x6", "minsum", 0.03, 0.05, 32),
    ("bb:6x6", "sumproduct", 0.03, 0.05, 32),
    ("bb:12x6", "minsum", 0.02, 0.05, 32),
    ("bb:12x6", "sumproduct", 0.02, 0.05, 32),
    ("rep:15", "minsum", 0.2, 0.1, 16),
    ("rep:15", "sumproduct", 0.2, 0.1, 16),
]


@pytest.mark.parametrize("form", ["resident", "stream"])
@pytest.mark.parametrize("name,bp,p,q,R", FAMILY_CASES)
def test_decode_families(L, orc, name, bp, p, q, R, form):
    code, dc = dcode(L, name)
    e0 = orc.sample_noise(code, p, 7, 1000, 333)
    P = L.DecodeParams(bp=bp, q=q, rounds=R)
    compare_decode(L, orc, name, P, e0, shot0=1000, form=form)


VARIANTS = [
    dict(retire=False),
    dict(evidence=False),
    dict(mask_density=1.0),
    dict(mask_density=0.0, rounds=3),
    dict(iters=0, rounds=5),
    dict(iters=1),
    dict(rounds=0),
    dict(alpha=1.0),
    dict(alpha=1.25),
    dict(clamp=4.0),
    dict(clamp=4.0, bp="sumproduct"),
    dict(q=0.3, seed=99),
    dict(bp="sumproduct", retire=False, rounds=10),
]


@pytest.mark.parametrize("form", ["resident", "stream"])
@pytest.mark.parametrize("var", VARIANTS, ids=[str(v) for v in VARIANTS])
def test_decode_variants(L, orc, var, form):
    """Knobs and degenerate settings (no sweeps, no rounds, every or no
    clock, no Evidence, an active clamp) on a ragged number of shots."""
    if var.get("alpha", 0.75) > 1.0 and form == "resident":
        form = "auto"  # min-sum with alpha > 1 runs in the stream form
    code, dc = dcode(L, "toric2d:6")
    e0 = orc.sample_noise(code, 0.06, 3, 0, 130)
    kw = dict(rounds=20)
    kw.update(var)
    P = L.DecodeParams(**kw)
    compare_decode(L, orc, "toric2d:6", P, e0, form=form, tag=str(var))


@pytest.mark.parametrize("form", ["resident", "stream"])
@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_decode_irregular_graphs(L, orc, bp, form):
    """Irregular Tanner graphs: the open chain (qubit degrees 1 and 2) and a
    code mixing check degrees 1..6 and qubit degrees 1..4."""
    open_chain = codes.repetition(12, periodic=False)
    rng = np.random.default_rng(5)
    H = np.zeros((20, 30), dtype=np.uint8)
    for r in range(20):
        H[r, rng.choice(30, size=int(rng.integers(1, 7)), replace=False)] = 1
    for v in range(30):
        if not H[:, v].any():
            H[rng.integers(0, 20), v] = 1
    # keep qubit degrees <= 4
    for v in range(30):
        rows = np.nonzero(H[:, v])[0]
        for r in rows[4:]:
            H[r, v] = 0
    mixed = codes.from_dense(H, name="mixed")
    for code in (open_chain, mixed):
        key = code.name
        _code_cache[key] = (code, L.Code(code, 0))
        e0 = orc.sample_noise(code, 0.15, 11, 0, 97)
        P = L.DecodeParams(bp=bp, q=0.1, rounds=12)
        compare_decode(L, orc, key, P, e0, form=form)


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_padded_degree2_variant(L, orc, bp):
    """Codes with checks of degree <= 6 and qubits of degree <= 2 that are not
    regular run the padded (6, 2) resident variant, in every launch shape: a
    random graph with check degrees 1..6 and qubit degrees 1..2, and the 2D
    toric code with alpha = 1 (its qubit-side clamp could bind, so the exact
    degree-2 kernel is not used)."""
    rng = np.random.default_rng(17)
    m, n = 48, 90
    H = np.zeros((m, n), dtype=np.uint8)
    deg = np.zeros(m, dtype=int)
    for v in range(n):
        for _ in range(int(rng.integers(1, 3))):
            free = np.nonzero((deg < 6) & (H[:, v] == 0))[0]
            r = int(rng.choice(free))
            H[r, v] = 1
            deg[r] += 1
    H = H[H.sum(1) > 0]
    assert H.sum(0).max() <= 2 and H.sum(1).max() <= 6 and H.sum(1).min() >= 1 and H.sum(0).min() >= 1
    graph = codes.from_dense(H, name="deg2-padded")
    _code_cache[graph.name] = (graph, L.Code(graph, 0))
    e0 = orc.sample_noise(graph, 0.1, 5, 0, 131)
    for cfg in (None, {"checks_per_thread": 1}, {"checks_per_thread": 2, "shots_per_block": 2},
                {"checks_per_thread": 4}, {"checks_per_thread": 8, "shots_per_block": 3}):
        compare_decode(L, orc, graph.name, L.DecodeParams(bp=bp, q=0.1, rounds=16), e0, cfg=cfg,
                       tag="padded (6, 2)")
    code, dc = dcode(L, "toric2d:8")
    e0 = orc.sample_noise(code, 0.06, 6, 0, 150)
    for cfg in (None, {"checks_per_thread": 8}):
        compare_decode(L, orc, "toric2d:8", L.DecodeParams(bp=bp, alpha=1.0, rounds=24), e0, cfg=cfg,
                       form="resident", tag="alpha 1")


def test_resident_launch_shapes_agree(L, orc):
    """Results do not depend on the resident launch shape."""
    code, dc = dcode(L, "toric2d:16")
    e0 = orc.sample_noise(code, 0.06, 0, 0, 200)
    P = L.DecodeParams(rounds=32)
    for cfg in ({"checks_per_thread": 1}, {"checks_per_thread": 2}, {"checks_per_thread": 4},
                {"checks_per_thread": 8}, {"checks_per_thread": 2, "shots_per_block": 2},
                {"checks_per_thread": 4, "shots_per_block": 3}):
        compare_decode(L, orc, "toric2d:16", P, e0, cfg=cfg, tag="shape")


def test_single_and_empty_batches(L, orc):
    import torch
    code, dc = dcode(L, "bb:6x6")
    e0 = orc.sample_noise(code, 0.05, 0, 42, 1)
    P = L.DecodeParams(rounds=16)
    compare_decode(L, orc, "bb:6x6", P, e0, shot0=42)
    empty = torch.zeros((0, code.n), dtype=torch.uint8, device="cuda")
    out = L.decode_rounds(dc, P, empty)
    assert out["z"].shape == (0, code.n)


def test_every_call_accepts_an_empty_batch(L):
    """Zero shots: every shot-batched call returns at once with empty outputs,
    whatever optional outputs are asked for, and an idle server step reports
    no event."""
    import torch
    code, dc = dcode(L, "toric2d:6")
    print("empty batch: noise, syndrome, failure", flush=True)
    e0 = L.sample_noise(dc, 0.05, 1, 0, 0)
    assert e0.shape == (0, code.n)
    assert L.syndrome(dc, e0).shape == (0, code.m)
    assert L.logical_failure(dc, e0, e0).shape == (0,)
    for form in ("resident", "stream"):
        for bp in ("minsum", "sumproduct"):
            print(f"empty batch: decode_rounds {form} {bp}", flush=True)
            out = L.decode_rounds(dc, L.DecodeParams(bp=bp, rounds=4), e0, form=form, want_beliefs=True,
                                  want_sweeps=True, want_fail=True)
            for k, shape in (("z", (0, code.n)), ("s", (0, code.m)), ("tclr", (0,)), ("L", (0, code.n)),
                             ("sweeps", (0,)), ("fail", (0,))):
                assert out[k].shape == shape, (form, bp, k)
    print("empty batch: decode_continuous", flush=True)
    out = L.decode_continuous(dc, L.ContinuousParams(dt=0.01, t_max=1.0), e0, want_fail=True,
                              want_steps=True)
    assert out["counts"].shape == (0, 2) and out["steps"].shape == (0,) and out["fail"].shape == (0,)
    print("empty batch: decode_bitcentric", flush=True)
    rc, rdc = dcode(L, "rep:7")
    e1 = torch.zeros((0, rc.n), dtype=torch.uint8, device="cuda")
    out = L.decode_bitcentric(rdc, 0.05, e1, 8, want_beliefs=True)
    assert out["z"].shape == (0, rc.n) and out["iclr"].shape == (0,) and out["L"].shape == (0, rc.n)
    print("empty batch: idle server step", flush=True)
    srv = L.Server(device=0, mem_budget=1 << 20, max_slots=4)
    assert srv.step() == []
    torch.cuda.synchronize()


def test_invalid_arguments_are_rejected(L):
    import torch
    code, dc = dcode(L, "toric2d:8")
    e0 = torch.zeros((4, code.n), dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LaimError) as ei:
        L.decode_rounds(dc, L.DecodeParams(q=1.5), e0)
    assert ei.value.status == L.EINVAL
    with pytest.raises(L.LaimError) as ei:
        L.decode_rounds(dc, L.DecodeParams(gauge=True), e0)
    assert ei.value.status == L.EUNSUP
    with pytest.raises(ValueError):
        L.decode_rounds(dc, L.DecodeParams(), e0[:, :10].contiguous())


def test_explicit_resident_form_it_cannot_take(L, orc):
    """Asking for the resident form where it cannot run is an error, with no
    workspace size, while the automatic choice runs the stream form."""
    import torch
    for name, P in (("toric3d_membrane:16", L.DecodeParams(q=0.125, rounds=2)),
                    ("toric2d:8", L.DecodeParams(alpha=1.25, rounds=6))):
        code, dc = dcode(L, name)
        print(f"[resident refused] {name} alpha={P.alpha}", flush=True)
        assert L.workspace_bytes(dc, P, 8, form="resident") == 0
        assert L.workspace_bytes(dc, P, 8, form="auto") == L.workspace_bytes(dc, P, 8, form="stream") > 0
        e0_np = orc.sample_noise(code, 0.03, 4, 0, 8)
        e0 = gpu_e0(L, dc, e0_np)
        with pytest.raises(L.LaimError) as ei:
            L.decode_rounds(dc, P, e0, form="resident")
        assert ei.value.status == L.EUNSUP
        assert b"resident" in L.lib().laim_last_error()
        a = L.decode_rounds(dc, P, e0, form="auto")
        b = L.decode_rounds(dc, P, e0, form="stream")
        for k in ("z", "s", "tclr"):
            assert torch.equal(a[k], b[k]), (name, k)


# ------------------------------------------------- full-size, sampled shots
@pytest.mark.timeout(600)
@pytest.mark.parametrize("form,bp,cfg", [("resident", "minsum", None), ("resident", "minsum", (8, 1)),
                                         ("resident", "sumproduct", None), ("stream", "minsum", None)])
def test_metric_config_full_size_sampled(L, orc, form, bp, cfg):
    """2D toric L = 32, p = 0.05, 65536 shots in one launch, 4L = 128 rounds
    of 20 sweeps: the launch the benchmark times (also in its tuned resident
    shape, 128 threads x 8 checks, one shot per block). 96 shots spread over
    the whole range are recomputed one by one by the oracle."""
    code, dc = dcode(L, "toric2d:32")
    S = 65536
    print(f"[parity] full size {form} {bp} cfg={cfg} S={S}", flush=True)
    e0 = L.sample_noise(dc, 0.05, 0, 0, S)
    P = L.DecodeParams(bp=bp, rounds=128)
    if cfg is None:
        g = L.decode_rounds(dc, P, e0, form=form)
    else:
        g = L.decode_rounds(dc, P, e0, cfg={"checks_per_thread": cfg[0], "shots_per_block": cfg[1]})
    f = L.logical_failure(dc, e0, g["z"])
    rng = np.random.default_rng(17)
    idx = np.unique(np.concatenate([[0, 1, S - 1], rng.integers(0, S, 93)]))
    e0s = to_np(e0[idx])
    assert np.array_equal(e0s, np.vstack([orc.sample_noise(code, 0.05, 0, int(i), 1) for i in idx]))
    zg, sg, tg, fg = to_np(g["z"][idx]), to_np(g["s"][idx]), to_np(g["tclr"][idx]), to_np(f[idx])
    from concurrent.futures import ThreadPoolExecutor
    op = oracle_params(orc, P)
    with ThreadPoolExecutor(NTHREADS) as ex:  # the oracle call releases the GIL
        refs = list(ex.map(lambda k: orc.decode(code, op, e0s[k:k + 1], shot0=int(idx[k])), range(len(idx))))
    for k, i in enumerate(idx):
        o = refs[k]
        assert np.array_equal(zg[k], o["z"][0]) and np.array_equal(sg[k], o["s"][0]) and tg[k] == o["tclr"][0], i
    assert np.array_equal(fg, orc.logical_failure(code, e0s, zg))
    # properties at every shot: s = H (e0 ^ z), t_clr consistent with s
    sfull = to_np(L.syndrome(dc, e0 ^ g["z"]))
    assert np.array_equal(sfull, to_np(g["s"]))
    t = to_np(g["tclr"])
    assert np.array_equal(to_np(g["s"]).any(1), t < 0)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,R", [("toric3d_point:24", 4), ("toric3d_membrane:16", 4)])
def test_large_codes_stream_form(L, orc, name, R):
    """Codes whose per-shot state exceeds the LDS run in the stream form."""
    code, dc = dcode(L, name)
    q = 0.125 if "membrane" in name else 0.05
    e0 = orc.sample_noise(code, 0.02, 0, 0, 24)
    P = L.DecodeParams(q=q, rounds=R)
    compare_decode(L, orc, name, P, e0, form="auto", beliefs=False)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("Lsz,p,bp", [(16, 0.01, "minsum"), (16, 0.10, "minsum"), (16, 0.10, "sumproduct")])
def test_2d_toric_sizes_full_launch_sampled(L, orc, Lsz, p, bp):
    """2D toric L = 16 at 65536 shots per launch, 4L rounds of 20 sweeps, in
    the default resident shape: sampled shots recomputed by the oracle; every
    shot checked against s = H (e0 ^ z). (L = 32 and 64 over the noise range:
    test_gpu_full_size.py.)"""
    from concurrent.futures import ThreadPoolExecutor
    name = f"toric2d:{Lsz}"
    code, dc = dcode(L, name)
    S = 65536
    print(f"[parity] {name} p={p} {bp} S={S}", flush=True)
    e0 = L.sample_noise(dc, p, 0, 0, S)
    P = L.DecodeParams(bp=bp, rounds=4 * Lsz)
    g = L.decode_rounds(dc, P, e0)
    idx = np.array([0, 1, 777, 32768, S - 1] + ([12345, 54321, 60000] if Lsz == 16 else []))
    e0s = to_np(e0[idx])
    op = oracle_params(orc, P)
    with ThreadPoolExecutor(NTHREADS) as ex:
        refs = list(ex.map(lambda k: orc.decode(code, op, e0s[k:k + 1], shot0=int(idx[k])), range(len(idx))))
    for k, i in enumerate(idx):
        assert np.array_equal(to_np(g["z"][i]), refs[k]["z"][0]), i
        assert int(g["tclr"][i]) == int(refs[k]["tclr"][0]), i
    sfull = to_np(L.syndrome(dc, e0 ^ g["z"]))
    assert np.array_equal(sfull, to_np(g["s"]))
    assert np.array_equal(sfull.any(1), to_np(g["tclr"]) < 0)


@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_stream_generic_paths_high_degrees(L, orc, bp):
    """Qubit degrees up to 6 and check degrees above 8: beyond the resident
    variants and the stream kernels' specialised gathers (qubit degree <= 4,
    check degree <= 8), so the stream form's generic loops run."""
    rng = np.random.default_rng(21)
    m, n = 24, 48
    H = np.zeros((m, n), dtype=np.uint8)
    for v in range(n):
        H[rng.choice(m, size=int(rng.integers(1, 7)), replace=False), v] = 1
    for r in range(m):
        if not H[r].any():
            H[r, rng.integers(0, n)] = 1
    code = codes.from_dense(H, name="high-degree")
    assert code.H.to_dense().sum(0).max() > 4 and code.H.to_dense().sum(1).max() > 8
    if code.name not in _code_cache:
        _code_cache[code.name] = (code, L.Code(code, 0))
    e0 = orc.sample_noise(code, 0.1, 4, 0, 300)
    for conflict in ("or", "xor", "sequential"):
        P = L.DecodeParams(bp=bp, q=0.1, rounds=10, conflict=conflict, retire=False)
        compare_decode(L, orc, code.name, P, e0, form="auto", tag=f"high-degree {conflict}")


@pytest.mark.parametrize("form", ["resident", "stream"])
def test_large_shot_ids_and_seed(L, orc, form):
    """Shot ids past 2^32 and a seed past 2^32 (the high words of the Philox
    counter and key) reach every random draw identically on both sides."""
    code, dc = dcode(L, "toric2d:8")
    shot0 = (1 << 33) + 123
    e0 = orc.sample_noise(code, 0.06, (1 << 40) + 7, shot0, 150)
    for conflict in ("or", "sequential"):
        P = L.DecodeParams(rounds=32, seed=(1 << 36) + 99, conflict=conflict)
        compare_decode(L, orc, "toric2d:8", P, e0, shot0=shot0, form=form, tag=f"large ids {conflict}")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("bp", ["minsum", "sumproduct"])
def test_2d_toric_l16_noise_sweep(L, orc, bp):
    """2D toric L = 16 over the whole noise range p = 0.01 .. 0.10 (4L = 64
    rounds, 8192 shots per p in one launch each): sampled shots against the
    oracle, and s = H (e0 ^ z) for every shot."""
    from concurrent.futures import ThreadPoolExecutor
    code, dc = dcode(L, "toric2d:16")
    P = L.DecodeParams(bp=bp, rounds=64)
    op = oracle_params(orc, P)
    idx = np.array([0, 4095, 8191])
    for k in range(1, 11):
        p = k / 100.0
        print(f"[parity] toric2d:16 {bp} p={p}", flush=True)
        e0 = L.sample_noise(dc, p, 0, 0, 8192)
        g = L.decode_rounds(dc, P, e0)
        e0s = to_np(e0[idx])
        with ThreadPoolExecutor(NTHREADS) as ex:
            refs = list(ex.map(lambda j: orc.decode(code, op, e0s[j:j + 1], shot0=int(idx[j])), range(len(idx))))
        for j, i in enumerate(idx):
            assert np.array_equal(to_np(g["z"][i]), refs[j]["z"][0]), (p, i)
            assert int(g["tclr"][i]) == int(refs[j]["tclr"][0]), (p, i)
        assert np.array_equal(to_np(L.syndrome(dc, e0 ^ g["z"])), to_np(g["s"])), p
