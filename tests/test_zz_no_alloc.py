"""laim_decode_rounds_static, the decode call that allocates nothing (its
scratch is a static device array), gives exactly what laim_decode_rounds
gives with a caller-owned workspace: in the resident and the stream form, on
two calls in a row with the second smaller (the array keeps the first call's
contents), and it refuses work that needs more scratch than the array
holds, before launching anything."""
import numpy as np
import pytest

from paper_2609_38139_amd import codes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU")
    from paper_2609_38139_amd import laim
    laim.lib()
    return laim


def _same(a, b, keys):
    import torch
    for k in keys:
        if a.get(k) is None:
            continue
        x, y = a[k], b[k]
        if x.dtype == torch.float32:
            x, y = x.view(torch.int32), y.view(torch.int32)
        assert torch.equal(x, y), k


@pytest.mark.parametrize("form,name,bp,sizes", [
    ("resident", "toric2d:16", "minsum", (700, 129)),
    ("resident", "bb:12x6", "sumproduct", (300, 1)),
    ("stream", "toric2d:8", "minsum", (1000, 257)),
    ("stream", "toric3d_membrane:4", "sumproduct", (300, 40)),
])
def test_static_scratch_equals_workspace_call(L, orc, form, name, bp, sizes):
    import torch
    spec = codes.by_name(name)
    code = L.Code(spec, 0)
    q = 0.125 if "membrane" in name else 0.05
    P = L.DecodeParams(bp=bp, q=q, rounds=24)
    for call, S in enumerate(sizes):
        print(f"[no-alloc] {form} {name} {bp} call {call}: {S} shots", flush=True)
        shot0 = 1000 * call + 3
        e0 = L.sample_noise(code, 0.04, 2, shot0, S)
        a = L.decode_rounds_static(code, P, e0, shot0=shot0, form=form, want_beliefs=True,
                                   want_sweeps=True, want_fail=True)
        b = L.decode_rounds(code, P, e0, shot0=shot0, form=form, want_beliefs=True, want_sweeps=True,
                            want_fail=True)
        torch.cuda.synchronize()
        _same(a, b, ("z", "s", "tclr", "L", "sweeps", "fail"))
        if call == 0:
            k = min(S, 16)
            o = orc.decode(spec, orc.DecodeParams(bp=bp, q=q, rounds=24), e0[:k].cpu().numpy(),
                           shot0=shot0, nthreads=8)
            assert np.array_equal(a["z"][:k].cpu().numpy(), o["z"])
            assert np.array_equal(a["tclr"][:k].cpu().numpy(), o["tclr"])


def test_static_scratch_refuses_work_beyond_its_size(L):
    """The stream form of 2D toric L=32 at 65536 shots needs about 2.4 GiB of
    scratch: the call fails with LAIM_ENOMEM and writes nothing; the resident
    form of the same batch needs only the shot queue and runs."""
    import torch
    code = L.Code(codes.toric_2d(32), 0)
    P = L.DecodeParams(rounds=4)
    S = 65536
    assert L.workspace_bytes(code, P, S, "stream") > L.STATIC_SCRATCH_BYTES
    e0 = L.sample_noise(code, 0.05, 0, 0, S)
    out = {"z": torch.full((S, code.n), 7, dtype=torch.uint8, device="cuda"),
           "s": torch.full((S, code.m), 7, dtype=torch.uint8, device="cuda"),
           "tclr": torch.full((S,), 7, dtype=torch.int32, device="cuda"), "L": None, "sweeps": None,
           "fail": None}
    with pytest.raises(L.LaimError) as ei:
        L.decode_rounds_static(code, P, e0, form="stream", out=out)
    assert ei.value.status == L.ENOMEM
    torch.cuda.synchronize()
    assert bool((out["z"] == 7).all()) and bool((out["tclr"] == 7).all())
    a = L.decode_rounds_static(code, P, e0, form="resident")
    b = L.decode_rounds(code, P, e0, form="resident")
    torch.cuda.synchronize()
    _same(a, b, ("z", "s", "tclr"))
