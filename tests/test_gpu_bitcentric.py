"""Parity of the bit-centric machine on the GPU with the oracle (SM "Setup
and algorithm"): corrections and clearing iterations bit for bit and the
double-precision beliefs of the last iteration equal, on periodic and open
repetition codes up to thousands of bits; and the paper's statement, on the
GPU at scale, that the machine fails exactly when more than half of the bits
are in error."""
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


def compare(L, orc, code, q, p, nshots, iters, seed=0):
    import torch
    print(f"[bitcentric] n={code.H.cols} q={q} p={p} shots={nshots} iters={iters}", flush=True)
    dc = L.Code(code, 0)
    e0 = orc.sample_noise(code, p, seed, 0, nshots)
    g = L.decode_bitcentric(dc, q, torch.from_numpy(e0).cuda(), iters, want_beliefs=True)
    torch.cuda.synchronize()
    z, ic, Lg = g["z"].cpu().numpy(), g["iclr"].cpu().numpy(), g["L"].cpu().numpy()
    for i in range(nshots):
        et, Lt, icl = orc.bitcentric_machine(code, q, e0[i], iters)
        e_last = et[-1] if iters > 0 else e0[i]
        assert np.array_equal(e0[i] ^ z[i], e_last), f"shot {i}: final error differs"
        assert ic[i] == icl, f"shot {i}: i_clr {ic[i]} vs {icl}"
        if iters > 0:
            assert np.array_equal(Lg[i], Lt[-1]), f"shot {i}: beliefs differ"
    return e0, z, ic


@pytest.mark.parametrize("d", [5, 11, 21, 101])
@pytest.mark.parametrize("p", [0.05, 0.25, 0.45])
def test_periodic_repetition(L, orc, d, p):
    compare(L, orc, codes.repetition(d, periodic=True), 0.1, p, 64, d + 3)


def test_open_chain_and_other_priors(L, orc):
    """Bits of degree 1 at the ends; several priors."""
    for q in (0.02, 0.3):
        compare(L, orc, codes.repetition(16, periodic=False), q, 0.2, 48, 20)


def test_long_chains_several_bits_per_thread(L, orc):
    """1001 bits (one per thread) and 2001 bits (two per thread, 148 KB of
    LDS); 2501 bits do not fit in LDS and are refused."""
    import torch
    compare(L, orc, codes.repetition(1001, periodic=True), 0.1, 0.3, 6, 60)
    compare(L, orc, codes.repetition(2001, periodic=True), 0.1, 0.45, 3, 40)
    dc = L.Code(codes.repetition(2501, periodic=True), 0)
    with pytest.raises(L.LaimError):
        L.decode_bitcentric(dc, 0.1, torch.zeros((1, 2501), dtype=torch.uint8, device="cuda"), 4)


def test_no_iterations_and_clear_start(L, orc):
    import torch
    code = codes.repetition(9)
    dc = L.Code(code, 0)
    e0 = np.zeros((2, 9), dtype=np.uint8)
    e0[1, 3] = 1
    g = L.decode_bitcentric(dc, 0.1, torch.from_numpy(e0).cuda(), 0)
    assert g["iclr"].cpu().tolist() == [0, -1]
    assert not g["z"].cpu().numpy().any()


def test_fails_exactly_above_half(L, orc):
    """The SM's theorem: after d iterations on the periodic repetition code
    the machine has not returned to the zero error exactly when |E| > d/2;
    checked on every shot of a large GPU run (so the logical error rate is
    the binomial tail)."""
    import torch
    for d, p in ((31, 0.3), (101, 0.45)):
        code = codes.repetition(d, periodic=True)
        dc = L.Code(code, 0)
        e0 = orc.sample_noise(code, p, 3, 0, 20000)
        g = L.decode_bitcentric(dc, 0.1, torch.from_numpy(e0).cuda(), d)
        e_fin = e0 ^ g["z"].cpu().numpy()
        ok = ~e_fin.any(axis=1)
        assert np.array_equal(ok, e0.sum(axis=1) < d / 2)


def test_rejects_codes_with_other_check_degrees(L):
    import torch
    dc = L.Code(codes.toric_2d(4), 0)
    e0 = torch.zeros((1, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LaimError):
        L.decode_bitcentric(dc, 0.1, e0, 5)
