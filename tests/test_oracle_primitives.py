"""Pins of the oracle's primitives: Philox4x32-10, Bernoulli sampling, the
FP32 functions behind the sum-product rule, and the Evidence thresholds.

Each primitive is checked against something other than itself: an
independent library implementation, a closed form, or a statistical law.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch_include():
    try:
        import torch
    except Exception:  # pragma: no cover
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")) else None


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    inc = _torch_include()
    if inc is None or shutil.which("g++") is None:
        pytest.skip("PyTorch headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("philox") / "torch_philox_ref")
    subprocess.run(["g++", "-O1", "-std=c++17", f"-I{inc}",
                    os.path.join(HERE, "philox_ref", "torch_philox_ref.cpp"), "-o", exe], check=True)

    def run(ctr, key):
        lines = "\n".join(" ".join(str(int(x)) for x in (*c, *k)) for c, k in zip(ctr, key))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
        return np.array([[int(w) for w in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint64)
    return run


def test_philox_matches_independent_implementation(orc, torch_philox):
    """Philox4x32-10 (Salmon et al., SC'11) word for word against ATen's engine."""
    rng = np.random.default_rng(123)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(2000, 2), dtype=np.uint64).astype(np.uint32)
    # include the corners of the counter space
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    key[1] = 0xFFFFFFFF
    mine = orc.philox(ctr, key).astype(np.uint64)
    ref = torch_philox(ctr, key)
    assert np.array_equal(mine, ref)


def test_philox_zero_vector(orc):
    """Counter 0, key 0: the well-known first output block of Philox4x32-10."""
    out = orc.philox([0, 0, 0, 0], [0, 0])[0]
    assert [hex(int(w)) for w in out] == ["0x6627e8d5", "0xe169c58d", "0xbc57ac4c", "0x9b00dbd8"]


def test_philox_uniformity(orc):
    """Chi-square of the top byte of 2^18 words is consistent with uniform."""
    k = 1 << 16
    ctr = np.zeros((k, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(k)
    ctr[:, 3] = 7
    key = np.tile(np.array([[5, 9]], dtype=np.uint32), (k, 1))
    w = orc.philox(ctr, key).ravel()
    counts = np.bincount((w >> 24).astype(np.int64), minlength=256)
    exp = w.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 255 dof: mean 255, sd ~22.6; 6 sigma band
    assert 120 < chi2 < 400
    # adjacent words uncorrelated
    u = w.astype(np.float64) / 2**32
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 0.01


def test_bernoulli_bound(orc):
    assert orc.bernoulli_bound(0.0) == 0
    assert orc.bernoulli_bound(-1.0) == 0
    assert orc.bernoulli_bound(1.0) == 2**32
    assert orc.bernoulli_bound(2.0) == 2**32
    assert orc.bernoulli_bound(0.5) == 2**31
    assert orc.bernoulli_bound(0.05) == int(np.floor(0.05 * 2**32))


def test_noise_rate_and_structure(orc):
    """i.i.d. Bernoulli(p) errors (SM, prior): rate, shot-id addressing and
    common random numbers across p."""
    from paper_2609_38139_amd import codes
    c = codes.toric_2d(16)
    e = orc.sample_noise(c, 0.05, 0, 0, 400)
    N = e.size
    rate = e.mean()
    assert abs(rate - 0.05) < 5 * np.sqrt(0.05 * 0.95 / N)
    # shot ids, not positions, address the stream
    assert np.array_equal(orc.sample_noise(c, 0.05, 0, 17, 5), e[17:22])
    # a different seed gives a different stream
    assert not np.array_equal(orc.sample_noise(c, 0.05, 1, 0, 4), e[:4])
    # the same words are thresholded for every p
    e2 = orc.sample_noise(c, 0.08, 0, 0, 400)
    assert np.all(e2 >= e)
    assert orc.sample_noise(c, 0.0, 0, 0, 3).sum() == 0
    assert orc.sample_noise(c, 1.0, 0, 0, 3).min() == 1
    # qubit v uses word v mod 4 of the block floor(v/4) of counter (shot, 0, v/4, 0)
    words = orc.philox([[3, 0, 5, 0]], [[0, 0]])[0]
    bound = orc.bernoulli_bound(0.05)
    one = orc.sample_noise(c, 0.05, 0, 3, 1)[0]
    assert [int(one[20 + j]) for j in range(4)] == [int(int(w) < bound) for w in words]


def test_exp_neg_accuracy(orc):
    x = np.concatenate([np.linspace(0, 80, 200001), [0.0, 1e-30, 1e-8, 0.34657359, 79.99]]).astype(np.float32)
    y = orc.exp_neg(x).astype(np.float64)
    ref = np.exp(-x.astype(np.float64))
    rel = np.abs(y - ref) / ref
    assert rel.max() < 3 * 2.0**-24
    assert orc.exp_neg([0.0])[0] == 1.0
    assert orc.exp_neg([80.5, np.inf])[1] == 0.0 and orc.exp_neg([80.5])[0] == 0.0


def test_log1p_unit_accuracy(orc):
    u = np.concatenate([np.linspace(0, 1, 200001), 2.0 ** -np.arange(1, 140)]).astype(np.float32)
    y = orc.log1p_unit(u).astype(np.float64)
    ref = np.log1p(u.astype(np.float64))
    ok = ref > 0
    assert (np.abs(y - ref)[ok] / ref[ok]).max() < 4 * 2.0**-24
    assert orc.log1p_unit([0.0])[0] == 0.0


def test_boxplus_is_the_check_rule_of_two_inputs(orc):
    """a [+] b equals 2 atanh(tanh(a/2) tanh(b/2)) (BP-LLR2 with two incoming
    messages), here evaluated in 80-bit long double from its definition."""
    rng = np.random.default_rng(7)
    a = np.concatenate([rng.standard_normal(100000) * 8, rng.uniform(-40, 40, 50000)]).astype(np.float32)
    b = np.concatenate([rng.standard_normal(100000) * 8, rng.uniform(-40, 40, 50000)]).astype(np.float32)
    y = orc.boxplus(a, b).astype(np.longdouble)
    ref = 2 * np.arctanh(np.tanh(a.astype(np.longdouble) / 2) * np.tanh(b.astype(np.longdouble) / 2))
    ok = np.isfinite(ref) & (np.abs(a) < 20) & (np.abs(b) < 20)  # long double tanh is exact enough here
    err = np.abs(y - ref)[ok]
    assert float((err / np.maximum(np.abs(ref[ok]), 1)).max()) < 1e-6
    # large arguments: the definition evaluated with 60 significant digits
    import mpmath
    mpmath.mp.dps = 60
    big = np.nonzero((np.abs(a) > 20) | (np.abs(b) > 20))[0][:400]
    for i in big:
        A, B = mpmath.mpf(float(a[i])), mpmath.mpf(float(b[i]))
        exact = 2 * mpmath.atanh(mpmath.tanh(A / 2) * mpmath.tanh(B / 2))
        assert abs(float(y[i]) - float(exact)) <= 2e-7 * max(1.0, abs(float(exact)))


def test_boxplus_symmetries(orc):
    rng = np.random.default_rng(8)
    a = (rng.standard_normal(50000) * 10).astype(np.float32)
    b = (rng.standard_normal(50000) * 10).astype(np.float32)
    y = orc.boxplus(a, b)
    assert np.array_equal(orc.boxplus(b, a), y)  # symmetric
    assert np.array_equal(orc.boxplus(-a, b), -y)  # odd in each argument
    assert np.array_equal(orc.boxplus(a, -b), -y)
    # +inf is the identity (an empty tanh product is 1)
    assert np.array_equal(orc.boxplus(np.full_like(a, np.inf), a), a)
    # a zero message annihilates
    assert np.all(orc.boxplus(np.zeros_like(a), a) == 0)
    # |a [+] b| <= min(|a|, |b|)
    assert np.all(np.abs(y) <= np.minimum(np.abs(a), np.abs(b)))


def test_evidence_thresholds(orc):
    """Evidence(c) >= 1/d_c with Pr = sigmoid(L) is L >= -log(d_c - 1)."""
    t = orc.evidence_thresholds(8)
    assert t[1] == np.inf
    assert t[2] == 0.0 and np.signbit(t[2])
    for d in range(2, 9):
        sig = 1 / (1 + np.exp(-np.float64(t[d])))
        assert abs(sig - 1 / d) < 1e-7
    assert t[4] == np.float32(-np.log(3.0))
    assert t[6] == np.float32(-np.log(5.0))


def _star(dc):
    """One check on dc qubits, each qubit in no other check."""
    from paper_2609_38139_amd import codes
    return codes.from_dense(np.ones((1, dc), dtype=np.uint8))


def _check_inputs(rng, dc, trial):
    kind = trial % 4
    if kind == 0:
        x = rng.standard_normal(dc) * 8
    elif kind == 1:
        x = rng.uniform(-40, 40, dc)
    elif kind == 2:
        x = rng.standard_normal(dc) * 0.5
    else:
        x = rng.uniform(-3, 3, dc) * rng.choice([1, 10], dc)
    return x.astype(np.float32)


def test_sum_product_order_against_definition_and_ascending_fold(orc):
    """The sum-product check rule (BP-LLR2) of the oracle evaluates output j
    as F_{j-1} [+] B_{j+1} (ascending prefix and descending suffix box-plus
    folds). Box-plus is the tanh product written in the log domain, so every
    order computes the same real number; this pins how far the FP32 order
    may move the result, for check degrees 2..8:
      - from the definition 2 atanh(prod_{i != j} tanh(m_i / 2)), evaluated
        with 50 significant digits: at most 1e-6 of max(1, |m|);
      - from the plain ascending fold ((m_0 [+] m_1) [+] m_2) ... of the
        other inputs (same FP32 box-plus): at most 8 ulp of max(1, |m|), and
        bit-identical for d_c <= 3, where the two orders coincide.
    Both include the sign (-1)^{s_c + d_c} and the clamp."""
    import mpmath
    mpmath.mp.dps = 50
    rng = np.random.default_rng(11)
    P = orc.DecodeParams(bp="sumproduct")
    ulp1 = 2.0 ** -23
    for dc in range(2, 9):
        spec = _star(dc)
        sig = (-1) ** dc  # s_c = 0
        for trial in range(240):
            x = _check_inputs(rng, dc, trial)
            mcv, _ = orc.bp_sweep(spec, P, np.zeros(dc, np.float32), np.zeros(1, np.uint8), x)
            for j in range(dc):
                others = [float(x[i]) for i in range(dc) if i != j]
                prod = mpmath.mpf(1)
                for o in others:
                    prod *= mpmath.tanh(mpmath.mpf(o) / 2)
                ref = float(sig * 2 * mpmath.atanh(prod)) if abs(prod) < 1 else sig * np.inf
                ref = min(1000.0, max(-1000.0, ref))
                got = float(mcv[j])
                assert abs(got - ref) <= 1e-6 * max(1.0, abs(ref)), (dc, trial, j, got, ref)
                acc = np.float32(others[0]) + np.float32(0.0)
                for o in others[1:]:
                    acc = orc.boxplus([acc], [o])[0]
                fold = float(np.float32(min(1000.0, max(-1000.0, sig * float(acc)))))
                if dc <= 3:
                    assert got == fold and np.signbit(got) == np.signbit(fold), (dc, j, got, fold)
                else:
                    assert abs(got - fold) <= 8 * ulp1 * max(1.0, abs(fold)), (dc, trial, j, got, fold)
