"""The oracle's pins have teeth: each plausible mistake below, planted in a
copy of the oracle's C source (on the CPU; the committed oracle is not
touched), makes at least one pin test fail.

Every mutation is compiled to a library of its own in a temporary folder and
the named pin tests run against it in a child process, stopping at the first
failure; the test passes when that child reports a failure."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "laim_oracle.c")

# name: (text in the oracle, replacement, pin test files, -k filter or "")
MUTATIONS = {
    "sign convention drops d_c": (
        "int sigma_neg = (int)((s_c + dc) & 1);", "int sigma_neg = (int)(s_c & 1);",
        ["test_oracle_pins.py"], "trees or window or open_chain"),
    "min-sum without alpha": (
        "float mag = P->alpha * minabs;", "float mag = minabs;",
        ["test_oracle_pins.py"], "window"),
    "min-sum ignores input signs": (
        "      if (mvc_row[i] < 0.0f) neg ^= 1;\n", "",
        ["test_oracle_pins.py"], "window or trees or star"),
    "qubit rule keeps its own edge": (
        "float acc = pi_v[v];\n      for (int32_t i = 0; i < dv; ++i)\n        if (i != j) acc",
        "float acc = pi_v[v];\n      for (int32_t i = 0; i < dv; ++i)\n        acc",
        ["test_oracle_pins.py"], "window or open_chain or trees"),
    "continuous machine's qubit rule keeps its own edge": (
        "float acc = pi;\n      for (int32_t i = 0; i < dv; ++i)\n        if (i != j) acc",
        "float acc = pi;\n      for (int32_t i = 0; i < dv; ++i)\n        acc",
        ["test_oracle_ctm.py"], "affine"),
    "beliefs without the prior": (
        "    float acc = pi_v[v];\n    for (int32_t i = T->vptr[v]; i < T->vptr[v + 1]; ++i) acc = acc + mcv[T->vedge[i]];",
        "    float acc = 0.0f;\n    for (int32_t i = T->vptr[v]; i < T->vptr[v + 1]; ++i) acc = acc + mcv[T->vedge[i]];",
        ["test_oracle_pins.py"], "window or open_chain or trees"),
    "round machine ignores the clock mask": (
        "      if (!((uint64_t)w[0] < R_bound)) continue;\n", "",
        ["test_oracle_pins.py"], "feedback_replays"),
    "round machine without the Evidence test": (
        "      if (P->evidence && !(Lmax >= thr[dc])) continue;\n", "",
        ["test_oracle_pins.py"], "feedback_replays"),
    "LocalMove takes the smallest belief": (
        "if (L[T->col[b + j]] > Lmax) Lmax = L[T->col[b + j]];",
        "if (L[T->col[b + j]] < Lmax) Lmax = L[T->col[b + j]];",
        ["test_oracle_pins.py"], "feedback_replays or special"),
    "LocalMove ties split by the wrong word": (
        "uint32_t pick = (uint32_t)(((uint64_t)w[1] * (uint64_t)ntie) >> 32);",
        "uint32_t pick = (uint32_t)(((uint64_t)w[2] * (uint64_t)ntie) >> 32);",
        ["test_oracle_pins.py"], "feedback_replays"),
    "clock draws of another counter": (
        "((uint32_t)r << 4) | 1u", "((uint32_t)r << 4) | 2u",
        ["test_oracle_pins.py"], "feedback_replays"),
    "Evidence bound of the wrong degree": (
        "(float)(-log((double)(d - 1)))", "(float)(-log((double)d))",
        ["test_oracle_primitives.py", "test_oracle_pins.py"], "evidence"),
    "t_clr counted from zero": (
        "if (!any && *tclr < 0) *tclr = rr + 1;", "if (!any && *tclr < 0) *tclr = rr;",
        ["test_oracle_pins.py"], "special"),
    "failure test without the row-space condition": (
        "fail_out[i] = (uint8_t)(any || !in_row_space(&B, n, r, work));", "fail_out[i] = (uint8_t)(any);",
        ["test_oracle_pins.py"], "homology or special"),
    "box-plus correction terms swapped": (
        "float mag = (mn + orc_softplus_neg(aa + ab)) - orc_softplus_neg(diff);",
        "float mag = (mn + orc_softplus_neg(diff)) - orc_softplus_neg(aa + ab);",
        ["test_oracle_primitives.py"], "boxplus"),
    "exp Taylor coefficient": (
        "p = fmaf(p, r, 1.0f / 120.0f);", "p = fmaf(p, r, 1.0f / 100.0f);",
        ["test_oracle_primitives.py"], "exp_neg"),
    "exp without the low part of ln 2": (
        "float r = fmaf(-kf, LN2_TAIL, fmaf(-kf, LN2_HEAD, x));", "float r = fmaf(-kf, LN2_HEAD, x);",
        ["test_oracle_primitives.py"], "exp_neg"),
    "Philox multiplier": (
        "const uint32_t MUL0 = 0xD2511F53u", "const uint32_t MUL0 = 0xD2511F51u",
        ["test_oracle_primitives.py"], "philox"),
    "syndrome of one bit too few": (
        "for (int32_t k = rowptr[c]; k < rowptr[c + 1]; ++k) x ^= e[(size_t)i * n + col[k]] & 1u;",
        "for (int32_t k = rowptr[c] + 1; k < rowptr[c + 1]; ++k) x ^= e[(size_t)i * n + col[k]] & 1u;",
        ["test_oracle_pins.py"], "special or homology or parity"),
    "multi-qubit move takes non-negative beliefs": (
        "          if (L[T->col[b + j]] > 0.0f) {", "          if (L[T->col[b + j]] >= 0.0f) {",
        ["test_oracle_pins.py"], "feedback_replays or positive_beliefs"),
    "multi-qubit move without the LocalMove fallback": (
        "        if (npos > 0) continue;", "        continue;",
        ["test_oracle_pins.py"], "feedback_replays"),
    "sequential rule re-tests the check within a multi-qubit move": (
        "      if (i == 0 || req[i].c != req[i - 1].c || req[i].key != req[i - 1].key) {",
        "      if (1) {",
        ["test_oracle_conflict.py"], "multi_qubit"),
    "online: the carried measurement correction is dropped": (
        "sw[tau * m + c] = (uint8_t)(D[(size_t)(a + tau) * m + c] ^ (tau == 0 ? bnd[c] : 0));",
        "sw[tau * m + c] = (uint8_t)(D[(size_t)(a + tau) * m + c]);",
        ["test_oracle_online.py"], "replay"),
    "online: every window numbers its rounds from 0": (
        "r1 = decode_core(Tw, P, thr, R_bound, pi, sw, shot, k * P->rounds, zw,",
        "r1 = decode_core(Tw, P, thr, R_bound, pi, sw, shot, 0, zw,",
        ["test_oracle_online.py"], "replay"),
    "online: the last round is not perfect": (
        "      if (t < N) {\n        philox_for", "      if (t <= N) {\n        philox_for",
        ["test_oracle_online.py"], "noise"),
    "online: data errors from the measurement counter": (
        "philox_for(seed, shot, (uint32_t)(v >> 2), ((uint32_t)t << 4) | 3u, w);",
        "philox_for(seed, shot, (uint32_t)(v >> 2), ((uint32_t)t << 4) | 4u, w);",
        ["test_oracle_online.py"], "noise"),
    "online: detectors without the previous measurement error": (
        "            if (t > 0) D[(size_t)t * m + c] ^= eps[(size_t)(t - 1) * m + c];\n", "",
        ["test_oracle_online.py"], "replay"),
    "online: a window commits all its rounds": (
        "const int32_t cr = last ? w : C; /* rounds committed */", "const int32_t cr = w;",
        ["test_oracle_online.py"], "replay"),
    "online: window graph without the previous round's measurement variable": (
        "      if (tau >= 1 && tau - 1 < w_eps) cl[k++] = w * n + (tau - 1) * m + c;\n", "",
        ["test_oracle_online.py"], "spacetime_graph"),
    "sequential rule with a stale syndrome": (
        "      for (int32_t k = T->rowptr[req[i].c]; k < T->rowptr[req[i].c + 1]; ++k) x ^= f[T->col[k]];\n", "",
        ["test_oracle_conflict.py"], "sequential"),
    "continuous machine damps by dt instead of dt / tau": (
        "  const float lam = (float)(C->dt / C->tau);\n  int32_t rc = 0;",
        "  const float lam = (float)(C->dt);\n  int32_t rc = 0;",
        ["test_oracle_ctm.py"], "clock_decisions"),
    "continuous machine's Euler steps damp by dt instead of dt / tau": (
        "  const float lam = (float)(C->dt / C->tau);\n  size_t E",
        "  const float lam = (float)(C->dt);\n  size_t E",
        ["test_oracle_ctm.py"], "affine"),
    "continuous machine applies an event one step late": (
        "while (nS > 0 && Tev <= tk)", "while (nS > 0 && Tev < tk - C->dt)",
        ["test_oracle_ctm.py"], "clock_decisions"),
    "continuous machine without the Evidence test": (
        "if (!C->evidence || Lmax >= thr[dc])", "if (1)",
        ["test_oracle_ctm.py"], "clock_decisions"),
}

RUNNER = r"""
import sys
sys.path.insert(0, {root!r})
from oracle import oracle as O
O.LIB = {lib!r}
O.SRC = {src!r}
O._lib = None
import pytest
args = ["-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + {files!r}
if {kexpr!r}:
    args += ["-k", {kexpr!r}]
sys.exit(pytest.main(args))
"""


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new, files, kexpr = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name!r} not unique in the oracle"
    msrc = tmp_path / "laim_oracle_mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = tmp_path / "liblaim_oracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                    "-fopenmp", "-w", "-o", str(lib), str(msrc), "-lm"], check=True)
    code = RUNNER.format(root=ROOT, lib=str(lib), src=str(msrc),
                         files=[os.path.join(ROOT, "tests", f) for f in files], kexpr=kexpr)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=str(tmp_path),
                       timeout=600)
    assert r.returncode == 1, (f"the pins did not catch {name!r} (pytest exit {r.returncode}):\n"
                               + r.stdout[-1500:])
