"""Benchmark of the decoder's hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic shots:
Philox noise -> syndrome, BP rounds with belief-guided moves (one resident
launch) -> homology-class failure test, for the 2D toric code L = 32 at
p = 0.05 with 65536 shots per step, 20 BP sweeps per round and 4L = 128
rounds (normalised min-sum, alpha = 0.75; shots retire once clear). Inputs
are generated on the device (shot ids advance every step) and every buffer
is resident in HBM before the timed region starts.

Prints one JSON line. `value` is decoded shots per second; the line also
carries message updates per second, the roofline of the dominant kernel
measured with HIP events on its stream, the same workload in the stream
form, with sum-product and without early retirement, and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Device peaks used for roofline fractions (MI355X, published).
HBM_PEAK_GBS = 8000.0
CU_COUNT = 256
CLOCK_GHZ = 2.4
# VALU issue: a CU issues up to two wave64 VALU instructions per clock (the
# dual-rate class -- FP32 add, sub, mul, multiply-add with a literal, 32-bit
# integer add, and, xor -- measured at 1.5-1.65 per clock by the probes;
# three-source and most other instructions issue at one per clock, measured
# at 0.88-1.05)
VALU_ISSUE_PER_CLK = 2
VALU_SINGLE_TOPS = CU_COUNT * 64 * CLOCK_GHZ / 1000.0  # 39.3 T lane-ops/s, one instruction per clock
VALU_PEAK_TOPS = VALU_ISSUE_PER_CLK * VALU_SINGLE_TOPS  # 78.6 T lane-ops/s
# LDS reads: 256 B per clock per CU (conflict-free 16-byte reads reach 97% of
# it in the probe); narrower reads and every write form run slower (the
# probe's table). The resident kernels' LDS side is priced by the measured
# rates of the two access forms their sweeps use.
LDS_BYTES_PER_CLK = 256  # per CU, reads
LDS_PEAK_TBS = CU_COUNT * LDS_BYTES_PER_CLK * CLOCK_GHZ / 1000.0  # 157.3 TB/s


RESIDENT_SOURCES = ("paper_2609_38139_amd/csrc/laim_kernels.hip", "paper_2609_38139_amd/csrc/device_math.h",
                    "paper_2609_38139_amd/csrc/laim_internal.h", "paper_2609_38139_amd/build.py")


STREAM_SOURCES = ("paper_2609_38139_amd/csrc/laim_stream.hip", "paper_2609_38139_amd/csrc/device_math.h",
                  "paper_2609_38139_amd/csrc/laim_internal.h", "paper_2609_38139_amd/build.py")


BITCENTRIC_SOURCES = ("paper_2609_38139_amd/csrc/laim_bitcentric.hip", "paper_2609_38139_amd/csrc/device_math.h",
                      "paper_2609_38139_amd/csrc/laim_internal.h", "paper_2609_38139_amd/build.py")


def profile_fields(profile: str, sources):
    """The machine-readable fields of a committed rocprofv3 summary, or None
    when the kernel sources (hashed in order) differ from the profiled ones."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ": " in line:
            k, v = line.strip().split(": ", 1)
            fields[k] = v
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return fields if fields.get("source_sha256") == h.hexdigest() else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the first three decode launches of a process run 3-10% slower than the
    # rest (6.26, 6.04, 5.85 ms, then 5.65-5.70 on the measured workload):
    # five untimed steps, then twenty timed ones
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--L", type=int, default=32)
    ap.add_argument("--p", type=float, default=0.05)
    ap.add_argument("--shots", type=int, default=65536)
    ap.add_argument("--rounds", type=int, default=0, help="default 4L")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--bp", default="minsum", choices=["minsum", "sumproduct"])
    ap.add_argument("--form", default="resident", choices=["resident", "stream", "auto"])
    ap.add_argument("--no-retire", action="store_true")
    ap.add_argument("--no-skip", action="store_true",
                    help="run every BP sweep (no skipping at a fixed point of the messages)")
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true", help="built-in resident launch shape")
    ap.add_argument("--cfg", default="", help="resident shape 'checks_per_thread,shots_per_block'")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="copy this many MiB device-to-device first (counter calibration)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-plan comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-seconds", type=float, default=4.0, help="open-loop time per arrival rate")
    ap.add_argument("--no-matrix", action="store_true",
                    help="skip the other benchmark configurations (2D sizes and p sweep, 3D, BB)")
    ap.add_argument("--probe-only", action="store_true", help="run the VALU and LDS probes and exit")
    ap.add_argument("--leg", default="", choices=["", "continuous", "matrix_3d", "matrix_bb", "online", "bitcentric"],
                    help="run one secondary measurement alone, print it as JSON and exit (for profiling)")
    return ap.parse_args()


def batch_vs_plain(laim, codes):
    """Several codes' shots in one batched plan (one persistent launch,
    replayed from a HIP graph) against plain launches: one stream-form decode
    per code (messages in HBM, one launch per sweep). Same shots, same
    outputs; shots/s of each."""
    import torch
    mix = [("bb:6x6", 0.005, 64, 65536), ("bb:12x6", 0.005, 64, 65536),
           ("toric2d:16", 0.05, 64, 16384), ("toric2d:32", 0.05, 128, 16384)]
    items = []
    for name, p, R, S in mix:
        code = laim.Code(codes.by_name(name), 0)
        P = laim.DecodeParams(rounds=R)
        e0 = laim.sample_noise(code, p, 0, 0, S)
        items.append({"code": code, "params": P, "e0": e0, "shot0": 0})
    plan = laim.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    outs = plan.launch()
    b.record()
    torch.cuda.synchronize()
    t_batch = a.elapsed_time(b) / 1000
    fails_b = [int(o["fail"].sum()) for o in outs]
    t_plain = 0.0
    fails_p = []
    for it in items:
        ws = torch.empty((laim.workspace_bytes(it["code"], it["params"], it["e0"].shape[0], "stream"),),
                         dtype=torch.uint8, device="cuda")
        a.record()
        r = laim.decode_rounds(it["code"], it["params"], it["e0"], form="stream", workspace=ws)
        f = laim.logical_failure(it["code"], it["e0"], r["z"])
        b.record()
        torch.cuda.synchronize()
        t_plain += a.elapsed_time(b) / 1000
        fails_p.append(int(f.sum()))
        del ws
    shots = sum(S for _, _, _, S in mix)
    return {"codes": [f"{n} p={p} R={R} S={S}" for n, p, R, S in mix],
            "batched_shots_per_s": round(shots / t_batch, 1),
            "plain_stream_shots_per_s": round(shots / t_plain, 1),
            "speedup": round(t_plain / t_batch, 2),
            "failures_batched": fails_b, "failures_plain": fails_p,
            "identical_failures": fails_b == fails_p}


def per_shot_plain(laim, codes):
    """The small configuration (2D toric L=8, p = 0.02..0.08, 1000 shots each,
    64 rounds): the plain method -- one decode launch per shot -- against one
    batched plan holding all 4000 shots. Same shots, bit-identical outputs;
    shots/s of each (wall time of the whole sequence, inputs resident)."""
    import time

    import torch
    code = laim.Code(codes.toric_2d(8), 0)
    ps = (0.02, 0.04, 0.06, 0.08)
    P = laim.DecodeParams(rounds=64)
    items = [{"code": code, "params": P, "e0": laim.sample_noise(code, p, 0, 0, 1000), "shot0": 0} for p in ps]
    plan = laim.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = plan.launch()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    n = code.n
    plain = []
    ws = torch.empty((max(laim.workspace_bytes(code, P, 1, "auto"), 256),), dtype=torch.uint8, device="cuda")
    for it in items:
        plain.append({"z": torch.empty((1000, n), dtype=torch.uint8, device="cuda"),
                      "s": torch.empty((1000, code.m), dtype=torch.uint8, device="cuda"),
                      "tclr": torch.empty((1000,), dtype=torch.int32, device="cuda")})
    laim.decode_rounds(code, P, items[0]["e0"][:1], workspace=ws)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it, o in zip(items, plain):
        for i in range(1000):
            laim.decode_rounds(code, P, it["e0"][i:i + 1], shot0=i, workspace=ws,
                               out={"z": o["z"][i:i + 1], "s": o["s"][i:i + 1],
                                    "tclr": o["tclr"][i:i + 1], "L": None})
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = all(torch.equal(a[k], b[k]) for a, b in zip(outs, plain) for k in ("z", "s", "tclr"))
    ler = {}
    for p, it, o in zip(ps, items, plain):
        f = laim.logical_failure(code, it["e0"], o["z"])
        ler[str(p)] = float(f.float().mean())
    res = {"workload": "2D toric L=8, p in {0.02,0.04,0.06,0.08}, seed 0, 1000 shots each, min-sum, "
                       "64 rounds, retire on clear",
           "plain_per_shot_shots_per_s": round(4000 / t_plain, 1),
           "batched_shots_per_s": round(4000 / t_batch, 1),
           "speedup": round(t_plain / t_batch, 1), "identical_outputs": bool(same),
           "logical_error_rate": ler}
    gpu = [{"e0": it["e0"].cpu().numpy(), "z": o["z"].cpu().numpy(), "s": o["s"].cpu().numpy(),
            "tclr": o["tclr"].cpu().numpy()} for it, o in zip(items, outs)]
    return res, gpu


# Shots per launch of the continuous machine. A shot holds one block until it
# clears or reaches t_max, and the shots that do not clear run about four times
# longer than the rest: with fewer shots than about 16 per block slot of the
# GPU, the end of a launch leaves most of the chip idle (sum-product at 2,048
# shots runs at 0.70 of its 16,384-shot rate).
CTM_SHOTS = 16384


def continuous_machine(laim, L, p, bp, nshots, t_max, reps=2):
    """The continuous-time machine (Algorithm 1 as stated) on the same code:
    Table S1's dt = 0.001 and tau = 0.1, a shot failing if not clear by
    t_max. Reports shots/s, Euler shot-steps/s and the VALU roofline of the
    kernel. Work per check and Euler step: the check update of the round
    machine (19 operations for a degree-4 check, gather included) plus, for
    each of the 2 d_c messages, the Euler update (subtract, multiply, add):
    19 + 6 d_c = 43. Every clamp is idle here (alpha < 1, dt/tau <= 1 and
    |pi|/(1 - alpha) < CLAMP: the Euler update is a convex combination) and
    is not executed; with the clamps it would be 23 + 8 d_c."""
    import math

    import torch

    from paper_2609_38139_amd import codes
    spec = codes.toric_2d(L)
    code = laim.Code(spec, 0)
    dt = 0.001
    P = laim.ContinuousParams(bp=bp, dt=dt, tau=0.1, t_max=t_max)
    e0 = laim.sample_noise(code, p, 0, 7 * 10**9, nshots)
    ws = torch.empty((laim.CONTINUOUS_WORKSPACE_BYTES,), dtype=torch.uint8, device="cuda")
    laim.decode_continuous(code, P, e0, shot0=7 * 10**9, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(reps):
        ev0.record(st)
        out = laim.decode_continuous(code, P, e0, shot0=7 * 10**9, want_fail=True, workspace=ws,
                                     want_steps=True)
        ev1.record(st)
        torch.cuda.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    sec = min(ms) / 1000.0
    computed = int(out["steps"].sum().item())
    # the same launch computing every Euler step (identical outputs)
    P_all = laim.ContinuousParams(bp=bp, dt=dt, tau=0.1, t_max=t_max, skip_fixed=False)
    ev0.record(st)
    laim.decode_continuous(code, P_all, e0, shot0=7 * 10**9, workspace=ws)
    ev1.record(st)
    torch.cuda.synchronize()
    sec_all = ev0.elapsed_time(ev1) / 1000.0
    tclr = out["tclr"].cpu().numpy()
    K = int(math.floor(t_max / dt + 0.5))
    # Euler steps run by each shot: up to the step whose time first reaches the
    # clearing event, or all K
    steps = 0
    for T in tclr:
        if T < 0:
            steps += K
        else:
            k = max(0, math.ceil(T / dt) - 1)
            while k * dt < T:
                k += 1
            steps += min(k, K)
    m = code.m
    dc = code.dc_max
    # the check and qubit rules (min-sum without its idle clamps; sum-product
    # as ops_per_check_sweep counts it), then the damped Euler update of both
    # directions: a subtract, a multiply-add and a clamp per message
    if bp == "minsum":
        ops_check = (dc * (code.dv_max - 1) + (dc + 1) // 2 + 1 + dc * max(0, (dc - 1) // 2) + 2 * dc
                     + 6 * dc)
    else:
        ops_check = ops_per_check_sweep("sumproduct", dc, code.dv_max, None) + 6 * dc
    res = {"workload": f"2D toric L={L}, p={p}, {bp}, dt={dt}, tau=0.1, t_max={t_max}, {nshots} shots",
           "shots_per_s": round(nshots / sec, 1), "decode_ms": round(sec * 1e3, 3),
           "euler_steps_computed_frac": round(computed / max(1, steps), 4),
           "euler_shot_steps_per_s": computed / sec, "msg_updates_per_s": 2 * code.E * computed / sec,
           "euler_shot_steps_of_the_method_per_s": steps / sec,
           "every_step": {"shots_per_s": round(nshots / sec_all, 1), "decode_ms": round(sec_all * 1e3, 3),
                          "what": "skip_fixed = 0: every Euler step computed; identical outputs"},
           "cleared": int((tclr >= 0).sum()), "logical_error_rate": float(out["fail"].float().mean().item()),
           "uncleared_at_t_max": float((tclr < 0).mean()),
           "wrong_class": float(((out["tclr"] >= 0) & (out["fail"] > 0)).float().mean().item()),
           "mean_tclr_cleared": float(tclr[tclr >= 0].mean()) if (tclr >= 0).any() else None}
    # only the computed steps count as work
    ach = computed * m * ops_check / sec / 1e12
    res["roofline"] = {"bound": "alu", "achieved": round(ach, 3), "peak": round(VALU_PEAK_TOPS, 1),
                       "unit": "Tops/s", "frac": round(ach / VALU_PEAK_TOPS, 4), "ops_per_check_step": ops_check}
    ach_all = steps * m * ops_check / sec_all / 1e12
    res["every_step"]["roofline"] = {"achieved": round(ach_all, 3), "frac": round(ach_all / VALU_PEAK_TOPS, 4)}
    return res


def bitcentric(laim, d=101, p=0.3, nshots=262144, q=0.1):
    """The bit-centric machine on the periodic repetition code (SM "Setup and
    algorithm"), d iterations: shots/s in the chain form (the default for
    chains; average of 10 launches) and in the block form (of 2), and the
    logical error rate beside the binomial tail P(|E| > d/2) it must equal."""
    import torch
    from scipy.stats import binom

    from paper_2609_38139_amd import codes
    code = laim.Code(codes.repetition(d, periodic=True), 0)
    e0 = laim.sample_noise(code, p, 5, 0, nshots)
    st = torch.cuda.current_stream()

    def timed(form, reps):
        # reps launches back to back, so the host's work for a launch overlaps
        # the previous one and the events time the kernels
        laim.decode_bitcentric(code, q, e0, d, form=form)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        for _ in range(reps):
            out = laim.decode_bitcentric(code, q, e0, d, stream=st, form=form)
        ev1.record(st)
        torch.cuda.synchronize()
        return out, ev0.elapsed_time(ev1) / 1000.0 / reps

    out, sec = timed("chain", 10)
    out_b, sec_b = timed("block", 2)
    fail = (e0 ^ out["z"]).any(dim=1).float().mean().item()
    ic = out["iclr"]
    # Work per bit and iteration in the frame of the current error, where the
    # chain form runs the machine: the two outgoing messages (prior plus the
    # other incoming message: 2 double adds), the belief (1 double add) and
    # the new error bit from the belief's sign (2 compares, > 0 and < 0): 5
    # operations, against one VALU instruction per CU per clock (FP64 is not
    # dual-rate). The machine as written (syndrome signs, LLR switches and the
    # syndrome update) takes 13 per bit and iteration; the frame change removes
    # 8 of them exactly.
    ops = 5
    ach = nshots * d * d * ops / sec / 1e12
    roof = {"bound": "alu", "achieved": round(ach, 3), "peak": round(VALU_SINGLE_TOPS, 1), "unit": "Tops/s",
            "frac": round(ach / VALU_SINGLE_TOPS, 4), "ops_per_bit_iteration": ops,
            "kernel": "bitchain_kernel (chain form)", "decode_ms_per_launch": round(sec * 1e3, 4), "launches_timed": 10}
    prof = profile_fields("bitchain_kernel_rep_d101.md", BITCENTRIC_SOURCES) \
        if (d, p, nshots, q) == (101, 0.3, 262144, 0.1) else None
    if prof is not None:
        roof["profile"] = {k: prof[k] for k in ("avg_timed_launch_ns", "executed_valu_per_bit_iteration",
                                                "valu_issue_frac", "source") if k in prof}
    return {"workload": f"periodic repetition d={d}, p={p}, q={q}, {d} iterations, {nshots} shots",
            "form": "chain", "shots_per_s": round(nshots / sec, 1), "decode_ms": round(sec * 1e3, 3),
            "logical_error_rate": fail, "binomial_tail": float(binom.sf(d // 2, d, p)),
            "mean_iclr_cleared": float(ic[ic > 0].float().mean().item()) if bool((ic > 0).any()) else None,
            "block_form": {"shots_per_s": round(nshots / sec_b, 1), "decode_ms": round(sec_b * 1e3, 3),
                           "same_results": bool(torch.equal(out["z"], out_b["z"]) and
                                                torch.equal(out["iclr"], out_b["iclr"]))},
            "roofline": roof}


def serving(laim, seconds):
    """Continuous batching of single-shot requests over the mixed workload:
    2D toric L=16/32/48, 3D toric L=12, bivariate-bicycle [[144,12,12]], each
    decoded for up to 8L rounds (96 for the 3D and BB codes) at p=0.03.
    Saturation is measured closed-loop (every request queued at once); then
    Poisson arrivals at 0.5, 0.8 and 0.95 of it."""
    from paper_2609_38139_amd import serve
    wl = serve.Workload(laim, nreq=4096, p=0.03)
    srv = laim.Server(0, mem_budget=2 << 30, max_slots=4096)
    serve.run(srv, wl, None, 64)  # warm-up
    sat = serve.run(srv, wl, None, 1024)
    out = {"workload": "toric2d L=16/32/48, toric3d_point L=12, bb 12x6; p=0.03; rounds 8L "
                       "(96 for 3D and BB); min-sum, retire on clear; request i = code i mod 5, "
                       "shot id i", "saturation": sat, "open_loop": []}
    for frac in (0.5, 0.8, 0.95):
        rate = frac * sat["requests_per_s"]
        n = max(32, min(4096, int(rate * seconds)))
        r = serve.run(srv, wl, rate, n, rng_seed=1)
        r["fraction_of_saturation"] = frac
        out["open_loop"].append(r)
    # the same 0.95x arrivals with the arena cut to half of what they used at
    # their peak: admission by memory binds, requests wait for room (FIFO)
    last = out["open_loop"][-1]
    budget = max(1 << 20, last["arena_bytes_peak"] // 2)
    srv_b = laim.Server(0, mem_budget=budget, max_slots=4096)
    serve.run(srv_b, wl, None, 64)  # warm-up
    r = serve.run(srv_b, wl, last["rate_req_per_s"], last["requests"], rng_seed=1)
    r["fraction_of_saturation"] = 0.95
    r["arena_budget_bytes"] = budget
    out["memory_bound"] = r
    return out


def ops_per_check_sweep(bp, dc, dv, P):
    """VALU operations that one sweep of one check needs on this instruction
    set, from the definition of the check and qubit rules (not from the
    kernel): the fewest instructions that evaluate the prescribed FP32
    operation sequence, three-input minimum, median and xor counting once.

    Min-sum (normalised, R5):
      d_c (d_v - 1)        qubit-side sums m_{v->c} = pi + sum of the others,
      + d_c                their clamps -- none on qubits of degree 2 with
                           alpha < 1 and |pi| / (1 - alpha) < CLAMP, where the
                           clamp provably cannot bind,
      + ceil(d_c / 2) + 1  sign parity of the inputs (three-input xors, the
                           check's sign folded into +-alpha),
      + d_c ceil((d_c - 2) / 2)  each output's smallest other |m| (three-input
                           minima),
      + 2 d_c              scale and sign of each output;
      = 19 for d_c = 4, d_v = 2.
    Sum-product (box-plus form, R6): the qubit side as above with its d_c
    clamps, 2 sign normalisations of the fold ends, 3 (d_c - 2) box-plus
    steps of 62 operations each (min, |difference|, sum; two softplus terms
    of 26: exp by range clamp, 2 for the reduction index, 2 reduction
    multiply-adds, 7 Horner multiply-adds, 2 for the 2^k scale, the result
    select, and log1p by 9 Horner multiply-adds and a product; the combine
    (2), its floor at 0 (1) and the sign of a nonzero result (4)), and the
    sign and clamp of each output (2 d_c); = 390 for d_c = 4, d_v = 2."""
    if bp == "minsum":
        pi = abs(np.log(P.q / (1.0 - P.q)))
        idle_clamp = dv == 2 and P.alpha < 1.0 and pi < 0.99 * P.clamp * (1.0 - P.alpha)
        return (dc * (dv - 1) + (0 if idle_clamp else dc) + (dc + 1) // 2 + 1
                + dc * max(0, (dc - 1) // 2) + 2 * dc)
    return dc * (dv - 1) + dc + 2 + 3 * (dc - 2) * 62 + 2 * dc


def roofline(laim, code, P, args, form, run, default_workload, steps=None):
    """Roofline of the decode launch of a run of timed steps (duration from
    HIP events on its stream, averaged over the timed launches).

    Resident form: bound by VALU issue, 256 CU x 64 lanes x 2.4 GHz x 2
    instructions per clock (the dual-rate class; one per clock for the others,
    reported beside it). The achieved rate counts ops_per_check_sweep() per
    computed check-sweep. Beside
    it, the on-chip traffic the method needs -- each check-to-qubit message
    written once (4 B) and read by the d_v - 1 other checks of its qubit
    (4 B each) per sweep -- as the time the LDS needs at the probe's measured
    rates for the same access forms, a fraction of the launch, and
    the HBM bytes the launch must move (e0 in; z, s, t_clr, failure out).
    Stream form: HBM bytes of the sweeps (each message 4 B in and out, 1 B of
    syndrome per check) against 8 TB/s."""
    steps = steps or args.steps
    E, m, n, S = code.E, code.m, code.n, args.shots
    dc, dv = code.dc_max, code.dv_max
    msg_per_launch = 2 * E * run["sweeps_exec"] / steps
    check_sweeps = m * run["sweeps_exec"] / steps
    dec_s = run["decode_ms"] / 1000.0
    if form == "stream":
        bytes_per_update = 4.0 + 1.0 / (2.0 * dc)
        if P.skip_fixed:
            # whole tiles skip sweeps: the sweeps computed are not counted per
            # shot, so the bytes of the launch are unknown here (the per-sweep
            # roofline is the plain form's, --no-skip)
            return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                    "traffic": None, "kernel": f"stream form decode (2D toric L={args.L}, {P.bp}, skip_fixed)",
                    "decode_ms_per_launch": round(run["decode_ms"], 3)}
        gbs = msg_per_launch * bytes_per_update / dec_s / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": f"stream form decode (2D toric L={args.L}, {P.bp})",
                "bytes_per_msg_update": bytes_per_update, "decode_ms_per_launch": round(run["decode_ms"], 3)}
    ops = ops_per_check_sweep(P.bp, dc, dv, P)
    tiled = code.resident_variant(P)["tiled"]
    tops = check_sweeps * ops / dec_s / 1e12
    # LDS: each message written once (4 B) and read by the d_v - 1 other
    # checks of its qubit (4 B each) per sweep; busy time at the measured
    # rates of the two access forms. In the tiled variant only the 12
    # messages on a tile's boundary (of 32 per 8 checks) go through LDS in a
    # sweep (the inner 20 are written and read back once per round that
    # swept, not counted here).
    rd_b, wr_b = 4 * dc * (dv - 1), 4 * dc
    if tiled:
        rd_b = wr_b = 4 * 12 / 8
    rates = lds_rates()
    lds_busy = check_sweeps * (rd_b / rates["read_b32"] + wr_b / rates["write2_stride65"]) / 1e12 / dec_s
    hbm_b = S * (2 * n + m + 5)
    shape = code.resident_cfg(P.bp)
    prof = None
    if default_workload:
        prof = profile_fields(f"resident_kernel_toric2d_L32_{P.bp}.md", RESIDENT_SOURCES)
        if prof is not None and prof.get("launch_shape") != f"{shape['checks_per_thread']},{shape['shots_per_block']}":
            prof = None
    traffic = float(prof["traffic_bytes_per_launch"]) if prof and "traffic_bytes_per_launch" in prof else None
    out = {"bound": "alu", "achieved": round(tops, 3), "peak": round(VALU_PEAK_TOPS, 1), "unit": "Tops/s",
           "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": traffic,
           "frac_of_single_issue": round(tops / VALU_SINGLE_TOPS, 4),
           "kernel": f"{'resident_tile_kernel' if tiled else 'resident_kernel'} (2D toric L={args.L}, {P.bp}, "
                     f"shape {shape['checks_per_thread']} checks per thread x {shape['shots_per_block']} shots "
                     f"per block{', 2x4 check tiles with inner messages in registers' if tiled else ''})",
           "ops_per_check_sweep": ops, "ops_per_msg_update": ops / (2.0 * dc),
           "decode_ms_per_launch": round(run["decode_ms"], 3), "launches_timed": steps,
           "check_sweeps_computed_per_launch": check_sweeps,
           "lds": {"read_bytes_per_check_sweep": rd_b, "write_bytes_per_check_sweep": wr_b,
                   "read_TBs": round(check_sweeps * rd_b / dec_s / 1e12, 2),
                   "write_TBs": round(check_sweeps * wr_b / dec_s / 1e12, 2),
                   "probe_read_b32_TBs": round(rates["read_b32"], 2),
                   "probe_write2_TBs": round(rates["write2_stride65"], 2),
                   "busy_frac": round(lds_busy, 4),
                   "what": "time the LDS needs for the sweeps' reads and writes at the probe's rates "
                           "for the same access forms, as a fraction of the launch"},
           "hbm": {"algorithmic_bytes_per_launch": hbm_b, "GBs": round(hbm_b / dec_s / 1e9, 1),
                   "frac": round(hbm_b / dec_s / 1e9 / HBM_PEAK_GBS, 5)}}
    if prof is not None:
        out["profile"] = {k: prof[k] for k in ("avg_timed_launch_ns", "executed_valu_per_check_sweep",
                                               "valu_issue_frac", "source") if k in prof}
    return out


def host_cores():
    """Threads for the CPU oracle -- every core this process may use: the CPU
    affinity mask, bounded by the cgroup CPU quota when there is one -- and
    what the host reports about itself."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = int(q) / int(per)
    except (OSError, ValueError):
        pass
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = aff if quota is None else max(1, min(aff, int(quota)))
    return threads, {"nproc": aff, "cpu_count": os.cpu_count(), "cgroup_cpu_quota": quota,
                     "cpu_model": model, "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def _probe_lib():
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2609_38139_amd", "liblaim_probe.so"))
    lib.laim_probe_valu.restype = C.c_double
    lib.laim_probe_valu.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p]
    lib.laim_probe_lds.restype = C.c_double
    lib.laim_probe_lds.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p]
    lib.laim_probe_valu_name.restype = C.c_char_p
    lib.laim_probe_valu_name.argtypes = [C.c_int32]
    lib.laim_probe_valu_kinds.restype = C.c_int32
    lib.laim_probe_lds_per_step.restype = C.c_int32
    return lib


LDS_MODES = (("read", 4), ("read", 8), ("read", 16), ("write", 4), ("write", 8), ("write", 16),
             ("write2_stride65", 8))


def lds_probe_tbs(lib, mode, out, blocks=2048, iters=2048):
    """Device-wide TB/s of LDS probe `mode` (32 KiB per block, 5 blocks per CU)."""
    import ctypes as C
    ms = lib.laim_probe_lds(mode, blocks, iters, C.c_void_p(out.data_ptr()))
    if ms <= 0:
        raise RuntimeError(f"LDS probe {mode} failed ({ms})")
    return blocks * 256 * iters * lib.laim_probe_lds_per_step() * LDS_MODES[mode][1] / (ms * 1e-3) / 1e12


_LDS_RATES = {}


def lds_rates():
    """Measured LDS rates (TB/s, whole device) of the access forms the
    resident sweeps use: conflict-free ds_read_b32 (the partner gathers) and
    ds_write2_b32 with the dwords 65 words apart (the message writes). Once
    per process."""
    import torch
    if not _LDS_RATES:
        lib = _probe_lib()
        out = torch.empty((2048 * 256,), dtype=torch.float32, device="cuda")
        _LDS_RATES["read_b32"] = lds_probe_tbs(lib, 0, out)
        _LDS_RATES["write2_stride65"] = lds_probe_tbs(lib, 6, out)
        del out
    return _LDS_RATES


def probes():
    """Issue rate of one VALU instruction class at a time (eight independent
    chains per lane, 2048 blocks of 256 threads) and LDS bandwidth of
    conflict-free 4-, 8- and 16-byte accesses, from the probe library built
    beside the decoder."""
    import ctypes as C

    import torch
    lib = _probe_lib()
    blocks, iters = 2048, 2048
    out = torch.empty((blocks * 256,), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    valu = {}
    for k in range(lib.laim_probe_valu_kinds()):
        ms = lib.laim_probe_valu(k, blocks, iters, C.c_void_p(out.data_ptr()))
        if ms <= 0:
            raise RuntimeError(f"VALU probe {k} failed ({ms})")
        rate = blocks * 256 * iters * 64 / (ms * 1e-3) / 1e12
        valu[lib.laim_probe_valu_name(k).decode()] = {
            "T_lane_ops_per_s": round(rate, 2), "per_CU_clock": round(rate / VALU_SINGLE_TOPS, 3)}
    lds = {}
    for mode, (what, width) in enumerate(LDS_MODES):
        tbs = lds_probe_tbs(lib, mode, out, blocks, iters)
        lds[f"{what}_b{8 * width}"] = {"TB_per_s": round(tbs, 2), "frac_of_peak": round(tbs / LDS_PEAK_TBS, 3),
                                       "bytes_per_CU_clock": round(tbs * 1e12 / (CU_COUNT * CLOCK_GHZ * 1e9), 1)}
    return {"valu_peak_T_lane_ops_per_s": round(VALU_PEAK_TOPS, 1),
            "valu_single_issue_T_lane_ops_per_s": round(VALU_SINGLE_TOPS, 1),
            "lds_peak_TB_per_s": round(LDS_PEAK_TBS, 1), "valu": valu, "lds": lds}


def one_launch(laim, code, P, p, S, seed=0, shot0=0, form="resident", reps=1):
    """One decode launch of S fresh shots (noise drawn first), timed with HIP
    events on the stream it runs on; the fastest of reps."""
    import torch
    st = torch.cuda.current_stream()
    e0 = laim.sample_noise(code, p, seed, shot0, S)
    out = laim.decode_rounds(code, P, e0, shot0=shot0, form=form, want_fail=True, want_sweeps=True)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        laim.decode_rounds(code, P, e0, shot0=shot0, form=form, workspace=out["workspace"], out=out)
        b.record(st)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    t = out["tclr"]
    f = out["fail"]
    return {"ms": round(best, 3), "shots_per_s": round(S / (best / 1000), 1),
            "logical_error_rate": float(f.float().mean().item()),
            "stuck": float((t < 0).float().mean().item()),
            "wrong_class": float(((t >= 0) & (f > 0)).float().mean().item()),
            "msg_updates_per_s": 2 * code.E * int(out["sweeps"].sum().item()) / (best / 1000)}


def matrix_2d(laim, codes, sizes=(16, 32, 64), S=65536):
    """2D toric L in {16, 32, 64}, p = 0.01 .. 0.10, both BP rules, 65536
    shots per launch, 4L rounds of 20 sweeps, retiring at clear, in the
    resident form with its built-in launch shape: one launch each."""
    rows = []
    for L in sizes:
        code = laim.Code(codes.toric_2d(L), 0)
        for bp in ("minsum", "sumproduct"):
            P = laim.DecodeParams(bp=bp, rounds=4 * L)
            for k in range(1, 11):
                p = k / 100.0
                r = one_launch(laim, code, P, p, S, shot0=0)
                rows.append(dict(code=f"toric2d:{L}", bp=bp, p=p, rounds=4 * L, shots=S, **r))
                print(f"[bench] 2D toric L={L} {bp} p={p}: {r['shots_per_s']:.0f} shots/s, "
                      f"LER {r['logical_error_rate']:.4f}", flush=True, file=sys.stderr)
    return rows


def plan_leg(laim, codes, spec_list, seed=1, reps=2):
    """One batched plan over (name, p, q, rounds, shots) items, replayed;
    per item the logical error rate, for the plan the shots/s of a replay."""
    import torch
    items = []
    for name, p, q, R, S in spec_list:
        code = laim.Code(codes.by_name(name), 0)
        P = laim.DecodeParams(q=q, rounds=R)
        items.append({"code": code, "params": P, "e0": laim.sample_noise(code, p, seed, 0, S), "shot0": 0,
                      "name": name, "p": p})
    plan = laim.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        outs = plan.launch()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    S = sum(it["e0"].shape[0] for it in items)
    per = [{"code": it["name"], "p": it["p"], "shots": it["e0"].shape[0], "rounds": it["params"].rounds,
            "logical_error_rate": float(o["fail"].float().mean().item()),
            "stuck": float((o["tclr"] < 0).float().mean().item())} for it, o in zip(items, outs)]
    return {"ms": round(best, 3), "shots_per_s": round(S / (best / 1000), 1), "items": per}, items, outs


def matrix_3d(laim, codes):
    """Both 3D toric sectors at L = 8, 16, 24 in one batched launch of 16384
    shots each (4L rounds, min-sum; prior 0.05 for the point sector, 0.125
    for the membrane sector), at the ends and middle of each sector's noise
    range: point 0.01, 0.04, 0.08; membrane 0.01, 0.03, 0.05."""
    out = []
    for pp, pm in ((0.01, 0.01), (0.04, 0.03), (0.08, 0.05)):
        spec = [(f"toric3d_point:{n}", pp, 0.05, 4 * n, 16384) for n in (8, 16, 24)]
        spec += [(f"toric3d_membrane:{n}", pm, 0.125, 4 * n, 16384) for n in (8, 16, 24)]
        r, _, _ = plan_leg(laim, codes, spec, reps=1)
        r["p_point"], r["p_membrane"] = pp, pm
        out.append(r)
        print(f"[bench] 3D mixed plan p={pp}/{pm}: {r['shots_per_s']:.0f} shots/s", flush=True, file=sys.stderr)
    return out


def matrix_bb(laim, codes):
    """Bivariate-bicycle (6,6) and (12,6) at 262144 shots per p, p = 0.001 ..
    0.010, with 2D toric L = 16 and 32 (p = 0.05), all in one batched launch
    (64 rounds for BB, 4L for toric, min-sum); then the same items as one
    resident launch per item, to isolate what one plan and one graph buy."""
    import torch
    spec = [(f"bb:{lm}", k / 1000.0, 0.05, 64, 262144) for lm in ("6x6", "12x6") for k in range(1, 11)]
    spec += [("toric2d:16", 0.05, 0.05, 64, 65536), ("toric2d:32", 0.05, 0.05, 128, 65536)]
    r, items, outs = plan_leg(laim, codes, spec, reps=2)
    st = torch.cuda.current_stream()
    singles = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for it in items:  # warm-up and outputs
        singles.append(laim.decode_rounds(it["code"], it["params"], it["e0"], want_fail=True))
    torch.cuda.synchronize()
    a.record(st)
    for it, o in zip(items, singles):
        laim.decode_rounds(it["code"], it["params"], it["e0"], workspace=o["workspace"], out=o)
    b.record(st)
    torch.cuda.synchronize()
    ms_single = a.elapsed_time(b)
    same = all(torch.equal(o[k], s[k]) for o, s in zip(outs, singles) for k in ("z", "s", "tclr", "fail"))
    S = sum(it["e0"].shape[0] for it in items)
    r["per_code_resident_launches"] = {"ms": round(ms_single, 3), "shots_per_s": round(S / (ms_single / 1000), 1),
                                       "identical_outputs": bool(same),
                                       "what": "one resident decode launch per item, back to back on one stream"}
    r["batched_over_per_code_resident"] = round(ms_single / r["ms"], 3)
    print(f"[bench] BB + toric plan: {r['shots_per_s']:.0f} shots/s; per-code resident "
          f"{r['per_code_resident_launches']['shots_per_s']:.0f}", flush=True, file=sys.stderr)
    return r


def online_leg(laim, codes, bp="sumproduct", S=65536):
    """Online decoding in overlapping spacetime windows: 2D toric L = 16, 16
    syndrome rounds (the last perfect), windows of 4 rounds committing 2,
    data and measurement error rates 0.01, 16 machine rounds per window."""
    import torch
    code = laim.Code(codes.toric_2d(16), 0)
    plan = laim.OnlinePlan(code, laim.OnlineParams(rounds_total=16, window=4, commit=2, p=0.01, p_meas=0.01))
    P = laim.DecodeParams(bp=bp, rounds=16)
    out = plan.decode(P, S)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    out = plan.decode(P, S, workspace=out["workspace"])
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    return {"workload": f"2D toric L=16, 16 rounds, windows of 4 committing 2, p = p_meas = 0.01, {bp}, "
                        f"16 machine rounds per window, {S} shots", "ms": round(ms, 3),
            "shots_per_s": round(S / (ms / 1000), 1), "windows_per_s": round(7 * S / (ms / 1000), 1),
            "logical_error_rate": float(out["fail"].float().mean().item()),
            "all_windows_cleared": float((out["cleared"] == 7).float().mean().item())}


def timed_steps(laim, code, P, args, steps, warmup, form, shot_base=0):
    """Runs warmup + steps passes (a pass: noise for fresh shots, then the
    decode with the failure test inside the launch); returns per-step and
    per-decode times (ms) from HIP events on the stream every kernel is
    launched on, plus the failures, rounds run and BP sweeps computed over the
    timed steps -- counted from each step's own outputs after the timed
    region, so that the bench's bookkeeping is not timed."""
    import torch
    S = args.shots
    st = torch.cuda.current_stream()
    e0 = torch.empty((S, code.n), dtype=torch.uint8, device="cuda")
    z = torch.empty((S, code.n), dtype=torch.uint8, device="cuda")
    s = torch.empty((S, code.m), dtype=torch.uint8, device="cuda")

    def outs():
        return {"z": z, "s": s, "tclr": torch.empty((S,), dtype=torch.int32, device="cuda"), "L": None,
                "sweeps": torch.empty((S,), dtype=torch.int32, device="cuda"),
                "fail": torch.empty((S,), dtype=torch.uint8, device="cuda")}

    out_w = outs()
    out_t = [outs() for _ in range(steps)]
    ws = torch.empty((max(laim.workspace_bytes(code, P, S, form), 256),), dtype=torch.uint8, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)

    def step(i, out, evs=None):
        shot0 = shot_base + i * S
        laim.sample_noise(code, args.p, 0, shot0, S, out=e0)
        if evs:
            evs[0].record(st)
        # the decoder failure test runs inside the decode launch (fail_out)
        laim.decode_rounds(code, P, e0, shot0=shot0, form=form, workspace=ws, out=out)
        if evs:
            evs[1].record(st)

    for i in range(warmup):
        step(i, out_w)
    torch.cuda.synchronize()
    t0.record(st)
    for i in range(steps):
        step(warmup + i, out_t[i], ev[i])
    t1.record(st)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    dec_ms = [a.elapsed_time(b) for a, b in ev]
    fails = sum(int(o["fail"].sum().item()) for o in out_t)
    rounds_exec = sum(int(torch.where(o["tclr"] >= 0, o["tclr"], torch.full_like(o["tclr"], P.rounds)).sum().item())
                      for o in out_t)
    sweeps_exec = sum(int(o["sweeps"].sum().item()) for o in out_t)
    return {"ms_per_step": total_ms / steps, "decode_ms": sum(dec_ms) / steps,
            "failures": fails, "rounds_exec": rounds_exec, "sweeps_exec": sweeps_exec, "shots": S * steps}


def cpu_baseline(args, spec, P_or, seconds, nthreads=None, max_shots=4096):
    """The oracle, as it is, on shot ids 0.. of the same workload, in chunks
    until `seconds` of wall time have passed."""
    from oracle import oracle as O
    if nthreads is None:
        nthreads = host_cores()[0]
    done = 0
    rounds = 0
    t0 = time.perf_counter()
    chunk = max(nthreads * 2, 8)
    while time.perf_counter() - t0 < seconds and done < max_shots:
        e0 = O.sample_noise(spec, args.p, 0, done, chunk)
        r = O.decode(spec, P_or, e0, shot0=done, nthreads=nthreads)
        O.logical_failure(spec, e0, r["z"])
        t = r["tclr"]
        rounds += int(((t >= 0) * t + (t < 0) * P_or.rounds).sum())
        done += chunk
    el = time.perf_counter() - t0
    return done, el, nthreads, rounds


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(shots are independent: N GPUs would each take a disjoint range of shot ids)",
              file=sys.stderr)
        return 2
    import torch

    from paper_2609_38139_amd import codes, laim
    torch.cuda.set_device(0)
    if args.probe_only:
        print(json.dumps({"probes": probes()}), flush=True)
        return 0
    if args.leg:
        legs = {"continuous": lambda: {bp: continuous_machine(laim, args.L, args.p, bp, CTM_SHOTS, 30.0)
                                       for bp in ("minsum", "sumproduct")},
                "matrix_3d": lambda: matrix_3d(laim, codes),
                "matrix_bb": lambda: matrix_bb(laim, codes),
                "online": lambda: {bp: online_leg(laim, codes, bp) for bp in ("minsum", "sumproduct")},
                "bitcentric": lambda: bitcentric(laim)}
        print(json.dumps({args.leg: legs[args.leg]()}), flush=True)
        return 0
    L = args.L
    R = args.rounds or 4 * L
    spec = codes.toric_2d(L)
    code = laim.Code(spec, 0)
    E = code.E
    skip = not args.no_skip
    P = laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=not args.no_retire, skip_fixed=skip)
    form = args.form
    if args.calibrate_copy_mb:
        src = torch.ones((args.calibrate_copy_mb << 20,), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuned = None
    if args.cfg:
        cpt, spb = (int(v) for v in args.cfg.split(","))
        code.set_resident_cfg(args.bp, {"checks_per_thread": cpt, "shots_per_block": spb})
    elif not args.no_tune and form != "stream":
        from paper_2609_38139_amd import autotune
        for bp in ("minsum", "sumproduct"):
            t = autotune.tune(code, bp, rounds=R, use_cache=False)
            if bp == args.bp:
                tuned = t
    print("[bench] main: timed steps", flush=True, file=sys.stderr)
    main_run = timed_steps(laim, code, P, args, args.steps, args.warmup, form)
    S_total = main_run["shots"]
    sec = main_run["ms_per_step"] * args.steps / 1000.0
    shots_per_s = S_total / sec
    # message updates the kernels computed (sweeps at a fixed point of the
    # messages are skipped, with identical results)
    msg_computed = 2 * E * main_run["sweeps_exec"]
    msg_per_s = msg_computed / sec
    msg_method = 2 * E * args.iters * main_run["rounds_exec"]
    dec_s = main_run["decode_ms"] / 1000.0
    msg_per_launch = msg_computed / args.steps
    sweeps_frac = main_run["sweeps_exec"] / max(1, args.iters * main_run["rounds_exec"])
    dc, dv = code.dc_max, code.dv_max
    default_workload = (L == 32 and args.p == 0.05 and args.shots == 65536 and R == 128
                        and args.iters == 20 and not args.no_retire)
    rl = roofline(laim, code, P, args, form, main_run, default_workload)

    extras = {}
    small_gpu = None
    sp_line = None
    if args.no_extras:
        args.no_batch = args.no_serve = args.no_matrix = True
    if not args.no_extras:
        print("[bench] probes", flush=True, file=sys.stderr)
        extras["probes"] = probes()
        print("[bench] the other BP rule", flush=True, file=sys.stderr)
        # the paper's BP rule on the same workload: its own timed steps
        other = "sumproduct" if args.bp == "minsum" else "minsum"
        P_o = laim.DecodeParams(bp=other, rounds=R, iters=args.iters, retire=not args.no_retire)
        ro = timed_steps(laim, code, P_o, args, max(2, args.steps // 4), 1, form, shot_base=3 * 10**9)
        sec_o = ro["ms_per_step"] * max(2, args.steps // 4) / 1000.0
        sp_line = {"bp": other, "shots_per_s": round(ro["shots"] / sec_o, 1),
                   "msg_updates_per_s": 2 * E * ro["sweeps_exec"] / sec_o,
                   "logical_error_rate": ro["failures"] / ro["shots"],
                   "sweeps_computed_frac": round(ro["sweeps_exec"] / max(1, args.iters * ro["rounds_exec"]), 4),
                   "ms_per_step": round(ro["ms_per_step"], 3), "decode_ms": round(ro["decode_ms"], 3),
                   "resident_shape": code.resident_cfg(other) if form != "stream" else None,
                   "roofline": roofline(laim, code, P_o, args, form, ro, default_workload,
                                        steps=max(2, args.steps // 4))}
        # stream form (messages in HBM, one launch per sweep): the plain baseline
        print("[bench] stream form", flush=True, file=sys.stderr)
        P_plain = laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=not args.no_retire,
                                    skip_fixed=False)
        rs = timed_steps(laim, code, P_plain, args, 1, 0, "stream", shot_base=10**9)
        # the same launch with the exact shortcuts (identical outputs)
        rk = timed_steps(laim, code, P, args, 1, 0, "stream", shot_base=10**9)
        sec_s = rs["ms_per_step"] / 1000.0
        upd = 2 * E * args.iters * rs["rounds_exec"]
        # each m_{c->v} read once by the partner gather and written once (4 B
        # each) per check-to-qubit update, plus 1 B of syndrome per check
        sweeps_bytes = upd * (4.0 + 1.0 / (2.0 * code.dc_max))
        src = torch.empty((1 << 30,), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        ca, cb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ca.record()
        for _ in range(5):
            dst.copy_(src)
        cb.record()
        torch.cuda.synchronize()
        copy_gbs = 5 * 2 * (1 << 30) / (ca.elapsed_time(cb) / 1000) / 1e9
        del src, dst
        pf = profile_fields("stream_sweep_toric2d_L32_minsum.md", STREAM_SOURCES) if default_workload else None
        sweep_prof = None
        if pf is not None:
            ns = float(pf["avg_launch_ns"])
            alg = 2 * E * 4.0 + code.m * 1.0  # bytes per shot and sweep: E messages in and out, s
            gbs = alg * args.shots / (ns * 1e-9) / 1e9
            sweep_prof = {"kernel": pf.get("kernel"), "avg_launch_ms": round(ns / 1e6, 4),
                          "algorithmic_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "traffic_bytes_per_launch": float(pf["traffic_bytes_per_launch"]),
                          "source": "profiles/stream_sweep_toric2d_L32_minsum.md"}
        extras["stream_form"] = {"shots_per_s": round(rs["shots"] / sec_s, 1),
                                 "sweep_kernel_rocprof": sweep_prof,
                                 "device_copy_GBs": round(copy_gbs, 1),
                                 "msg_updates_per_s": upd / sec_s,
                                 "decode_ms": round(rs["decode_ms"], 2),
                                 "algorithmic_hbm_GBs": round(sweeps_bytes / (rs["decode_ms"] / 1000) / 1e9, 1),
                                 "failures": rs["failures"],
                                 "what": "every sweep of every round (skip_fixed = 0)",
                                 "with_shortcuts": {
                                     "shots_per_s": round(rk["shots"] / (rk["ms_per_step"] / 1000), 1),
                                     "decode_ms": round(rk["decode_ms"], 2), "failures": rk["failures"],
                                     "identical_failures": rk["failures"] == rs["failures"],
                                     "what": "skip_fixed = 1: tiles of 256 shots all retired or at a fixed "
                                             "point skip the sweep; stuck shots stop (identical outputs)"}}
        if skip:
            # the same launch running every sweep: identical results
            rn = timed_steps(laim, code, laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters,
                                                           retire=not args.no_retire, skip_fixed=False),
                             args, 2, 1, form)
            sec_n = rn["ms_per_step"] * 2 / 1000
            extras["every_sweep"] = {
                "shots_per_s": round(rn["shots"] / sec_n, 1),
                "decode_ms": round(rn["decode_ms"], 3),
                "msg_updates_per_s": 2 * E * rn["sweeps_exec"] / sec_n,
                "failures_per_shot": rn["failures"] / rn["shots"],
                "what": "skip_fixed = 0: every BP sweep computed; same z, s, t_clr as the value"}
            if form != "stream":
                rr = roofline(laim, code, laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters,
                                                            retire=not args.no_retire, skip_fixed=False),
                              args, form, rn, False, steps=2)
                extras["every_sweep"]["roofline"] = {k: rr[k] for k in ("achieved", "peak", "unit", "frac")}
        P_fix = laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=False)
        rf = timed_steps(laim, code, P_fix, args, 1, 0, form, shot_base=2 * 10**9)
        extras["fixed_rounds"] = {"shots_per_s": round(rf["shots"] / (rf["ms_per_step"] / 1000), 1),
                                  "msg_updates_per_s": 2 * E * rf["sweeps_exec"] / (rf["ms_per_step"] / 1000),
                                  "failures": rf["failures"]}
        extras["conflict_rules"] = {}
        for rule in ("or", "xor", "sequential"):
            P_c = laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=not args.no_retire,
                                    conflict=rule)
            rc_ = timed_steps(laim, code, P_c, args, 1, 0, form, shot_base=5 * 10**9)
            extras["conflict_rules"][rule] = {
                "shots_per_s": round(rc_["shots"] / (rc_["ms_per_step"] / 1000), 1),
                "failures": rc_["failures"], "logical_error_rate": rc_["failures"] / rc_["shots"],
                "mean_rounds_run": round(rc_["rounds_exec"] / rc_["shots"], 3)}
        extras["moves"] = {}
        for bp in ("minsum", "sumproduct"):
            for mv in ("single", "multi"):
                P_m = laim.DecodeParams(bp=bp, rounds=R, iters=args.iters, retire=not args.no_retire, move=mv)
                rm = timed_steps(laim, code, P_m, args, 1, 0, form, shot_base=6 * 10**9)
                extras["moves"][f"{bp}/{mv}"] = {
                    "shots_per_s": round(rm["shots"] / (rm["ms_per_step"] / 1000), 1),
                    "logical_error_rate": rm["failures"] / rm["shots"],
                    "mean_rounds_run": round(rm["rounds_exec"] / rm["shots"], 3)}
        print("[bench] online decoding", flush=True, file=sys.stderr)
        extras["online"] = {bp: online_leg(laim, codes, bp) for bp in ("minsum", "sumproduct")}
    if not args.no_matrix:
        extras["matrix_2d_toric"] = matrix_2d(laim, codes)
        extras["matrix_3d_toric"] = matrix_3d(laim, codes)
        extras["matrix_bb_with_toric"] = matrix_bb(laim, codes)
    if not args.no_batch:
        extras["batched_vs_plain_stream"] = batch_vs_plain(laim, codes)
        extras["per_shot_plain"], small_gpu = per_shot_plain(laim, codes)
    if not args.no_serve:
        print("[bench] serving", flush=True, file=sys.stderr)
        extras["serving"] = serving(laim, args.serve_seconds)
    if not args.no_extras:
        print("[bench] bit-centric and continuous machines", flush=True, file=sys.stderr)
        extras["bitcentric"] = bitcentric(laim)
        extras["continuous_machine"] = {
            bp: continuous_machine(laim, L, args.p, bp, CTM_SHOTS, 30.0) for bp in ("minsum", "sumproduct")}
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle", flush=True, file=sys.stderr)
        from oracle import oracle as O
        nth, host = host_cores()
        P_or = O.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=not args.no_retire)
        n_done, el, nth, rounds = cpu_baseline(args, spec, P_or, args.cpu_seconds, nthreads=nth)
        cpu = {"value": round(n_done / el, 2), "unit": "shots/s", "cores": nth, "kind": "oracle",
               "host": host,
               "msg_updates_per_s": 2 * E * args.iters * rounds / el,
               "sample": f"shot ids 0..{n_done - 1} of the same workload ({el:.1f} s wall, "
                         f"{nth} OpenMP threads over shots: every core this process may use)"}
        n1, el1, _, _ = cpu_baseline(args, spec, P_or, min(3.0, args.cpu_seconds), nthreads=1, max_shots=256)
        cpu["single_thread"] = {"value": round(n1 / el1, 2), "unit": "shots/s", "cores": 1,
                                "sample": f"shot ids 0..{n1 - 1} ({el1:.1f} s wall)"}
        if small_gpu is not None:
            spec8 = codes.toric_2d(8)
            P8 = O.DecodeParams(rounds=64)
            t0 = time.perf_counter()
            refs = [O.decode(spec8, P8, g["e0"], nthreads=nth) for g in small_gpu]
            el8 = time.perf_counter() - t0
            same8 = all(np.array_equal(r[k], g[k]) for r, g in zip(refs, small_gpu) for k in ("z", "s", "tclr"))
            cpu["small_config"] = {"value": round(4000 / el8, 1), "unit": "shots/s", "cores": nth,
                                   "sample": "all 4000 shots of 2D toric L=8, p = 0.02..0.08, 64 rounds",
                                   "identical_to_gpu": bool(same8)}

    line = {
        "metric": "shots/s and BP msg-updates/s (2D toric L=32, p=0.05); served p50/p99 latency",
        "value": round(shots_per_s, 1),
        "unit": "shots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D toric code L={L}, i.i.d. Z noise p={args.p}, {args.shots} shots per "
                               f"step (fresh shot ids each step), {args.iters} BP sweeps x {R} rounds, "
                               f"{args.bp}{' alpha=0.75' if args.bp == 'minsum' else ''}, clocks at "
                               f"density 0.5, {'retire on clear' if not args.no_retire else 'fixed rounds'}, "
                               f"{form} form",
                   "code": f"toric2d:{L}", "p": args.p, "shots_per_step": args.shots, "rounds": R,
                   "iters": args.iters, "bp": args.bp, "form": form, "retire": not args.no_retire,
                   "skip_fixed": skip,
                   "resident_shape": code.resident_cfg(args.bp) if form != "stream" else None,
                   "autotuned": tuned is not None},
        "msg_updates_per_s": msg_per_s,
        "logical_error_rate": main_run["failures"] / S_total,
        "sumproduct": sp_line,
        "served_latency": (
            {"p50_round_ms": extras["serving"]["open_loop"][1]["p50_round_ms"],
             "p99_round_ms": extras["serving"]["open_loop"][1]["p99_round_ms"],
             "requests_per_s": extras["serving"]["open_loop"][1]["requests_per_s"],
             "at": "Poisson arrivals at 0.8x the saturation rate of the mixed serving workload"}
            if "serving" in extras else None),
        "roofline": rl,
        "cpu_baseline": cpu,
        "extras": dict(extras, sweeps_not_computed={
            "msg_updates_of_the_method_per_s": msg_method / sec,
            "what": "the method's count: every sweep of every round run, including the identity sweeps "
                    "at a fixed point that the kernel skips (not computed; msg_updates_per_s counts the "
                    "computed ones)", "sweeps_computed_frac": round(sweeps_frac, 4)}),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
