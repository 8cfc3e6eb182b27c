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
LANES_PER_CU = 64  # one VALU instruction per lane per clock per CU (4 SIMD x 16 lanes)
VALU_PEAK_TOPS = CU_COUNT * LANES_PER_CU * CLOCK_GHZ / 1000.0  # 39.3 T lane-ops/s


RESIDENT_SOURCES = ("paper_2609_38139_amd/csrc/laim_kernels.hip", "paper_2609_38139_amd/csrc/device_math.h",
                    "paper_2609_38139_amd/csrc/laim_internal.h", "paper_2609_38139_amd/build.py")


STREAM_SOURCES = ("paper_2609_38139_amd/csrc/laim_stream.hip", "paper_2609_38139_amd/csrc/device_math.h",
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


def profiled_traffic(profile: str, shape: str, sources=RESIDENT_SOURCES):
    """HBM bytes per launch from a committed rocprofv3 summary (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy's counts), or None when the kernel
    sources (hashed in order) or the launch shape differ from the profiled
    ones."""
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
    if fields.get("source_sha256") != h.hexdigest() or fields.get("launch_shape") != shape:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
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
    ops_check = (dc * (code.dv_max - 1) + (dc + 1) // 2 + 1 + dc * max(0, (dc - 1) // 2) + 2 * dc
                 + 6 * dc) if bp == "minsum" else None
    res = {"workload": f"2D toric L={L}, p={p}, {bp}, dt={dt}, tau=0.1, t_max={t_max}, {nshots} shots",
           "shots_per_s": round(nshots / sec, 1), "decode_ms": round(sec * 1e3, 3),
           "euler_steps_computed_frac": round(computed / max(1, steps), 4),
           "euler_shot_steps_per_s": computed / sec, "msg_updates_per_s": 2 * code.E * computed / sec,
           "euler_shot_steps_of_the_method_per_s": steps / sec,
           "every_step": {"shots_per_s": round(nshots / sec_all, 1), "decode_ms": round(sec_all * 1e3, 3),
                          "what": "skip_fixed = 0: every Euler step computed; identical outputs"},
           "cleared": int((tclr >= 0).sum()), "logical_error_rate": float(out["fail"].float().mean().item()),
           "mean_tclr_cleared": float(tclr[tclr >= 0].mean()) if (tclr >= 0).any() else None}
    if ops_check is not None:
        # only the computed steps count as work
        ach = computed * m * ops_check / sec / 1e12
        res["roofline"] = {"bound": "alu", "achieved": round(ach, 3), "peak": round(VALU_PEAK_TOPS, 1),
                           "unit": "Tops/s", "frac": round(ach / VALU_PEAK_TOPS, 4),
                           "ops_per_check_step": ops_check}
        ach_all = steps * m * ops_check / sec_all / 1e12
        res["every_step"]["roofline"] = {"achieved": round(ach_all, 3), "frac": round(ach_all / VALU_PEAK_TOPS, 4)}
    return res


def bitcentric(laim, d=101, p=0.3, nshots=262144, q=0.1):
    """The bit-centric machine on the periodic repetition code (SM "Setup and
    algorithm"), d iterations: shots/s, and its logical error rate beside the
    binomial tail P(|E| > d/2) it must equal."""
    import torch
    from scipy.stats import binom

    from paper_2609_38139_amd import codes
    code = laim.Code(codes.repetition(d, periodic=True), 0)
    e0 = laim.sample_noise(code, p, 5, 0, nshots)
    laim.decode_bitcentric(code, q, e0, d)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(st)
    out = laim.decode_bitcentric(code, q, e0, d)
    ev1.record(st)
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / 1000.0
    fail = (e0 ^ out["z"]).any(dim=1).float().mean().item()
    ic = out["iclr"]
    return {"workload": f"periodic repetition d={d}, p={p}, q={q}, {d} iterations, {nshots} shots",
            "shots_per_s": round(nshots / sec, 1), "decode_ms": round(sec * 1e3, 3),
            "logical_error_rate": fail, "binomial_tail": float(binom.sf(d // 2, d, p)),
            "mean_iclr_cleared": float(ic[ic > 0].float().mean().item()) if bool((ic > 0).any()) else None}


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


def timed_steps(laim, code, P, args, steps, warmup, form, shot_base=0):
    """Runs warmup + steps passes; returns per-step and per-decode times (ms)
    from HIP events on the stream every kernel is launched on, plus the
    rounds run and BP sweeps computed over the timed steps."""
    import torch
    S = args.shots
    st = torch.cuda.current_stream()
    e0 = torch.empty((S, code.n), dtype=torch.uint8, device="cuda")
    out = {"z": torch.empty((S, code.n), dtype=torch.uint8, device="cuda"),
           "s": torch.empty((S, code.m), dtype=torch.uint8, device="cuda"),
           "tclr": torch.empty((S,), dtype=torch.int32, device="cuda"), "L": None,
           "sweeps": torch.empty((S,), dtype=torch.int32, device="cuda"),
           "fail": torch.empty((S,), dtype=torch.uint8, device="cuda")}
    ws = torch.empty((max(laim.workspace_bytes(code, P, S, form), 256),), dtype=torch.uint8, device="cuda")
    fails = torch.zeros((), dtype=torch.int64, device="cuda")
    rounds_exec = torch.zeros((), dtype=torch.int64, device="cuda")
    sweeps_exec = torch.zeros((), dtype=torch.int64, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)

    def step(i, evs=None):
        shot0 = shot_base + i * S
        laim.sample_noise(code, args.p, 0, shot0, S, out=e0)
        if evs:
            evs[0].record(st)
        # the decoder failure test runs inside the decode launch (fail_out)
        laim.decode_rounds(code, P, e0, shot0=shot0, form=form, workspace=ws, out=out)
        if evs:
            evs[1].record(st)
        fails.add_(out["fail"].sum())
        t = out["tclr"]
        rounds_exec.add_(torch.where(t >= 0, t, torch.full_like(t, P.rounds)).sum())
        sweeps_exec.add_(out["sweeps"].sum())

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    fails.zero_()
    rounds_exec.zero_()
    sweeps_exec.zero_()
    t0.record(st)
    for i in range(steps):
        step(warmup + i, ev[i])
    t1.record(st)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    dec_ms = [a.elapsed_time(b) for a, b in ev]
    return {"ms_per_step": total_ms / steps, "decode_ms": sum(dec_ms) / steps,
            "failures": int(fails.item()), "rounds_exec": int(rounds_exec.item()),
            "sweeps_exec": int(sweeps_exec.item()), "shots": S * steps}


def cpu_baseline(args, spec, P_or, seconds, nthreads=None, max_shots=4096):
    """The oracle, as it is, on shot ids 0.. of the same workload, in chunks
    until `seconds` of wall time have passed."""
    from oracle import oracle as O
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
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
    main_run = timed_steps(laim, code, P, args, args.steps, args.warmup, form)
    S_total = main_run["shots"]
    sec = main_run["ms_per_step"] * args.steps / 1000.0
    shots_per_s = S_total / sec
    # message updates of the method (every sweep of every round run) and
    # those the kernels computed (sweeps at a fixed point are skipped)
    msg_updates = 2 * E * args.iters * main_run["rounds_exec"]
    msg_computed = 2 * E * main_run["sweeps_exec"]
    msg_per_s = msg_computed / sec
    dec_s = main_run["decode_ms"] / 1000.0
    msg_per_launch = msg_computed / args.steps
    sweeps_frac = main_run["sweeps_exec"] / max(1, args.iters * main_run["rounds_exec"])

    # Roofline of the dominant kernel. The resident decode launch keeps every
    # message on chip, so HBM carries only e0 in and z, s, t_clr out; its
    # bound is VALU issue (256 CU x 64 lanes x 2.4 GHz). Achieved work is the
    # operation count of the sweeps on this instruction set (three-input min,
    # median and xor exist), per check and sweep:
    #   d_c (d_v - 1) qubit-side sums, plus d_c clamps -- except for min-sum
    #                 on qubits of degree 2 with alpha < 1 and |pi|/(1 - alpha)
    #                 < CLAMP, where the clamp provably cannot bind and the
    #                 kernel does not execute it
    #   ceil(d_c/2)+1 sign parity by three-input xors, folded into +-alpha
    #   d_c ceil((d_c - 2)/2)  smallest other |m| per output by three-input mins
    #   2 d_c         scale and sign per output
    # = 19 for d_c = 4, d_v = 2 (2.375 per message update; 23 with the
    # clamps). Sum-product has no fixed count: each of its 3 (d_c - 2)
    # box-plus steps evaluates exp only for arguments up to 80 (a larger one
    # gives 0 at once), so its work depends on the message magnitudes --
    # about 66 VALU per step for small ones, little more than half of that
    # once |m| is large. Its roofline therefore reports no fraction.
    # Beside it: the rate the stream form's HBM traffic would need for the
    # same sweeps (each check-to-qubit message written once and read once by
    # its partner's gather, 4 B each way, i.e. 4 B per message update
    # counting both directions, plus 1 B of syndrome per check and sweep).
    # In the stream form the sweeps themselves stream through HBM and the
    # roofline is that traffic against the 8 TB/s peak.
    # Only computed sweeps count as work: with the fixed-point skip the
    # kernel also spends time comparing each new message with the one it
    # replaces, and the feedback phase is a larger share of the launch.
    dc, dv = code.dc_max, code.dv_max
    ops_check = None
    if args.bp == "minsum":
        pi = abs(np.log(P.q / (1.0 - P.q)))
        idle_clamp = dv == 2 and P.alpha < 1.0 and pi < 0.99 * P.clamp * (1.0 - P.alpha)
        ops_check = (dc * (dv - 1) + (0 if idle_clamp else dc) + (dc + 1) // 2 + 1
                     + dc * max(0, (dc - 1) // 2) + 2 * dc)
    ops_per_update = ops_check / (2.0 * dc) if ops_check is not None else None
    bytes_per_update = 4.0 + 1.0 / (2.0 * dc)
    hbm_equiv_gbs = msg_per_launch * bytes_per_update / dec_s / 1e9
    default_workload = (L == 32 and args.p == 0.05 and args.shots == 65536 and R == 128
                        and args.iters == 20 and args.bp == "minsum" and not args.no_retire)
    if form != "stream":
        shape = code.resident_cfg(args.bp)
        traffic = None
        if default_workload:
            traffic = profiled_traffic("resident_kernel_toric2d_L32_minsum.md",
                                       f"{shape['checks_per_thread']},{shape['shots_per_block']}")
        achieved_tops = msg_per_launch * ops_per_update / dec_s / 1e12 if ops_per_update else None
        rl = {"bound": "alu", "achieved": round(achieved_tops, 3) if achieved_tops else None,
              "peak": round(VALU_PEAK_TOPS, 1), "unit": "Tops/s",
              "frac": round(achieved_tops / VALU_PEAK_TOPS, 4) if achieved_tops else None, "traffic": traffic,
              "kernel": f"resident_kernel (2D toric L={L}, {args.bp})",
              "ops_per_msg_update": ops_per_update, "decode_ms_per_launch": round(main_run["decode_ms"], 3),
              "msg_updates_per_launch": msg_per_launch, "sweeps_computed_frac": round(sweeps_frac, 4),
              "hbm_equivalent_GBs": round(hbm_equiv_gbs, 1),
              "hbm_equivalent_frac": round(hbm_equiv_gbs / HBM_PEAK_GBS, 3)}
    else:
        rl = {"bound": "hbm", "achieved": round(hbm_equiv_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(hbm_equiv_gbs / HBM_PEAK_GBS, 4), "traffic": None,
              "kernel": f"stream form decode, sweeps and feedback kernels (2D toric L={L}, {args.bp})",
              "bytes_per_msg_update": bytes_per_update, "decode_ms_per_launch": round(main_run["decode_ms"], 3),
              "msg_updates_per_launch": msg_per_launch}

    extras = {}
    small_gpu = None
    if args.no_extras:
        args.no_batch = args.no_serve = True
    if not args.no_extras:
        # stream form (messages in HBM, one launch per sweep): the plain baseline
        rs = timed_steps(laim, code, P, args, 1, 0, "stream", shot_base=10**9)
        sec_s = rs["ms_per_step"] / 1000.0
        upd = 2 * E * args.iters * rs["rounds_exec"]
        # each m_{c->v} read once by the partner gather and written once (4 B
        # each) per check-to-qubit update, plus 1 B of syndrome per check
        sweeps_bytes = upd * (4.0 + 1.0 / (2.0 * code.dc_max))
        # context for the HBM fraction: what a plain 1 GiB device copy reaches
        # (bytes read + bytes written over its time)
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
        # the sweep kernel alone, from its committed rocprofv3 summary (only
        # while the stream sources are the profiled ones)
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
                                 "failures": rs["failures"]}
        if skip:
            # the same launch running every sweep: identical results
            rn = timed_steps(laim, code, laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters,
                                                           retire=not args.no_retire, skip_fixed=False),
                             args, 2, 1, form)
            sec_n = rn["ms_per_step"] * 2 / 1000  # two timed steps
            extras["every_sweep"] = {
                "shots_per_s": round(rn["shots"] / sec_n, 1),
                "decode_ms": round(rn["decode_ms"], 3),
                "msg_updates_per_s": 2 * E * rn["sweeps_exec"] / sec_n,
                "failures_per_shot": rn["failures"] / rn["shots"],
                "what": "skip_fixed = 0: every BP sweep computed; same z, s, t_clr as the value"}
            if ops_per_update and form != "stream":
                upd_launch = 2 * E * rn["sweeps_exec"] / 2  # two timed launches
                ach = upd_launch * ops_per_update / (rn["decode_ms"] / 1000) / 1e12
                extras["every_sweep"]["roofline"] = {"achieved": round(ach, 3), "peak": round(VALU_PEAK_TOPS, 1),
                                                     "unit": "Tops/s", "frac": round(ach / VALU_PEAK_TOPS, 4)}
        P_fix = laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=False)
        rf = timed_steps(laim, code, P_fix, args, 1, 0, form, shot_base=2 * 10**9)
        extras["fixed_rounds"] = {"shots_per_s": round(rf["shots"] / (rf["ms_per_step"] / 1000), 1),
                                  "msg_updates_per_s": 2 * E * args.iters * rf["rounds_exec"] / (rf["ms_per_step"] / 1000),
                                  "failures": rf["failures"]}
        other = "sumproduct" if args.bp == "minsum" else "minsum"
        P_o = laim.DecodeParams(bp=other, rounds=R, iters=args.iters, retire=not args.no_retire)
        ro = timed_steps(laim, code, P_o, args, 1, 1, form, shot_base=3 * 10**9)
        extras[other] = {"shots_per_s": round(ro["shots"] / (ro["ms_per_step"] / 1000), 1),
                         "msg_updates_per_s": 2 * E * ro["sweeps_exec"] / (ro["ms_per_step"] / 1000),
                         "sweeps_computed_frac": round(ro["sweeps_exec"] / max(1, args.iters * ro["rounds_exec"]), 4),
                         "decode_ms": round(ro["decode_ms"], 2), "failures": ro["failures"],
                         "logical_error_rate": ro["failures"] / ro["shots"],
                         "resident_shape": code.resident_cfg(other) if form != "stream" else None}
        # conflict rules for the round's move requests (ablation): same
        # workload and shots, each rule
        extras["conflict_rules"] = {}
        for k, rule in enumerate(("or", "xor", "sequential")):
            P_c = laim.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=not args.no_retire,
                                    conflict=rule)
            rc_ = timed_steps(laim, code, P_c, args, 1, 0, form, shot_base=5 * 10**9)
            extras["conflict_rules"][rule] = {
                "shots_per_s": round(rc_["shots"] / (rc_["ms_per_step"] / 1000), 1),
                "failures": rc_["failures"], "logical_error_rate": rc_["failures"] / rc_["shots"],
                "mean_rounds_run": round(rc_["rounds_exec"] / rc_["shots"], 3)}
    if not args.no_batch:
        extras["batched_vs_plain"] = batch_vs_plain(laim, codes)
        extras["per_shot_plain"], small_gpu = per_shot_plain(laim, codes)
    if not args.no_serve:
        extras["serving"] = serving(laim, args.serve_seconds)
    if not args.no_extras:
        extras["bitcentric"] = bitcentric(laim)
        extras["continuous_machine"] = {
            "minsum": continuous_machine(laim, L, args.p, "minsum", 4096, 30.0),
            "sumproduct": continuous_machine(laim, L, args.p, "sumproduct", 2048, 30.0)}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        P_or = O.DecodeParams(bp=args.bp, rounds=R, iters=args.iters, retire=not args.no_retire)
        n_done, el, nth, rounds = cpu_baseline(args, spec, P_or, args.cpu_seconds)
        cpu = {"value": round(n_done / el, 2), "unit": "shots/s", "cores": nth, "kind": "oracle",
               "msg_updates_per_s": 2 * E * args.iters * rounds / el,
               "sample": f"shot ids 0..{n_done - 1} of the same workload ({el:.1f} s wall, "
                         f"{nth} OpenMP threads over shots)"}
        n1, el1, _, _ = cpu_baseline(args, spec, P_or, min(3.0, args.cpu_seconds), nthreads=1, max_shots=256)
        cpu["single_thread"] = {"value": round(n1 / el1, 2), "unit": "shots/s", "cores": 1,
                                "sample": f"shot ids 0..{n1 - 1} ({el1:.1f} s wall)"}
        if small_gpu is not None:
            # the small configuration whole (4 x 1000 shots of 2D toric L=8), by
            # the oracle on the host cores, compared bit for bit with the GPU's
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
                   "skip_fixed": skip and form != "stream",
                   "resident_shape": code.resident_cfg(args.bp) if form != "stream" else None,
                   "autotuned": tuned is not None},
        "msg_updates_per_s": msg_per_s,
        "msg_updates_of_the_method_per_s": msg_updates / sec,
        "logical_error_rate": main_run["failures"] / S_total,
        "served_latency": (
            {"p50_round_ms": extras["serving"]["open_loop"][1]["p50_round_ms"],
             "p99_round_ms": extras["serving"]["open_loop"][1]["p99_round_ms"],
             "requests_per_s": extras["serving"]["open_loop"][1]["requests_per_s"],
             "at": "Poisson arrivals at 0.8x the saturation rate of the mixed serving workload"}
            if "serving" in extras else None),
        "roofline": rl,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
