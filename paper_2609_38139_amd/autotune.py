"""Launch-shape autotuner for the resident decode form.

For one code and BP rule it times every valid resident launch shape
(checks per thread x shots per block) on a fixed batch of shots decoded as
a run decodes them (shots retire once clear), checks that all shapes produce
identical outputs, installs the fastest with ``laim_set_resident_cfg`` and
caches the choice per device name and code in a JSON file
(``$LAIM_TUNE_CACHE``, default ``~/.cache/laim/resident_shapes.json``).
"""
from __future__ import annotations

import json
import os

CACHE = os.environ.get("LAIM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "laim",
                                                      "resident_shapes.json"))


def _key(code, bp: str) -> str:
    import torch
    name = torch.cuda.get_device_name(code.device)
    spec = code.spec
    return f"{name}|{spec.name}|m{code.m}|n{code.n}|E{code.E}|{bp}"


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def candidates(code, bp: str):
    """Every resident shape the library accepts for this code."""
    from . import laim
    out = []
    for cpt in (1, 2, 4, 8):
        for spb in (0, 1, 2, 4, 8):
            cfg = {"checks_per_thread": cpt, "shots_per_block": spb}
            try:
                code.set_resident_cfg(bp, cfg)
                got = code.resident_cfg(bp)
            except laim.LaimError:
                continue
            if got not in out:
                out.append(got)
    code.set_resident_cfg(bp, None)
    return out


def tune(code, bp: str = "minsum", nshots: int = 16384, rounds: int = 64, iters: int = 20,
         p: float = 0.05, q: float = 0.05, use_cache: bool = True, verbose: bool = False) -> dict:
    """Returns {'cfg': best shape, 'ms': {shape: time}} and installs the best shape.

    Each shape decodes the same batch for `rounds` rounds with shots retiring
    at clear, as decoding runs: a block of several shots waits for its
    slowest, and shots that clear or freeze early end their work, so fewer
    or shorter runs would rank the shapes differently."""
    import torch

    from . import laim
    key = _key(code, bp)
    cache = _load() if use_cache else {}
    if key in cache:
        cfg = cache[key]["cfg"]
        code.set_resident_cfg(bp, cfg)
        return cache[key]
    P = laim.DecodeParams(bp=bp, rounds=rounds, iters=iters, q=q, retire=True)
    e0 = laim.sample_noise(code, p, 0, 0, nshots)
    results = {}
    ref = None
    for cfg in candidates(code, bp):
        out = laim.decode_rounds(code, P, e0, cfg=cfg)  # warm-up and output check
        torch.cuda.synchronize()
        if ref is None:
            ref = out
        else:
            for k in ("z", "s", "tclr"):
                if not torch.equal(ref[k], out[k]):
                    raise RuntimeError(f"launch shape {cfg} changed the results ({k})")
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(2):
            laim.decode_rounds(code, P, e0, cfg=cfg, workspace=out["workspace"], out=out)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 2
        results[json.dumps(cfg, sort_keys=True)] = ms
        if verbose:
            print(f"[autotune] {code.spec.name} {bp} {cfg}: {ms:.3f} ms", flush=True)
    best = min(results, key=results.get)
    entry = {"cfg": json.loads(best), "ms": results}
    code.set_resident_cfg(bp, entry["cfg"])
    if use_cache:
        cache[key] = entry
        _save(cache)
    return entry
