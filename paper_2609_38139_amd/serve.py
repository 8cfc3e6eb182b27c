"""Load generator and statistics for the continuous-batching server.

Requests are single shots of a mix of codes, each decoded for up to its own
number of rounds (a shot retires once its syndrome clears); the server draws
each request's error on the device when it admits it. Arrivals form a
Poisson process; every step the server admits what fits and advances each
resident request by one round. Reported: requests/s, shots/s, rounds/s and
the p50/p99 of the per-round latency (from a round's input being ready --
arrival for the first round, the previous round's completion otherwise -- to
its results being on the host).
"""
from __future__ import annotations

import time

import numpy as np

# The mixed workload: (code, rounds) with rounds = 8L, and the distance
# proxy sqrt(n) = 12 for the [[144,12,12]] bivariate-bicycle code.
DEFAULT_MIX = [("toric2d:16", 128), ("toric2d:32", 256), ("toric2d:48", 384),
               ("toric3d_point:12", 96), ("bb:12x6", 96)]


class Workload:
    """Request i uses code i mod len(mix) (the codes take equal shares) and
    shot id i; its error is drawn by the server on the device from (seed,
    shot id, p) when the request is admitted."""

    def __init__(self, laim, mix=DEFAULT_MIX, p=0.03, nreq=2048, bp="minsum", seed=0):
        from . import codes
        self.laim = laim
        self.codes = []
        self.params = []
        for name, rounds in mix:
            spec = codes.by_name(name)
            self.codes.append(laim.Code(spec, 0))
            self.params.append(laim.DecodeParams(bp=bp, rounds=rounds, seed=seed,
                                                 q=0.125 if "membrane" in name else 0.05))
        self.nreq = nreq
        self.p = p
        self.seed = seed

    def request(self, i):
        k = i % len(self.codes)
        return self.codes[k], self.params[k], i


def run(server, wl: Workload, rate: float | None, nreq: int, rng_seed: int = 0,
        time_limit: float = 60.0) -> dict:
    """Drives `nreq` requests through `server`. rate=None submits them all at
    once (saturation); otherwise arrivals are Poisson with that rate (1/s)."""
    rng = np.random.default_rng(rng_seed)
    if rate is None:
        arrivals = np.zeros(nreq)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    lat = []
    done = 0
    rounds = 0
    nxt = 0
    t0 = time.perf_counter()
    resident_peak = 0
    bytes_peak = 0
    waiting_peak = 0
    pending = 0
    while done < nreq:
        now = time.perf_counter() - t0
        if now > time_limit:
            break
        while nxt < nreq and arrivals[nxt] <= now:
            code, P, shot = wl.request(nxt)
            server.submit(code, P, shot, None, wl.p)
            nxt += 1
            pending += 1
        if pending == 0:
            time.sleep(min(0.001, max(0.0, arrivals[nxt] - now)) if nxt < nreq else 0.0)
            continue
        evs = server.step()
        st = server.stats()
        resident_peak = max(resident_peak, st["resident"])
        bytes_peak = max(bytes_peak, st["bytes"])
        waiting_peak = max(waiting_peak, st["waiting"])
        for e in evs:
            lat.append(e["latency_ns"])
            rounds += 1
            if e["done"]:
                server.result(e["ticket"])
                done += 1
                pending -= 1
    el = time.perf_counter() - t0
    lat = np.array(lat, dtype=np.float64) / 1e6
    return {"rate_req_per_s": rate, "requests": done, "seconds": round(el, 3),
            "requests_per_s": round(done / el, 1), "rounds_per_s": round(rounds / el, 1),
            "p50_round_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_round_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
            "resident_peak": resident_peak, "arena_bytes_peak": bytes_peak, "waiting_peak": waiting_peak}
