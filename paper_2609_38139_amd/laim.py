"""Python binding of the C ABI declared in ``include/laim.h``.

Argument marshalling only: every step of the decoder runs in the HIP
library ``liblaim.so`` built next to this file. PyTorch provides device
memory and the stream each call is enqueued on. Importing this module does
not need a GPU; the calls do, and there is no CPU fallback: without the
built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblaim.so")

OK, EINVAL, ENOMEM, EHIP, EUNSUP, EBUSY = 0, -1, -2, -3, -4, -5
FORM_AUTO, FORM_RESIDENT, FORM_STREAM = 0, 1, 2
FORMS = {"auto": FORM_AUTO, "resident": FORM_RESIDENT, "stream": FORM_STREAM}

# Every symbol the header declares (checked by the tests).
SYMBOLS = [
    "laim_last_error", "laim_version", "laim_build_tanner", "laim_build_tanner_ex",
    "laim_free_code", "laim_code_info", "laim_code_logicals", "laim_host_logicals",
    "laim_sample_noise", "laim_syndrome", "laim_workspace_bytes", "laim_decode_rounds",
    "laim_decode_rounds_cfg", "laim_set_resident_cfg", "laim_get_resident_cfg",
    "laim_logical_failure", "laim_batch_plan_create", "laim_batch_plan_launch",
    "laim_batch_plan_destroy", "laim_server_create", "laim_server_submit", "laim_server_step",
    "laim_server_result", "laim_server_stats", "laim_server_destroy", "laim_decode_continuous",
    "laim_decode_bitcentric", "laim_decode_rounds_static", "laim_online_plan_create",
    "laim_online_plan_destroy", "laim_online_workspace_bytes", "laim_decode_online",
    "laim_decode_bitcentric_form", "laim_resident_variant",
]

STATIC_SCRATCH_BYTES = 32 << 20  # LAIM_STATIC_SCRATCH_BYTES


class LaimError(RuntimeError):
    def __init__(self, status: int, where: str, text: str):
        super().__init__(f"{where} failed with status {status}: {text}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("bp", C.c_int32), ("alpha", C.c_float), ("q", C.c_double), ("clamp", C.c_float),
                ("iters", C.c_int32), ("rounds", C.c_int32), ("mask_density", C.c_double),
                ("gauge", C.c_int32), ("evidence", C.c_int32), ("retire", C.c_int32),
                ("seed", C.c_uint64), ("conflict", C.c_int32), ("skip_fixed", C.c_int32),
                ("move", C.c_int32)]


# LAIM_CONFLICT_*: how one round's move requests combine
CONFLICT_RULES = {"or": 0, "xor": 1, "sequential": 2}
# LAIM_MOVE_*: the local move of an acting check
MOVES = {"single": 0, "multi": 1}


class ResidentCfg(C.Structure):
    _fields_ = [("threads_per_shot", C.c_int32), ("checks_per_thread", C.c_int32),
                ("shots_per_block", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("code", C.c_void_p), ("params", Params), ("e0", C.c_void_p), ("shot0", C.c_uint64),
                ("nshots", C.c_int32), ("z_out", C.c_void_p), ("s_out", C.c_void_p),
                ("tclr_out", C.c_void_p), ("fail_out", C.c_void_p)]


class ServerEvent(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("round", C.c_int32), ("done", C.c_int32),
                ("tclr", C.c_int32), ("flips", C.c_int32), ("defects", C.c_int32),
                ("fail", C.c_int32), ("latency_ns", C.c_int64)]


@dataclass
class DecodeParams:
    """Knobs of the round machine (defaults: Table S1's q and CLAMP for the
    2D toric code; 20 BP sweeps per round; clocks ring with probability 0.5)."""

    bp: str = "minsum"
    alpha: float = 0.75
    q: float = 0.05
    clamp: float = 1000.0
    iters: int = 20
    rounds: int = 64
    mask_density: float = 0.5
    gauge: bool = False
    evidence: bool = True
    retire: bool = True
    seed: int = 0
    conflict: str = "or"  # "or", "xor" or "sequential"
    skip_fixed: bool = True  # skip sweeps once a shot's messages are a fixed point (same results)
    move: str = "single"  # "single": LocalMove; "multi": every qubit of the check with L_v > 0

    def c(self) -> Params:
        if self.bp not in ("minsum", "sumproduct"):
            raise ValueError("bp must be 'minsum' or 'sumproduct'")
        if self.conflict not in CONFLICT_RULES:
            raise ValueError("conflict must be 'or', 'xor' or 'sequential'")
        if self.move not in MOVES:
            raise ValueError("move must be 'single' or 'multi'")
        return Params(1 if self.bp == "sumproduct" else 0, self.alpha, self.q, self.clamp,
                      self.iters, self.rounds, self.mask_density, int(self.gauge),
                      int(self.evidence), int(self.retire), self.seed, CONFLICT_RULES[self.conflict],
                      int(self.skip_fixed), MOVES[self.move])


class ContinuousParamsC(C.Structure):
    _fields_ = [("bp", C.c_int32), ("alpha", C.c_float), ("q", C.c_double), ("clamp", C.c_float),
                ("dt", C.c_double), ("tau", C.c_double), ("t_max", C.c_double),
                ("evidence", C.c_int32), ("seed", C.c_uint64), ("skip_fixed", C.c_int32)]


@dataclass
class ContinuousParams:
    """Knobs of the continuous-time machine (defaults: Table S1, 2D toric code
    row: dt = 0.001, tau = 0.1, q = 0.05, CLAMP = 1000)."""

    bp: str = "minsum"
    alpha: float = 0.75
    q: float = 0.05
    clamp: float = 1000.0
    dt: float = 0.001
    tau: float = 0.1
    t_max: float = 100.0
    evidence: bool = True
    seed: int = 0
    skip_fixed: bool = True  # skip Euler steps at a fixed point of the messages (same results)

    def c(self) -> ContinuousParamsC:
        if self.bp not in ("minsum", "sumproduct"):
            raise ValueError("bp must be 'minsum' or 'sumproduct'")
        return ContinuousParamsC(1 if self.bp == "sumproduct" else 0, self.alpha, self.q, self.clamp,
                                 self.dt, self.tau, self.t_max, int(self.evidence), self.seed,
                                 int(self.skip_fixed))


class OnlineParamsC(C.Structure):
    _fields_ = [("rounds_total", C.c_int32), ("window", C.c_int32), ("commit", C.c_int32),
                ("p", C.c_double), ("p_meas", C.c_double)]


@dataclass
class OnlineParams:
    """Online decoding: N syndrome rounds (the last one perfect), windows of
    W rounds of which the first C are committed, data and measurement error
    rates."""

    rounds_total: int = 8
    window: int = 4
    commit: int = 2
    p: float = 0.01
    p_meas: float = 0.01

    def c(self) -> OnlineParamsC:
        return OnlineParamsC(self.rounds_total, self.window, self.commit, self.p, self.p_meas)


CONTINUOUS_WORKSPACE_BYTES = 256

_lib = None


def lib():
    """Loads ``liblaim.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() or "
                               "python paper_2609_38139_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, u64, sz = C.c_void_p, C.c_int32, C.c_uint64, C.c_size_t
        i32p = C.POINTER(C.c_int32)
        L.laim_last_error.restype = C.c_char_p
        L.laim_version.restype = i32
        L.laim_build_tanner_ex.argtypes = [i32, i32, i32p, i32p, i32, i32p, i32p, i32, i32p, i32p,
                                           i32, C.POINTER(vp)]
        L.laim_build_tanner.argtypes = [i32, i32, i32p, i32p, i32, i32p, i32p, i32, C.POINTER(vp)]
        L.laim_free_code.argtypes = [vp]
        L.laim_free_code.restype = None
        L.laim_code_info.argtypes = [vp] + [i32p] * 6
        L.laim_code_logicals.argtypes = [vp, vp]
        L.laim_host_logicals.argtypes = [i32, i32, i32p, i32p, i32, i32p, i32p, i32, vp, i32p]
        L.laim_sample_noise.argtypes = [vp, C.c_double, u64, u64, i32, vp, vp]
        L.laim_syndrome.argtypes = [vp, vp, i32, vp, vp]
        L.laim_workspace_bytes.argtypes = [vp, C.POINTER(Params), i32, i32]
        L.laim_workspace_bytes.restype = sz
        L.laim_decode_rounds.argtypes = [vp, C.POINTER(Params), vp, u64, i32, vp, sz, vp, vp, vp, vp,
                                         vp, vp, i32, vp]
        L.laim_decode_rounds_cfg.argtypes = [vp, C.POINTER(Params), vp, u64, i32, vp, sz, vp, vp, vp,
                                             vp, vp, vp, C.POINTER(ResidentCfg), vp]
        L.laim_set_resident_cfg.argtypes = [vp, i32, C.POINTER(ResidentCfg)]
        L.laim_get_resident_cfg.argtypes = [vp, i32, C.POINTER(ResidentCfg)]
        L.laim_logical_failure.argtypes = [vp, vp, vp, i32, vp, vp]
        L.laim_batch_plan_create.argtypes = [C.POINTER(BatchItem), i32, vp, C.POINTER(vp)]
        L.laim_batch_plan_launch.argtypes = [vp, vp]
        L.laim_batch_plan_destroy.argtypes = [vp]
        L.laim_batch_plan_destroy.restype = None
        L.laim_server_create.argtypes = [i32, sz, i32, C.POINTER(vp)]
        L.laim_server_submit.argtypes = [vp, vp, C.POINTER(Params), u64, vp, C.c_double, C.POINTER(u64)]
        L.laim_server_step.argtypes = [vp, C.POINTER(ServerEvent), i32, i32p]
        L.laim_server_result.argtypes = [vp, u64, vp, vp, i32p]
        L.laim_server_stats.argtypes = [vp, i32p, i32p, C.POINTER(sz)]
        L.laim_server_destroy.argtypes = [vp]
        L.laim_decode_continuous.argtypes = [vp, C.POINTER(ContinuousParamsC), vp, u64, i32, vp, sz,
                                             vp, vp, vp, vp, vp, vp, i32, vp]
        L.laim_decode_bitcentric.argtypes = [vp, C.c_double, vp, i32, i32, vp, vp, vp, vp]
        L.laim_decode_bitcentric_form.argtypes = [vp, C.c_double, vp, i32, i32, i32, vp, vp, vp, vp]
        L.laim_resident_variant.argtypes = [vp, C.POINTER(Params), vp, i32p, i32p, i32p, i32p]
        L.laim_decode_rounds_static.argtypes = [vp, C.POINTER(Params), vp, u64, i32, vp, vp, vp, vp,
                                                vp, vp, i32, vp]
        L.laim_online_plan_create.argtypes = [vp, C.POINTER(OnlineParamsC), C.POINTER(vp)]
        L.laim_online_plan_destroy.argtypes = [vp]
        L.laim_online_plan_destroy.restype = None
        L.laim_online_workspace_bytes.argtypes = [vp, C.POINTER(Params), i32]
        L.laim_online_workspace_bytes.restype = sz
        L.laim_decode_online.argtypes = [vp, C.POINTER(Params), u64, i32, vp, vp, vp, sz, vp, vp, vp, vp, vp]
        L.laim_server_destroy.restype = None
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != OK:
        raise LaimError(status, where, lib().laim_last_error().decode(errors="replace"))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Code:
    """A code on a device (``laim_build_tanner``)."""

    def __init__(self, code, device: int | None = None, logicals: str = "auto"):
        import torch
        self.spec = code
        self.device = torch.cuda.current_device() if device is None else device
        H, G = code.H, code.G
        hr, hrp = _i32(H.rowptr)
        hc, hcp = _i32(H.col if H.col.size else np.zeros(1))
        gr, grp = _i32(G.rowptr)
        gc, gcp = _i32(G.col if G.col.size else np.zeros(1))
        h = C.c_void_p()
        Lg = getattr(code, "logicals", None)
        if logicals == "auto" and Lg is not None:
            lr, lrp = _i32(Lg.rowptr)
            lc, lcp = _i32(Lg.col if Lg.col.size else np.zeros(1))
            st = lib().laim_build_tanner_ex(H.rows, H.cols, hrp, hcp, G.rows, grp, gcp, Lg.rows, lrp,
                                            lcp, self.device, C.byref(h))
        else:
            st = lib().laim_build_tanner(H.rows, H.cols, hrp, hcp, G.rows, grp, gcp, self.device,
                                         C.byref(h))
        check(st, "laim_build_tanner")
        self.handle = h
        vals = [C.c_int32() for _ in range(6)]
        check(lib().laim_code_info(h, *[C.byref(v) for v in vals]), "laim_code_info")
        self.m, self.n, self.E, self.k, self.dc_max, self.dv_max = [v.value for v in vals]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.laim_free_code(h)
            self.handle = None

    def logical_matrix(self) -> np.ndarray:
        out = np.zeros((self.k, self.n), dtype=np.uint8)
        check(lib().laim_code_logicals(self.handle, out.ctypes.data_as(C.c_void_p)), "laim_code_logicals")
        return out

    def resident_cfg(self, bp: str = "minsum") -> dict:
        cfg = ResidentCfg()
        check(lib().laim_get_resident_cfg(self.handle, 1 if bp == "sumproduct" else 0, C.byref(cfg)),
              "laim_get_resident_cfg")
        return {"threads_per_shot": cfg.threads_per_shot, "checks_per_thread": cfg.checks_per_thread,
                "shots_per_block": cfg.shots_per_block}

    def resident_variant(self, params: "DecodeParams", cfg: dict | None = None) -> dict:
        """``laim_resident_variant``: the resident kernel a decode with these
        parameters (and launch shape) would run."""
        c = None
        if cfg is not None:
            c = ResidentCfg(cfg.get("threads_per_shot", 0), cfg.get("checks_per_thread", 0),
                            cfg.get("shots_per_block", 0))
        P = params.c()
        out = [C.c_int32() for _ in range(4)]
        check(lib().laim_resident_variant(self.handle, C.byref(P), C.byref(c) if c is not None else None,
                                          *[C.byref(o) for o in out]), "laim_resident_variant")
        return {"dc": out[0].value, "dv": out[1].value, "checks_per_thread": out[2].value,
                "tiled": bool(out[3].value)}

    def set_resident_cfg(self, bp: str, cfg: dict | None):
        c = None
        if cfg is not None:
            c = ResidentCfg(cfg.get("threads_per_shot", 0), cfg.get("checks_per_thread", 0),
                            cfg.get("shots_per_block", 0))
        check(lib().laim_set_resident_cfg(self.handle, 1 if bp == "sumproduct" else 0,
                                          C.byref(c) if c is not None else None), "laim_set_resident_cfg")


def host_logicals(code, kmax: int = 4096) -> np.ndarray:
    """GF(2) logical basis computed by the library's host code (no device)."""
    H, G = code.H, code.G
    hr, hrp = _i32(H.rowptr)
    hc, hcp = _i32(H.col if H.col.size else np.zeros(1))
    gr, grp = _i32(G.rowptr)
    gc, gcp = _i32(G.col if G.col.size else np.zeros(1))
    out = np.zeros((kmax, H.cols), dtype=np.uint8)
    k = C.c_int32()
    check(lib().laim_host_logicals(H.rows, H.cols, hrp, hcp, G.rows, grp, gcp, kmax,
                                   out.ctypes.data_as(C.c_void_p), C.byref(k)), "laim_host_logicals")
    return out[:k.value]


def sample_noise(code: Code, p: float, seed: int, shot0: int, nshots: int, out=None, stream=None):
    import torch
    e = out if out is not None else torch.empty((nshots, code.n), dtype=torch.uint8,
                                                device=f"cuda:{code.device}")
    _dev(e, torch.uint8, (nshots, code.n), "e_out")
    check(lib().laim_sample_noise(code.handle, p, seed, shot0, nshots, _ptr(e), _stream(stream)),
          "laim_sample_noise")
    return e


def syndrome(code: Code, e, stream=None):
    import torch
    _dev(e, torch.uint8, (e.shape[0], code.n), "e")
    s = torch.empty((e.shape[0], code.m), dtype=torch.uint8, device=e.device)
    check(lib().laim_syndrome(code.handle, _ptr(e), e.shape[0], _ptr(s), _stream(stream)), "laim_syndrome")
    return s


def workspace_bytes(code: Code, params: DecodeParams, nshots: int, form: str = "auto") -> int:
    P = params.c()
    return int(lib().laim_workspace_bytes(code.handle, C.byref(P), nshots, FORMS[form]))


def decode_rounds(code: Code, params: DecodeParams, e0, shot0: int = 0, form: str = "auto",
                  want_beliefs: bool = False, cfg: dict | None = None, workspace=None, out=None,
                  stream=None, want_sweeps: bool = False, want_fail: bool = False) -> dict:
    """``laim_decode_rounds``: returns device tensors z, s, tclr (and L; with
    want_sweeps the BP sweeps computed per shot; with want_fail the decoder
    failure of each shot)."""
    import torch
    ns = e0.shape[0]
    _dev(e0, torch.uint8, (ns, code.n), "e0")
    P = params.c()
    dev = e0.device
    if out is None:
        out = {"z": torch.empty((ns, code.n), dtype=torch.uint8, device=dev),
               "s": torch.empty((ns, code.m), dtype=torch.uint8, device=dev),
               "tclr": torch.empty((ns,), dtype=torch.int32, device=dev),
               "L": torch.empty((ns, code.n), dtype=torch.float32, device=dev) if want_beliefs else None}
    if want_sweeps and out.get("sweeps") is None:
        out["sweeps"] = torch.empty((ns,), dtype=torch.int32, device=dev)
    if want_fail and out.get("fail") is None:
        out["fail"] = torch.empty((ns,), dtype=torch.uint8, device=dev)
    f = FORM_RESIDENT if cfg is not None else FORMS[form]
    need = int(lib().laim_workspace_bytes(code.handle, C.byref(P), ns, f))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty((max(need, 256),), dtype=torch.uint8, device=dev)
    if cfg is None:
        st = lib().laim_decode_rounds(code.handle, C.byref(P), _ptr(e0), shot0, ns, _ptr(workspace),
                                      workspace.numel(), _ptr(out["z"]), _ptr(out["s"]),
                                      _ptr(out["tclr"]), _ptr(out.get("L")), _ptr(out.get("sweeps")),
                                      _ptr(out.get("fail")), f, _stream(stream))
    else:
        rc = ResidentCfg(cfg.get("threads_per_shot", 0), cfg.get("checks_per_thread", 0),
                         cfg.get("shots_per_block", 0))
        st = lib().laim_decode_rounds_cfg(code.handle, C.byref(P), _ptr(e0), shot0, ns, _ptr(workspace),
                                          workspace.numel(), _ptr(out["z"]), _ptr(out["s"]),
                                          _ptr(out["tclr"]), _ptr(out.get("L")), _ptr(out.get("sweeps")),
                                          _ptr(out.get("fail")), C.byref(rc), _stream(stream))
    check(st, "laim_decode_rounds")
    out["workspace"] = workspace
    return out


def decode_rounds_static(code: Code, params: DecodeParams, e0, shot0: int = 0, form: str = "auto",
                         want_beliefs: bool = False, want_sweeps: bool = False,
                         want_fail: bool = False, out=None, stream=None) -> dict:
    """``laim_decode_rounds_static``: as decode_rounds, with the library's
    static device scratch instead of a workspace (the call allocates no
    device memory; ``out`` may hold preallocated outputs)."""
    import torch
    ns = e0.shape[0]
    _dev(e0, torch.uint8, (ns, code.n), "e0")
    dev = e0.device
    if out is None:
        out = {"z": torch.empty((ns, code.n), dtype=torch.uint8, device=dev),
               "s": torch.empty((ns, code.m), dtype=torch.uint8, device=dev),
               "tclr": torch.empty((ns,), dtype=torch.int32, device=dev),
               "L": torch.empty((ns, code.n), dtype=torch.float32, device=dev) if want_beliefs else None,
               "sweeps": torch.empty((ns,), dtype=torch.int32, device=dev) if want_sweeps else None,
               "fail": torch.empty((ns,), dtype=torch.uint8, device=dev) if want_fail else None}
    P = params.c()
    check(lib().laim_decode_rounds_static(code.handle, C.byref(P), _ptr(e0), shot0, ns, _ptr(out["z"]),
                                          _ptr(out["s"]), _ptr(out["tclr"]), _ptr(out.get("L")),
                                          _ptr(out.get("sweeps")), _ptr(out.get("fail")), FORMS[form],
                                          _stream(stream)), "laim_decode_rounds_static")
    return out


def decode_continuous(code: Code, params: ContinuousParams, e0, shot0: int = 0,
                      checks_per_thread: int = 0, want_fail: bool = False, workspace=None,
                      stream=None, want_steps: bool = False) -> dict:
    """``laim_decode_continuous``: returns device tensors z, s, tclr (float64),
    counts ([nshots, 2] int32: events, moves) and, with want_fail, fail; with
    want_steps the Euler steps computed per shot."""
    import torch
    ns = e0.shape[0]
    _dev(e0, torch.uint8, (ns, code.n), "e0")
    dev = e0.device
    out = {"z": torch.empty((ns, code.n), dtype=torch.uint8, device=dev),
           "s": torch.empty((ns, code.m), dtype=torch.uint8, device=dev),
           "tclr": torch.empty((ns,), dtype=torch.float64, device=dev),
           "counts": torch.empty((ns, 2), dtype=torch.int32, device=dev),
           "fail": torch.empty((ns,), dtype=torch.uint8, device=dev) if want_fail else None,
           "steps": torch.empty((ns,), dtype=torch.int32, device=dev) if want_steps else None}
    if workspace is None:
        workspace = torch.empty((CONTINUOUS_WORKSPACE_BYTES,), dtype=torch.uint8, device=dev)
    P = params.c()
    check(lib().laim_decode_continuous(code.handle, C.byref(P), _ptr(e0), shot0, ns, _ptr(workspace),
                                       workspace.numel(), _ptr(out["z"]), _ptr(out["s"]),
                                       _ptr(out["tclr"]), _ptr(out["counts"]), _ptr(out["steps"]),
                                       _ptr(out["fail"]), checks_per_thread, _stream(stream)),
          "laim_decode_continuous")
    return out


BITCENTRIC_FORMS = {"auto": 0, "chain": 1, "block": 2}


def decode_bitcentric(code: Code, q: float, e0, iters: int, want_beliefs: bool = False,
                      stream=None, form: str = "auto") -> dict:
    """``laim_decode_bitcentric_form``: returns device tensors z, iclr and
    (with want_beliefs) L, the float64 beliefs of the last iteration. form:
    "auto", "chain" (one wavefront per shot, chains only) or "block"."""
    import torch
    ns = e0.shape[0]
    _dev(e0, torch.uint8, (ns, code.n), "e0")
    dev = e0.device
    out = {"z": torch.empty((ns, code.n), dtype=torch.uint8, device=dev),
           "iclr": torch.empty((ns,), dtype=torch.int32, device=dev),
           "L": torch.empty((ns, code.n), dtype=torch.float64, device=dev) if want_beliefs else None}
    if form not in BITCENTRIC_FORMS:
        raise ValueError(f"unknown bit-centric form {form!r}")
    check(lib().laim_decode_bitcentric_form(code.handle, q, _ptr(e0), ns, iters, BITCENTRIC_FORMS[form],
                                            _ptr(out["z"]), _ptr(out["iclr"]), _ptr(out["L"]),
                                            _stream(stream)),
          "laim_decode_bitcentric_form")
    return out


def logical_failure(code: Code, e0, z, stream=None):
    import torch
    ns = e0.shape[0]
    _dev(e0, torch.uint8, (ns, code.n), "e0")
    _dev(z, torch.uint8, (ns, code.n), "z")
    f = torch.empty((ns,), dtype=torch.uint8, device=e0.device)
    check(lib().laim_logical_failure(code.handle, _ptr(e0), _ptr(z), ns, _ptr(f), _stream(stream)),
          "laim_logical_failure")
    return f


class OnlinePlan:
    """``laim_online_plan_*``: the window codes of one code for online
    decoding with these OnlineParams."""

    def __init__(self, code: Code, op: OnlineParams):
        self.code = code
        self.op = op
        O = op.c()
        h = C.c_void_p()
        check(lib().laim_online_plan_create(code.handle, C.byref(O), C.byref(h)), "laim_online_plan_create")
        self.handle = h

    def workspace_bytes(self, params: DecodeParams, nshots: int) -> int:
        P = params.c()
        return int(lib().laim_online_workspace_bytes(self.handle, C.byref(P), nshots))

    def decode(self, params: DecodeParams, nshots: int, shot0: int = 0, e_in=None, eps_in=None,
               workspace=None, want_E: bool = True, want_fail: bool = True, want_cleared: bool = True,
               stream=None) -> dict:
        """``laim_decode_online``: device tensors z [nshots, n] and, as asked,
        E (the final error), fail and cleared (windows that cleared)."""
        import torch
        code = self.code
        dev = f"cuda:{code.device}"
        N = self.op.rounds_total
        if (e_in is None) != (eps_in is None):
            raise ValueError("give both e_in and eps_in or neither")
        if e_in is not None:
            _dev(e_in, torch.uint8, (nshots, N, code.n), "e_in")
            _dev(eps_in, torch.uint8, (nshots, N, code.m), "eps_in")
        out = {"z": torch.empty((nshots, code.n), dtype=torch.uint8, device=dev),
               "E": torch.empty((nshots, code.n), dtype=torch.uint8, device=dev) if want_E else None,
               "fail": torch.empty((nshots,), dtype=torch.uint8, device=dev) if want_fail else None,
               "cleared": torch.empty((nshots,), dtype=torch.int32, device=dev) if want_cleared else None}
        need = self.workspace_bytes(params, nshots)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty((max(need, 256),), dtype=torch.uint8, device=dev)
        P = params.c()
        check(lib().laim_decode_online(self.handle, C.byref(P), shot0, nshots, _ptr(e_in), _ptr(eps_in),
                                       _ptr(workspace), workspace.numel(), _ptr(out["z"]), _ptr(out["E"]),
                                       _ptr(out["fail"]), _ptr(out["cleared"]), _stream(stream)),
              "laim_decode_online")
        out["workspace"] = workspace
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.laim_online_plan_destroy(h)
            self.handle = None


class BatchPlan:
    """``laim_batch_plan_*``: one persistent launch over shots of several
    codes, captured in a HIP graph. ``items`` is a list of dicts with keys
    code, params, e0 (device uint8 [nshots, n]) and optionally shot0 and
    want_fail; outputs are allocated here and rewritten by every launch."""

    def __init__(self, items, stream=None):
        import torch
        self.items = []
        arr = (BatchItem * len(items))()
        for i, it in enumerate(items):
            code, P, e0 = it["code"], it["params"], it["e0"]
            ns = e0.shape[0]
            _dev(e0, torch.uint8, (ns, code.n), "e0")
            o = {"code": code, "e0": e0, "shot0": it.get("shot0", 0),
                 "z": torch.empty((ns, code.n), dtype=torch.uint8, device=e0.device),
                 "s": torch.empty((ns, code.m), dtype=torch.uint8, device=e0.device),
                 "tclr": torch.empty((ns,), dtype=torch.int32, device=e0.device),
                 "fail": torch.empty((ns,), dtype=torch.uint8, device=e0.device)
                 if it.get("want_fail", True) else None}
            self.items.append(o)
            arr[i] = BatchItem(code.handle, P.c(), C.c_void_p(e0.data_ptr()), o["shot0"], ns,
                               C.c_void_p(o["z"].data_ptr()), C.c_void_p(o["s"].data_ptr()),
                               C.c_void_p(o["tclr"].data_ptr()),
                               C.c_void_p(o["fail"].data_ptr()) if o["fail"] is not None else None)
        h = C.c_void_p()
        check(lib().laim_batch_plan_create(arr, len(items), _stream(stream), C.byref(h)),
              "laim_batch_plan_create")
        self.handle = h

    def launch(self, stream=None):
        check(lib().laim_batch_plan_launch(self.handle, _stream(stream)), "laim_batch_plan_launch")
        return self.items

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.laim_batch_plan_destroy(h)
            self.handle = None


class Server:
    """``laim_server_*``: continuous batching of single-shot decode requests
    with device-resident state; every ``step`` advances each resident request
    by one round and returns its per-round event."""

    def __init__(self, device: int = 0, mem_budget: int = 1 << 30, max_slots: int = 4096):
        h = C.c_void_p()
        check(lib().laim_server_create(device, mem_budget, max_slots, C.byref(h)), "laim_server_create")
        self.handle = h
        self.max_slots = max_slots
        self._ev = (ServerEvent * max_slots)()
        self._codes = {}

    def submit(self, code: Code, params: DecodeParams, shot_id: int, e0=None, p: float = 0.0) -> int:
        """Queues one shot. With e0 given (n host bits) it is copied; with
        e0 None the server samples the error on the device from
        (params.seed, shot_id, p)."""
        ptr = None
        if e0 is not None:
            e0 = np.ascontiguousarray(e0, dtype=np.uint8).ravel()
            if e0.size != code.n:
                raise ValueError("e0 must hold n bits")
            ptr = e0.ctypes.data_as(C.c_void_p)
        P = params.c()
        t = C.c_uint64()
        check(lib().laim_server_submit(self.handle, code.handle, C.byref(P), shot_id, ptr, float(p),
                                       C.byref(t)), "laim_server_submit")
        self._codes[t.value] = code
        return t.value

    def step(self, max_events: int | None = None) -> list:
        """One server step; at most max_events requests (default: every
        slot) advance."""
        k = self.max_slots if max_events is None else min(int(max_events), self.max_slots)
        n = C.c_int32()
        check(lib().laim_server_step(self.handle, self._ev, k, C.byref(n)), "laim_server_step")
        out = []
        for i in range(n.value):
            e = self._ev[i]
            out.append({"ticket": e.ticket, "round": e.round, "done": bool(e.done), "tclr": e.tclr,
                        "flips": e.flips, "defects": e.defects, "fail": e.fail,
                        "latency_ns": e.latency_ns})
        return out

    def result(self, ticket: int) -> dict:
        code = self._codes.pop(ticket)
        z = np.zeros(code.n, dtype=np.uint8)
        s = np.zeros(code.m, dtype=np.uint8)
        t = C.c_int32()
        check(lib().laim_server_result(self.handle, ticket, z.ctypes.data_as(C.c_void_p),
                                       s.ctypes.data_as(C.c_void_p), C.byref(t)), "laim_server_result")
        return {"z": z, "s": s, "tclr": t.value}

    def stats(self) -> dict:
        r, w = C.c_int32(), C.c_int32()
        b = C.c_size_t()
        check(lib().laim_server_stats(self.handle, C.byref(r), C.byref(w), C.byref(b)), "laim_server_stats")
        return {"resident": r.value, "waiting": w.value, "bytes": b.value}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.laim_server_destroy(h)
            self.handle = None
