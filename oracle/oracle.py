"""Python access to the CPU oracle (``laim_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark. The product library never imports it,
and it never imports the product package: codes are passed in as anything
with ``H``/``G`` attributes holding ``rows``, ``cols``, ``rowptr``, ``col``.

``build()`` compiles the C file with gcc (FP32 without contraction, OpenMP
over shots) into ``oracle/liblaim_oracle.so``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "laim_oracle.c")
LIB = os.path.join(HERE, "liblaim_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle (always when ``force``)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


class Params(C.Structure):
    _fields_ = [("bp", C.c_int32), ("alpha", C.c_float), ("q", C.c_double), ("clamp", C.c_float),
                ("iters", C.c_int32), ("rounds", C.c_int32), ("mask_density", C.c_double),
                ("gauge", C.c_int32), ("evidence", C.c_int32), ("retire", C.c_int32),
                ("seed", C.c_uint64), ("conflict", C.c_int32), ("move", C.c_int32)]


CONFLICT_RULES = {"or": 0, "xor": 1, "sequential": 2}
MOVES = {"single": 0, "multi": 1}


@dataclass
class DecodeParams:
    """Decoder knobs (defaults: Table S1's q, CLAMP; 20 iterations; rho = 0.5)."""

    bp: str = "minsum"  # "minsum" or "sumproduct"
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
    conflict: str = "or"  # how one round's move requests combine: "or", "xor", "sequential"
    move: str = "single"  # "single": LocalMove; "multi": every qubit of N(c) with L_v > 0

    def c(self) -> Params:
        return Params(1 if self.bp == "sumproduct" else 0, self.alpha, self.q, self.clamp,
                      self.iters, self.rounds, self.mask_density, int(self.gauge),
                      int(self.evidence), int(self.retire), self.seed,
                      CONFLICT_RULES[self.conflict], MOVES[self.move])


class OnlineParamsC(C.Structure):
    _fields_ = [("rounds_total", C.c_int32), ("window", C.c_int32), ("commit", C.c_int32),
                ("p", C.c_double), ("p_meas", C.c_double)]


@dataclass
class OnlineParams:
    """Online decoding: N syndrome rounds (the last perfect), windows of W
    rounds of which the first C are committed, data and measurement error
    rates."""

    rounds_total: int = 8
    window: int = 4
    commit: int = 2
    p: float = 0.01
    p_meas: float = 0.01

    def c(self) -> OnlineParamsC:
        return OnlineParamsC(self.rounds_total, self.window, self.commit, self.p, self.p_meas)

    def layout(self):
        """(number of windows, rounds of the last window)."""
        k = 0
        while k * self.commit + self.window < self.rounds_total:
            k += 1
        return k + 1, self.rounds_total - k * self.commit


class CtmParams(C.Structure):
    _fields_ = [("bp", C.c_int32), ("alpha", C.c_float), ("q", C.c_double), ("clamp", C.c_float),
                ("dt", C.c_double), ("tau", C.c_double), ("max_steps", C.c_int32),
                ("evidence", C.c_int32), ("seed", C.c_uint64)]


@dataclass
class ContinuousParams:
    """Continuous-time machine knobs (defaults: Table S1, 2D toric code row)."""

    bp: str = "minsum"
    alpha: float = 0.75
    q: float = 0.05
    clamp: float = 1000.0
    dt: float = 0.001
    tau: float = 0.1
    t_max: float = 100.0  # clock units; the run stops unsuccessfully after t_max / dt steps
    evidence: bool = True
    seed: int = 0

    @property
    def max_steps(self) -> int:
        return int(math.floor(self.t_max / self.dt + 0.5))

    def c(self) -> CtmParams:
        return CtmParams(1 if self.bp == "sumproduct" else 0, self.alpha, self.q, self.clamp,
                         self.dt, self.tau, self.max_steps, int(self.evidence), self.seed)


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        i32p, u8p, f32p, u32p = (C.POINTER(C.c_int32), C.POINTER(C.c_uint8),
                                 C.POINTER(C.c_float), C.POINTER(C.c_uint32))
        L.orc_version.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_bernoulli_bound.restype = C.c_uint64
        L.orc_bernoulli_bound.argtypes = [C.c_double]
        for nm in ("orc_exp_neg", "orc_log1p_unit", "orc_softplus_neg"):
            getattr(L, nm).restype = C.c_float
            getattr(L, nm).argtypes = [C.c_float]
        L.orc_boxplus.restype = C.c_float
        L.orc_boxplus.argtypes = [C.c_float, C.c_float]
        for nm in ("orc_vec_exp_neg", "orc_vec_log1p_unit"):
            getattr(L, nm).argtypes = [f32p, C.c_int32, f32p]
        L.orc_vec_boxplus.argtypes = [f32p, f32p, C.c_int32, f32p]
        L.orc_vec_philox.argtypes = [u32p, u32p, C.c_int32, u32p]
        L.orc_sample_noise.argtypes = [C.c_int32, C.c_double, C.c_uint64, C.c_uint64, C.c_int32, u8p]
        L.orc_syndrome.argtypes = [C.c_int32, C.c_int32, i32p, i32p, u8p, C.c_int32, u8p]
        L.orc_decode.restype = C.c_int32
        L.orc_decode.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.POINTER(Params), u8p,
                                 C.c_uint64, C.c_int32, u8p, u8p, i32p, f32p, u8p, u8p, C.c_int32]
        L.orc_bp_sweep.restype = C.c_int32
        L.orc_bp_sweep.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.POINTER(Params), f32p, u8p,
                                   f32p, f32p, f32p]
        L.orc_logical_failure.restype = C.c_int32
        L.orc_logical_failure.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.c_int32, i32p, i32p,
                                          u8p, u8p, C.c_int32, u8p]
        L.orc_gf2_rank.restype = C.c_int32
        L.orc_gf2_rank.argtypes = [C.c_int32, C.c_int32, i32p, i32p]
        L.orc_evidence_thresholds.argtypes = [C.c_int32, f32p]
        f64p = C.POINTER(C.c_double)
        L.orc_ln_unit.restype = C.c_double
        L.orc_ln_unit.argtypes = [C.c_double]
        L.orc_vec_ln_unit.argtypes = [f64p, C.c_int32, f64p]
        L.orc_ctm_bp_steps.restype = C.c_int32
        L.orc_ctm_bp_steps.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.POINTER(CtmParams), u8p,
                                       C.c_int32, f32p, f32p]
        L.orc_ctm_decode.restype = C.c_int32
        L.orc_ctm_decode.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.POINTER(CtmParams), u8p,
                                     C.c_uint64, C.c_int32, u8p, u8p, f64p, i32p, f64p, C.c_int32,
                                     C.c_int32]
        L.orc_resolve_moves.restype = C.c_int32
        L.orc_resolve_moves.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.c_int32, u8p, C.c_int32,
                                        i32p, i32p, u32p, u8p]
        L.orc_bitcentric_machine.restype = C.c_int32
        L.orc_bitcentric_machine.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.c_double, u8p,
                                             C.c_int32, u8p, C.POINTER(C.c_double), i32p]
        L.orc_online_noise.argtypes = [C.c_int32, C.c_int32, C.POINTER(OnlineParamsC), C.c_uint64, C.c_uint64,
                                       C.c_int32, u8p, u8p]
        L.orc_online_decode.restype = C.c_int32
        L.orc_online_decode.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.c_int32, i32p, i32p,
                                        C.POINTER(Params), C.POINTER(OnlineParamsC), C.c_uint64, C.c_int32,
                                        u8p, u8p, u8p, u8p, u8p, i32p, u8p, u8p, C.c_int32]
        L.orc_decode_syndrome.restype = C.c_int32
        L.orc_decode_syndrome.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.POINTER(Params), u8p, C.c_uint64,
                                          C.c_int32, C.c_int32, u8p, u8p, i32p]
        L.orc_window_code.restype = C.c_int32
        L.orc_window_code.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.c_int32, C.c_int32, i32p, i32p]
        _lib = L
    return _lib


def _csr(M):
    rp = np.ascontiguousarray(M.rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(M.col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    return rp, cl


# ---------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 on arrays of counters [k,4] and keys [k,2] (uint32)."""
    ctr = np.ascontiguousarray(np.atleast_2d(ctr), dtype=np.uint32)
    key = np.ascontiguousarray(np.atleast_2d(key), dtype=np.uint32)
    out = np.zeros_like(ctr)
    lib().orc_vec_philox(_p(ctr, C.c_uint32), _p(key, C.c_uint32), ctr.shape[0], _p(out, C.c_uint32))
    return out


def bernoulli_bound(p: float) -> int:
    return int(lib().orc_bernoulli_bound(p))


def _vec(name, x):
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    y = np.zeros_like(x)
    getattr(lib(), name)(_p(x, C.c_float), x.size, _p(y, C.c_float))
    return y


def exp_neg(x):
    return _vec("orc_vec_exp_neg", x)


def log1p_unit(x):
    return _vec("orc_vec_log1p_unit", x)


def boxplus(a, b):
    """a [+] b = 2 atanh(tanh(a/2) tanh(b/2)) in the oracle's FP32 evaluation."""
    a = np.ascontiguousarray(a, dtype=np.float32).ravel()
    b = np.ascontiguousarray(b, dtype=np.float32).ravel()
    y = np.zeros_like(a)
    lib().orc_vec_boxplus(_p(a, C.c_float), _p(b, C.c_float), a.size, _p(y, C.c_float))
    return y


def evidence_thresholds(dmax: int) -> np.ndarray:
    t = np.zeros(dmax + 1, dtype=np.float32)
    lib().orc_evidence_thresholds(dmax, _p(t, C.c_float))
    return t


# ---------------------------------------------------------------- method
def sample_noise(code, p: float, seed: int, shot0: int, nshots: int) -> np.ndarray:
    n = code.H.cols
    e = np.zeros((nshots, n), dtype=np.uint8)
    lib().orc_sample_noise(n, p, seed, shot0, nshots, _p(e, C.c_uint8))
    return e


def syndrome(code, e) -> np.ndarray:
    e = np.ascontiguousarray(np.atleast_2d(e), dtype=np.uint8)
    rp, cl = _csr(code.H)
    s = np.zeros((e.shape[0], code.H.rows), dtype=np.uint8)
    lib().orc_syndrome(code.H.rows, code.H.cols, _p(rp, C.c_int32), _p(cl, C.c_int32),
                       _p(e, C.c_uint8), e.shape[0], _p(s, C.c_uint8))
    return s


def resolve_moves(code, conflict: str, s, req_c, req_v, req_key) -> np.ndarray:
    """Flip vector of one round's move requests (check req_c[i] asks for qubit
    req_v[i] at ring time req_key[i]) under a conflict rule, from the
    syndrome s at the start of the move step."""
    m, n = code.H.rows, code.H.cols
    rp, cl = _csr(code.H)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    rc_ = np.ascontiguousarray(req_c, dtype=np.int32)
    rv = np.ascontiguousarray(req_v, dtype=np.int32)
    rk = np.ascontiguousarray(req_key, dtype=np.uint32)
    if rc_.size == 0:
        rc_, rv, rk = np.zeros(1, np.int32), np.zeros(1, np.int32), np.zeros(1, np.uint32)
    f = np.zeros(n, dtype=np.uint8)
    rc = lib().orc_resolve_moves(m, n, _p(rp, C.c_int32), _p(cl, C.c_int32), CONFLICT_RULES[conflict],
                                 _p(s, C.c_uint8), len(req_c), _p(rc_, C.c_int32), _p(rv, C.c_int32),
                                 _p(rk, C.c_uint32), _p(f, C.c_uint8))
    if rc != 0:
        raise RuntimeError(f"oracle resolve_moves failed with status {rc}")
    return f


def decode(code, params: DecodeParams, e0, shot0: int = 0, nthreads: int = 1,
           want_beliefs: bool = False, trace: bool = False) -> dict:
    """Run the round machine on every row of e0 (shot ids shot0, shot0+1, ...)."""
    e0 = np.ascontiguousarray(np.atleast_2d(e0), dtype=np.uint8)
    ns, n = e0.shape
    m = code.H.rows
    assert n == code.H.cols
    rp, cl = _csr(code.H)
    z = np.zeros((ns, n), dtype=np.uint8)
    s = np.zeros((ns, m), dtype=np.uint8)
    t = np.zeros(ns, dtype=np.int32)
    L = np.zeros((ns, n), dtype=np.float32) if want_beliefs else None
    st = zt = None
    if trace:
        assert ns == 1, "traces are per shot"
        st = np.zeros((params.rounds, m), dtype=np.uint8)
        zt = np.zeros((params.rounds, n), dtype=np.uint8)
    P = params.c()
    rc = lib().orc_decode(m, n, _p(rp, C.c_int32), _p(cl, C.c_int32), C.byref(P), _p(e0, C.c_uint8),
                          shot0, ns, _p(z, C.c_uint8), _p(s, C.c_uint8), _p(t, C.c_int32),
                          _p(L, C.c_float) if L is not None else None,
                          _p(st, C.c_uint8) if st is not None else None,
                          _p(zt, C.c_uint8) if zt is not None else None, nthreads)
    if rc != 0:
        raise RuntimeError(f"oracle decode failed with status {rc}")
    return {"z": z, "s": s, "tclr": t, "L": L, "s_trace": st, "z_trace": zt}


def bp_sweep(code, params: DecodeParams, pi_v, s, mvc):
    """One check phase then one qubit phase. Returns (m_cv, m_vc)."""
    rp, cl = _csr(code.H)
    E = code.H.nnz
    pi_v = np.ascontiguousarray(pi_v, dtype=np.float32)
    s = np.ascontiguousarray(s, dtype=np.uint8)
    mvc = np.ascontiguousarray(mvc, dtype=np.float32)
    mcv_o = np.zeros(E, dtype=np.float32)
    mvc_o = np.zeros(E, dtype=np.float32)
    P = params.c()
    rc = lib().orc_bp_sweep(code.H.rows, code.H.cols, _p(rp, C.c_int32), _p(cl, C.c_int32),
                            C.byref(P), _p(pi_v, C.c_float), _p(s, C.c_uint8), _p(mvc, C.c_float),
                            _p(mcv_o, C.c_float), _p(mvc_o, C.c_float))
    assert rc == 0
    return mcv_o, mvc_o


def logical_failure(code, e0, z) -> np.ndarray:
    e0 = np.ascontiguousarray(np.atleast_2d(e0), dtype=np.uint8)
    z = np.ascontiguousarray(np.atleast_2d(z), dtype=np.uint8)
    hr, hc = _csr(code.H)
    gr, gc = _csr(code.G)
    f = np.zeros(e0.shape[0], dtype=np.uint8)
    rc = lib().orc_logical_failure(code.H.rows, code.H.cols, _p(hr, C.c_int32), _p(hc, C.c_int32),
                                   code.G.rows, _p(gr, C.c_int32), _p(gc, C.c_int32),
                                   _p(e0, C.c_uint8), _p(z, C.c_uint8), e0.shape[0], _p(f, C.c_uint8))
    assert rc == 0
    return f


def gf2_rank(M) -> int:
    rp, cl = _csr(M)
    return int(lib().orc_gf2_rank(M.rows, M.cols, _p(rp, C.c_int32), _p(cl, C.c_int32)))


def bitcentric_machine(code, q: float, e0, iters: int):
    """Discrete bit-centric machine (double precision). Returns
    (e_trace [iters, n], L_trace [iters, n], i_clr)."""
    rp, cl = _csr(code.H)
    e0 = np.ascontiguousarray(e0, dtype=np.uint8).ravel()
    n = code.H.cols
    et = np.zeros((iters, n), dtype=np.uint8)
    Lt = np.zeros((iters, n), dtype=np.float64)
    ic = np.zeros(1, dtype=np.int32)
    rc = lib().orc_bitcentric_machine(code.H.rows, n, _p(rp, C.c_int32), _p(cl, C.c_int32), q,
                                      _p(e0, C.c_uint8), iters, _p(et, C.c_uint8),
                                      Lt.ctypes.data_as(C.POINTER(C.c_double)), _p(ic, C.c_int32))
    assert rc == 0
    return et, Lt, int(ic[0])


# ---------------------------------------------------------------- continuous-time machine
def ln_unit(x) -> np.ndarray:
    """The oracle's FP64 natural logarithm on (0, 1]."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.zeros_like(x)
    lib().orc_vec_ln_unit(x.ctypes.data_as(C.POINTER(C.c_double)), x.size,
                          y.ctypes.data_as(C.POINTER(C.c_double)))
    return y


def ctm_bp_steps(code, params: ContinuousParams, s, K: int):
    """K Euler steps of the damped Jacobi BP from m = 0 on the fixed syndrome
    s. Returns (m_cv, m_vc) in edge order."""
    rp, cl = _csr(code.H)
    E = code.H.nnz
    s = np.ascontiguousarray(s, dtype=np.uint8).ravel()
    mcv = np.zeros(E, dtype=np.float32)
    mvc = np.zeros(E, dtype=np.float32)
    P = params.c()
    rc = lib().orc_ctm_bp_steps(code.H.rows, code.H.cols, _p(rp, C.c_int32), _p(cl, C.c_int32),
                                C.byref(P), _p(s, C.c_uint8), K, _p(mcv, C.c_float), _p(mvc, C.c_float))
    assert rc == 0
    return mcv, mvc


def ctm_decode(code, params: ContinuousParams, e0, shot0: int = 0, nthreads: int = 1,
               trace_cap: int = 0) -> dict:
    """Run the continuous-time machine on every row of e0. With one shot and
    trace_cap > 0 the first trace_cap events are returned as rows
    (time, |S| before, ringing check, flipped qubit or -1)."""
    e0 = np.ascontiguousarray(np.atleast_2d(e0), dtype=np.uint8)
    ns, n = e0.shape
    m = code.H.rows
    rp, cl = _csr(code.H)
    z = np.zeros((ns, n), dtype=np.uint8)
    s = np.zeros((ns, m), dtype=np.uint8)
    t = np.zeros(ns, dtype=np.float64)
    cnt = np.zeros((ns, 2), dtype=np.int32)
    tr = np.zeros((max(trace_cap, 1), 4), dtype=np.float64)
    P = params.c()
    f64p = C.POINTER(C.c_double)
    rc = lib().orc_ctm_decode(m, n, _p(rp, C.c_int32), _p(cl, C.c_int32), C.byref(P),
                              _p(e0, C.c_uint8), shot0, ns, _p(z, C.c_uint8), _p(s, C.c_uint8),
                              t.ctypes.data_as(f64p), _p(cnt, C.c_int32),
                              tr.ctypes.data_as(f64p) if trace_cap > 0 else None, trace_cap, nthreads)
    if rc != 0:
        raise RuntimeError(f"oracle ctm_decode failed with status {rc}")
    out = {"z": z, "s": s, "tclr": t, "events": cnt[:, 0].copy(), "moves": cnt[:, 1].copy()}
    if trace_cap > 0:
        k = min(int(cnt[0, 0]), trace_cap)
        out["trace"] = tr[:k].copy()
    return out


# ---------------------------------------------------------------- online decoding
def online_noise(code, params: OnlineParams, seed: int, shot0: int, nshots: int):
    """Spacetime errors: e [nshots, N, n] (new data errors of each round) and
    eps [nshots, N, m] (measurement errors; the last round's are 0)."""
    n, m, N = code.H.cols, code.H.rows, params.rounds_total
    e = np.zeros((nshots, N, n), dtype=np.uint8)
    eps = np.zeros((nshots, N, m), dtype=np.uint8)
    O = params.c()
    lib().orc_online_noise(n, m, C.byref(O), seed, shot0, nshots, _p(e, C.c_uint8), _p(eps, C.c_uint8))
    return e, eps


def window_code(code, w: int, w_eps: int):
    """CSR (rowptr, col, number of variables) of a window of w rounds with
    measurement variables for its first w_eps rounds."""
    rp, cl = _csr(code.H)
    m = code.H.rows
    rpo = np.zeros(w * m + 1, dtype=np.int32)
    clo = np.zeros(max(1, w * (code.H.nnz + 2 * m)), dtype=np.int32)
    nv = lib().orc_window_code(m, code.H.cols, _p(rp, C.c_int32), _p(cl, C.c_int32), w, w_eps,
                               _p(rpo, C.c_int32), _p(clo, C.c_int32))
    assert nv >= 0
    return rpo, clo[:rpo[-1]].copy(), int(nv)


def online_decode(code, params: DecodeParams, online: OnlineParams, shot0: int = 0, nshots: int = 1,
                  e_in=None, eps_in=None, nthreads: int = 1, trace: bool = False) -> dict:
    """The online (spacetime-window) decoder on nshots shots; with e_in and
    eps_in ([nshots, N, n], [nshots, N, m]) the given errors replace the
    sampled ones."""
    n, m, N = code.H.cols, code.H.rows, online.rounds_total
    hr, hc = _csr(code.H)
    gr, gc = _csr(code.G)
    if e_in is not None:
        e_in = np.ascontiguousarray(e_in, dtype=np.uint8).reshape(nshots, N, n)
        eps_in = np.ascontiguousarray(eps_in, dtype=np.uint8).reshape(nshots, N, m)
    z = np.zeros((nshots, n), dtype=np.uint8)
    E = np.zeros((nshots, n), dtype=np.uint8)
    f = np.zeros(nshots, dtype=np.uint8)
    cl = np.zeros(nshots, dtype=np.int32)
    nwin, _ = online.layout()
    W = online.window
    ts = tz = None
    if trace:
        assert nshots == 1
        ts = np.zeros((nwin, W * m), dtype=np.uint8)
        tz = np.zeros((nwin, W * (n + m)), dtype=np.uint8)
    P = params.c()
    O = online.c()
    rc = lib().orc_online_decode(m, n, _p(hr, C.c_int32), _p(hc, C.c_int32), code.G.rows, _p(gr, C.c_int32),
                                 _p(gc, C.c_int32), C.byref(P), C.byref(O), shot0, nshots,
                                 _p(e_in, C.c_uint8) if e_in is not None else None,
                                 _p(eps_in, C.c_uint8) if eps_in is not None else None,
                                 _p(z, C.c_uint8), _p(E, C.c_uint8), _p(f, C.c_uint8), _p(cl, C.c_int32),
                                 _p(ts, C.c_uint8) if ts is not None else None,
                                 _p(tz, C.c_uint8) if tz is not None else None, nthreads)
    if rc != 0:
        raise RuntimeError(f"oracle online_decode failed with status {rc}")
    return {"z": z, "E": E, "fail": f, "cleared": cl, "windows": nwin, "trace_s": ts, "trace_z": tz}


def decode_syndrome(H, params: DecodeParams, s0, shot0: int = 0, r0: int = 0) -> dict:
    """The round machine on the Tanner graph of H (a CSR with rows, cols,
    rowptr, col) from start syndromes s0 [nshots, m], its rounds numbered
    from r0."""
    s0 = np.ascontiguousarray(np.atleast_2d(s0), dtype=np.uint8)
    ns = s0.shape[0]
    rp = np.ascontiguousarray(H.rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(H.col if len(H.col) else np.zeros(1), dtype=np.int32)
    z = np.zeros((ns, H.cols), dtype=np.uint8)
    s = np.zeros((ns, H.rows), dtype=np.uint8)
    t = np.zeros(ns, dtype=np.int32)
    P = params.c()
    rc = lib().orc_decode_syndrome(H.rows, H.cols, _p(rp, C.c_int32), _p(cl, C.c_int32), C.byref(P),
                                   _p(s0, C.c_uint8), shot0, r0, ns, _p(z, C.c_uint8), _p(s, C.c_uint8),
                                   _p(t, C.c_int32))
    if rc != 0:
        raise RuntimeError(f"oracle decode_syndrome failed with status {rc}")
    return {"z": z, "s": s, "tclr": t}
