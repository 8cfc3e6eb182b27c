// laim_online.hip -- online decoding in overlapping spacetime windows.
//
// The Discussion's next step for the machine: faults and syndrome rounds
// keep arriving, the Tanner graph is promoted to a spacetime decoding graph
// and the local dynamics runs inside overlapping windows of it. The rules
// here (the paper gives none):
//  - N syndrome rounds t = 1..N. Before round t every qubit gets a new Z
//    error e_t[v] ~ Bernoulli(p) (word v mod 4 of Philox(seed, (shot_lo,
//    shot_hi, v / 4, 16 t + 3))); round t reads m_t = H E_t ^ eps_t with
//    E_t the sum of e_1..e_t and measurement errors eps_t[c] ~ Bernoulli(p_meas)
//    (word c mod 4 of Philox(seed, (shot_lo, shot_hi, c / 4, 16 t + 4))),
//    except the last round, which is perfect.
//  - Detectors D_t = m_t ^ m_{t-1} = H e_t ^ eps_t ^ eps_{t-1}.
//  - A window of w rounds is a code of its own: one variable per data error
//    (tau, v) -> tau n + v and per measurement error (tau, c) -> w n + tau m + c
//    of its first w_eps rounds (w_eps = w, or w - 1 for the window ending
//    with the perfect round); detector (tau, c) is check tau m + c.
//  - Window k covers rounds k C + 1 .. min(k C + W, N); the last is the
//    first to reach N. Its syndrome is the detectors of its rounds, with the
//    measurement corrections committed for round k C added to its first
//    round. The round machine decodes it from fresh messages with its rounds
//    numbered from k R. The corrections of the window's first C rounds (all
//    rounds in the last window) are committed: data corrections accumulate
//    into z, and the measurement corrections of the last committed round are
//    carried into the next window.
//  - The result is z and the failure test of the offline decoder applied to
//    E_N and z.
// All shots of a call advance window by window; each window is one launch
// of the resident (or stream) form on its window code.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "device_math.h"
#include "laim_internal.h"

namespace laim {

// One block per shot: for each round, the new data errors (kept in LDS and
// summed into E) and the round's measurement errors, then the round's
// detectors. LDS: the round's data errors (n bytes), E (n bytes), this and
// the previous round's measurement errors (2 m bytes).
__global__ void __launch_bounds__(256) online_noise_kernel(DevCode c, int32_t N, uint64_t bd, uint64_t bm,
                                                           uint64_t seed, uint64_t shot0,
                                                           const uint8_t* __restrict__ e_in,
                                                           const uint8_t* __restrict__ eps_in,
                                                           uint8_t* __restrict__ D, uint8_t* __restrict__ E) {
  extern __shared__ uint8_t sm[];
  const int32_t n = c.n, m = c.m;
  uint8_t* et = sm;
  uint8_t* Ea = sm + n;
  uint8_t* ep[2] = {sm + 2 * n, sm + 2 * n + m};
  const int64_t i = bid_x();
  const uint64_t shot = shot0 + (uint64_t)i;
  const uint32_t s_lo = (uint32_t)shot, s_hi = (uint32_t)(shot >> 32);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int32_t v = tid_x(); v < n; v += bdim_x()) Ea[v] = 0;
  // round t writes its measurement errors to ep[t & 1] and reads eps_{t-1}
  // from the other buffer: eps_0 = 0 goes to ep[0]
  for (int32_t ch = tid_x(); ch < m; ch += bdim_x()) ep[0][ch] = 0;
  for (int32_t t = 1; t <= N; ++t) {
    uint8_t* ec = ep[t & 1];
    const uint8_t* eq = ep[(t & 1) ^ 1];
    if (e_in) {
      const uint8_t* row = e_in + (i * N + (t - 1)) * (int64_t)n;
      for (int32_t v = tid_x(); v < n; v += bdim_x()) et[v] = row[v] & 1u;
      const uint8_t* mrow = eps_in + (i * N + (t - 1)) * (int64_t)m;
      for (int32_t ch = tid_x(); ch < m; ch += bdim_x()) ec[ch] = (t < N) ? (mrow[ch] & 1u) : 0;
    } else {
      for (int32_t b = tid_x(); 4 * b < n; b += bdim_x()) {
        const Philox4 w = philox4x32_10(s_lo, s_hi, (uint32_t)b, ((uint32_t)t << 4) | 3u, k0, k1);
        const uint32_t ww[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (4 * b + q < n) et[4 * b + q] = below(ww[q], bd) ? 1 : 0;
      }
      for (int32_t b = tid_x(); 4 * b < m; b += bdim_x()) {
        uint32_t ww[4] = {0u, 0u, 0u, 0u};
        if (t < N) {
          const Philox4 w = philox4x32_10(s_lo, s_hi, (uint32_t)b, ((uint32_t)t << 4) | 4u, k0, k1);
          ww[0] = w.w0;
          ww[1] = w.w1;
          ww[2] = w.w2;
          ww[3] = w.w3;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (4 * b + q < m) ec[4 * b + q] = (t < N && below(ww[q], bm)) ? 1 : 0;
      }
    }
    __syncthreads();
    for (int32_t v = tid_x(); v < n; v += bdim_x()) Ea[v] ^= et[v];
    uint8_t* Drow = D + (i * N + (t - 1)) * (int64_t)m;
    for (int32_t ch = tid_x(); ch < m; ch += bdim_x()) {
      const int32_t d = c.chk_deg[ch];
      uint32_t x = ec[ch] ^ eq[ch];
      for (int32_t j = 0; j < d; ++j) x ^= et[c.chk_var[(int64_t)ch * c.dcmax + j]];
      Drow[ch] = (uint8_t)(x & 1u);
    }
    __syncthreads();
  }
  for (int32_t v = tid_x(); v < n; v += bdim_x()) E[i * (int64_t)n + v] = Ea[v];
}

// Syndrome of window k for every shot: rows a .. a + w - 1 of the
// detectors, the carried correction added to the first.
__global__ void __launch_bounds__(256) online_window_syndrome(int32_t m, int32_t N, int32_t a, int32_t w,
                                                              const uint8_t* __restrict__ D,
                                                              const uint8_t* __restrict__ bnd,
                                                              uint8_t* __restrict__ sw) {
  const int64_t i = bid_y();
  const int32_t j = bid_x() * bdim_x() + tid_x();
  if (j >= w * m) return;
  uint8_t x = D[(i * N + a) * (int64_t)m + j];
  if (j < m) x ^= bnd[i * (int64_t)m + j];
  sw[i * (int64_t)w * m + j] = x;
}

// Commit of window k: the data corrections of its first cr rounds into z,
// the measurement corrections of round cr - 1 into the carry (unless it is
// the last window), and the window's clearing into the count.
__global__ void __launch_bounds__(256) online_commit(int32_t n, int32_t m, int32_t w, int32_t nvw, int32_t cr,
                                                     int32_t last, const uint8_t* __restrict__ zw,
                                                     const int32_t* __restrict__ tclr_w,
                                                     uint8_t* __restrict__ z, uint8_t* __restrict__ bnd,
                                                     int32_t* __restrict__ cleared) {
  const int64_t i = bid_y();
  const int32_t j = bid_x() * bdim_x() + tid_x();
  const uint8_t* row = zw + i * (int64_t)nvw;
  if (j < n) {
    uint8_t x = z[i * (int64_t)n + j];
    for (int32_t tau = 0; tau < cr; ++tau) x ^= row[tau * n + j];
    z[i * (int64_t)n + j] = x & 1u;
  }
  if (!last && j < m) bnd[i * (int64_t)m + j] = row[w * n + (cr - 1) * m + j];
  if (cleared && j == 0) cleared[i] += (tclr_w[i] >= 0) ? 1 : 0;
}

__global__ void __launch_bounds__(256) online_clear(uint8_t* __restrict__ a, int64_t na, int32_t* __restrict__ b,
                                                    int64_t nb) {
  const int64_t j = (int64_t)bid_x() * bdim_x() + tid_x();
  if (j < na) a[j] = 0;
  if (j < nb) b[j] = 0;
}

}  // namespace laim

using namespace laim;

struct laim_online_plan {
  const laim_code* base = nullptr;
  laim_online_params op;
  int32_t nwin = 0, w_last = 0;
  laim_code* win_full = nullptr;  // W rounds, measurement variables on every round (nwin > 1)
  laim_code* win_last = nullptr;  // w_last rounds, ending with the perfect round
};

namespace {

// The window's spacetime check matrix in CSR: detector (tau, c) holds the
// data errors of its round, then the measurement errors of rounds tau - 1
// and tau (where the window has them), in ascending variable order.
void window_csr(const laim_code* b, int32_t w, int32_t w_eps, std::vector<int32_t>* rp,
                std::vector<int32_t>* col) {
  const int32_t m = b->m, n = b->n;
  rp->assign((size_t)w * m + 1, 0);
  col->clear();
  col->reserve((size_t)w * (b->E + 2 * m));
  for (int32_t tau = 0; tau < w; ++tau) {
    const int32_t data0 = tau * n;
    const int32_t meas_prev = (tau >= 1 && tau - 1 < w_eps) ? w * n + (tau - 1) * m : -1;
    const int32_t meas_own = (tau < w_eps) ? w * n + tau * m : -1;
    for (int32_t c = 0; c < m; ++c) {
      for (int32_t k = b->h_rowptr[c]; k < b->h_rowptr[c + 1]; ++k) col->push_back(data0 + b->h_col[k]);
      if (meas_prev >= 0) col->push_back(meas_prev + c);
      if (meas_own >= 0) col->push_back(meas_own + c);
      (*rp)[(size_t)tau * m + c + 1] = (int32_t)col->size();
    }
  }
}

laim_status build_window(const laim_code* b, int32_t w, int32_t w_eps, laim_code** out) {
  std::vector<int32_t> rp, col;
  window_csr(b, w, w_eps, &rp, &col);
  const int32_t nv = w * b->n + w_eps * b->m;
  const int32_t zero = 0;
  // no commuting stabilisers and no logicals: the window code is only decoded
  return laim_build_tanner_ex(w * b->m, nv, rp.data(), col.data(), 0, &zero, &zero, 0, &zero, &zero,
                              b->device, out);
}

struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// Form and workspace of a window decode: resident when the window code fits
// it, else stream.
size_t window_decode_bytes(const laim_code* wc, const KParams& kp, int32_t nshots, bool* resident,
                           ResidentShape* sh) {
  const bool seq = kp.conflict == kConflictSequential;
  const laim_resident_cfg* want = wc->has_cfg[kp.bp] ? &wc->cfg[kp.bp] : nullptr;
  *resident = !(kp.bp == 0 && kp.alpha > 1.0f) &&
              resident_shape(wc->dev, kp.bp, want, sh, wc->device, seq, reg_dv2_ok(kp));
  return *resident ? resident_workspace_bytes() : stream_workspace_bytes(wc->dev, nshots, seq);
}

struct OnlineWS {
  uint8_t *D, *E, *bnd, *sw, *zw, *sout;
  int32_t* tclr;
  void* dec;
  size_t total;
};

OnlineWS carve(const laim_online_plan* P, const KParams& kp, int32_t nshots, void* base) {
  const laim_code* b = P->base;
  const int32_t N = P->op.rounds_total, W = std::max(P->op.window, P->w_last);
  const size_t S = (size_t)nshots;
  const int32_t nv_max = std::max(P->win_last->n, P->win_full ? P->win_full->n : 0);
  size_t dec = 0;
  for (const laim_code* wc : {P->win_full, P->win_last}) {
    if (!wc) continue;
    bool res;
    ResidentShape sh;
    dec = std::max(dec, window_decode_bytes(wc, kp, nshots, &res, &sh));
  }
  char* p = (char*)base;
  OnlineWS w;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = p ? p + off : nullptr;
    off += al256(bytes);
    return q;
  };
  w.D = (uint8_t*)take(S * N * b->m);
  w.E = (uint8_t*)take(S * b->n);
  w.bnd = (uint8_t*)take(S * b->m);
  w.sw = (uint8_t*)take(S * W * b->m);
  w.zw = (uint8_t*)take(S * nv_max);
  w.sout = (uint8_t*)take(S * W * b->m);
  w.tclr = (int32_t*)take(S * 4);
  w.dec = take(dec);
  w.total = off;
  return w;
}

}  // namespace

extern "C" {

laim_status laim_online_plan_create(const laim_code* code, const laim_online_params* op,
                                    laim_online_plan** out) {
  if (!code || !op || !out) {
    set_error("laim_online_plan_create: bad arguments");
    return LAIM_EINVAL;
  }
  *out = nullptr;
  if (op->rounds_total < 1 || op->window < 1 || op->commit < 1 || op->commit > op->window ||
      op->p != op->p || op->p_meas != op->p_meas) {
    set_error("need rounds_total >= 1, 1 <= commit <= window and rates that are numbers");
    return LAIM_EINVAL;
  }
  laim_online_plan* P = new (std::nothrow) laim_online_plan();
  if (!P) {
    set_error("out of host memory");
    return LAIM_ENOMEM;
  }
  P->base = code;
  P->op = *op;
  int32_t k = 0;
  while ((int64_t)k * op->commit + op->window < op->rounds_total) ++k;
  P->nwin = k + 1;
  P->w_last = op->rounds_total - k * op->commit;
  if ((int64_t)std::max(op->window, P->w_last) * (code->n + code->m) > (int64_t)1 << 30) {
    delete P;
    set_error("the window code is too large");
    return LAIM_EUNSUP;
  }
  laim_status st = build_window(code, P->w_last, P->w_last - 1, &P->win_last);
  if (st == LAIM_OK && P->nwin > 1) st = build_window(code, op->window, op->window, &P->win_full);
  if (st != LAIM_OK) {
    laim_online_plan_destroy(P);
    return st;
  }
  *out = P;
  return LAIM_OK;
}

void laim_online_plan_destroy(laim_online_plan* plan) {
  if (!plan) return;
  laim_free_code(plan->win_full);
  laim_free_code(plan->win_last);
  delete plan;
}

size_t laim_online_workspace_bytes(const laim_online_plan* plan, const laim_decode_params* params,
                                   int32_t nshots) {
  if (!plan || !params || nshots < 0) return 0;
  KParams kp;
  if (resolve_params(params, &kp) != LAIM_OK) return 0;
  return carve(plan, kp, nshots, nullptr).total;
}

laim_status laim_decode_online(const laim_online_plan* plan, const laim_decode_params* params,
                               uint64_t shot0, int32_t nshots, const uint8_t* e_in,
                               const uint8_t* eps_in, void* workspace, size_t ws_bytes,
                               uint8_t* z_out, uint8_t* E_out, uint8_t* fail_out,
                               int32_t* cleared_out, laim_stream stream) {
  if (!plan || !params || nshots < 0 || (nshots > 0 && !z_out) || (!e_in) != (!eps_in)) {
    set_error("laim_decode_online: bad arguments");
    return LAIM_EINVAL;
  }
  KParams kp;
  laim_status st = resolve_params(params, &kp);
  if (st != LAIM_OK) return st;
  const laim_code* b = plan->base;
  if (fail_out && b->dev.kw > 64) {
    set_error("more than 2048 logicals are not supported");
    return LAIM_EUNSUP;
  }
  if (nshots == 0) return LAIM_OK;
  const OnlineWS need = carve(plan, kp, nshots, nullptr);
  if (!workspace || ws_bytes < need.total) {
    set_error("workspace of %zu bytes needed (got %zu)", need.total, ws_bytes);
    return LAIM_ENOMEM;
  }
  if (((uintptr_t)workspace) % 256) {
    set_error("workspace must be 256-byte aligned");
    return LAIM_EINVAL;
  }
  const OnlineWS w = carve(plan, kp, nshots, workspace);
  DeviceGuard g(b->device);
  hipStream_t s = (hipStream_t)stream;
  const int32_t N = plan->op.rounds_total, C = plan->op.commit, n = b->n, m = b->m;
  uint8_t* E = E_out ? E_out : w.E;
  const dim3 blk(256);
  // start: z = 0, no carried correction, no cleared window
  const int64_t zn = (int64_t)nshots * n, bn = (int64_t)nshots * m;
  hipLaunchKernelGGL(online_clear, dim3((unsigned)((std::max(zn, (int64_t)nshots) + 255) / 256)), blk, 0, s,
                     z_out, zn, cleared_out, cleared_out ? (int64_t)nshots : 0);
  hipLaunchKernelGGL(online_clear, dim3((unsigned)((bn + 255) / 256)), blk, 0, s, w.bnd, bn, nullptr, 0);
  const size_t lds = (size_t)2 * n + 2 * m;
  if (lds > 64 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(online_noise_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
  }
  hipLaunchKernelGGL(online_noise_kernel, dim3((unsigned)nshots), blk, lds, s, b->dev, N,
                     bernoulli_bound(plan->op.p), bernoulli_bound(plan->op.p_meas), kp.seed, shot0, e_in,
                     eps_in, w.D, E);
  hipError_t er = hipGetLastError();
  for (int32_t k = 0; k < plan->nwin && er == hipSuccess; ++k) {
    const bool last = k == plan->nwin - 1;
    const laim_code* wc = last ? plan->win_last : plan->win_full;
    const int32_t wr = last ? plan->w_last : plan->op.window;
    hipLaunchKernelGGL(online_window_syndrome, dim3((unsigned)((wr * m + 255) / 256), (unsigned)nshots), blk, 0,
                       s, m, N, k * C, wr, w.D, w.bnd, w.sw);
    bool res;
    ResidentShape sh;
    window_decode_bytes(wc, kp, nshots, &res, &sh);
    if (res)
      er = launch_resident(wc->dev, kp, sh, nullptr, shot0, nshots, w.dec, w.zw, w.sout, w.tclr, nullptr,
                           nullptr, nullptr, s, w.sw, k * kp.rounds);
    else
      er = launch_stream(wc->dev, kp, nullptr, shot0, nshots, w.dec, w.zw, w.sout, w.tclr, nullptr, s, w.sw,
                         k * kp.rounds);
    if (er != hipSuccess) break;
    const int32_t cr = last ? wr : C;
    hipLaunchKernelGGL(online_commit, dim3((unsigned)((std::max(n, m) + 255) / 256), (unsigned)nshots), blk, 0,
                       s, n, m, wr, wc->n, cr, last ? 1 : 0, w.zw, w.tclr, z_out, w.bnd, cleared_out);
    er = hipGetLastError();
  }
  if (er == hipSuccess && fail_out) er = launch_failure(b->dev, E, z_out, nshots, fail_out, s);
  return er == hipSuccess ? LAIM_OK : hip_fail(er, "online decode kernels");
}

}  // extern "C"
