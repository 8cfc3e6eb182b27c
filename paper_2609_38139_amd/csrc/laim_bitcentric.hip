// laim_bitcentric.hip -- the discrete bit-centric machine of the SM ("Setup
// and algorithm") on gfx950, for codes whose checks have degree 2 (the
// repetition code of the paper's bit-centric analysis).
//
// Iteration i, all updates from the state of iteration i - 1 (Jacobi):
//   check-to-bit  m_{c->v} = (-1)^{s_c} m_{w->c}, w the other bit of c
//                 (BP-LLR2 with d_c = 2: the tanh product of one input);
//   bit-to-check  m_{v->c} = pi_v + sum over c' in N(v)\c of m_{c'->v};
//   beliefs       L_v = pi_v + sum over c in N(v) of m_{c->v} (ascending c);
//   feedback      f_v = [L_v > 0]; s_c ^= XOR over N(c) of f;
//   LLR switch    pi_v, the new m_{v->c} and m_{c->v} of flipped bits negated.
// Messages start at 0 and pi_v at log(q / (1 - q)); all in double precision,
// where every operation above is exact up to the additions' rounding.
//
// One block per shot; thread t owns bits t + k nt and writes the new
// messages on their edges, with its edge indices and its checks' bits kept
// in registers. LDS: old and new messages by edge (check-major edge order,
// double-buffered), pi, f and s.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device_math.h"
#include "laim_internal.h"

namespace laim {

// Bits (and checks) per thread: the thread's edge indices and its checks'
// bits stay in registers for all iterations.
constexpr int kBcMaxBits = 3;
constexpr int kBcMaxDv = 4;
// Bits per lane of the chain form: chains of up to 16 x 64 bits.
constexpr int kBcChainMaxK = 16;

__global__ void __launch_bounds__(1024) bitcentric_kernel(DevCode c, double pi0, const uint8_t* e0,
                                                          int32_t iters, uint8_t* z_out,
                                                          int32_t* iclr_out, double* L_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int32_t t = tid_x();
  const int32_t nt = bdim_x();
  const int64_t shot = bid_x();
  const int32_t E = c.E;
  // messages by edge (check-major: edge 2 ch + j), two buffers each
  double* cv[2] = {reinterpret_cast<double*>(smem), reinterpret_cast<double*>(smem) + E};
  double* vc[2] = {cv[1] + E, cv[1] + 2 * E};
  double* piv = vc[1] + E;                             // [n]
  uint8_t* f = reinterpret_cast<uint8_t*>(piv + c.n);  // [n]
  uint8_t* s = f + c.n;                                // [m]
  __shared__ int32_t any_s;

  // per-thread tables: for bit v = t + k nt its degree and the LDS index
  // 2 ch + j of each of its edges (ascending check); for check t + k nt its
  // two bits
  int32_t bdv[kBcMaxBits];
  int32_t bix[kBcMaxBits][kBcMaxDv];
  int32_t cb0[kBcMaxBits], cb1[kBcMaxBits];
#pragma unroll
  for (int k = 0; k < kBcMaxBits; ++k) {
    const int32_t v = t + k * nt;
    bdv[k] = (v < c.n) ? c.var_deg[v] : 0;
#pragma unroll
    for (int q = 0; q < kBcMaxDv; ++q) {
      int32_t ix = 0;
      if (q < bdv[k]) {
        const int32_t e = c.var_edge[(int64_t)v * c.dvmax + q];
        ix = edge_check(e) * 2 + edge_slot(e);
      }
      bix[k][q] = ix;
    }
    const int32_t ch = t + k * nt;
    cb0[k] = (ch < c.m) ? c.chk_var[(int64_t)ch * c.dcmax] : 0;
    cb1[k] = (ch < c.m) ? c.chk_var[(int64_t)ch * c.dcmax + 1] : 0;
  }

  const uint8_t* e0row = e0 + shot * c.n;
  for (int32_t e = t; e < E; e += nt) {
    cv[0][e] = 0.0;
    vc[0][e] = 0.0;
  }
  for (int32_t v = t; v < c.n; v += nt) piv[v] = pi0;
#pragma unroll
  for (int k = 0; k < kBcMaxBits; ++k) {
    const int32_t ch = t + k * nt;
    if (ch < c.m) s[ch] = (uint8_t)((e0row[cb0[k]] ^ e0row[cb1[k]]) & 1u);
  }
  if (t == 0) any_s = 0;
  __syncthreads();
  for (int32_t ch = t; ch < c.m; ch += nt)
    if (s[ch]) any_s = 1;
  __syncthreads();
  int32_t iclr = any_s ? -1 : 0;
  uint32_t zbits = 0;  // correction of this thread's bits t + k nt
  int cur = 0;

  for (int32_t it = 1; it <= iters; ++it) {
    const double* mcv = cv[cur];
    const double* mvc = vc[cur];
    double* ncv = cv[cur ^ 1];
    double* nvc = vc[cur ^ 1];
    // new messages and beliefs of the owned bits from the old state; the LLR
    // switch of a flipped bit negates its prior and its new messages
#pragma unroll
    for (int k = 0; k < kBcMaxBits; ++k) {
      const int32_t v = t + k * nt;
      if (v >= c.n) continue;
      const int32_t dv = bdv[k];
      const double pv = piv[v];
      double m_in[kBcMaxDv];
#pragma unroll
      for (int q = 0; q < kBcMaxDv; ++q) m_in[q] = (q < dv) ? mcv[bix[k][q]] : 0.0;
      double L = pv;
#pragma unroll
      for (int q = 0; q < kBcMaxDv; ++q)
        if (q < dv) L = L + m_in[q];
      const bool flip = L > 0.0;
      if (L_out && it == iters) L_out[shot * c.n + v] = L;
#pragma unroll
      for (int q = 0; q < kBcMaxDv; ++q) {
        if (q >= dv) continue;
        const int32_t ix = bix[k][q];
        const double other = mvc[ix ^ 1];          // the check's other edge
        const double mc = s[ix >> 1] ? -other : other;
        double acc = pv;
#pragma unroll
        for (int q2 = 0; q2 < kBcMaxDv; ++q2)
          if (q2 < dv && q2 != q) acc = acc + m_in[q2];
        ncv[ix] = flip ? -mc : mc;
        nvc[ix] = flip ? -acc : acc;
      }
      f[v] = flip ? 1 : 0;
      if (flip) {
        piv[v] = -pv;
        zbits ^= 1u << k;
      }
    }
    if (t == 0) any_s = 0;
    __syncthreads();
    // syndrome update s_c ^= XOR over N(c) of f
#pragma unroll
    for (int k = 0; k < kBcMaxBits; ++k) {
      const int32_t ch = t + k * nt;
      if (ch >= c.m) continue;
      const uint32_t x = (uint32_t)(s[ch] ^ f[cb0[k]] ^ f[cb1[k]]) & 1u;
      s[ch] = (uint8_t)x;
      if (x) any_s = 1;
    }
    __syncthreads();
    if (!any_s && iclr < 0) iclr = it;
    cur ^= 1;
  }
#pragma unroll
  for (int k = 0; k < kBcMaxBits; ++k) {
    const int32_t v = t + k * nt;
    if (v < c.n) z_out[shot * c.n + v] = (uint8_t)((zbits >> k) & 1u);
  }
  if (t == 0) iclr_out[shot] = iclr;
}

bool bitcentric_shape(const DevCode& c, int device, int32_t* nt, size_t* lds) {
  if (c.dcmax != 2 || c.dvmax > 4) {
    set_error("the bit-centric machine needs checks of degree 2 and qubit degree <= 4");
    return false;
  }
  *nt = (c.n < 1024) ? ((c.n + 63) / 64) * 64 : 1024;
  if ((int64_t)c.n > (int64_t)kBcMaxBits * *nt || (int64_t)c.m > (int64_t)kBcMaxBits * *nt) {
    set_error("the bit-centric machine supports at most %d bits and checks", kBcMaxBits * 1024);
    return false;
  }
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      lds_max <= 0)
    lds_max = 64 * 1024;
  *lds = ((size_t)4 * c.E + c.n) * 8 + (size_t)c.n + c.m;
  *lds = (*lds + 15) / 16 * 16;
  if (*lds > (size_t)lds_max) {
    set_error("the bit-centric machine needs %zu bytes of LDS (device limit %d)", *lds, lds_max);
    return false;
  }
  return true;
}

hipError_t launch_bitcentric(const DevCode& c, double q, const uint8_t* e0, int32_t nshots,
                             int32_t iters, int32_t nt, size_t lds, uint8_t* z, int32_t* iclr,
                             double* L, hipStream_t st) {
  if (nshots <= 0) return hipSuccess;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(bitcentric_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bitcentric_kernel, dim3((unsigned)nshots), dim3(nt), lds, st, c,
                     log(q / (1.0 - q)), e0, iters, z, iclr, L);
  return hipGetLastError();
}

// ---- chain form
// On a chain (checks (v, v + 1), and (d - 1, 0) when periodic) the machine can
// be carried in the frame of its current error x = e0 ^ z. With
// M_{c->v} = (-1)^{x_v} m_{c->v} and Y_{v->c} = (-1)^{x_v} m_{v->c}, the
// syndrome sign of a check of degree 2 (s_c = x_v ^ x_w) and the LLR switch
// cancel, and one iteration is a shift and an add:
//   Y^i_{v->c} = P_v + M^{i-1}_{c'->v},  P_v = (-1)^{e0_v} pi0, c' the other check;
//   M^i_{c->v} = Y^{i-1}_{w->c},         w the other bit of c;
//   L^i_v = (-1)^{x^{i-1}_v} (P_v + sum over c of M^{i-1}_{c->v}) (ascending c),
// and x^i_v is 1 where the bracket is positive, 0 where it is negative, and
// x^{i-1}_v where it is zero. Negation commutes with round-to-nearest, so the
// doubles are the machine's up to the sign of a zero, which no decision reads
// (a zero belief is written as +0, the sign the machine gives it). The
// syndrome is zero exactly when x is constant along the chain.
//
// Messages of iteration i come from iteration i - 2 only, so the even and odd
// iterations are two independent recursions; a neighbour's message is
// exchanged across lanes one iteration before it is needed.
//
// A wavefront holds S shots, each on a segment of nl lanes. The first nl - r
// lanes of a segment hold K bits and the last r (r = nl K - d <= nl) hold
// K - 1, in order along the chain, so a lane's last bit is in slot K - 1 or
// K - 2 whatever d is. Lanes outside the segments, and segments past the
// last shot, are idle (prior 0, messages 0, their own neighbours); an open
// chain's ends take their missing message from lane 63, which is idle. x is
// held as a 64-lane mask per slot, and so are the shots not yet cleared.
// Up to 8 bits per lane the launch bounds hold the kernel to 128 VGPRs,
// four wavefronts per SIMD.
__device__ inline double bperm_f64(int32_t addr, double x) {
  const int32_t lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
  const int32_t hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

template <int K, bool PERIODIC>
__global__ void __launch_bounds__(256, K <= 8 ? 4 : 1) bitchain_kernel(int32_t d, int32_t nl, int32_t S, double pi0,
                                                       const uint8_t* __restrict__ e0, int32_t nshots,
                                                       int32_t iters, uint8_t* __restrict__ z_out,
                                                       int32_t* __restrict__ iclr_out,
                                                       double* __restrict__ L_out) {
  const int32_t lane = tid_x() & 63;
  const int64_t shot0 = ((int64_t)bid_x() * (bdim_x() >> 6) + (tid_x() >> 6)) * S;
  if (shot0 >= nshots) return;  // whole wavefronts
  const int32_t seg = lane / nl;
  const int32_t lam = lane - seg * nl;  // lane within the segment
  const int64_t shot = shot0 + seg;
  const bool act = seg < S && shot < nshots;
  const int32_t full = nl - (nl * K - d);  // lanes with K bits
  const bool part = K > 1 && lam >= full;  // K - 1 bits: slot K - 1 unused
  const int32_t b0 = lam * K - (lam > full ? lam - full : 0);  // the lane's first bit
  const int32_t nb = act ? (part ? K - 1 : K) : 0;
  const uint8_t* er = e0 + (act ? shot : 0) * d;

  double P[K];
  uint64_t X[K], V[K];
  uint32_t ebits = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool ok = k < nb;
    const uint32_t e = ok ? (uint32_t)(er[b0 + k] & 1u) : 0u;
    ebits |= e << k;
    P[k] = ok ? (e ? -pi0 : pi0) : 0.0;
    X[k] = __builtin_amdgcn_ballot_w64(e != 0);
    V[k] = __builtin_amdgcn_ballot_w64(ok);
  }
  const int32_t srcl = !act ? lane : lam > 0 ? lane - 1 : PERIODIC ? lane + nl - 1 : 63;
  const int32_t srcr = !act ? lane : lam < nl - 1 ? lane + 1 : PERIODIC ? lane - nl + 1 : 63;
  const int32_t al = srcl * 4, ar = srcr * 4;
  // bit 0 of a periodic chain lists its right check (0, 1) before the wrap
  // check, so it sums its right message first
  const bool first_swapped = PERIODIC && act && lam == 0;
  const uint64_t seg0 = (nl >= 64) ? ~0ull : ((1ull << nl) - 1ull);

  // [parity][slot]: Y towards the right and the left check; r*: the
  // neighbours' boundary Y of the same parity
  double YR[2][K], YL[2][K], rR[2], rL[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int k = 0; k < K; ++k) YR[p][k] = YL[p][k] = 0.0;
    rR[p] = rL[p] = 0.0;
  }
  // The syndrome of a shot is zero when no two neighbouring bits of its
  // segment differ in x (a ring's wrap check then agrees too). walls(): the
  // lanes holding the left bit of such a pair, the wrap excepted.
  const uint64_t v_full = __builtin_amdgcn_ballot_w64(act && !part);
  const uint64_t v_part = __builtin_amdgcn_ballot_w64(act && part);
  const uint64_t v_inner = __builtin_amdgcn_ballot_w64(act && lam < nl - 1);
  auto walls = [&]() {
    uint64_t w = 0;
#pragma unroll
    for (int k = 0; k + 1 < K; ++k) w |= (X[k] ^ X[k + 1]) & V[k + 1];
    const uint64_t lastx = (X[K - 1] & v_full) | (X[K > 1 ? K - 2 : 0] & v_part);
    return w | ((lastx ^ (X[0] >> 1)) & v_inner);
  };
  // this lane's segment, as a lane mask
  const uint64_t myseg = act ? (seg0 << (seg * nl)) : 0ull;
  int32_t iclr = ((walls() & myseg) == 0) ? 0 : -1;
  // lanes of the shots whose syndrome has not been zero yet
  uint64_t pend = __builtin_amdgcn_ballot_w64(act && iclr < 0);

  // One iteration of one parity, in place: Y^i from Y^{i-2} (the lane's own
  // and the neighbours' boundary ones), the beliefs, new x.
  auto step = [&](double (&yr)[K], double (&yl)[K], double& rr, double& rl, int32_t it) {
    const double ml0 = rr;
    // towards the right check: from the left neighbour's, highest slot first
    // so each old value is read before it is replaced
#pragma unroll
    for (int k = K - 1; k >= 0; --k) yr[k] = P[k] + (k ? yr[k - 1] : ml0);
    // towards the left check: from the right neighbour's, lowest slot first
    double Lg[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double mr = (k < K - 1) ? yl[k + 1] : rl;
      if (k == K - 2) mr = part ? rl : mr;  // a K - 1 bit lane's last bit
      yl[k] = P[k] + mr;
      Lg[k] = yr[k] + mr;
    }
    if (PERIODIC) {
      const double alt = yl[0] + ml0;
      Lg[0] = first_swapped ? alt : Lg[0];
    }
    const double sr = (K > 1 && part) ? yr[K > 1 ? K - 2 : 0] : yr[K - 1];
    rr = bperm_f64(al, sr);
    rl = bperm_f64(ar, yl[0]);
    if (L_out && it == iters) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k < nb) {
          const double Lo = ((X[k] >> lane) & 1u) ? -Lg[k] : Lg[k];
          L_out[shot * d + b0 + k] = Lo + 0.0;
        }
      }
    }
    // x <- 1 where the belief bracket is positive, 0 where negative (lanes
    // outside a chain may change; every use masks them)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint64_t gt = __builtin_amdgcn_ballot_w64(Lg[k] > 0.0);
      const uint64_t lt = __builtin_amdgcn_ballot_w64(Lg[k] < 0.0);
      X[k] = gt | (X[k] & ~lt);
    }
    if (pend) {
      const uint64_t w = walls();
      const uint64_t clr = __builtin_amdgcn_ballot_w64((w & myseg) == 0);
      const uint64_t first = clr & pend;  // shots whose syndrome is zero for the first time
      if (first) {
        if ((first >> lane) & 1ull) iclr = it;
        pend &= ~clr;
      }
    }
  };

  // four iterations per trip, so that the two parities' neighbour values
  // stay in their registers from one trip to the next
  int32_t it = 1;
  for (; it + 3 <= iters; it += 4) {
    step(YR[1], YL[1], rR[1], rL[1], it);
    step(YR[0], YL[0], rR[0], rL[0], it + 1);
    step(YR[1], YL[1], rR[1], rL[1], it + 2);
    step(YR[0], YL[0], rR[0], rL[0], it + 3);
  }
  for (; it <= iters; it += 2) {
    step(YR[1], YL[1], rR[1], rL[1], it);
    if (it + 1 <= iters) step(YR[0], YL[0], rR[0], rL[0], it + 1);
  }

#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k < nb)
      z_out[shot * d + b0 + k] = (uint8_t)(((uint32_t)(X[k] >> lane) & 1u) ^ ((ebits >> k) & 1u));
  }
  if (act && lam == 0) iclr_out[shot] = iclr;
}

bool bitchain_shape(int32_t d, bool periodic, int32_t* K, int32_t* nl, int32_t* S) {
  // an open chain keeps lane 63 idle: its ends read their missing message there
  const int32_t cap = periodic ? 64 : 63;
  if (d < (periodic ? 3 : 2)) return false;
  // Bits per lane: the fewest VALU instructions per shot and iteration --
  // about 5 per slot and 7 per lane (the wrap bit's sum order and the
  // selects of a lane with K - 1 bits), shared by the S shots of a wavefront
  // -- weighed by occupancy: the kernel takes about 13 K + 25 VGPRs (at
  // most 128 up to K = 8, whose launch bounds ask for four wavefronts per
  // SIMD), and below four wavefronts per SIMD the measured time per
  // instruction grows (by about 10% at three and 40% at two). One bit per
  // lane is never the cheapest.
  int32_t best = 0;
  double best_cost = 0.0;
  for (int32_t k = 2; k <= kBcChainMaxK; ++k) {
    const int32_t n_l = (d + k - 1) / k;
    // lanes hold K or K - 1 bits: at most one unused slot per lane
    if (n_l > cap || n_l * k - d > n_l) continue;
    const int32_t s = cap / n_l;
    const int32_t vgpr = k <= 8 ? 128 : (13 * k + 25 + 7) / 8 * 8;
    const int32_t waves = std::min(8, 512 / vgpr);
    const double slow = waves >= 4 ? 1.0 : waves == 3 ? 1.1 : waves == 2 ? 1.4 : 2.0;
    const double cost = (5.0 * k + 7.0) / s * slow;
    if (!best || cost < best_cost) {
      best = k;
      best_cost = cost;
    }
  }
  if (!best) return false;
  *K = best;
  *nl = (d + best - 1) / best;
  *S = cap / *nl;
  return true;
}

#define LAIM_BCHAIN_CASE(KK)                                                                  \
  case KK:                                                                                     \
    if (periodic)                                                                              \
      hipLaunchKernelGGL((bitchain_kernel<KK, true>), grid, dim3(256), 0, st, d, nl, S, pi0,    \
                         e0, nshots, iters, z, iclr, L);                                       \
    else                                                                                       \
      hipLaunchKernelGGL((bitchain_kernel<KK, false>), grid, dim3(256), 0, st, d, nl, S, pi0,   \
                         e0, nshots, iters, z, iclr, L);                                       \
    break;

hipError_t launch_bitchain(int32_t d, bool periodic, int32_t K, int32_t nl, int32_t S, double q,
                           const uint8_t* e0, int32_t nshots, int32_t iters, uint8_t* z,
                           int32_t* iclr, double* L, hipStream_t st) {
  if (nshots <= 0) return hipSuccess;
  if (S < 1 || nl < 1 || nl * S > 64) return hipErrorInvalidValue;
  const double pi0 = log(q / (1.0 - q));
  // four wavefronts of S shots per workgroup
  const int64_t per_block = 4 * (int64_t)S;
  const dim3 grid((unsigned)((nshots + per_block - 1) / per_block));
  switch (K) {
    LAIM_BCHAIN_CASE(2)
    LAIM_BCHAIN_CASE(3)
    LAIM_BCHAIN_CASE(4)
    LAIM_BCHAIN_CASE(5)
    LAIM_BCHAIN_CASE(6)
    LAIM_BCHAIN_CASE(7)
    LAIM_BCHAIN_CASE(8)
    LAIM_BCHAIN_CASE(9)
    LAIM_BCHAIN_CASE(10)
    LAIM_BCHAIN_CASE(11)
    LAIM_BCHAIN_CASE(12)
    LAIM_BCHAIN_CASE(13)
    LAIM_BCHAIN_CASE(14)
    LAIM_BCHAIN_CASE(15)
    LAIM_BCHAIN_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
#undef LAIM_BCHAIN_CASE

}  // namespace laim
