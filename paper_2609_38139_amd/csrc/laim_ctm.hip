// laim_ctm.hip -- the continuous-time machine of Algorithm 1 on gfx950.
//
// BP relaxes by tau dm/dt = F_BP(m; S) - m, integrated with Euler steps of
// dt (SM "Numerical details"), in the Jacobi form: one step computes both
// message directions from the state before it,
//   m_{c->v} <- clamp(m_{c->v} + lambda (F_c - m_{c->v})),  F_c by (BP-LLR2),
//   m_{v->c} <- clamp(m_{v->c} + lambda (F_v - m_{v->c})),  F_v by (BP-LLR1),
// lambda = dt / tau. Unit-rate Poisson clocks ring at the checks; only active
// checks can act, so the next ring is a waiting time ~ Exp(|S|) and a
// uniformly chosen active check. Event j draws Philox(seed; shot, j, 2):
// w0 gives its waiting time -ln((w0 + 1) 2^-32) / |S| (FP64), w1 the ringing
// check (active check number floor(w1 |S| / 2^32), ascending), w2 the
// LocalMove tie. An event at time T acts on the BP state of the last Euler
// step at or before T. A ringing check with Evidence flips its LocalMove
// qubit: z_v ^= 1, s ^= H e_v. t_clr is the time of the clearing event.
//
// One block runs one shot at a time (shots come from a queue). Thread t owns
// checks t + k nt (k < CPT); it keeps the m_{v->c} and m_{c->v} of its
// checks' edges in registers and publishes m_{c->v} in LDS, in tiles of 64
// checks with a 65-word slot stride, for the partner gathers. Events are
// handled by the first wavefront between Euler steps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.h"
#include "laim_internal.h"

namespace laim {

namespace {

constexpr int kCtmStride = 65;
constexpr int kCtmWords = 18;  // scratch words after the messages
// scratch word indices
// (the words start 8-byte aligned; the FP64 ones sit at even indices)
constexpr int kCwZero = 0, kCwLpar = 1 /* 4 words */, kCwNs = 5, kCwMoved = 6, kCwJ = 7,
              kCwTev = 8 /* 2 words */, kCwEvents = 10, kCwMoves = 11, kCwClear = 12 /* 2 words */,
              kCwChg = 15, kCwSkipped = 16, kCwQueue = 17;
constexpr int kCtmFusedWords = 4;

template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};

template <int DC>
__device__ __forceinline__ int32_t ctm_word(int32_t c, int32_t j) {
  return ((c >> 6) * DC + j) * kCtmStride + (c & 63);
}

// Words of messages for mpad checks, rounded up to even so that the scratch
// words after them are 8-byte aligned; the first scratch word is the slot
// padded partners point at.
__host__ __device__ __forceinline__ int32_t ctm_zslot(int32_t dc, int32_t mpad) {
  return ((mpad >> 6) * dc * kCtmStride + 1) & ~1;
}

__global__ void ctm_zero_counter(uint32_t* p) {
  if (tid_x() == 0) p[0] = 0u;
}

// ln(u) for 0 < u <= 1 in double: u = f 2^e with f in [sqrt(1/2), sqrt(2)),
// ln f = 2 atanh(s) = 2 s (1 + s^2/3 + ... + s^24/25), s = (f - 1)/(f + 1).
__device__ double ctm_ln_unit(double u) {
  const uint64_t b = (uint64_t)__double_as_longlong(u);
  int32_t e = (int32_t)((b >> 52) & 0x7ffu) - 1023;
  double f = __longlong_as_double((long long)((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
  if (f > 1.4142135623730951) {
    f = f * 0.5;
    e = e + 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 25.0;
#pragma unroll
  for (int k = 11; k >= 0; --k) p = p * s2 + 1.0 / (double)(2 * k + 1);
  return (double)e * 0.6931471805599453 + 2.0 * s * p;
}

__device__ __forceinline__ Philox4 ctm_words(const CtmParamsDev& P, uint64_t shot, uint32_t j) {
  return philox4x32_10((uint32_t)shot, (uint32_t)(shot >> 32), j, 2u, (uint32_t)P.seed,
                       (uint32_t)(P.seed >> 32));
}

// The Euler step at which an event at time T acts: the least k >= 0 with
// T <= k dt (k dt evaluated in double as in the step loop), or
// max_steps + 1 if it would come after the last step.
__device__ int32_t ctm_step_of(double T, double dt, int32_t max_steps) {
  if (!(T <= (double)max_steps * dt)) return max_steps + 1;
  double q = ceil(T / dt);
  int32_t k = (q < 0.0) ? 0 : (int32_t)q;
  while (k > 0 && (double)(k - 1) * dt >= T) --k;
  while ((double)k * dt < T) ++k;
  return k;
}

__device__ __forceinline__ double ctm_wait(uint32_t w0, int32_t nS) {
  const double u = ((double)w0 + 1.0) * (1.0 / 4294967296.0);
  return -ctm_ln_unit(u) / (double)nS;
}

// Check rule (BP-LLR2) of one check from its m_{v->c} (x; slots >= deg hold
// +inf), clamped. Min-sum: (-1)^{s_c + d_c} alpha min |other| prod sg(other).
template <int DC, int BP, bool REG>
__device__ __forceinline__ void ctm_check_rule(const CtmParamsDev& P, const float* x, int32_t deg,
                                               uint32_t sigma_neg, float* out) {
  const float C = P.clamp;
  if (BP == 0) {
    uint32_t par = sigma_neg << 31;
#pragma unroll
    for (int j = 0; j + 1 < DC; j += 2) par = xor3(par, __float_as_uint(x[j]), __float_as_uint(x[j + 1]));
    if (DC & 1) par ^= __float_as_uint(x[DC - 1]);
    const float alpha_s = __uint_as_float(__float_as_uint(P.alpha) ^ (par & 0x80000000u));
    float ex[DC];
    if (DC == 2) {
      ex[0] = fabsf(x[1]);
      ex[1] = fabsf(x[0]);
    } else if (DC == 4) {
      ex[0] = min3_abs(x[1], x[2], x[3]);
      ex[1] = min3_abs(x[0], x[2], x[3]);
      ex[2] = min3_abs(x[0], x[1], x[3]);
      ex[3] = min3_abs(x[0], x[1], x[2]);
    } else {
      float pre[DC], suf[DC];
      pre[1] = fabsf(x[0]);
#pragma unroll
      for (int j = 2; j < DC; ++j) pre[j] = fminf(pre[j - 1], fabsf(x[j - 1]));
      suf[DC - 2] = fabsf(x[DC - 1]);
#pragma unroll
      for (int j = DC - 3; j >= 0; --j) suf[j] = fminf(suf[j + 1], fabsf(x[j + 1]));
      ex[0] = suf[0];
      ex[DC - 1] = pre[DC - 1];
#pragma unroll
      for (int j = 1; j < DC - 1; ++j) ex[j] = fminf(pre[j], suf[j]);
    }
#pragma unroll
    for (int j = 0; j < DC; ++j) {
      // The regular-code kernels run with alpha <= 1 only (others use the
      // padded variant): every input is clamped, so alpha min |m| <= C and
      // the output clamp cannot bind. The padded variant clamps (a
      // degree-1 check's minimum is empty, and alpha may exceed 1).
      float v = alpha_s * ex[j];
      if (!REG) v = __builtin_amdgcn_fmed3f(v, -C, C);
      out[j] = __uint_as_float(__float_as_uint(v) ^ (__float_as_uint(x[j]) & 0x80000000u));
    }
  } else {
    float acc[DC];
    boxplus_others<DC, REG>(x, deg, acc);
#pragma unroll
    for (int j = 0; j < DC; ++j) out[j] = __builtin_amdgcn_fmed3f(sigma_neg ? -acc[j] : acc[j], -C, C);
  }
}

// Every event due by time tk, in order, handled by the first wavefront of
// the block (nl = min(64, block size) lanes). Every lane keeps the same
// event state (|S|, event counter, pending time, counts; identical
// arithmetic in each). The search for the ringing check is spread over the
// lanes: lane l counts the active checks of syndrome words l, l + nl, ...,
// and a prefix sum over the lanes finds the word holding it. Lane 0 applies
// the flip to the LDS bitmaps; the wavefront executes in order, so the next
// event's search sees it.
// With qubits of degree 2 (regular codes) a qubit's two messages are the
// check's own and the one named by the partner table, and a flip toggles
// those two checks: one table read per qubit instead of the qubit's degree
// and edge list read one after the other, on the path every other wavefront
// of the block waits for.
template <int DC, int DV, bool REG>
__device__ void ctm_events(const DevCode& c, const CtmParamsDev& P, uint64_t shot, double tk,
                           const float* msg, int32_t* gw, uint32_t* zw, uint32_t* sw, int32_t nl) {
  constexpr bool PAIR = REG && DV == 2;
  const int32_t lane = tid_x();
  int32_t nS = gw[kCwNs];
  uint32_t j = (uint32_t)gw[kCwJ];
  int32_t events = gw[kCwEvents], moves = gw[kCwMoves];
  double Tev = *reinterpret_cast<const double*>(gw + kCwTev);
  const int32_t mw = (c.m + 31) >> 5;
  int32_t moved = 0;
  while (nS > 0 && Tev <= tk) {
    const Philox4 w = ctm_words(P, shot, j);
    uint32_t idx = (uint32_t)(((uint64_t)w.w1 * (uint64_t)nS) >> 32);
    // the idx-th active check in ascending order
    int32_t ch = -1;
    for (int32_t base = 0; base < mw && ch < 0; base += nl) {
      const int32_t q = base + lane;
      const uint32_t word = (q < mw) ? sw[q] : 0u;
      const uint32_t pc = (uint32_t)__popc(word);
      uint32_t incl = pc;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
      }
      const uint32_t total = __shfl(incl, nl - 1);
      if (idx >= total) {
        idx -= total;
        continue;
      }
      const bool mine = idx >= incl - pc && idx < incl;
      const int32_t src = (int32_t)__builtin_ctzll(__ballot(mine));
      int32_t bpos = 0;
      if (mine) {
        uint32_t wd = word;
        for (uint32_t r = idx - (incl - pc); r > 0; --r) wd &= wd - 1u;
        bpos = __builtin_ctz(wd);
      }
      ch = (base + src) * 32 + __shfl(bpos, src);
    }
    int32_t chosen = -1, chosen_c2 = -1;
    const int32_t d = (ch >= 0) ? (REG ? DC : c.chk_deg[ch]) : 0;
    if (d > 0) {
      // the beliefs of the check's qubits (every lane the same), their two
      // messages added to pi in ascending check order as everywhere
      const int32_t* nb = c.chk_var + (int64_t)ch * c.dcmax;
      float Lv[DC];
      int32_t c2v[DC];
      float Lmax = 0.0f;
#pragma unroll
      for (int jj = 0; jj < DC; ++jj) {
        if (jj >= d) continue;
        float acc = P.pi;
        if (PAIR) {
          const int32_t pe = c.partner[(int64_t)ch * DC + jj];
          const int32_t c2 = edge_check(pe);
          const float own = msg[ctm_word<DC>(ch, jj)];
          const float oth = msg[ctm_word<DC>(c2, edge_slot(pe))];
          acc = c2 < ch ? (acc + oth) + own : (acc + own) + oth;
          c2v[jj] = c2;
        } else {
          const int32_t v = nb[jj];
          const int32_t dv = c.var_deg[v];
          for (int32_t q = 0; q < dv; ++q) {
            const int32_t e = c.var_edge[(int64_t)v * c.dvmax + q];
            acc = acc + msg[ctm_word<DC>(edge_check(e), edge_slot(e))];
          }
        }
        acc = clampf(acc, P.clamp);
        Lv[jj] = acc;
        if (jj == 0 || acc > Lmax) Lmax = acc;
      }
      if (!P.evidence || Lmax >= c.thr[d]) {
        uint32_t ntie = 0;
#pragma unroll
        for (int jj = 0; jj < DC; ++jj)
          if (jj < d && Lv[jj] == Lmax) ++ntie;
        uint32_t pick = (uint32_t)(((uint64_t)w.w2 * (uint64_t)ntie) >> 32);
#pragma unroll
        for (int jj = 0; jj < DC; ++jj) {
          if (jj < d && Lv[jj] == Lmax && chosen < 0) {
            if (pick == 0) {
              chosen = nb[jj];
              if (PAIR) chosen_c2 = c2v[jj];
            } else {
              --pick;
            }
          }
        }
      }
    }
    if (chosen >= 0) {
      int32_t nS_new = nS;
      if (lane == 0) {
        zw[chosen >> 5] ^= 1u << (chosen & 31);
        auto toggle = [&](int32_t c2) {
          const uint32_t bit = 1u << (c2 & 31);
          const uint32_t nw2 = sw[c2 >> 5] ^ bit;
          sw[c2 >> 5] = nw2;
          nS_new += (nw2 & bit) ? 1 : -1;
        };
        if (PAIR) {  // the qubit's two checks: this one and its partner
          toggle(ch);
          toggle(chosen_c2);
        } else {
          const int32_t dv = c.var_deg[chosen];
          for (int32_t q = 0; q < dv; ++q) toggle(edge_check(c.var_edge[(int64_t)chosen * c.dvmax + q]));
        }
      }
      __builtin_amdgcn_wave_barrier();
      nS = __shfl(nS_new, 0);
      ++moves;
      moved = 1;
    }
    ++events;
    ++j;
    if (nS == 0) {
      if (lane == 0) *reinterpret_cast<double*>(gw + kCwClear) = Tev;
      break;
    }
    Tev = Tev + ctm_wait(ctm_words(P, shot, j).w0, nS);
  }
  if (lane == 0) {
    gw[kCwNs] = nS;
    gw[kCwJ] = (int32_t)j;
    gw[kCwEvents] = events;
    gw[kCwMoves] = moves;
    gw[kCwMoved] = moved;
    *reinterpret_cast<double*>(gw + kCwTev) = Tev;
  }
}

}  // namespace

// SKIP: the kernel skips steps at a fixed point (P.skip); the instance
// without it carries none of that bookkeeping.
template <int DC, int DV, int CPT, int BP, bool REG, bool SKIP>
__global__ void __launch_bounds__(1024) ctm_kernel(DevCode c, CtmParamsDev P, CtmArgs a) {
  // min-sum on qubits of degree 2 (exact variants, run only when
  // ctm_reg_dv2_ok holds): no clamp can bind
  constexpr bool kNoClamp = (BP == 0 && REG && DV == 2);
  extern __shared__ __align__(16) unsigned char smem[];
  const int32_t t = tid_x();
  const int32_t nt = a.nt;
  float* msg = reinterpret_cast<float*>(smem);
  const int32_t zslot = ctm_zslot(DC, a.mpad);
  int32_t* gw = reinterpret_cast<int32_t*>(msg + zslot);
  const int32_t nw = (c.n + 31) >> 5;
  const int32_t mw = (c.m + 31) >> 5;
  uint32_t* zw = reinterpret_cast<uint32_t*>(gw + kCtmWords);
  uint32_t* sw = zw + nw;
  const float C = P.clamp;
  // lambda and pi are held in vector registers: the step uses them as
  // operands of every update, and scalar registers run short in the
  // skipping instance (the compiler would otherwise spill them to lanes
  // of a vector register and read them back in every step)
  float lam = P.lam;
  float piv = P.pi;
  asm volatile("" : "+v"(lam), "+v"(piv));

  // ---- per-thread graph tables (for the whole launch). Checks t + k nt
  // from m on pad the last tile: their LDS slots exist (mpad >= nt CPT) and
  // they are stepped like the others -- inputs from the zero word, syndrome
  // 0 -- so that the step needs no per-check condition; nothing reads them.
  int32_t cidx[CPT];
  int32_t deg[CPT];
  int32_t pidx[CPT][DC][DV > 1 ? DV - 1 : 1];
  uint32_t vmask = 0u;  // bit k: check k of this thread is one of the code's checks
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int32_t ch = t + k * nt;
    const bool valid = ch < c.m;
    cidx[k] = ch;
    vmask |= (valid ? 1u : 0u) << k;
    deg[k] = (valid && !REG) ? c.chk_deg[ch] : DC;
#pragma unroll
    for (int j = 0; j < DC; ++j) {
#pragma unroll
      for (int p = 0; p < DV - 1; ++p) {
        int32_t e = -1;
        if (valid && j < c.dcmax && p < c.dvmax - 1)
          e = c.partner[((int64_t)ch * c.dcmax + j) * (c.dvmax - 1) + p];
        pidx[k][j][p] = (e >= 0) ? ctm_word<DC>(edge_check(e), edge_slot(e)) : zslot;
      }
    }
  }

  for (;;) {
    __syncthreads();
    if (t == 0) gw[kCwQueue] = (int32_t)atomicAdd(a.counter, 1u);
    __syncthreads();
    const int32_t si = gw[kCwQueue];
    if (si >= a.nshots) break;
    const uint64_t shot = a.shot0 + (uint64_t)si;
    const uint8_t* e0row = a.e0 + (int64_t)si * c.n;

    // ---- start: m = 0, z = 0, s = H e0
    float mvc[CPT][DC], mcv[CPT][DC];
    uint32_t sb = 0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
#pragma unroll
      for (int j = 0; j < DC; ++j) {
        mvc[k][j] = 0.0f;
        mcv[k][j] = 0.0f;
      }
      float* mk = msg + ctm_word<DC>(cidx[k], 0);
#pragma unroll
      for (int j = 0; j < DC; ++j) mk[j * kCtmStride] = 0.0f;
      if (!((vmask >> k) & 1u)) continue;
      uint32_t x = 0;
      for (int32_t j = 0; j < deg[k]; ++j) x ^= e0row[c.chk_var[(int64_t)cidx[k] * c.dcmax + j]];
      sb |= (x & 1u) << k;
    }
    if (t == 0) {
      gw[kCwZero] = (int32_t)0x80000000u;  // -0.0f, the padded partners' message
      for (int w = 1; w < kCtmWords - 1; ++w) gw[w] = 0;
    }
#pragma unroll 1
    for (int32_t w = t; w < nw + mw; w += nt) zw[w] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CPT; ++k)
      if ((sb >> k) & 1u) atomicOr(&sw[cidx[k] >> 5], 1u << (cidx[k] & 31));
    if (sb) atomicAdd(&gw[kCwNs], __popc(sb));
    __syncthreads();
    // Every thread derives the start state itself (the values are uniform);
    // thread 0 keeps the LDS copies the event handler works on.
    int32_t nS = gw[kCwNs];
    double Tev = 0.0;
    double tclr = 0.0;
    if (nS > 0) {
      Tev = ctm_wait(ctm_words(P, shot, 0u).w0, nS);
      tclr = -1.0;
    }
    __syncthreads();
    if (t == 0) *reinterpret_cast<double*>(gw + kCwTev) = Tev;

    int32_t kev = (nS > 0) ? ctm_step_of(Tev, P.dt, P.max_steps) : 0;
    // conv: the messages are a fixed point of the Euler step for the current
    // syndrome -- a step left every message bit for bit as it was. The step
    // is a fixed map of (messages, syndrome), so every step up to the next
    // move is the identity and the loop goes straight to the next event
    // step (thread 0 adds the skipped steps to kCwSkipped); events are still
    // handled one by one. With P.skip, compared steps raise kCwChg if a
    // message changed; every other step clears it, after every thread has
    // read the last one. A jump happens only on a clear flag, and nothing
    // raises it until the next compared step, so the steps after a jump find
    // it clear as well. The compared steps: the 7th after the start and
    // after every move, then at intervals that double (8, 16, ... 256 steps)
    // while compares find a changed message -- sum-product, for one, drifts
    // in its last bits without reaching a fixed point, and a compare costs
    // extra instructions on every message. Which steps compare changes no
    // result: a step is skipped only after a compare found the messages
    // fixed.
    bool conv = false;
    int32_t k = 0;
    int32_t cmp_gap = 8, next_cmp = 7;
    for (;; ++k) {
      if (nS > 0 && k >= kev) {
        if (t < 64) ctm_events<DC, DV, REG>(c, P, shot, (double)k * P.dt, msg, gw, zw, sw, nt < 64 ? nt : 64);
        __syncthreads();
        nS = gw[kCwNs];
        Tev = *reinterpret_cast<const double*>(gw + kCwTev);
        if (nS == 0) tclr = *reinterpret_cast<const double*>(gw + kCwClear);
        else kev = ctm_step_of(Tev, P.dt, P.max_steps);
        if (gw[kCwMoved]) {
          uint32_t nsb = 0;
#pragma unroll
          for (int kk = 0; kk < CPT; ++kk)
            if ((vmask >> kk) & 1u) nsb |= ((sw[cidx[kk] >> 5] >> (cidx[kk] & 31)) & 1u) << kk;
          sb = nsb;
          conv = false;
          cmp_gap = 8;
          next_cmp = k + 7;
        }
      }
      if (nS == 0 || k >= P.max_steps) break;
      if (SKIP && conv) {
        const int32_t next = (nS > 0 && kev < P.max_steps) ? kev : P.max_steps;  // > k here
        if (t == 0) gw[kCwSkipped] += next - k;
        k = next - 1;
        continue;
      }
      const bool cmp = SKIP && k == next_cmp;

      // ---- one Euler step: both directions from the state before it
      float Fv[CPT][DC], Fc[CPT][DC];
#pragma unroll
      for (int kk = 0; kk < CPT; ++kk) {
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          float acc = piv;
#pragma unroll
          for (int p = 0; p < DV - 1; ++p) acc = acc + msg[pidx[kk][j][p]];
          Fv[kk][j] = kNoClamp ? acc : __builtin_amdgcn_fmed3f(acc, -C, C);
        }
        float x[DC];
#pragma unroll
        for (int j = 0; j < DC; ++j) x[j] = (!REG && j >= deg[kk]) ? __builtin_inff() : mvc[kk][j];
        const uint32_t sigma_neg = ((sb >> kk) ^ (uint32_t)deg[kk]) & 1u;
        ctm_check_rule<DC, BP, REG>(P, x, deg[kk], sigma_neg, Fc[kk]);
      }
      __syncthreads();
      if (SKIP && !cmp && t == 0) gw[kCwChg] = 0;
      uint32_t diff = 0u;
      // the update, written twice so that the compare costs nothing on the
      // steps that do not compare
      auto update = [&](auto cmp_tag) {
        constexpr bool CMP = decltype(cmp_tag)::value;
#pragma unroll
        for (int kk = 0; kk < CPT; ++kk) {
          float* mk = msg + ctm_word<DC>(cidx[kk], 0);
          uint32_t dk = 0u;
#pragma unroll
          for (int j = 0; j < DC; ++j) {
            if (!REG && j >= deg[kk]) continue;
            const float nv = mvc[kk][j] + lam * (Fv[kk][j] - mvc[kk][j]);
            const float nc = mcv[kk][j] + lam * (Fc[kk][j] - mcv[kk][j]);
            const float v2 = kNoClamp ? nv : __builtin_amdgcn_fmed3f(nv, -C, C);
            const float c2 = kNoClamp ? nc : __builtin_amdgcn_fmed3f(nc, -C, C);
            if (CMP)
              dk |= (__float_as_uint(v2) ^ __float_as_uint(mvc[kk][j])) |
                    (__float_as_uint(c2) ^ __float_as_uint(mcv[kk][j]));
            mvc[kk][j] = v2;
            mcv[kk][j] = c2;
            mk[j * kCtmStride] = c2;
          }
          if (CMP) diff |= ((vmask >> kk) & 1u) ? dk : 0u;  // padding checks are not compared
        }
      };
      if (SKIP && cmp)
        update(BoolTag<true>());
      else
        update(BoolTag<false>());
      if (cmp && diff) gw[kCwChg] = 1;
      __syncthreads();
      if (cmp) {
        conv = gw[kCwChg] == 0;
        if (!conv && cmp_gap < 256) cmp_gap *= 2;
        next_cmp = k + cmp_gap;
      }
    }

    // ---- results
    for (int32_t v = t; v < c.n; v += nt)
      a.z[(int64_t)si * c.n + v] = (uint8_t)((zw[v >> 5] >> (v & 31)) & 1u);
#pragma unroll
    for (int k = 0; k < CPT; ++k)
      if ((vmask >> k) & 1u) a.s[(int64_t)si * c.m + cidx[k]] = (uint8_t)((sb >> k) & 1u);
    if (a.fail && c.kw <= kCtmFusedWords) {
      uint32_t lp[kCtmFusedWords] = {0u, 0u, 0u, 0u};
#pragma unroll 1
      for (int32_t v = t; v < c.n; v += nt) {
        if (!((e0row[v] ^ (zw[v >> 5] >> (v & 31))) & 1u)) continue;
#pragma unroll
        for (int w = 0; w < kCtmFusedWords; ++w)
          if (w < c.kw) lp[w] ^= c.lcol[(int64_t)v * c.kw + w];
      }
#pragma unroll
      for (int w = 0; w < kCtmFusedWords; ++w)
        if (lp[w]) atomicXor(reinterpret_cast<uint32_t*>(&gw[kCwLpar + w]), lp[w]);
    }
    __syncthreads();
    if (t == 0) {
      a.tclr[si] = tclr;
      if (a.counts) {
        a.counts[2 * (int64_t)si] = gw[kCwEvents];
        a.counts[2 * (int64_t)si + 1] = gw[kCwMoves];
      }
      if (a.steps) a.steps[si] = k - gw[kCwSkipped];  // the loop ended at step k
      if (a.fail && c.kw <= kCtmFusedWords) {
        uint32_t f = (tclr < 0.0) ? 1u : 0u;
        for (int w = 0; w < kCtmFusedWords; ++w) f |= (uint32_t)gw[kCwLpar + w];
        a.fail[si] = f ? 1 : 0;
      }
    }
  }
}

// ---- instantiation table
namespace {

typedef void (*CtmKernel)(DevCode, CtmParamsDev, CtmArgs);

struct CtmVariant {
  int dc, dv, cpt, bp, reg;
  CtmKernel fn;       // every Euler step
  CtmKernel fn_skip;  // steps at a fixed point skipped
};

#define LAIM_CTM(DC, DV, CPT)                                                                        \
  {DC, DV, CPT, 0, 1, ctm_kernel<DC, DV, CPT, 0, true, false>, ctm_kernel<DC, DV, CPT, 0, true, true>}, \
      {DC, DV, CPT, 1, 1, ctm_kernel<DC, DV, CPT, 1, true, false>, ctm_kernel<DC, DV, CPT, 1, true, true>}
#define LAIM_CTM_IRR(DC, DV, CPT)                                                                       \
  {DC, DV, CPT, 0, 0, ctm_kernel<DC, DV, CPT, 0, false, false>, ctm_kernel<DC, DV, CPT, 0, false, true>}, \
      {DC, DV, CPT, 1, 0, ctm_kernel<DC, DV, CPT, 1, false, false>, ctm_kernel<DC, DV, CPT, 1, false, true>}

const CtmVariant kCtmVariants[] = {
    LAIM_CTM(2, 2, 1), LAIM_CTM(2, 2, 2), LAIM_CTM(2, 2, 4),
    LAIM_CTM(4, 2, 1), LAIM_CTM(4, 2, 2), LAIM_CTM(4, 2, 4), LAIM_CTM(4, 2, 8),
    LAIM_CTM(6, 2, 1), LAIM_CTM(6, 2, 2), LAIM_CTM(6, 2, 4),
    LAIM_CTM(4, 4, 1), LAIM_CTM(4, 4, 2), LAIM_CTM(4, 4, 4),
    LAIM_CTM(6, 3, 1), LAIM_CTM(6, 3, 2), LAIM_CTM(6, 3, 4),
    LAIM_CTM_IRR(8, 4, 1), LAIM_CTM_IRR(8, 4, 2), LAIM_CTM_IRR(8, 4, 4),
};

// Template degrees: exact ones for regular codes, else the padded (8, 4)
// variant -- also for min-sum with alpha > 1 (its outputs need the clamp)
// and, for qubit degree 2, when reg2 is false (the exact degree-2 min-sum
// kernels skip the clamps, see ctm_reg_dv2_ok).
bool ctm_degrees(const DevCode& c, bool allow_reg, bool reg2, int* dc, int* dv, int* reg) {
  static const int exact[][2] = {{2, 2}, {4, 2}, {6, 2}, {4, 4}, {6, 3}};
  if (c.regular && allow_reg)
    for (auto& e : exact)
      if (e[0] == c.dcmax && e[1] == c.dvmax && (reg2 || e[1] != 2)) {
        *dc = e[0];
        *dv = e[1];
        *reg = 1;
        return true;
      }
  if (c.dcmax <= 8 && c.dvmax <= 4) {
    *dc = 8;
    *dv = 4;
    *reg = 0;
    return true;
  }
  return false;
}

const CtmVariant* ctm_find(int dc, int dv, int cpt, int bp, int reg) {
  for (const auto& v : kCtmVariants)
    if (v.dc == dc && v.dv == dv && v.cpt == cpt && v.bp == bp && v.reg == reg) return &v;
  return nullptr;
}

}  // namespace

bool ctm_shape(const DevCode& c, const CtmParamsDev& P, int32_t cpt_want, int device, CtmShape* out) {
  const int bp = P.bp;
  int dc, dv, reg;
  if (!ctm_degrees(c, !(bp == 0 && P.alpha > 1.0f), ctm_reg_dv2_ok(P), &dc, &dv, &reg)) {
    set_error("the continuous machine needs check degree <= 8 and qubit degree <= 4 (have %d, %d)",
              c.dcmax, c.dvmax);
    return false;
  }
  int cpt = cpt_want;
  if (cpt <= 0) {
    cpt = 8;
    for (int a : {1, 2, 4, 8})
      if ((c.m + a - 1) / a <= 512 && ctm_find(dc, dv, a, bp, reg)) {
        cpt = a;
        break;
      }
    while (cpt > 1 && !ctm_find(dc, dv, cpt, bp, reg)) cpt /= 2;
  }
  if (!ctm_find(dc, dv, cpt, bp, reg)) {
    set_error("no continuous-machine kernel for checks_per_thread = %d (degrees %d/%d)", cpt, dc, dv);
    return false;
  }
  const int nt = (c.m + cpt - 1) / cpt;
  if (nt > 1024) {
    set_error("%d threads per shot exceed 1024 (m = %d, checks_per_thread = %d)", nt, c.m, cpt);
    return false;
  }
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      lds_max <= 0)
    lds_max = 64 * 1024;
  const int mpad = (nt * cpt + 63) / 64 * 64;
  const size_t lds = ((size_t)ctm_zslot(dc, mpad) + kCtmWords + (c.n + 31) / 32 + (c.m + 31) / 32) * 4;
  if (lds > (size_t)lds_max) {
    set_error("the continuous machine needs %zu bytes of LDS per block (device limit %d)", lds, lds_max);
    return false;
  }
  out->nt = nt;
  out->cpt = cpt;
  out->mpad = mpad;
  out->lds = (lds + 15) / 16 * 16;
  out->dc = dc;
  out->dv = dv;
  out->reg = reg;
  return true;
}

hipError_t launch_ctm(const DevCode& c, const CtmParamsDev& P, const CtmShape& sh, const uint8_t* e0,
                      uint64_t shot0, int32_t nshots, void* ws, uint8_t* z, uint8_t* s, double* tclr,
                      int32_t* counts, int32_t* steps, uint8_t* fail, hipStream_t st) {
  if (nshots <= 0) return hipSuccess;
  // the degrees the shape was sized for; the exact degree-2 min-sum kernels
  // skip the clamps, so the parameters must allow them
  if (sh.reg && sh.dv == 2 && !ctm_reg_dv2_ok(P)) return hipErrorInvalidValue;
  const int dc = sh.dc, dv = sh.dv, reg = sh.reg;
  const CtmVariant* var = ctm_find(dc, dv, sh.cpt, P.bp, reg);
  if (!var) return hipErrorInvalidValue;
  CtmArgs a;
  a.e0 = e0;
  a.shot0 = shot0;
  a.nshots = nshots;
  a.counter = reinterpret_cast<uint32_t*>(ws);
  a.z = z;
  a.s = s;
  a.tclr = tclr;
  a.counts = counts;
  a.steps = steps;
  a.fail = (c.kw <= kCtmFusedWords) ? fail : nullptr;
  a.nt = sh.nt;
  a.mpad = sh.mpad;
  const CtmKernel kfn = P.skip ? var->fn_skip : var->fn;
  const void* fn = reinterpret_cast<const void*>(kfn);
  if (sh.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, sh.nt, sh.lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  const int64_t want = (int64_t)per_cu * cus;
  const unsigned blocks = (unsigned)(want < nshots ? want : nshots);
  hipLaunchKernelGGL(ctm_zero_counter, dim3(1), dim3(64), 0, st, a.counter);
  hipLaunchKernelGGL(kfn, dim3(blocks), dim3(sh.nt), sh.lds, st, c, P, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (fail && c.kw > kCtmFusedWords) return launch_failure(c, e0, z, nshots, fail, st);
  return hipSuccess;
}

}  // namespace laim
