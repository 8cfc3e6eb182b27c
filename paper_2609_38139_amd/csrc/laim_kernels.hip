// laim_kernels.hip -- gfx950 kernels of the decoder and their launchers.
//
// Notation: m checks, n qubits, an edge (c, j) is the j-th qubit of check c
// (SM Definition "Tanner graph"); m_{c->v} / m_{v->c} are the LLR messages
// of Eqs. (BP-LLR1), (BP-LLR2); pi = log(q / (1 - q)).
//
// Both decode forms keep only the check-to-qubit messages m_{c->v} as
// state: a sweep's qubit phase m_{v->c} = clamp(pi + sum_{c' != c} m_{c'->v})
// is recomputed, in ascending check order, where the next check phase reads
// it. This is the same arithmetic as a stored two-phase sweep (check phase
// from m_{v->c}, then qubit phase), with the very first check phase of a
// shot reading m_{v->c} = 0.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.h"
#include "laim_internal.h"

namespace laim {

// ---------------------------------------------------------------- noise
// One thread per (shot, block of 4 qubits): one Philox call gives the four
// uniform words of qubits 4b .. 4b+3. Block (x, y) covers shot x, qubit
// blocks 256 y .. 256 y + 255; rows of a multiple of 4 qubits on a 4-byte
// aligned buffer take one 32-bit store per thread.
__global__ void __launch_bounds__(256) noise_kernel(int32_t n, int32_t nb4, uint64_t bound,
                                                    uint64_t seed, uint64_t shot0, int32_t word_rows,
                                                    uint8_t* __restrict__ e) {
  const int64_t i = bid_x();
  const int32_t b = (int32_t)bid_y() * 256 + (int32_t)tid_x();
  if (b >= nb4) return;
  const uint64_t shot = shot0 + (uint64_t)i;
  const Philox4 w = philox4x32_10((uint32_t)shot, (uint32_t)(shot >> 32), (uint32_t)b, 0u,
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
  uint8_t* row = e + i * (int64_t)n;
  const int32_t v = 4 * b;
  const uint32_t q0 = below(w.w0, bound) ? 1u : 0u, q1 = below(w.w1, bound) ? 1u : 0u;
  const uint32_t q2 = below(w.w2, bound) ? 1u : 0u, q3 = below(w.w3, bound) ? 1u : 0u;
  if (word_rows) {
    *reinterpret_cast<uint32_t*>(row + v) = q0 | (q1 << 8) | (q2 << 16) | (q3 << 24);
  } else {
    if (v + 0 < n) row[v + 0] = (uint8_t)q0;
    if (v + 1 < n) row[v + 1] = (uint8_t)q1;
    if (v + 2 < n) row[v + 2] = (uint8_t)q2;
    if (v + 3 < n) row[v + 3] = (uint8_t)q3;
  }
}

hipError_t launch_noise(const DevCode& c, uint64_t bound, uint64_t seed, uint64_t shot0,
                        int32_t nshots, uint8_t* e, hipStream_t st) {
  if (nshots <= 0) return hipSuccess;
  const int32_t nb4 = (c.n + 3) / 4;
  const int32_t word_rows = (c.n % 4 == 0 && ((uintptr_t)e % 4) == 0) ? 1 : 0;
  if ((nb4 + 255) / 256 > 65535) return hipErrorInvalidValue;  // grid y limit: n <= 2^26
  const dim3 grid((unsigned)nshots, (unsigned)((nb4 + 255) / 256));
  hipLaunchKernelGGL(noise_kernel, grid, dim3(256), 0, st, c.n, nb4, bound, seed, shot0, word_rows, e);
  return hipGetLastError();
}

// ------------------------------------------------------------- syndrome
__global__ void __launch_bounds__(256) syndrome_kernel(DevCode c, const uint8_t* __restrict__ e,
                                                       int64_t total, uint8_t* __restrict__ s) {
  const int64_t idx = (int64_t)bid_x() * bdim_x() + tid_x();
  if (idx >= total) return;
  const int64_t i = idx / c.m;
  const int32_t ch = (int32_t)(idx - i * c.m);
  const uint8_t* row = e + i * (int64_t)c.n;
  const int32_t d = c.chk_deg[ch];
  uint32_t x = 0;
  for (int32_t j = 0; j < d; ++j) x ^= row[c.chk_var[(int64_t)ch * c.dcmax + j]];
  s[idx] = (uint8_t)(x & 1u);
}

hipError_t launch_syndrome(const DevCode& c, const uint8_t* e, int32_t nshots, uint8_t* s,
                           hipStream_t st) {
  if (nshots <= 0) return hipSuccess;
  const int64_t total = (int64_t)c.m * nshots;
  hipLaunchKernelGGL(syndrome_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, c,
                     e, total, s);
  return hipGetLastError();
}

// -------------------------------------------------------------- failure
// One block per shot: r = e0 ^ z; fail = any(H r) or any odd overlap of r
// with a logical (the logical parities are folded into LDS words).
constexpr int kFailMaxWords = 64;

__global__ void __launch_bounds__(256) failure_kernel(DevCode c, const uint8_t* __restrict__ e0,
                                                      const uint8_t* __restrict__ z,
                                                      uint8_t* __restrict__ fail) {
  __shared__ uint32_t par[kFailMaxWords];
  __shared__ int32_t anys;
  const int64_t i = bid_x();
  const uint8_t* a = e0 + i * (int64_t)c.n;
  const uint8_t* b = z + i * (int64_t)c.n;
  for (int w = tid_x(); w < kFailMaxWords; w += bdim_x()) par[w] = 0u;
  if (tid_x() == 0) anys = 0;
  __syncthreads();
  uint32_t local[4] = {0u, 0u, 0u, 0u};
  for (int32_t v = tid_x(); v < c.n; v += bdim_x()) {
    if ((a[v] ^ b[v]) & 1u) {
      for (int32_t w = 0; w < c.kw; ++w) {
        const uint32_t bits = c.lcol[(int64_t)v * c.kw + w];
        if (w < 4)
          local[w] ^= bits;
        else if (bits)
          atomicXor(&par[w], bits);
      }
    }
  }
  for (int32_t w = 0; w < c.kw && w < 4; ++w)
    if (local[w]) atomicXor(&par[w], local[w]);
  int32_t mine = 0;
  for (int32_t ch = tid_x(); ch < c.m; ch += bdim_x()) {
    const int32_t d = c.chk_deg[ch];
    uint32_t x = 0;
    for (int32_t j = 0; j < d; ++j) {
      const int32_t v = c.chk_var[(int64_t)ch * c.dcmax + j];
      x ^= (uint32_t)(a[v] ^ b[v]);
    }
    mine |= (int32_t)(x & 1u);
  }
  if (mine) anys = 1;
  __syncthreads();
  if (tid_x() == 0) {
    uint32_t f = (uint32_t)anys;
    for (int32_t w = 0; w < c.kw; ++w) f |= par[w];
    fail[i] = f ? 1 : 0;
  }
}

// The same test with r packed into an LDS bitmap first: lane l packs
// qubits 32 l .. 32 l + 31 from 16-byte loads of both rows (bit 0 of each
// byte, gathered four at a time by one multiply), then the checks and the
// logical parities read bits. Needs rows of a multiple of 32 bytes and
// 16-byte aligned e0 and z; the bitmap takes n / 8 bytes of LDS.
constexpr int kFailPackedMaxN = 1 << 18;

__device__ __forceinline__ uint32_t pack_bit0(uint4 x) {
  // (b0 + b1 2^8 + b2 2^16 + b3 2^24) * (2^28 + 2^21 + 2^14 + 2^7) puts
  // b0..b3 at bits 28..31 with no carries from the other products
  const uint32_t m = 0x01010101u, k = 0x10204080u;
  return (((x.x & m) * k) >> 28) | ((((x.y & m) * k) >> 28) << 4) | ((((x.z & m) * k) >> 28) << 8) |
         ((((x.w & m) * k) >> 28) << 12);
}

__global__ void __launch_bounds__(256) failure_packed_kernel(DevCode c, const uint8_t* __restrict__ e0,
                                                             const uint8_t* __restrict__ z,
                                                             uint8_t* __restrict__ fail) {
  extern __shared__ uint32_t rb[];  // [n / 32] bits of r, then [kw] logical parities
  __shared__ int32_t anys;
  const int32_t nw = c.n >> 5;
  uint32_t* par = rb + nw;
  const int64_t i = bid_x();
  const uint4* a = reinterpret_cast<const uint4*>(e0 + i * (int64_t)c.n);
  const uint4* b = reinterpret_cast<const uint4*>(z + i * (int64_t)c.n);
  for (int32_t w = tid_x(); w < c.kw; w += bdim_x()) par[w] = 0u;
  if (tid_x() == 0) anys = 0;
  for (int32_t w = tid_x(); w < nw; w += bdim_x()) {
    const uint4 a0 = a[2 * w], a1 = a[2 * w + 1], b0 = b[2 * w], b1 = b[2 * w + 1];
    const uint4 r0 = make_uint4(a0.x ^ b0.x, a0.y ^ b0.y, a0.z ^ b0.z, a0.w ^ b0.w);
    const uint4 r1 = make_uint4(a1.x ^ b1.x, a1.y ^ b1.y, a1.z ^ b1.z, a1.w ^ b1.w);
    rb[w] = pack_bit0(r0) | (pack_bit0(r1) << 16);
  }
  __syncthreads();
  // logical parities: the rows of lcol of the qubits in r. With one word
  // per qubit (at most 32 logicals) a lane reads the rows of its 32 qubits
  // as eight independent 16-byte loads and keeps those whose bit is set.
  uint32_t local[4] = {0u, 0u, 0u, 0u};
  for (int32_t w = tid_x(); w < nw; w += bdim_x()) {
    uint32_t bits = rb[w];
    if (!bits) continue;
    if (c.kw == 1) {
      const uint4* lc = reinterpret_cast<const uint4*>(c.lcol + ((int64_t)w << 5));
      uint32_t acc = 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint4 q = lc[u];
        const uint32_t nib = bits >> (4 * u);
        acc ^= ((nib & 1u) ? q.x : 0u) ^ ((nib & 2u) ? q.y : 0u) ^ ((nib & 4u) ? q.z : 0u) ^
               ((nib & 8u) ? q.w : 0u);
      }
      local[0] ^= acc;
      continue;
    }
    while (bits) {
      const int32_t v = (w << 5) + __builtin_ctz(bits);
      bits &= bits - 1u;
      for (int32_t q = 0; q < c.kw; ++q) {
        const uint32_t lb = c.lcol[(int64_t)v * c.kw + q];
        if (q < 4)
          local[q] ^= lb;
        else if (lb)
          atomicXor(&par[q], lb);
      }
    }
  }
  for (int32_t q = 0; q < c.kw && q < 4; ++q)
    if (local[q]) atomicXor(&par[q], local[q]);
  // syndrome: every entry of a check's row at once (padding entries are -1)
  int32_t mine = 0;
  if (c.dcmax <= 8) {
#pragma unroll 2
    for (int32_t ch = tid_x(); ch < c.m; ch += bdim_x()) {
      const int32_t* nb = c.chk_var + (int64_t)ch * c.dcmax;
      int32_t vv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) vv[j] = (j < c.dcmax) ? nb[j] : -1;
      uint32_t x = 0u;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (vv[j] >= 0) x ^= rb[vv[j] >> 5] >> (vv[j] & 31);
      mine |= (int32_t)(x & 1u);
    }
  } else {
    for (int32_t ch = tid_x(); ch < c.m; ch += bdim_x()) {
      const int32_t d = c.chk_deg[ch];
      const int32_t* nb = c.chk_var + (int64_t)ch * c.dcmax;
      uint32_t x = 0u;
      for (int32_t j = 0; j < d; ++j) {
        const int32_t v = nb[j];
        x ^= rb[v >> 5] >> (v & 31);
      }
      mine |= (int32_t)(x & 1u);
    }
  }
  if (mine) anys = 1;
  __syncthreads();
  if (tid_x() == 0) {
    uint32_t f = (uint32_t)anys;
    for (int32_t q = 0; q < c.kw; ++q) f |= par[q];
    fail[i] = f ? 1 : 0;
  }
}

hipError_t launch_failure(const DevCode& c, const uint8_t* e0, const uint8_t* z, int32_t nshots,
                          uint8_t* fail, hipStream_t st) {
  if (nshots <= 0) return hipSuccess;
  if (c.kw > kFailMaxWords) return hipErrorInvalidValue;
  const bool packed = c.n % 32 == 0 && c.n <= kFailPackedMaxN && ((uintptr_t)e0 % 16) == 0 &&
                      ((uintptr_t)z % 16) == 0;
  if (packed) {
    const size_t lds = (size_t)(c.n / 32 + c.kw) * 4;
    hipLaunchKernelGGL(failure_packed_kernel, dim3((unsigned)nshots), dim3(256), lds, st, c, e0, z, fail);
  } else {
    hipLaunchKernelGGL(failure_kernel, dim3((unsigned)nshots), dim3(256), 0, st, c, e0, z, fail);
  }
  return hipGetLastError();
}

// ====================================================================
// Resident form. A block runs "units": up to `spb` shots of one code at
// once, one shot per group of `nt` threads, in lockstep through the same
// rounds. Thread t of a group owns checks t + k nt (k < CPT) and qubits
// t + k nt (k < vpt). Per group, LDS holds the current m_{c->v} in
// tiles of 64 checks, slot-major within a tile: message (c, j) is word
// ((c / 64) DC + j) S + c mod 64 with a slot stride S of 65 words, so
// consecutive lanes touch consecutive words, the slots of one check sit at
// fixed offsets (immediate operands of the LDS writes) and neighbouring
// checks' messages in different slots fall in different banks. After the
// messages come a few scratch words -- the first holds -0.0, which padded
// qubit-side partners point at (x + (-0.0) == x for every x) -- and four
// bitmaps: flip requests of the current feedback step (n bits), the
// correction z (n bits), the syndrome s (m bits) and the initial error
// (n bits). A shot either
// starts fresh from its initial error or resumes from state saved in device
// memory (used by the serving loop, which runs one round per launch).
// ====================================================================

// LDS word of message (check c, slot j) in the resident layout. A slot of
// a tile spans kSlotStride words (64 used), so that messages of
// neighbouring checks in different slots fall in different LDS banks.
constexpr int kSlotStride = kResSlotStride;
template <int DC>
__device__ __forceinline__ int32_t msg_word(int32_t c, int32_t j) {
  return resident_msg_word(DC, c, j);
}

// Tiled variant (DevCode::tile_*): a thread's 8 checks form a 2 x 4 tile, so
// 10 of the qubits they touch lie inside the tile. The message a check needs
// on such a qubit is the other tile check's output of the previous sweep,
// kept in a register; only the 12 messages on the tile's boundary go through
// LDS during the sweeps. tile_partner(k, g) is the (check, direction) whose
// output check k's input in direction g (0 left, 1 right, 2 up, 3 down)
// reads, or -1 on the boundary.
__host__ __device__ constexpr int tile_partner(int k, int g) {
  return g == 0 ? ((k & 3) > 0 ? 4 * (k - 1) + 1 : -1)
       : g == 1 ? ((k & 3) < 3 ? 4 * (k + 1) + 0 : -1)
       : g == 2 ? ((k >> 2) == 1 ? 4 * (k - 4) + 3 : -1)
                : ((k >> 2) == 0 ? 4 * (k + 4) + 2 : -1);
}

// What one group of a unit works on.
struct GroupJob {
  int32_t alive;
  int32_t r0;            // number of the first round run here (Philox counter)
  uint64_t shot;         // logical shot id
  const uint8_t* e0row;  // [n] initial error
  const uint8_t* s0row;  // [m] start syndrome, or null: the start syndrome is H e0
  float* st_msg;         // resumable state or null: [m * dcmax] m_{c->v} in ELL order,
  uint8_t* st_z;         //   [n] correction, [m] syndrome,
  uint8_t* st_s;
  int32_t* st_hdr;       //   [0] t_clr, [1] messages at a fixed point
  uint8_t* z_out;        // results or null: [n] z, [m] s, t_clr, [n] beliefs,
  uint8_t* s_out;
  int32_t* t_out;
  float* L_out;
  uint8_t* f_out;        //   logical failure (0/1)
  int32_t* ev_out;       //   [4] flips and syndrome weight of the last round run, t_clr, failure
                         //   (bit 0) and frozen (bit 1)
  int32_t* sw_out;       //   BP sweeps computed
};

constexpr int kCtrlWords = 64;  // [0] queue value, [1 + g] group still working (bit 0)
                                // and needing sweeps (bit 1), [kCtrlChg0, kCtrlChg1]
                                // "a message changed" in even / odd sweeps,
                                // [kCtrlSeq0 .. + 2] sequential-rule pass flags
constexpr int kCtrlChg0 = 56, kCtrlChg1 = 57;
constexpr int kCtrlSeq0 = 60;
constexpr uint8_t kNoRequest = 0x7F;
constexpr int kMaxShotsPerBlock = 31;
constexpr int kGroupWords = 16;  // per-group scratch words after msg
// scratch word indices
constexpr int kGwZero = 0, kGwLpar = 1 /* 4 words */, kGwFlips = 5, kGwDefects = 6, kGwInit = 7,
              kGwAct0 = 8, kGwAct1 = 9, kGwChg0 = 10, kGwChg1 = 11, kGwLive = 12;
constexpr int kFusedMaxWords = 4;  // logicals folded in LDS by the fused failure test

template <bool B>
struct BoolTag {
  static constexpr bool value = B;
};

__device__ __forceinline__ GroupJob dead_job() {
  GroupJob j;
  j.alive = 0;
  j.r0 = 0;
  j.shot = 0;
  j.e0row = nullptr;
  j.s0row = nullptr;
  j.st_msg = nullptr;
  j.st_z = j.st_s = nullptr;
  j.st_hdr = nullptr;
  j.z_out = j.s_out = nullptr;
  j.t_out = nullptr;
  j.L_out = nullptr;
  j.f_out = nullptr;
  j.ev_out = nullptr;
  j.sw_out = nullptr;
  return j;
}

// Applies a flip of qubit v to the correction and syndrome bitmaps.
// s ^= H e_v: toggles the syndrome bits of qubit v's checks.
template <int DV, bool REG>
__device__ __forceinline__ void toggle_checks(const DevCode& c, int32_t v, uint32_t* sw) {
  const int32_t dv = REG ? DV : c.var_deg[v];
#pragma unroll
  for (int32_t q = 0; q < (REG ? DV : dv); ++q) {
    const int32_t c2 = edge_check(c.var_edge[(int64_t)v * c.dvmax + q]);
    atomicXor(&sw[c2 >> 5], 1u << (c2 & 31));
  }
}

template <int DV, bool REG>
__device__ __forceinline__ void flip_qubit(const DevCode& c, int32_t v, uint32_t* zw, uint32_t* sw) {
  atomicXor(&zw[v >> 5], 1u << (v & 31));
  toggle_checks<DV, REG>(c, v, sw);
}

// Bits 0..3 of `nib` to bit 0 of bytes 0..3: the four shifted copies
// nib 2^(7i) occupy disjoint bits, so the product has no carries.
__device__ __forceinline__ uint32_t spread4(uint32_t nib) { return (nib * 0x00204081u) & 0x01010101u; }

// Runs the units `src` hands out, one after another, all with the same
// code and launch shape: the per-thread graph tables are built once and
// stay in registers. Every thread of the block calls it (threads beyond
// spb * nt only take part in the barriers).
template <int DC, int DV, int CPT, int BP, bool REG, class Src, bool TILE = false>
__device__ void run_units(const DevCode& c, const KParams& kp, const UnitCtx& u, Src& src,
                          unsigned char* smem, int32_t* ctrl) {
  static_assert(!TILE || (DC == 4 && DV == 2 && CPT == 8 && BP == 0 && REG),
                "the tiled variant is min-sum on the 2D toric layout");
  const int32_t spb = u.spb;
  const int32_t tid = tid_x();
  const int32_t g = tid / u.nt;
  const bool member = g < spb;
  const int32_t t = member ? tid - g * u.nt : 0;
  float* msg = reinterpret_cast<float*>(smem + (size_t)(member ? g : 0) * u.group_bytes);
  const int32_t zslot = (u.mpad >> 6) * DC * kSlotStride;  // mpad is a multiple of 64
  int32_t* gw = reinterpret_cast<int32_t*>(msg + zslot);
  const int32_t nw = (c.n + 31) >> 5;
  uint32_t* flw = reinterpret_cast<uint32_t*>(gw + kGroupWords);  // [nw] flip requests
  uint32_t* zw = flw + nw;                                         // [nw] correction
  uint32_t* sw = zw + nw;                                          // [(m + 31) / 32] syndrome
  uint32_t* e0w = sw + ((c.m + 31) >> 5);                          // [nw] initial error
  // sequential conflict rule only: ring time and request byte per check
  // (bits 0-6 the slot of the requested qubit, kNoRequest if none; bit 7
  // whether the request applies)
  uint32_t* rkey = e0w + nw;                                       // [m]
  uint8_t* rq = reinterpret_cast<uint8_t*>(rkey + c.m);            // [m]
  const float C = kp.clamp;
  const float pi = kp.pi;
  const float thr_reg = REG ? c.thr[DC] : 0.0f;  // Evidence bound of the one check degree
  // this thread's check k: its index in the code, and its index in the LDS
  // layout (the same except in the tiled variant); the LDS word of message
  // (check, row slot) of any check
  // (a tile's checks are (2I + r) L + 4J + q: its first check plus an offset)
  const int32_t tile0 = (TILE && member) ? c.tile_chk[t] : 0;
  // Recomputed where used (one or two instructions) rather than kept for
  // every k: registers are the resident kernels' limit.
  auto own_ch = [&](int32_t k) -> int32_t {
    int32_t b = TILE ? tile0 : t;
    asm volatile("" : "+v"(b));
    return TILE ? b + (k >> 2) * c.tile_L + (k & 3) : b + k * u.nt;
  };

  auto mword = [&](int32_t ch, int32_t j) -> int32_t {
    return TILE ? c.tile_word[ch * DC + j] : msg_word<DC>(ch, j);
  };

  // ---- per-thread graph tables
  // A member owns checks t + k nt, k < CPT; those from m on pad the last
  // tile. Their LDS slots exist (mpad >= nt CPT) and they are swept like
  // the others -- inputs from the zero word, syndrome 0 -- so that the
  // sweep needs no per-check condition; nothing reads what they write.
  // In the tiled variant slot j of a check's LDS messages is lattice
  // direction j, whose row slot is tile_jo; pidx of an input inside the tile
  // is not used.
  int32_t deg[CPT];
  int32_t pidx[CPT][DC][DV > 1 ? DV - 1 : 1];
  uint32_t vmask = 0u;  // bit k: check k of this thread is one of the code's checks
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int32_t vk = t + k * u.nt;
    const bool valid = member && vk < c.m;
    const int32_t ch = (TILE && valid) ? own_ch(k) : vk;
    vmask |= (valid ? 1u : 0u) << k;
    deg[k] = (valid && !REG) ? c.chk_deg[ch] : DC;
#pragma unroll
    for (int j = 0; j < DC; ++j) {
      const int32_t jr = (TILE && valid) ? c.tile_jo[vk * DC + j] : j;
#pragma unroll
      for (int p = 0; p < DV - 1; ++p) {
        int32_t e = -1;
        if (valid && jr < c.dcmax && p < c.dvmax - 1)
          e = c.partner[((int64_t)ch * c.dcmax + jr) * (c.dvmax - 1) + p];
        pidx[k][j][p] = (e >= 0) ? mword(edge_check(e), edge_slot(e)) : zslot;
      }
    }
  }
  // the tile's inner outputs of the last sweep (tiled variant)
  float io[TILE ? CPT : 1][DC];

  while (src.next(ctrl)) {
  const Src& job_at = src;
  // The job is read several times (here, at the start and for the results)
  // rather than kept in registers through the rounds: only the shot id and
  // first round live on.
  bool alive;
  uint64_t shot;
  int32_t r0;
  {
    const GroupJob job = member ? job_at(g) : dead_job();
    alive = member && job.alive;
    shot = job.shot;
    r0 = job.r0;
  }
  // ---- start: messages, bitmaps, scratch words; bit k of sb is the
  // syndrome of check t + k nt (kept in registers for the sweeps)
  uint32_t sb = 0;
  int32_t tclr = -1;
  if (member) {
    const GroupJob job = job_at(g);
    if (t == 0) {
      gw[kGwZero] = (int32_t)0x80000000u;  // -0.0f
      for (int w = 1; w < kGroupWords; ++w) gw[w] = 0;
    }
#pragma unroll 1
    for (int32_t w = t; w < 3 * nw + ((c.m + 31) >> 5); w += u.nt) flw[w] = 0u;
    if (kp.conflict == kConflictSequential) {
#pragma unroll 1
      for (int32_t ch = t; ch < c.m; ch += u.nt) rq[ch] = kNoRequest;
    }
#pragma unroll 1
    for (int k = 0; k < CPT; ++k) {
      const int32_t ch = t + k * u.nt;  // no resume in the tiled variant: its LDS index
      float* mk = msg + msg_word<DC>(ch, 0);
      if (!TILE && u.resume && alive && ch < c.m) {
        for (int j = 0; j < DC; ++j)
          mk[j * kSlotStride] = (j < c.dcmax) ? job.st_msg[(int64_t)ch * c.dcmax + j] : 0.0f;
      } else {  // fresh start, or a padding check
        for (int j = 0; j < DC; ++j) mk[j * kSlotStride] = 0.0f;
      }
    }
  }
  __syncthreads();
  // the initial error as an LDS bitmap, read once from HBM; the syndrome
  // of a fresh start and the failure test at the end take it from there.
  // A row of a multiple of 16 bytes at a 16-byte aligned address is read
  // 16 bytes per thread (independent loads, bits packed by multiplies);
  // other rows a byte per thread.
  if (member && alive) {
    const GroupJob job = job_at(g);
    if (job.e0row) {
      const uint8_t* row = job.e0row;
      if ((c.n & 15) == 0 && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
#pragma unroll 4
        for (int32_t q = t; q < (c.n >> 4); q += u.nt) {
          const uint32_t b = pack_bit0(*reinterpret_cast<const uint4*>(row + 16 * q));  // qubits 16q ..
          if (b) atomicOr(&e0w[q >> 1], b << ((q & 1) * 16));
        }
      } else {
#pragma unroll 4
        for (int32_t v = t; v < c.n; v += u.nt)
          if (row[v] & 1u) atomicOr(&e0w[v >> 5], 1u << (v & 31));
      }
    }
  }
  __syncthreads();
  // the start syndrome: from a fresh start s = H e0, accumulated from the
  // qubits of e0 (few) toggling the bits of their checks; on resume or from
  // a given syndrome, each thread reads its checks' bits
  bool from_e0 = false;
  if (member && alive) {
    const GroupJob job = job_at(g);
    if (!u.resume && !job.s0row) {
      from_e0 = true;
#pragma unroll 1
      for (int32_t wq = t; wq < nw; wq += u.nt) {
        uint32_t r = e0w[wq];
        while (r) {
          const int32_t v = (wq << 5) + __builtin_ctz(r);
          r &= r - 1u;
          toggle_checks<DV, REG>(c, v, sw);
        }
      }
    } else {
#pragma unroll 1
      for (int k = 0; k < CPT; ++k) {
        if (t + k * u.nt >= c.m) continue;
        const int32_t ch = own_ch(k);
        const uint32_t x = u.resume ? job.st_s[ch] : job.s0row[ch];
        sb |= (x & 1u) << k;
      }
    }
  }
  __syncthreads();
  if (member && alive) {
    if (from_e0) {
#pragma unroll
      for (int k = 0; k < CPT; ++k)
        if ((vmask >> k) & 1u) {
          const int32_t ch = own_ch(k);
          sb |= ((sw[ch >> 5] >> (ch & 31)) & 1u) << k;
        }
    } else {
      if (u.resume) {
        const GroupJob job = job_at(g);
#pragma unroll 1
        for (int32_t v = t; v < c.n; v += u.nt)
          if (job.st_z[v] & 1u) atomicOr(&zw[v >> 5], 1u << (v & 31));
      }
#pragma unroll 1
      for (int k = 0; k < CPT; ++k)
        if ((sb >> k) & 1u) {
          const int32_t ch = own_ch(k);
          atomicOr(&sw[ch >> 5], 1u << (ch & 31));
        }
    }
  }
  if (member && sb) gw[kGwInit] = 1;
  __syncthreads();
  if (member) {
    if (u.resume)
      tclr = alive ? job_at(g).st_hdr[0] : -1;
    else
      tclr = gw[kGwInit] ? -1 : 0;
  }
  bool working = alive && !(kp.retire && tclr >= 0);
  bool fresh = !u.resume;
  int32_t flips_last = 0;
  // conv: the group's messages are a fixed point of the sweep for its
  // current syndrome -- a sweep wrote every message back bit for bit. The
  // sweep is a deterministic map of (messages, syndrome), so every further
  // sweep is the identity until a flip changes the syndrome, and the group
  // skips them (with kp.skip; the results are those of all the sweeps).
  bool conv = kp.skip && member && u.resume && alive && job_at(g).st_hdr[1] != 0;
  bool frozen = false;
  int32_t nsweeps = 0;
  // this thread's active checks that failed the Evidence test in the last
  // feedback (valid while the group stays at a fixed point: same beliefs,
  // same syndrome, so the same outcome)
  uint32_t noev = 0u;

  for (int32_t rr = 0; rr < u.rounds; ++rr) {
    const int32_t r = r0 + rr;
    __syncthreads();
    if (member && t == 0) {
      ctrl[1 + g] = working ? (conv ? 1 : 3) : 0;
      gw[((rr + 1) & 1) ? kGwAct1 : kGwAct0] = 0;
      gw[kGwFlips] = 0;
      gw[kGwChg0] = 0;
      gw[kGwChg1] = 0;
      gw[kGwLive] = 0;
    }
    if (tid == 0) {
      ctrl[kCtrlChg0] = 0;
      ctrl[kCtrlChg1] = 0;
    }
    __syncthreads();
    int32_t anyw = 0;
    for (int32_t h = 0; h < spb; ++h) anyw |= ctrl[1 + h];
    if (!anyw) break;

    // ---- BP sweeps, only while some working group is not at a fixed point
    const bool same_state = conv;  // nothing changed since the last feedback
    bool sweep = working && !conv;
    bool swept = false;  // this group computed a sweep in this round
    if (anyw & 2) {
      int32_t it0 = 0;
      if (fresh && REG && kp.iters > 0) {
        // First sweep of a shot: every m_{v->c} is 0, so each check sends
        // (-1)^{s_c + d_c} * 0 (min-sum: alpha * 0; sum-product: 0 [+] 0 = +0).
        if (sweep) {
#pragma unroll
          for (int k = 0; k < CPT; ++k) {
            const float z0 = (((sb >> k) ^ (uint32_t)DC) & 1u) ? -0.0f : 0.0f;
            float* mk = msg + msg_word<DC>(t + k * u.nt, 0);  // LDS index of check k
#pragma unroll
            for (int j = 0; j < DC; ++j) {
              mk[j * kSlotStride] = z0;
              if (TILE) io[TILE ? k : 0][j] = z0;
            }
          }
        }
        fresh = false;
        it0 = 1;
        nsweeps += (sweep && nsweeps != 0x7fffffff) ? 1 : 0;  // saturating
        __syncthreads();
      }
      if (TILE && sweep && it0 == 0) {
        // the tile's inner messages from LDS (written there by the flush of
        // the last round that swept, or by the start): registers hold them
        // only while the sweeps run
#pragma unroll
        for (int k = 0; k < CPT; ++k)
#pragma unroll
          for (int j = 0; j < DC; ++j)
            if (tile_partner(k, j) >= 0) io[TILE ? k : 0][j] = msg[msg_word<DC>(t + k * u.nt, j)];
      }
      // With CMP, a sweep may also compare each new message with the one
      // it replaces; comparing costs half a sweep's worth of extra VALU per
      // check, so it is done every eighth sweep and at the last of the
      // round, and a fixed point is found at most seven sweeps late (those
      // sweeps are identities).
      // The flags of successive compared sweeps alternate, so that a flag
      // is cleared only after every thread has read it. A shot's first
      // sweep (m_{v->c} = 0 rather than pi + sum m_{c->v}) is another map
      // and never counts as a fixed point.
      auto sweeps = [&](auto cmp_tag) {
        constexpr bool CMP_ON = decltype(cmp_tag)::value;
        int32_t ncmp = 0;  // compared sweeps so far in this round
        for (int32_t it = it0; it < kp.iters; ++it) {
          const bool CMP = CMP_ON && ((it & 7) == 7 || it == kp.iters - 1);
          const int32_t f = ncmp & 1;
          const bool first = fresh;
          float x[CPT][DC];
          if (sweep) {
            if (!REG && fresh) {
#pragma unroll
              for (int k = 0; k < CPT; ++k)
#pragma unroll
                for (int j = 0; j < DC; ++j) x[k][j] = (j >= deg[k]) ? __builtin_inff() : 0.0f;
            } else {
#pragma unroll
              for (int k = 0; k < CPT; ++k) {
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                  // (inside a tile the input is formed after the barrier,
                  // from a register)
                  if (TILE && tile_partner(k, j) >= 0) continue;
                  float acc = pi;
#pragma unroll
                  for (int p = 0; p < DV - 1; ++p) acc = acc + msg[pidx[k][j][p]];
                  // min-sum on qubits of degree 2 (exact variants, run only when
                  // alpha < 1 and |pi| / (1 - alpha) < CLAMP): |m_{v->c}| stays
                  // below |pi| / (1 - alpha), so the clamp cannot bind
                  if (!(BP == 0 && REG && DV == 2)) acc = __builtin_amdgcn_fmed3f(acc, -C, C);
                  if (!REG && j >= deg[k]) acc = __builtin_inff();
                  x[k][j] = acc;
                }
              }
            }
          }
          __syncthreads();
          if (CMP) {
            if (member && t == 0) gw[f ? kGwChg0 : kGwChg1] = 0;
            if (tid == 0) ctrl[f ? kCtrlChg0 : kCtrlChg1] = 0;
          }
          uint32_t diff = 0u;
          if (sweep) {
            // Inside a tile the checks' outputs replace the last sweep's in
            // place: when check k runs, the inputs that its outputs feed in
            // a later check are formed first (xpre), from the old outputs;
            // the inputs it takes from an earlier check were formed there.
            float xpre[TILE ? CPT : 1][DC];
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
              if (TILE) {
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                  const int tp = tile_partner(k, j);
                  if (tp < 0) continue;
                  x[k][j] = (tp >> 2) < k ? xpre[TILE ? k : 0][j] : pi + io[TILE ? tp >> 2 : 0][tp & 3];
                }
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                  const int tp = tile_partner(k, j);
                  if (tp >= 0 && (tp >> 2) > k) xpre[TILE ? tp >> 2 : 0][tp & 3] = pi + io[TILE ? k : 0][j];
                }
              }
              const uint32_t sigma_neg = ((sb >> k) ^ (uint32_t)(REG ? DC : deg[k])) & 1u;
              float out[DC];
              if (BP == 0) {
                // normalised min-sum: alpha * (smallest other |m|) with the
                // sign product. No input is -0 (pi + messages with pi != -0,
                // or +0 on a fresh sweep), so the sign bit is sg(). The sign
                // product of all inputs goes into the scale (alpha * min
                // rounds the same for either sign); each output then removes
                // its own input's sign with one bit operation.
                uint32_t par = sigma_neg << 31;
#pragma unroll
                for (int j = 0; j + 1 < DC; j += 2)
                  par = xor3(par, __float_as_uint(x[k][j]), __float_as_uint(x[k][j + 1]));
                if (DC & 1) par ^= __float_as_uint(x[k][DC - 1]);
                const float alpha_s = __uint_as_float(__float_as_uint(kp.alpha) ^ (par & 0x80000000u));
                float ex[DC];  // smallest |m| over the other inputs
                if (DC == 2) {
                  ex[0] = fabsf(x[k][1]);
                  ex[1] = fabsf(x[k][0]);
                } else if (DC == 4) {
                  ex[0] = min3_abs(x[k][1], x[k][2], x[k][3]);
                  ex[1] = min3_abs(x[k][0], x[k][2], x[k][3]);
                  ex[2] = min3_abs(x[k][0], x[k][1], x[k][3]);
                  ex[3] = min3_abs(x[k][0], x[k][1], x[k][2]);
                } else {
                  float pre[DC], suf[DC];
                  pre[1] = fabsf(x[k][0]);
#pragma unroll
                  for (int j = 2; j < DC; ++j) pre[j] = fminf(pre[j - 1], fabsf(x[k][j - 1]));
                  suf[DC - 2] = fabsf(x[k][DC - 1]);
#pragma unroll
                  for (int j = DC - 3; j >= 0; --j) suf[j] = fminf(suf[j + 1], fabsf(x[k][j + 1]));
                  ex[0] = suf[0];
                  ex[DC - 1] = pre[DC - 1];
#pragma unroll
                  for (int j = 1; j < DC - 1; ++j) ex[j] = fminf(pre[j], suf[j]);
                }
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                  // With degree >= 2 there is an input to take the minimum of,
                  // so |v| <= alpha * clamp <= clamp (the resident min-sum path
                  // runs only with alpha <= 1) and the output clamp cannot bind;
                  // a degree-1 check of an irregular code has an empty minimum
                  // (+inf) and is clamped.
                  float v = alpha_s * ex[j];
                  if (!REG) v = __builtin_amdgcn_fmed3f(v, -C, C);
                  out[j] = __uint_as_float(__float_as_uint(v) ^ (__float_as_uint(x[k][j]) & 0x80000000u));
                }
              } else {
                // sum-product: box-plus of the other inputs (prefix/suffix folds)
                float acc[DC];
                boxplus_others<DC, REG>(x[k], deg[k], acc);
#pragma unroll
                for (int j = 0; j < DC; ++j) out[j] = __builtin_amdgcn_fmed3f(sigma_neg ? -acc[j] : acc[j], -C, C);
              }
              float* mk = msg + msg_word<DC>(t + k * u.nt, 0);
              if (CMP) {  // padding checks and the padding slots of irregular checks are never read
                uint32_t dk = 0u;
#pragma unroll
                for (int j = 0; j < DC; ++j) {
                  const float old = (TILE && tile_partner(k, j) >= 0) ? io[TILE ? k : 0][j] : mk[j * kSlotStride];
                  if (REG || j < deg[k]) dk |= __float_as_uint(old) ^ __float_as_uint(out[j]);
                }
                diff |= ((vmask >> k) & 1u) ? dk : 0u;
              }
#pragma unroll
              for (int j = 0; j < DC; ++j) {
                if (TILE && tile_partner(k, j) >= 0)
                  io[TILE ? k : 0][j] = out[j];  // read from a register within the tile
                else
                  mk[j * kSlotStride] = out[j];
              }
            }
          }
          swept = swept || sweep;
          if (CMP && sweep && (diff || first)) {
            gw[f ? kGwChg1 : kGwChg0] = 1;
            ctrl[f ? kCtrlChg1 : kCtrlChg0] = 1;
          }
          fresh = false;
          __syncthreads();
          nsweeps += (sweep && nsweeps != 0x7fffffff) ? 1 : 0;  // saturating
          if (CMP) {
            ++ncmp;
            if (sweep && gw[f ? kGwChg1 : kGwChg0] == 0) {
              sweep = false;
              conv = true;
            }
            if (ctrl[f ? kCtrlChg1 : kCtrlChg0] == 0) break;  // no group changed
          }
        }
      };
      if (kp.skip)
        sweeps(BoolTag<true>());
      else
        sweeps(BoolTag<false>());
      if (TILE) {
        // the tile's inner messages back to LDS, for the feedback and the
        // next round's sweeps (anyw is the same in every thread of the block)
        if (swept) {
#pragma unroll
          for (int k = 0; k < CPT; ++k)
#pragma unroll
            for (int j = 0; j < DC; ++j)
              if (tile_partner(k, j) >= 0) msg[msg_word<DC>(t + k * u.nt, j)] = io[TILE ? k : 0][j];
        }
        __syncthreads();
      }
    }

    // ---- feedback: every active check whose clock rang tests Evidence
    // and requests a flip of its LocalMove qubit. A lane visits only its
    // own active checks, so a wavefront runs as many passes as its busiest
    // lane has defects. Requests combine by the conflict rule:
    //   OR   the request that sets a qubit's bit first applies the flip;
    //   XOR  every request applies (two on one qubit cancel);
    //   SEQUENTIAL  requests are recorded and resolved below.
    // Applying a flip toggles the qubit's correction bit and the syndrome
    // bits of its checks (z ^= f, s ^= H f); the flip bitmap is toggled
    // too, so that its population -- the net count kept in kGwFlips -- is
    // the number of qubits that changed.
    uint32_t reqm = 0;  // this thread's checks with a recorded request (sequential rule)
    if (working) {
      if (!same_state) noev = 0u;
      uint32_t act = sb & ~noev;
      int32_t nflip = 0;
      // regular codes with qubits of degree 2: the qubits of an active check
      // and the other check of each are read together (one round trip), and
      // those of the next active check are requested before this one is
      // evaluated, so that the round trip overlaps the evaluation
      int32_t pe_n[DC], nb_n[DC], ow_n[DC], pw_n[DC];
      auto fetch_rows = [&](int32_t kk) {
        const int32_t chn = own_ch(kk);
        const int32_t* prow = c.partner + (int64_t)chn * DC;
        const int32_t* nrow = c.chk_var + (int64_t)chn * c.dcmax;
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          pe_n[j] = prow[j];
          nb_n[j] = nrow[j];
          if (TILE) {  // the LDS words of the check's messages and of the other check's
            ow_n[j] = c.tile_word[chn * DC + j];
            pw_n[j] = c.tile_word[edge_check(pe_n[j]) * DC + edge_slot(pe_n[j])];
          }
        }
      };
      if (REG && DV == 2 && act) fetch_rows(__builtin_ctz(act));
#pragma unroll 1
      while (act) {
        const int32_t k = __builtin_ctz(act);
        act &= act - 1u;
        const int32_t ch = own_ch(k);
        const int32_t d = REG ? DC : c.chk_deg[ch];
        const int32_t* nb = c.chk_var + (int64_t)ch * c.dcmax;
        float Lv[DC];
        float Lmax = -__builtin_inff();
        int32_t pe[DC], nbv[DC], ow[DC], pw[DC];
        if (REG && DV == 2) {
          // Qubit j has two messages: the check's own and the one of the
          // other check of the qubit, added to pi in ascending check order
          // as everywhere. (A regular variant runs only on codes whose every
          // check has degree DC and every qubit degree DV, so a row holds DC
          // entries.)
#pragma unroll
          for (int j = 0; j < DC; ++j) {
            pe[j] = pe_n[j];
            nbv[j] = nb_n[j];
            ow[j] = ow_n[j];
            pw[j] = pw_n[j];
          }
          if (act) fetch_rows(__builtin_ctz(act));
#pragma unroll
          for (int j = 0; j < DC; ++j) {
            const int32_t c2 = edge_check(pe[j]);
            const float own = msg[TILE ? ow[j] : msg_word<DC>(ch, j)];
            const float oth = msg[TILE ? pw[j] : msg_word<DC>(c2, edge_slot(pe[j]))];
            const float acc = clampf(c2 < ch ? (pi + oth) + own : (pi + own) + oth, C);
            Lv[j] = acc;
            if (j == 0 || acc > Lmax) Lmax = acc;
          }
        } else {
#pragma unroll
          for (int j = 0; j < DC; ++j) {
            if (j >= d) continue;
            const int32_t v = nb[j];
            const int32_t dv = REG ? DV : c.var_deg[v];
            float acc = pi;
#pragma unroll
            for (int32_t q = 0; q < (REG ? DV : dv); ++q) {
              const int32_t e = c.var_edge[(int64_t)v * c.dvmax + q];
              acc = acc + msg[mword(edge_check(e), edge_slot(e))];
            }
            acc = clampf(acc, C);
            Lv[j] = acc;
            if (j == 0 || acc > Lmax) Lmax = acc;
          }
        }
        if (d == 0) continue;
        // The move needs both the Evidence bound and the check's clock; the
        // bound is tested first, so the random words are drawn only when
        // it holds.
        if (kp.evidence && !(Lmax >= (REG ? thr_reg : c.thr[d]))) {
          noev |= 1u << k;
          continue;
        }
        const Philox4 w = philox4x32_10((uint32_t)shot, (uint32_t)(shot >> 32), (uint32_t)ch,
                                        ((uint32_t)r << 4) | 1u, (uint32_t)kp.seed,
                                        (uint32_t)(kp.seed >> 32));
        if (!below(w.w0, kp.mask_bound)) continue;
        uint32_t ntie = 0;
#pragma unroll
        for (int j = 0; j < DC; ++j)
          if (j < d && Lv[j] == Lmax) ++ntie;
        uint32_t pick = (uint32_t)(((uint64_t)w.w1 * (uint64_t)ntie) >> 32);
        int32_t slot = -1;
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          if (j < d && Lv[j] == Lmax && slot < 0) {
            if (pick == 0)
              slot = j;
            else
              --pick;
          }
        }
        if (slot < 0) continue;
        if (kp.conflict == kConflictSequential) {
          // provisionally applies: the check is active at the round's start
          // (single-qubit moves only: the host refuses multi-qubit ones here)
          rkey[ch] = w.w2;
          rq[ch] = (uint8_t)(0x80 | slot);
          reqm |= 1u << k;
          continue;
        }
        // The slots the check asks to flip: its LocalMove qubit, or for a
        // multi-qubit move every qubit of the check with a positive belief
        // (Pr_BP(e_v = 1 | s) > 1/2), falling back to the LocalMove qubit.
        uint32_t fmask = 1u << slot;
        if (kp.move) {
          uint32_t pos = 0u;
#pragma unroll
          for (int j = 0; j < DC; ++j)
            if (j < d && Lv[j] > 0.0f) pos |= 1u << j;
          if (pos) fmask = pos;
        }
#pragma unroll 1
        while (fmask) {
          const int32_t jj = __builtin_ctz(fmask);
          fmask &= fmask - 1u;
          int32_t chosen, c2 = 0;
          if (REG && DV == 2) {  // from registers: the qubit and its other check
            chosen = nbv[0];
            c2 = edge_check(pe[0]);
#pragma unroll
            for (int j = 1; j < DC; ++j)
              if (jj == j) {
                chosen = nbv[j];
                c2 = edge_check(pe[j]);
              }
          } else {
            chosen = nb[jj];
          }
          const uint32_t bit = 1u << (chosen & 31);
          uint32_t had;
          if (kp.conflict == kConflictOr) {
            if (atomicOr(&flw[chosen >> 5], bit) & bit) continue;  // already requested
            had = 0;
          } else {
            had = atomicXor(&flw[chosen >> 5], bit) & bit;
          }
          if (REG && DV == 2) {  // z ^= e_v; s ^= H e_v over the qubit's two checks
            atomicXor(&zw[chosen >> 5], bit);
            atomicXor(&sw[ch >> 5], 1u << (ch & 31));
            atomicXor(&sw[c2 >> 5], 1u << (c2 & 31));
          } else {
            flip_qubit<DV, REG>(c, chosen, zw, sw);
          }
          nflip += had ? -1 : 1;
        }
      }
      if (nflip) atomicAdd(&gw[kGwFlips], nflip);
      if (sb & ~noev) gw[kGwLive] = 1;  // an active check passed the Evidence test
    }
    if (kp.conflict == kConflictSequential) {
      // Sequential rule: request i applies iff its check's start syndrome
      // (1) toggled by every applied request that rang earlier -- ring
      // time, then check index -- and asks for a qubit of the check is 1.
      // The requests form a directed acyclic graph in ring-time order, so
      // the relaxation below reaches the unique solution after at most
      // (longest chain + 1) passes; a pass that changes nothing in the
      // block ends it. Three flags rotate so that a flag is cleared only
      // after every thread has read it.
      if (tid == 0) ctrl[kCtrlSeq0] = 0;
      __syncthreads();
#pragma unroll 1
      for (int32_t pass = 0; pass <= c.m + 1; ++pass) {
        const int32_t fi = kCtrlSeq0 + pass % 3;
        if (tid == 0) ctrl[kCtrlSeq0 + (pass + 1) % 3] = 0;
        bool changed = false;
        uint32_t pend = reqm;
#pragma unroll 1
        while (pend) {
          const int32_t k = __builtin_ctz(pend);
          pend &= pend - 1u;
          const int32_t ch = own_ch(k);
          const uint32_t key = rkey[ch];
          const int32_t d = REG ? DC : c.chk_deg[ch];
          const int32_t* nb = c.chk_var + (int64_t)ch * c.dcmax;
          uint32_t x = 1u;
#pragma unroll
          for (int j = 0; j < DC; ++j) {
            if (j >= d) continue;
            const int32_t v = nb[j];
            const int32_t dv = REG ? DV : c.var_deg[v];
#pragma unroll
            for (int32_t q = 0; q < (REG ? DV : dv); ++q) {
              const int32_t e = c.var_edge[(int64_t)v * c.dvmax + q];
              const int32_t c2 = edge_check(e);
              const uint32_t r2 = rq[c2];
              if (c2 == ch || (r2 & 0x7Fu) != (uint32_t)edge_slot(e)) continue;
              const uint32_t k2 = rkey[c2];
              if (k2 < key || (k2 == key && c2 < ch)) x ^= r2 >> 7;
            }
          }
          const uint32_t cur = rq[ch];
          if ((cur >> 7) != x) {
            rq[ch] = (uint8_t)((x << 7) | (cur & 0x7Fu));
            changed = true;
          }
        }
        if (changed) ctrl[fi] = 1;
        __syncthreads();
        if (!ctrl[fi]) break;
      }
      if (working && reqm) {
        int32_t nflip = 0;
        uint32_t pend = reqm;
#pragma unroll 1
        while (pend) {
          const int32_t k = __builtin_ctz(pend);
          pend &= pend - 1u;
          const int32_t ch = own_ch(k);
          const uint32_t cur = rq[ch];
          rq[ch] = kNoRequest;
          if (!(cur >> 7)) continue;
          const int32_t chosen = c.chk_var[(int64_t)ch * c.dcmax + (cur & 0x7Fu)];
          const uint32_t bit = 1u << (chosen & 31);
          const uint32_t had = atomicXor(&flw[chosen >> 5], bit) & bit;
          flip_qubit<DV, REG>(c, chosen, zw, sw);
          nflip += had ? -1 : 1;
        }
        if (nflip) atomicAdd(&gw[kGwFlips], nflip);
      }
    }
    __syncthreads();
    // ---- the new syndrome bits of this thread's checks (unchanged when
    // no qubit of the group flipped this round)
    const int32_t nfl = member ? gw[kGwFlips] : 0;
    if (working) {
      if (nfl) {
        uint32_t nsb = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k)
          if ((vmask >> k) & 1u) {
            const int32_t ch = own_ch(k);
            nsb |= ((sw[ch >> 5] >> (ch & 31)) & 1u) << k;
          }
        sb = nsb;
      }
      if (sb) gw[(rr & 1) ? kGwAct1 : kGwAct0] = 1;
    }
    __syncthreads();
    if (working) {
      if (nfl) {
#pragma unroll 1
        for (int32_t w = t; w < nw; w += u.nt) flw[w] = 0u;
      }
      const bool any = gw[(rr & 1) ? kGwAct1 : kGwAct0] != 0;
      if (!any && tclr < 0) tclr = r + 1;
      flips_last = nfl;
      if (nfl) conv = false;  // the syndrome changed
      if (kp.retire && tclr >= 0) working = false;
      // Frozen: at a fixed point, no flip, and no active check passes the
      // Evidence test. The next round then repeats this one exactly -- no
      // sweep changes anything, the same checks fail the test, nothing
      // flips -- and so does every round after it: the shot's z, s, t_clr
      // and beliefs are final and it stops here.
      if (conv && !gw[kGwLive]) {
        working = false;
        frozen = true;
      }
    }
  }

  // ---- results. The group index passes through an empty asm statement so
  // that the job's output pointers are not computed before the rounds and
  // kept in registers through them.
  int32_t g_res = g;
  asm volatile("" : "+v"(g_res));
  if (alive) {
    const GroupJob job = job_at(g_res);
    if (job.z_out) {
      uint8_t* zrow = job.z_out;
      if ((c.n & 15) == 0 && (reinterpret_cast<uintptr_t>(zrow) & 15) == 0) {
        // 16 bytes per thread from 16 bits of the bitmap
#pragma unroll 1
        for (int32_t q = t; q < (c.n >> 4); q += u.nt) {
          const uint32_t b = zw[q >> 1] >> ((q & 1) * 16);
          *reinterpret_cast<uint4*>(zrow + 16 * q) =
              make_uint4(spread4(b & 15u), spread4((b >> 4) & 15u), spread4((b >> 8) & 15u), spread4((b >> 12) & 15u));
        }
      } else {
#pragma unroll 1
        for (int32_t v = t; v < c.n; v += u.nt) zrow[v] = (uint8_t)((zw[v >> 5] >> (v & 31)) & 1u);
      }
    }
    if (job.s_out) {
#pragma unroll 1
      for (int k = 0; k < CPT; ++k)
        if (t + k * u.nt < c.m) job.s_out[own_ch(k)] = (uint8_t)((sb >> k) & 1u);
    }
    if (job.t_out && t == 0) job.t_out[0] = tclr;
    if (job.sw_out && t == 0) job.sw_out[0] = nsweeps;
    if (job.L_out) {
#pragma unroll 1
      for (int32_t v = t; v < c.n; v += u.nt) {
        const int32_t dv = c.var_deg[v];
        float acc = pi;
        for (int32_t q = 0; q < dv; ++q) {
          const int32_t e = c.var_edge[(int64_t)v * c.dvmax + q];
          acc = acc + msg[mword(edge_check(e), edge_slot(e))];
        }
        job.L_out[v] = clampf(acc, C);
      }
    }
    if (job.st_msg) {
#pragma unroll 1
      for (int k = 0; k < CPT; ++k) {
        if (t + k * u.nt >= c.m) continue;
        const int32_t ch = own_ch(k);
        for (int j = 0; j < c.dcmax && j < DC; ++j)
          job.st_msg[(int64_t)ch * c.dcmax + j] = msg[mword(ch, j)];
        job.st_s[ch] = (uint8_t)((sb >> k) & 1u);
      }
#pragma unroll 1
      for (int32_t v = t; v < c.n; v += u.nt) job.st_z[v] = (uint8_t)((zw[v >> 5] >> (v & 31)) & 1u);
      if (t == 0) {
        job.st_hdr[0] = tclr;
        job.st_hdr[1] = conv ? 1 : 0;
      }
    }
    // fused success test: odd overlap of e0 ^ z with a logical, or s != 0
    if (job.f_out || job.ev_out) {
      uint32_t lp[kFusedMaxWords] = {0u, 0u, 0u, 0u};
#pragma unroll 1
      for (int32_t wq = t; wq < nw; wq += u.nt) {
        uint32_t r = e0w[wq] ^ zw[wq];
        while (r) {
          const int32_t v = (wq << 5) + __builtin_ctz(r);
          r &= r - 1u;
#pragma unroll
          for (int w = 0; w < kFusedMaxWords; ++w)
            if (w < c.kw) lp[w] ^= c.lcol[(int64_t)v * c.kw + w];
        }
      }
#pragma unroll
      for (int w = 0; w < kFusedMaxWords; ++w)
        if (lp[w]) atomicXor(reinterpret_cast<uint32_t*>(&gw[kGwLpar + w]), lp[w]);
    }
    if (job.ev_out && sb) atomicAdd(&gw[kGwDefects], __popc(sb));
  }
  __syncthreads();
  if (alive && t == 0) {
    const GroupJob job = job_at(g_res);
    uint32_t f = (tclr < 0) ? 1u : 0u;
    for (int w = 0; w < kFusedMaxWords; ++w) f |= (uint32_t)gw[kGwLpar + w];
    if (job.f_out) job.f_out[0] = f ? 1 : 0;
    if (job.ev_out) {
      job.ev_out[0] = flips_last;
      job.ev_out[1] = gw[kGwDefects];
      job.ev_out[2] = tclr;
      job.ev_out[3] = (f ? 1 : 0) | (frozen ? 2 : 0);
    }
  }
  }  // units
}

// ---- the single-code persistent kernel
struct ResArgs {
  UnitCtx u;
  const GroupItemDev* items;  // [nitems] or null: a single item given by the fields below
  int32_t nitems;
  const uint8_t* e0;  // [nshots][n] initial errors, or null when s0 is given
  const uint8_t* s0;  // [nshots][m] start syndromes, or null: H e0
  int32_t r0;         // number of the first round (the clocks' Philox counter)
  uint64_t shot0;
  int32_t nshots;
  uint32_t* counter;  // queue head, zeroed before the launch
  uint8_t* z;
  uint8_t* s;
  int32_t* tclr;
  float* L;
  uint8_t* fail;
  int32_t* sweeps;
};

struct ResJobs {
  // copied by value: taking the address of a kernel argument would force it
  // into scratch memory
  const GroupItemDev* items;
  int32_t nitems;
  const uint8_t* e0;
  const uint8_t* s0;
  int32_t r0;
  uint64_t shot0;
  int32_t nshots, n, m, base;
  uint8_t* z;
  uint8_t* s;
  int32_t* tclr;
  float* L;
  uint8_t* fail;
  int32_t* sweeps;
  uint32_t* counter;
  int32_t spb;
  // Takes the next spb shots from the launch's queue; false once it is empty.
  __device__ bool next(int32_t* ctrl) {
    __syncthreads();
    if (tid_x() == 0) ctrl[0] = (int32_t)atomicAdd(counter, (uint32_t)spb);
    __syncthreads();
    base = ctrl[0];
    return base < nshots;
  }
  __device__ GroupJob operator()(int32_t g) const {
    GroupJob j = dead_job();
    const int32_t idx = base + g;
    if (idx >= nshots) return j;
    if (items) {
      // the item holding launch shot idx (items ascend in `first`)
      int32_t it = 0;
      while (it + 1 < nitems && items[it + 1].first <= idx) ++it;
      const GroupItemDev& I = items[it];
      const int32_t li = idx - I.first;
      j.alive = 1;
      j.r0 = 0;
      j.shot = I.shot0 + (uint64_t)li;
      j.e0row = I.e0 + (int64_t)li * n;
      j.z_out = I.z + (int64_t)li * n;
      j.s_out = I.s + (int64_t)li * m;
      j.t_out = I.tclr + li;
      j.f_out = I.fail ? I.fail + li : nullptr;
      return j;
    }
    j.alive = 1;
    j.r0 = r0;
    j.shot = shot0 + (uint64_t)idx;
    j.e0row = e0 ? e0 + (int64_t)idx * n : nullptr;
    j.s0row = s0 ? s0 + (int64_t)idx * m : nullptr;
    j.z_out = z + (int64_t)idx * n;
    j.s_out = s + (int64_t)idx * m;
    j.t_out = tclr + idx;
    j.L_out = L ? L + (int64_t)idx * n : nullptr;
    j.f_out = fail ? fail + idx : nullptr;
    j.sw_out = sweeps ? sweeps + idx : nullptr;
    return j;
  }
};

template <int DC, int DV, int CPT, int BP, bool REG, bool TILE>
__device__ __forceinline__ void resident_body(const DevCode& c, const KParams& kp, const ResArgs& a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // control words after the groups, so that group 0's messages start at
  // LDS address 0 and the slot offsets fit the LDS instructions' offset fields
  int32_t* ctrl = reinterpret_cast<int32_t*>(smem + (size_t)a.u.spb * a.u.group_bytes);
  ResJobs jobs{a.items, a.nitems, a.e0,     a.s0,     a.r0,      a.shot0,   a.nshots, c.n, c.m, 0,
               a.z,     a.s,      a.tclr,   a.L,      a.fail,    a.sweeps,  a.counter, a.u.spb};
  run_units<DC, DV, CPT, BP, REG, ResJobs, TILE>(c, kp, a.u, jobs, smem, ctrl);
}

template <int DC, int DV, int CPT, int BP, bool REG>
__global__ void __launch_bounds__(1024) resident_kernel(DevCode c, KParams kp, ResArgs a) {
  resident_body<DC, DV, CPT, BP, REG, false>(c, kp, a);
}

// The tiled variant runs blocks of at most kTileMaxThreads threads with at
// least kTileWavesPerSimd wavefronts per SIMD (128 VGPRs), as the plain
// variant: measured on 2D toric L = 32, two and three wavefronts per SIMD
// (no spills) ran 57% and 13% slower than four (a few spills outside the
// sweeps).
constexpr int kTileMaxThreads = 512;
constexpr int kTileWavesPerSimd = 4;
__global__ void __launch_bounds__(kTileMaxThreads, kTileWavesPerSimd)
    resident_tile_kernel(DevCode c, KParams kp, ResArgs a) {
  resident_body<4, 2, 8, 0, true, true>(c, kp, a);
}

__global__ void zero_u32_kernel(uint32_t* p, int32_t k) {
  const int32_t i = bid_x() * bdim_x() + tid_x();
  if (i < k) p[i] = 0u;
}

// ---- serving: one round for every scheduled request, state in HBM
struct ServerJobs {
  const ServerReqDev* R;
  int32_t first, count;
  bool given;
  __device__ bool next(int32_t*) {  // a single unit
    const bool once = !given;
    given = true;
    return once;
  }
  __device__ GroupJob operator()(int32_t g) const {
    GroupJob j = dead_job();
    if (g >= count) return j;
    const ServerReqDev& q = R[first + g];
    j.alive = 1;
    j.r0 = q.round;
    j.shot = q.shot;
    j.e0row = q.e0;
    j.st_msg = q.msg;
    j.st_z = q.z;
    j.st_s = q.s;
    j.st_hdr = q.hdr;
    j.f_out = q.fail;
    j.ev_out = q.ev;
    return j;
  }
};

// The (degrees, checks per thread) variants compiled into the multi-code
// kernels; the host picks one per code (batch_variant below).
#define LAIM_BATCH_SWITCH(V, BP, CALL)                \
  switch (V) {                                        \
    case 0: CALL(2, 2, 1, BP, true); break;           \
    case 1: CALL(2, 2, 2, BP, true); break;           \
    case 2: CALL(4, 2, 1, BP, true); break;           \
    case 3: CALL(4, 2, 2, BP, true); break;           \
    case 4: CALL(4, 2, 4, BP, true); break;           \
    case 5: CALL(6, 2, 1, BP, true); break;           \
    case 6: CALL(6, 2, 2, BP, true); break;           \
    case 7: CALL(4, 4, 1, BP, true); break;           \
    case 8: CALL(4, 4, 2, BP, true); break;           \
    case 9: CALL(6, 3, 1, BP, true); break;           \
    case 10: CALL(6, 3, 2, BP, true); break;          \
    case 11: CALL(6, 2, 1, BP, false); break;         \
    default: CALL(8, 4, 1, BP, false); break;         \
  }

static const int kBatchVariants[][4] = {  // dc, dv, cpt, regular
    {2, 2, 1, 1}, {2, 2, 2, 1}, {4, 2, 1, 1}, {4, 2, 2, 1}, {4, 2, 4, 1}, {6, 2, 1, 1},
    {6, 2, 2, 1}, {4, 4, 1, 1}, {4, 4, 2, 1}, {6, 3, 1, 1}, {6, 3, 2, 1}, {6, 2, 1, 0}, {8, 4, 1, 0}};

template <int BP>
__global__ void __launch_bounds__(1024) server_kernel(const BatchItemDev* items,
                                                      const ServerUnitDev* units,
                                                      const ServerReqDev* reqs, int32_t ctrl_off) {
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t* ctrl = reinterpret_cast<int32_t*>(smem + ctrl_off);
  const ServerUnitDev U = units[bid_x()];
  const BatchItemDev* I = items + U.item;
  const DevCode c = I->c;
  const KParams kp = I->kp;
  UnitCtx ctx = I->u;
  ctx.rounds = U.rounds;
  ctx.resume = U.resume;
  ctx.events = 1;
  ServerJobs jobs{reqs, U.first, U.count, false};
#define LAIM_CALL(DC, DV, CPT, BPV, REG) run_units<DC, DV, CPT, BPV, REG>(c, kp, ctx, jobs, smem, ctrl)
  LAIM_BATCH_SWITCH(I->variant, BP, LAIM_CALL)
#undef LAIM_CALL
}

// ---- instantiation table
typedef void (*ResKernel)(DevCode, KParams, ResArgs);

struct ResVariant {
  int dc, dv, cpt, bp, reg, tile;
  ResKernel fn;
};

#define LAIM_RES(DC, DV, CPT)                                                     \
  {DC, DV, CPT, 0, 1, 0, resident_kernel<DC, DV, CPT, 0, true>},                 \
      {DC, DV, CPT, 1, 1, 0, resident_kernel<DC, DV, CPT, 1, true>}
#define LAIM_RES_IRR(DC, DV, CPT)                                                 \
  {DC, DV, CPT, 0, 0, 0, resident_kernel<DC, DV, CPT, 0, false>},                \
      {DC, DV, CPT, 1, 0, 0, resident_kernel<DC, DV, CPT, 1, false>}

static const ResVariant kResVariants[] = {
    LAIM_RES(2, 2, 1), LAIM_RES(2, 2, 2), LAIM_RES(2, 2, 4), LAIM_RES(2, 2, 8),
    LAIM_RES(4, 2, 1), LAIM_RES(4, 2, 2), LAIM_RES(4, 2, 4), LAIM_RES(4, 2, 8),
    LAIM_RES(6, 2, 1), LAIM_RES(6, 2, 2), LAIM_RES(6, 2, 4), LAIM_RES(6, 2, 8),
    LAIM_RES(4, 4, 1), LAIM_RES(4, 4, 2), LAIM_RES(4, 4, 4),
    LAIM_RES(6, 3, 1), LAIM_RES(6, 3, 2), LAIM_RES(6, 3, 4),
    LAIM_RES_IRR(6, 2, 1), LAIM_RES_IRR(6, 2, 2), LAIM_RES_IRR(6, 2, 4), LAIM_RES_IRR(6, 2, 8),
    LAIM_RES_IRR(8, 4, 1), LAIM_RES_IRR(8, 4, 2), LAIM_RES_IRR(8, 4, 4),
    {4, 2, 8, 0, 1, 1, resident_tile_kernel},
};

// Template degrees for a code: exact ones for the regular families, a
// padded variant otherwise -- (6, 2) for checks of degree <= 6 on qubits of
// degree <= 2 (the spacetime window codes of online decoding among them),
// else (8, 4) -- and for qubit degree 2 when reg2 is false (min-sum whose
// qubit-side clamp could bind; the exact variant skips it).
static bool pick_degrees(const DevCode& c, bool reg2, int* dc, int* dv, int* reg) {
  static const int exact[][2] = {{2, 2}, {4, 2}, {6, 2}, {4, 4}, {6, 3}};
  if (c.regular) {
    for (auto& e : exact)
      if (e[0] == c.dcmax && e[1] == c.dvmax && (reg2 || e[1] != 2)) {
        *dc = e[0];
        *dv = e[1];
        *reg = 1;
        return true;
      }
  }
  if (c.dcmax <= 6 && c.dvmax <= 2) {
    *dc = 6;
    *dv = 2;
    *reg = 0;
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

static const ResVariant* find_variant(int dc, int dv, int cpt, int bp, int reg, int tile = 0) {
  for (const auto& v : kResVariants)
    if (v.dc == dc && v.dv == dv && v.cpt == cpt && v.bp == bp && v.reg == reg && v.tile == tile) return &v;
  return nullptr;
}

// msg, scratch words, flip and correction bitmaps (n bits each), syndrome
// bitmap (m bits), initial-error bitmap (n bits); with the sequential
// conflict rule also a ring time
// (m words) and a request byte (m bytes) per check
static size_t group_bytes_for(int dc, int mpad, int n, int m, bool seq) {
  size_t b = (size_t)(dc * (mpad / 64) * kSlotStride + kGroupWords + 3 * ((n + 31) / 32) + (m + 31) / 32) * 4;
  if (seq) b += (size_t)m * 5;
  return (b + 15) / 16 * 16;
}

bool resident_shape(const DevCode& c, int bp, const laim_resident_cfg* want, ResidentShape* out,
                    int device, bool seq, bool reg2) {
  int dc, dv, reg;
  if (!pick_degrees(c, reg2, &dc, &dv, &reg)) {
    set_error("resident form needs check degree <= 8 and qubit degree <= 4 (have %d, %d)", c.dcmax,
              c.dvmax);
    return false;
  }
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
          hipSuccess ||
      lds_max <= 0)
    lds_max = 64 * 1024;
  int cpt = want ? want->checks_per_thread : 0;
  int nt = want ? want->threads_per_shot : 0;
  int spb = want ? want->shots_per_block : 0;
  // min-sum on the 2D toric layout: the tiled variant, faster than the
  // other shapes at every L measured (8 to 64)
  const bool tile_ok = c.tile_chk && bp == 0 && dc == 4 && dv == 2 && reg && !seq;
  if (cpt <= 0 && nt <= 0 && tile_ok) cpt = 8;
  if (cpt <= 0) {
    if (nt > 0)
      cpt = (c.m + nt - 1) / nt;
    else
      cpt = (c.m <= 256) ? 1 : (c.m <= 512 ? 2 : (c.m <= 1024 ? 4 : 8));
    int allowed[] = {1, 2, 4, 8};
    int pick = -1;
    for (int a : allowed)
      if (a >= cpt && find_variant(dc, dv, a, bp, reg)) {
        pick = a;
        break;
      }
    if (pick < 0)
      for (int i = 3; i >= 0; --i)
        if (find_variant(dc, dv, allowed[i], bp, reg)) {
          pick = allowed[i];
          break;
        }
    cpt = pick;
  }
  if (!find_variant(dc, dv, cpt, bp, reg)) {
    set_error("no resident kernel for checks_per_thread = %d (degrees %d/%d)", cpt, dc, dv);
    return false;
  }
  if (nt <= 0) nt = (c.m + cpt - 1) / cpt;
  if (nt * cpt < c.m) {
    set_error("threads_per_shot * checks_per_thread = %d < m = %d", nt * cpt, c.m);
    return false;
  }
  const int vpt = (c.n + nt - 1) / nt;
  if (spb <= 0 && tile_ok && cpt == 8 && nt * 8 == c.m) {
    // blocks near 128 threads with wavefronts at least 80% full (measured:
    // 128 threads best at L = 8 and 32, 216 at L = 24, 64-128 at L = 16)
    int best = 0, gap = 0;
    for (int s = 1; nt * s <= kTileMaxThreads; ++s) {
      const int th = nt * s, waves = (th + 63) / 64;
      if (5 * th < 4 * 64 * waves) continue;
      const int d = th > 128 ? th - 128 : 128 - th;
      if (!best || d < gap) {
        best = s;
        gap = d;
      }
    }
    spb = best > 0 ? best : 1;
  }
  if (spb <= 0) spb = (nt >= 256) ? 1 : 256 / nt;
  if (spb > kMaxShotsPerBlock) spb = kMaxShotsPerBlock;
  if (nt * spb > 1024) {
    set_error("block of %d threads exceeds 1024", nt * spb);
    return false;
  }
  const int mpad = (nt * cpt + 63) / 64 * 64;
  const size_t gb = group_bytes_for(dc, mpad, c.n, c.m, seq);
  const size_t lds = kCtrlWords * 4 + gb * (size_t)spb;
  if (lds > (size_t)lds_max) {
    set_error("resident form needs %zu bytes of LDS per block (device limit %d)", lds, lds_max);
    return false;
  }
  out->nt = nt;
  out->cpt = cpt;
  out->vpt = vpt;
  out->spb = spb;
  out->mpad = mpad;
  out->group_bytes = (int32_t)gb;
  out->lds = lds;
  out->dc = dc;
  out->dv = dv;
  out->reg = reg;
  // the tiled variant: min-sum on the 2D toric layout with its shape (8
  // checks per thread, m / 8 threads per shot); the sequential rule keeps
  // the plain variant
  out->tile = (c.tile_chk && bp == 0 && dc == 4 && dv == 2 && reg && cpt == 8 && nt * 8 == c.m && !seq &&
               nt * spb <= kTileMaxThreads) ? 1 : 0;
  return true;
}


// Variant and unit shape of a code inside the multi-code kernels. The
// launch shape follows the code's resident shape, with checks per thread
// limited to the compiled variants (at most the shape's value).
bool batch_variant(const DevCode& c, int bp, const laim_resident_cfg* want, int device, bool seq,
                   bool reg2, UnitCtx* u, int* variant, size_t* lds, int* block) {
  ResidentShape sh;
  if (!resident_shape(c, bp, want, &sh, device, seq, reg2)) return false;
  const int dc = sh.dc, dv = sh.dv, reg = sh.reg;
  int best = -1;
  for (int i = 0; i < (int)(sizeof(kBatchVariants) / sizeof(kBatchVariants[0])); ++i) {
    const int* v = kBatchVariants[i];
    if (v[0] != dc || v[1] != dv || v[3] != reg) continue;
    if (v[2] <= sh.cpt && (best < 0 || v[2] > kBatchVariants[best][2])) best = i;
  }
  if (best < 0) {
    set_error("no batched variant for degrees %d/%d", dc, dv);
    return false;
  }
  const int cpt = kBatchVariants[best][2];
  laim_resident_cfg cfg = {0, cpt, want ? want->shots_per_block : 0};
  if (cpt != sh.cpt && !resident_shape(c, bp, &cfg, &sh, device, seq, reg2)) return false;
  u->nt = sh.nt;
  u->vpt = sh.vpt;
  u->spb = sh.spb;
  u->mpad = sh.mpad;
  u->group_bytes = sh.group_bytes;
  u->rounds = 0;
  u->resume = 0;
  u->events = 0;
  *variant = best;
  *lds = sh.lds;
  *block = sh.nt * sh.spb;
  return true;
}

hipError_t launch_server(int bp, const BatchItemDev* items, const ServerUnitDev* units,
                         int32_t nunits, const ServerReqDev* reqs, size_t lds, int block,
                         hipStream_t st) {
  if (nunits <= 0) return hipSuccess;
  const void* fn = bp ? reinterpret_cast<const void*>(server_kernel<1>)
                      : reinterpret_cast<const void*>(server_kernel<0>);
  if (lds > 64 * 1024) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
  }
  const int32_t ctrl_off = (int32_t)(lds - kCtrlWords * 4);
  if (bp)
    hipLaunchKernelGGL(server_kernel<1>, dim3(nunits), dim3(block), lds, st, items, units, reqs, ctrl_off);
  else
    hipLaunchKernelGGL(server_kernel<0>, dim3(nunits), dim3(block), lds, st, items, units, reqs, ctrl_off);
  return hipGetLastError();
}

// A shot runs every round until it retires: t_clr rounds if it cleared and
// retires, else all of them (a shot clear from the start runs none).
__global__ void __launch_bounds__(256) sweep_count_kernel(int32_t iters, int32_t rounds, int32_t retire,
                                                          const int32_t* __restrict__ tclr,
                                                          int32_t nshots, int32_t* __restrict__ sweeps) {
  const int32_t i = bid_x() * bdim_x() + tid_x();
  if (i >= nshots) return;
  const int32_t t = tclr[i];
  const int64_t k = (int64_t)iters * ((retire && t >= 0) ? t : rounds);
  sweeps[i] = (int32_t)(k < 2147483647 ? k : 2147483647);
}

hipError_t launch_sweep_count(const KParams& kp, const int32_t* tclr, int32_t nshots, int32_t* sweeps,
                              hipStream_t st) {
  if (nshots <= 0 || !sweeps) return hipSuccess;
  hipLaunchKernelGGL(sweep_count_kernel, dim3((unsigned)((nshots + 255) / 256)), dim3(256), 0, st,
                     kp.iters, kp.rounds, kp.retire, tclr, nshots, sweeps);
  return hipGetLastError();
}

size_t resident_workspace_bytes() { return 256; }

// The persistent launch of a resident kernel variant: as many blocks as fit
// on the device at once (at most one per group of shots); the shot queue
// in a.counter is cleared first by a kernel (no memset node in a graph).
static hipError_t launch_resident_args(const DevCode& c, const KParams& kp, const ResidentShape& sh,
                                       ResArgs& a, int32_t total, hipStream_t st) {
  if (sh.reg && sh.dv == 2 && !reg_dv2_ok(kp)) return hipErrorInvalidValue;
  const ResVariant* var = find_variant(sh.dc, sh.dv, sh.cpt, kp.bp, sh.reg, sh.tile);
  if (!var) return hipErrorInvalidValue;
  a.u.nt = sh.nt;
  a.u.vpt = sh.vpt;
  a.u.spb = sh.spb;
  a.u.mpad = sh.mpad;
  a.u.group_bytes = sh.group_bytes;
  a.u.rounds = kp.rounds;
  a.u.resume = 0;
  a.u.events = 0;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, st, a.counter, 1);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (sh.lds > 64 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(var->fn),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
    (void)hipGetLastError();
  }
  int per_cu = 0;
  err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(var->fn),
                                                     sh.nt * sh.spb, sh.lds);
  if (err != hipSuccess) return err;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus <= 0) cus = 256;
  const int64_t groups = ((int64_t)total + sh.spb - 1) / sh.spb;
  int64_t blocks = (int64_t)per_cu * cus;
  if (blocks > groups) blocks = groups;
  hipLaunchKernelGGL(var->fn, dim3((unsigned)blocks), dim3(sh.nt * sh.spb), sh.lds, st, c, kp, a);
  return hipGetLastError();
}

hipError_t launch_resident(const DevCode& c, const KParams& kp, const ResidentShape& sh,
                           const uint8_t* e0, uint64_t shot0, int32_t nshots, void* ws, uint8_t* z,
                           uint8_t* s, int32_t* tclr, float* L, uint8_t* fail, int32_t* sweeps,
                           hipStream_t st, const uint8_t* s0, int32_t r0) {
  if (s0 && fail) return hipErrorInvalidValue;  // the failure test needs e0
  if (nshots <= 0) return hipSuccess;
  ResArgs a;
  a.items = nullptr;
  a.nitems = 0;
  a.e0 = e0;
  a.s0 = s0;
  a.r0 = r0;
  a.shot0 = shot0;
  a.nshots = nshots;
  a.counter = reinterpret_cast<uint32_t*>(ws);
  a.z = z;
  a.s = s;
  a.tclr = tclr;
  a.L = L;
  a.fail = fail;
  a.sweeps = sweeps;
  return launch_resident_args(c, kp, sh, a, nshots, st);
}

hipError_t launch_resident_group(const DevCode& c, const KParams& kp, const ResidentShape& sh,
                                 const GroupItemDev* items, int32_t nitems, int32_t total, void* ws,
                                 hipStream_t st) {
  if (total <= 0) return hipSuccess;
  ResArgs a;
  a.items = items;
  a.nitems = nitems;
  a.e0 = nullptr;
  a.s0 = nullptr;
  a.r0 = 0;
  a.shot0 = 0;
  a.nshots = total;
  a.counter = reinterpret_cast<uint32_t*>(ws);
  a.z = nullptr;
  a.s = nullptr;
  a.tclr = nullptr;
  a.L = nullptr;
  a.fail = nullptr;
  a.sweeps = nullptr;
  return launch_resident_args(c, kp, sh, a, total, st);
}

}  // namespace laim
