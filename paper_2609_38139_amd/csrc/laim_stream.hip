// laim_stream.hip -- the stream form of the decoder: BP messages in HBM,
// one launch per sweep, plus the per-round feedback kernels. As in the
// resident form only m_{c->v} is stored; each sweep recomputes
// m_{v->c} = clamp(pi + sum_{c' != c} m_{c'->v}) in ascending check order
// where the check phase reads it (Eqs. (BP-LLR1), (BP-LLR2)).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.h"
#include "laim_internal.h"

namespace laim {

// ====================================================================
// Stream form: messages live in HBM in tiles of 256 shots,
// msg[tile][edge][shot in tile] with edges in ELL order (c * dcmax + j).
// A wavefront handles one row (one check or qubit, all shots of a tile);
// lane l holds shots 4l .. 4l + 3, so every data access is a contiguous
// row (1 KiB of messages, 256 B of bytes) read or written with 16- or
// 4-byte vector accesses, and every graph lookup is uniform across the
// wavefront. One launch per BP sweep (double-buffered m_{c->v}) and a few
// small launches per round for the feedback step.
// ====================================================================
constexpr int kSV = 4;  // shots per lane
static_assert(kStreamTile == 64 * kSV, "a stream tile is one wavefront of kSV shots per lane");

struct StreamWS {
  float* msg[2];     // [ntile][m * dcmax][kStreamTile]
  uint8_t* s;        // [ntile][m][kStreamTile]
  uint8_t* z;        // [ntile][n][kStreamTile]
  uint8_t* fl;       // [ntile][n][kStreamTile]
  uint32_t* anys;    // [ntile * kStreamTile]
  int32_t* tclr;     // [ntile * kStreamTile]
  uint8_t* done;     // [ntile * kStreamTile]: retired (or frozen) shots and the last tile's padding
  uint8_t* newdone;  // [ntile * kStreamTile]
  // exact shortcuts (kp.skip), per shot:
  uint8_t* conv;     // the messages are a fixed point of the sweep for the current syndrome
  uint8_t* chg;      // a compared sweep changed a message
  uint8_t* evid;     // an active check passed Evidence in this round's feedback step
  // live-shot compaction (with the exact shortcuts):
  int32_t* sid;      // [ntile * kStreamTile]: the shot (0 .. nshots - 1) in each slot, -1 for none
  int32_t* sid2;     // [ntile * kStreamTile]: scratch
  int32_t* inv;      // [ntile * kStreamTile]: new slot -> old slot of a compaction
  int32_t* ctl;      // [4]: tiles in use, compaction pending, live shots, tiles after it
  uint8_t* s2;       // [ntile][m][kStreamTile]: scratch
  // sequential conflict rule only (else null)
  uint8_t* rq;       // [ntile][m][kStreamTile]: slot of the requested qubit (bits 0-6,
                     //   kStreamNoRequest if none), bit 7 whether the request applies
  uint32_t* rkey;    // [ntile][m][kStreamTile]: ring time of the request
};

constexpr uint8_t kStreamNoRequest = 0x7F;

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static StreamWS stream_carve(const DevCode& c, int32_t nshots, void* ws, size_t* total, bool seq) {
  const int64_t ntile = ((int64_t)nshots + kStreamTile - 1) / kStreamTile;
  const int64_t ns = ntile * kStreamTile;
  const size_t msg_b = align256((size_t)ns * c.m * c.dcmax * 4);
  const size_t s_b = align256((size_t)ns * c.m);
  const size_t z_b = align256((size_t)ns * c.n);
  const size_t sh4 = align256((size_t)ns * 4);
  const size_t sh1 = align256((size_t)ns);
  StreamWS w;
  char* p = reinterpret_cast<char*>(ws);
  size_t off = 0;
  w.msg[0] = reinterpret_cast<float*>(p + off);
  off += msg_b;
  w.msg[1] = reinterpret_cast<float*>(p + off);
  off += msg_b;
  w.s = reinterpret_cast<uint8_t*>(p + off);
  off += s_b;
  w.z = reinterpret_cast<uint8_t*>(p + off);
  off += z_b;
  w.fl = reinterpret_cast<uint8_t*>(p + off);
  off += z_b;
  w.anys = reinterpret_cast<uint32_t*>(p + off);
  off += sh4;
  w.tclr = reinterpret_cast<int32_t*>(p + off);
  off += sh4;
  w.done = reinterpret_cast<uint8_t*>(p + off);
  off += sh1;
  w.newdone = reinterpret_cast<uint8_t*>(p + off);
  off += sh1;
  w.conv = reinterpret_cast<uint8_t*>(p + off);
  off += sh1;
  w.chg = reinterpret_cast<uint8_t*>(p + off);
  off += sh1;
  w.evid = reinterpret_cast<uint8_t*>(p + off);
  off += sh1;
  w.sid = reinterpret_cast<int32_t*>(p + off);
  off += sh4;
  w.sid2 = reinterpret_cast<int32_t*>(p + off);
  off += sh4;
  w.inv = reinterpret_cast<int32_t*>(p + off);
  off += sh4;
  w.ctl = reinterpret_cast<int32_t*>(p + off);
  off += 256;
  w.s2 = reinterpret_cast<uint8_t*>(p + off);
  off += s_b;
  w.rq = nullptr;
  w.rkey = nullptr;
  if (seq) {
    w.rq = reinterpret_cast<uint8_t*>(p + off);
    off += s_b;
    w.rkey = reinterpret_cast<uint32_t*>(p + off);
    off += align256((size_t)ns * c.m * 4);
  }
  if (total) *total = off;
  return w;
}

size_t stream_workspace_bytes(const DevCode& c, int32_t nshots, bool seq) {
  size_t t = 0;
  stream_carve(c, nshots, nullptr, &t, seq);
  return t;
}

constexpr int kStreamRowsPerBlock = 4;  // 256 threads: one row per wavefront

// Row handled by this wavefront (uniform, so table reads become scalar loads).
__device__ __forceinline__ int32_t stream_row() {
  return (int32_t)bid_x() * kStreamRowsPerBlock + __builtin_amdgcn_readfirstlane(tid_x() >> 6);
}

// Offset of this lane's first shot in row `row` of tile `tile` of an array of rows.
__device__ __forceinline__ int64_t stream_at(int64_t tile, int32_t rows, int64_t row, int32_t lane) {
  return (tile * rows + row) * kStreamTile + kSV * lane;
}

__device__ __forceinline__ uint32_t ld4b(const uint8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }

// Messages stream through HBM, each read once per sweep: non-temporal
// 16-byte accesses.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 nt_load4(const float* p) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store4(float* p, float a, float b, float c, float d) {
  f32x4 v = {a, b, c, d};
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
}
__device__ __forceinline__ void st4b(uint8_t* p, uint32_t v) { *reinterpret_cast<uint32_t*>(p) = v; }

// Shot start: z = 0, no flip requests.
__global__ void __launch_bounds__(256) stream_init_var(DevCode c, StreamWS w) {
  const int32_t lane = tid_x() & 63;
  const int32_t v = stream_row();
  if (v >= c.n) return;
  const int64_t o = stream_at(bid_y(), c.n, v, lane);
  st4b(w.z + o, 0u);
  st4b(w.fl + o, 0u);
}

// Shot start: s = H e0 (or s0 when given) and messages 0 (shots beyond
// nshots get s = 0).
__global__ void __launch_bounds__(256) stream_init_chk(DevCode c, StreamWS w, const uint8_t* e0,
                                                       const uint8_t* s0, int32_t nshots) {
  const int32_t lane = tid_x() & 63;
  const int32_t ch = stream_row();
  const int64_t tile = bid_y();
  if (ch >= c.m) return;
  const int32_t d = c.chk_deg[ch];
  uint32_t x4 = 0;
#pragma unroll
  for (int q = 0; q < kSV; ++q) {
    const int64_t i = tile * kStreamTile + kSV * lane + q;
    if (i >= nshots) continue;
    uint32_t x = 0;
    if (s0)
      x = s0[i * c.m + ch];
    else
      for (int32_t j = 0; j < d; ++j) x ^= e0[i * c.n + c.chk_var[(int64_t)ch * c.dcmax + j]];
    x &= 1u;
    x4 |= x << (8 * q);
    if (x) w.anys[i] = 1u;
  }
  st4b(w.s + stream_at(tile, c.m, ch, lane), x4);
  if (w.rq) st4b(w.rq + stream_at(tile, c.m, ch, lane), 0x01010101u * kStreamNoRequest);
  for (int32_t j = 0; j < c.dcmax; ++j)
    *reinterpret_cast<float4*>(w.msg[0] + stream_at(tile, c.m * c.dcmax, (int64_t)ch * c.dcmax + j, lane)) =
        make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// The check rule for one shot: x[j] = m_{v->c} of the check's j-th qubit
// (j < d), out[j] = m_{c->v}.
template <int DCT>
__device__ __forceinline__ void stream_check_rule(const KParams& kp, const float* x, int32_t d,
                                                  uint32_t sigma_neg, float* out) {
  const float C = kp.clamp;
  if (kp.bp == 0) {
    float mn1 = __builtin_inff(), mn2 = __builtin_inff();
    uint32_t par = sigma_neg;
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      if (j >= d) continue;
      const float av = fabsf(x[j]);
      par ^= (x[j] < 0.0f) ? 1u : 0u;
      mn2 = fminf(mn2, fmaxf(mn1, av));
      mn1 = fminf(mn1, av);
    }
    const float m1 = clampf(kp.alpha * mn1, C);
    const float m2 = clampf(kp.alpha * mn2, C);
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      if (j >= d) continue;
      const float mag = (fabsf(x[j]) == mn1) ? m2 : m1;
      const uint32_t ng = par ^ ((x[j] < 0.0f) ? 1u : 0u);
      out[j] = ng ? -mag : mag;
    }
  } else {
    float acc[DCT];
    boxplus_others<DCT, false>(x, d, acc);
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      if (j >= d) continue;
      out[j] = clampf(sigma_neg ? -acc[j] : acc[j], C);
    }
  }
}

// m_{v->c} for the d slots of one check and the kSV shots of this lane:
// pi plus the PW partner messages of each slot in ascending check order.
// `mine` holds entry `lane` of the check's partner block. Every load is
// issued before any is used, and without branches: a missing partner reads
// the tile's first row instead and contributes +0, which leaves the sum
// unchanged (the sum starts at pi, which is never -0, so it is never -0).
template <int DCT, int PW>
__device__ __forceinline__ void stream_gather(const DevCode& c, const float* __restrict__ src, int64_t tile,
                                              int32_t erows, int32_t lane, int32_t mine, int32_t d,
                                              int32_t pstride, bool live, float4* acc) {
  int32_t eix[PW][DCT];
  float4 v[PW][DCT];
#pragma unroll
  for (int p = 0; p < PW; ++p) {
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      const int32_t e = __builtin_amdgcn_readlane(mine, j * pstride + p);
      eix[p][j] = (j < d) ? e : -1;
      v[p][j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
  if (live) {  // a lane whose shots are all idle requests no memory
#pragma unroll
    for (int p = 0; p < PW; ++p) {
#pragma unroll
      for (int j = 0; j < DCT; ++j) {
        const int32_t e = eix[p][j];
        const int64_t row = (e >= 0) ? (int64_t)edge_check(e) * c.dcmax + edge_slot(e) : 0;
        v[p][j] = nt_load4(src + stream_at(tile, erows, row, lane));
      }
    }
  }
#pragma unroll
  for (int p = 0; p < PW; ++p) {
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      const bool ok = eix[p][j] >= 0;
      acc[j].x = acc[j].x + (ok ? v[p][j].x : 0.0f);
      acc[j].y = acc[j].y + (ok ? v[p][j].y : 0.0f);
      acc[j].z = acc[j].z + (ok ? v[p][j].z : 0.0f);
      acc[j].w = acc[j].w + (ok ? v[p][j].w : 0.0f);
    }
  }
}

// One BP sweep: m_{c->v} (src) -> m_{c->v} (dst), one wavefront per (tile,
// check). `fresh` marks the first sweep of every shot (m_{v->c} = 0). A tile
// whose shots have all retired is skipped; the other tiles are swept whole,
// since the messages of retired shots are never read again.
//
// Exact shortcuts (kp.skip): a compared sweep (`cmp`) also reads the old
// messages of its own rows and marks every shot one of whose messages
// changed (w.chg); stream_conv then records the shots whose messages are a
// fixed point of the sweep (w.conv). The sweep is a fixed map of the
// messages while the syndrome does not change, so at a fixed point every
// later sweep rewrites the same values, and both message buffers already
// hold them: a tile whose shots are all retired or at a fixed point skips
// the sweep, and within a swept tile a lane whose four shots are all idle
// (retired, or with the shortcuts at a fixed point) neither reads nor
// writes; the outputs are those of sweeping everything. (Retired shots'
// messages are never read again.)
template <int DCT>
__global__ void __launch_bounds__(256) stream_sweep(DevCode c, KParams kp, StreamWS w,
                                                    const float* __restrict__ src,
                                                    float* __restrict__ dst, int32_t fresh, int32_t cmp) {
  const int32_t lane = tid_x() & 63;
  const int32_t ch = stream_row();
  const int64_t tile = bid_y();
  if (ch >= c.m || tile >= w.ctl[0]) return;
  const float C = kp.clamp;
  const int32_t pw = c.dvmax - 1;           // partners per edge
  const int32_t pstride = pw > 0 ? pw : 1;  // the partner table's row length
  const int32_t erows = c.m * c.dcmax;
  const int32_t nidx = c.dcmax * pstride;   // partner entries of this check
  // The check's degree and partner edges are wavefront-uniform: lane l loads
  // entry l of the check's partner block, and every edge is then broadcast
  // from its lane, so all table reads cost one memory round trip; they and
  // the syndrome bytes are requested together with the retirement flags.
  const int32_t* pblk = c.partner + (int64_t)ch * nidx;
  const int32_t mine_raw = pblk[lane < nidx ? lane : 0];  // in bounds for every lane
  const int32_t d_raw = c.chk_deg[ch];
  const uint32_t s4 = ld4b(w.s + stream_at(tile, c.m, ch, lane));
  uint32_t idle4 = ld4b(w.done + tile * kStreamTile + kSV * lane);
  if (kp.skip) idle4 |= ld4b(w.conv + tile * kStreamTile + kSV * lane);
  if (!__any(idle4 != 0x01010101u)) return;
  const bool live = idle4 != 0x01010101u;
  const int32_t mine = (lane < nidx) ? mine_raw : -1;
  const int32_t d = __builtin_amdgcn_readfirstlane(d_raw);
  float4 acc[DCT];
#pragma unroll
  for (int j = 0; j < DCT; ++j) acc[j] = make_float4(kp.pi, kp.pi, kp.pi, kp.pi);
  if (DCT <= 8 && nidx <= 64 && pw == 1)
    stream_gather<DCT, 1>(c, src, tile, erows, lane, mine, d, pstride, live, acc);
  else if (DCT <= 8 && nidx <= 64 && pw == 2)
    stream_gather<DCT, 2>(c, src, tile, erows, lane, mine, d, pstride, live, acc);
  else if (DCT <= 8 && nidx <= 64 && pw == 3)
    stream_gather<DCT, 3>(c, src, tile, erows, lane, mine, d, pstride, live, acc);
  else if (live) {
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      if (j >= d) continue;
      for (int32_t p = 0; p < pw; ++p) {
        const int32_t e = pblk[j * pstride + p];
        if (e < 0) break;
        const float4 w4 = *reinterpret_cast<const float4*>(
            src + stream_at(tile, erows, (int64_t)edge_check(e) * c.dcmax + edge_slot(e), lane));
        acc[j].x = acc[j].x + w4.x;
        acc[j].y = acc[j].y + w4.y;
        acc[j].z = acc[j].z + w4.z;
        acc[j].w = acc[j].w + w4.w;
      }
    }
  }
  float x[kSV][DCT];
#pragma unroll
  for (int j = 0; j < DCT; ++j) {
    if (j >= d) continue;
    x[0][j] = fresh ? 0.0f : clampf(acc[j].x, C);
    x[1][j] = fresh ? 0.0f : clampf(acc[j].y, C);
    x[2][j] = fresh ? 0.0f : clampf(acc[j].z, C);
    x[3][j] = fresh ? 0.0f : clampf(acc[j].w, C);
  }
  float4 old[DCT];
  if (cmp && live) {
#pragma unroll
    for (int j = 0; j < DCT; ++j)
      if (j < d) old[j] = nt_load4(src + stream_at(tile, erows, (int64_t)ch * c.dcmax + j, lane));
  }
  float out[kSV][DCT];
#pragma unroll
  for (int q = 0; q < kSV; ++q)
    stream_check_rule<DCT>(kp, x[q], d, ((s4 >> (8 * q)) ^ (uint32_t)d) & 1u, out[q]);
  if (!live) return;
#pragma unroll
  for (int j = 0; j < DCT; ++j) {
    if (j >= d) continue;
    // streamed out: read once, by the partner gather of the next sweep
    nt_store4(dst + stream_at(tile, erows, (int64_t)ch * c.dcmax + j, lane), out[0][j], out[1][j], out[2][j],
              out[3][j]);
  }
  if (cmp) {
    uint32_t dq[kSV] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      if (j >= d) continue;
      dq[0] |= __float_as_uint(out[0][j]) ^ __float_as_uint(old[j].x);
      dq[1] |= __float_as_uint(out[1][j]) ^ __float_as_uint(old[j].y);
      dq[2] |= __float_as_uint(out[2][j]) ^ __float_as_uint(old[j].z);
      dq[3] |= __float_as_uint(out[3][j]) ^ __float_as_uint(old[j].w);
    }
    // every writer stores the same value: plain byte stores suffice
#pragma unroll
    for (int q = 0; q < kSV; ++q)
      if (dq[q]) w.chg[tile * kStreamTile + kSV * lane + q] = 1;
  }
}

// After a compared sweep: a live shot none of whose messages changed is at a
// fixed point (kept until its syndrome changes); the change marks are cleared.
__global__ void __launch_bounds__(256) stream_conv(StreamWS w, int32_t ntot) {
  const int32_t i = bid_x() * bdim_x() + tid_x();
  if (i >= ntot) return;
  if (!w.done[i]) w.conv[i] = w.chg[i] ? 0 : 1;
  w.chg[i] = 0;
}

// Belief of qubit v for shot column `col` of a tile.
__device__ __forceinline__ float stream_belief(const DevCode& c, const float* msg, int64_t tile,
                                               int32_t col, int32_t v, float pi, float C) {
  float acc = pi;
  const int32_t dv = c.var_deg[v];
  for (int32_t q = 0; q < dv; ++q) {
    const int32_t e = c.var_edge[(int64_t)v * c.dvmax + q];
    acc = acc + msg[((tile * c.m + edge_check(e)) * c.dcmax + edge_slot(e)) * kStreamTile + col];
  }
  return clampf(acc, C);
}

// One shot's move request from the beliefs Lv of the check's d qubits:
// Evidence first, then the clock, then the tie pick; the request is
// recorded by the conflict rule.
template <int DCT>
__device__ __forceinline__ void stream_request(const DevCode& c, const KParams& kp, StreamWS& w, int32_t ch,
                                               int32_t d, const int32_t* nb, const float* Lv, int64_t tile,
                                               int32_t lane, int32_t q, int32_t r, uint64_t shot0) {
  const int32_t col = kSV * lane + q;
  const uint64_t shot = shot0 + (uint64_t)w.sid[tile * kStreamTile + col];
  float Lmax = 0.0f;
#pragma unroll
  for (int j = 0; j < DCT; ++j)
    if (j < d && (j == 0 || Lv[j] > Lmax)) Lmax = Lv[j];
  if (kp.evidence && !(Lmax >= c.thr[d])) return;  // Evidence first, then the clock
  if (kp.skip) w.evid[tile * kStreamTile + col] = 1;
  const Philox4 rw = philox4x32_10((uint32_t)shot, (uint32_t)(shot >> 32), (uint32_t)ch,
                                   ((uint32_t)r << 4) | 1u, (uint32_t)kp.seed, (uint32_t)(kp.seed >> 32));
  if (!below(rw.w0, kp.mask_bound)) return;
  uint32_t ntie = 0;
#pragma unroll
  for (int j = 0; j < DCT; ++j)
    if (j < d) ntie += (Lv[j] == Lmax) ? 1u : 0u;
  uint32_t pick = (uint32_t)(((uint64_t)rw.w1 * (uint64_t)ntie) >> 32);
  int32_t slot = -1;
#pragma unroll
  for (int j = 0; j < DCT; ++j) {
    if (j < d && Lv[j] == Lmax && slot < 0) {
      if (pick == 0)
        slot = j;
      else
        --pick;
    }
  }
  if (slot < 0) return;
  if (kp.conflict == kConflictSequential) {
    // recorded, provisionally applying; resolved by stream_resolve
    // (single-qubit moves only: the host refuses multi-qubit ones here)
    const int64_t o = stream_at(tile, c.m, ch, lane) + q;
    w.rkey[o] = rw.w2;
    w.rq[o] = (uint8_t)(0x80 | slot);
    return;
  }
  // the LocalMove qubit, or for a multi-qubit move every qubit of the check
  // with a positive belief (if any)
  bool multi = false;
  if (kp.move) {
#pragma unroll
    for (int j = 0; j < DCT; ++j) multi |= (j < d && Lv[j] > 0.0f);
  }
#pragma unroll
  for (int j = 0; j < DCT; ++j) {
    if (j >= d || !(multi ? (Lv[j] > 0.0f) : (j == slot))) continue;
    const int64_t fo = (tile * c.n + nb[j]) * kStreamTile + col;
    if (kp.conflict == kConflictOr)
      w.fl[fo] = 1;
    else  // XOR: the byte of this shot in the 4-byte word holding it
      atomicXor(reinterpret_cast<uint32_t*>(w.fl + (fo & ~(int64_t)3)), 1u << (8 * (fo & 3)));
  }
}

// Adds to L4[j] (pi for 4 shots) the messages m_{c->v} of the DV edges of
// the qubit in slot j, in ascending check order; `el` holds, in lane
// j * DV + q, edge q of that qubit (or -1). Every message row is requested
// before the first add.
template <int DCT, int DV>
__device__ __forceinline__ void stream_belief_rows(const DevCode& c, const float* __restrict__ msg, int64_t tile,
                                                   int32_t erows, int32_t lane, int32_t el, float4* L4) {
  int32_t eix[DV][DCT];
  float4 v[DV][DCT];
#pragma unroll
  for (int q = 0; q < DV; ++q) {
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      const int32_t e = __builtin_amdgcn_readlane(el, j * DV + q);
      eix[q][j] = e;
      const int64_t row = (e >= 0) ? (int64_t)edge_check(e) * c.dcmax + edge_slot(e) : 0;
      v[q][j] = *reinterpret_cast<const float4*>(msg + stream_at(tile, erows, row, lane));
    }
  }
#pragma unroll
  for (int q = 0; q < DV; ++q) {
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      const bool ok = eix[q][j] >= 0;
      L4[j].x = L4[j].x + (ok ? v[q][j].x : 0.0f);
      L4[j].y = L4[j].y + (ok ? v[q][j].y : 0.0f);
      L4[j].z = L4[j].z + (ok ? v[q][j].z : 0.0f);
      L4[j].w = L4[j].w + (ok ? v[q][j].w : 0.0f);
    }
  }
}

// Feedback: active checks whose Evidence holds and whose clock rang request
// a flip of their LocalMove qubit. One wavefront per (tile, check); a
// wavefront with no active shot leaves at once. For checks of degree <= 8
// whose qubits have degree <= kMovesMaxDv, the beliefs of the check's
// qubits are computed for all 4 shots of a lane at once: the check's qubits
// and their edges are wavefront-uniform (loaded cooperatively, broadcast by
// readlane), and every message row is requested before the first add. A
// missing edge reads a valid row and adds +0, exact since the sum starts at
// pi (never -0).
constexpr int kMovesMaxDv = 4;
template <int DCT>
__global__ void __launch_bounds__(256) stream_moves(DevCode c, KParams kp, StreamWS w,
                                                    const float* __restrict__ msg, int32_t r,
                                                    int32_t fresh, uint64_t shot0) {
  const int32_t lane = tid_x() & 63;
  const int32_t ch = stream_row();
  const int64_t tile = bid_y();
  if (ch >= c.m || tile >= w.ctl[0]) return;
  const uint32_t s4 = ld4b(w.s + stream_at(tile, c.m, ch, lane));
  const uint32_t dn = ld4b(w.done + tile * kStreamTile + kSV * lane);
  const uint32_t act = s4 & ~dn & 0x01010101u;
  if (!__any(act != 0u)) return;
  const int32_t d = __builtin_amdgcn_readfirstlane(c.chk_deg[ch]);
  if (d == 0) return;
  const int32_t* nb = c.chk_var + (int64_t)ch * c.dcmax;
  const int32_t dvm = c.dvmax;
  if (DCT <= 8 && dvm <= kMovesMaxDv) {
    // lane l: qubit of slot l, and edge (l mod dvm) of the qubit of slot l / dvm
    const int32_t nbl = nb[lane < c.dcmax ? lane : 0];
    const int32_t jl = lane / dvm;
    const int32_t ql = lane - jl * dvm;
    // slots j >= d hold no qubit (-1): read slot 0's entries there instead
    const int32_t vq = __shfl(nbl, jl < d ? jl : 0);
    const int32_t el_raw = c.var_edge[(int64_t)vq * dvm + ql];
    const int32_t el = (jl < d) ? el_raw : -1;
    const int32_t erows = c.m * c.dcmax;
    float4 L4[DCT];
#pragma unroll
    for (int j = 0; j < DCT; ++j) L4[j] = make_float4(kp.pi, kp.pi, kp.pi, kp.pi);
    if (!fresh) {  // on a fresh sweep every message is +0 and L = pi
      if (dvm == 1)
        stream_belief_rows<DCT, 1>(c, msg, tile, erows, lane, el, L4);
      else if (dvm == 2)
        stream_belief_rows<DCT, 2>(c, msg, tile, erows, lane, el, L4);
      else if (dvm == 3)
        stream_belief_rows<DCT, 3>(c, msg, tile, erows, lane, el, L4);
      else
        stream_belief_rows<DCT, 4>(c, msg, tile, erows, lane, el, L4);
    }
    float Lq[kSV][DCT];
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      Lq[0][j] = clampf(L4[j].x, kp.clamp);
      Lq[1][j] = clampf(L4[j].y, kp.clamp);
      Lq[2][j] = clampf(L4[j].z, kp.clamp);
      Lq[3][j] = clampf(L4[j].w, kp.clamp);
    }
#pragma unroll
    for (int q = 0; q < kSV; ++q)
      if ((act >> (8 * q)) & 1u) stream_request<DCT>(c, kp, w, ch, d, nb, Lq[q], tile, lane, q, r, shot0);
    return;
  }
#pragma unroll 1
  for (int q = 0; q < kSV; ++q) {
    if (!((act >> (8 * q)) & 1u)) continue;
    const int32_t col = kSV * lane + q;
    float Lv[DCT];
#pragma unroll
    for (int j = 0; j < DCT; ++j) {
      if (j >= d) continue;
      float L;
      if (fresh) {
        L = kp.pi;
        for (int32_t qq = 0; qq < c.var_deg[nb[j]]; ++qq) L = L + 0.0f;
        L = clampf(L, kp.clamp);
      } else {
        L = stream_belief(c, msg, tile, col, nb[j], kp.pi, kp.clamp);
      }
      Lv[j] = L;
    }
    stream_request<DCT>(c, kp, w, ch, d, nb, Lv, tile, lane, q, r, shot0);
  }
}

// Sequential conflict rule: request i applies iff its check's start
// syndrome (1), toggled by every applied request that rang earlier (ring
// time, then check index) and asks for a qubit of the check, is 1. One
// thread per shot relaxes the requests of its shot in place, pass after
// pass over the checks; the requests form a directed acyclic graph in
// ring-time order, so a pass without change comes after at most (longest
// chain + 2) passes. Then the applied requests become flip requests
// (f ^= e_v) and the records are cleared.
__global__ void __launch_bounds__(256) stream_resolve(DevCode c, StreamWS w) {
  const int32_t col = tid_x();
  const int64_t tile = bid_x();
  if (tile >= w.ctl[0] || w.done[tile * kStreamTile + col]) return;
  uint8_t* rq = w.rq + tile * c.m * kStreamTile + col;
  const uint32_t* rk = w.rkey + tile * c.m * kStreamTile + col;
#pragma unroll 1
  for (int32_t pass = 0; pass <= c.m + 1; ++pass) {
    bool changed = false;
#pragma unroll 1
    for (int32_t ch = 0; ch < c.m; ++ch) {
      const uint32_t cur = rq[(int64_t)ch * kStreamTile];
      if ((cur & 0x7Fu) == kStreamNoRequest) continue;
      const uint32_t key = rk[(int64_t)ch * kStreamTile];
      const int32_t d = c.chk_deg[ch];
      uint32_t x = 1u;
      for (int32_t j = 0; j < d; ++j) {
        const int32_t v = c.chk_var[(int64_t)ch * c.dcmax + j];
        for (int32_t q = 0; q < c.var_deg[v]; ++q) {
          const int32_t e = c.var_edge[(int64_t)v * c.dvmax + q];
          const int32_t c2 = edge_check(e);
          const uint32_t r2 = rq[(int64_t)c2 * kStreamTile];
          if (c2 == ch || (r2 & 0x7Fu) != (uint32_t)edge_slot(e)) continue;
          const uint32_t k2 = rk[(int64_t)c2 * kStreamTile];
          if (k2 < key || (k2 == key && c2 < ch)) x ^= r2 >> 7;
        }
      }
      if ((cur >> 7) != x) {
        rq[(int64_t)ch * kStreamTile] = (uint8_t)((x << 7) | (cur & 0x7Fu));
        changed = true;
      }
    }
    if (!changed) break;
  }
#pragma unroll 1
  for (int32_t ch = 0; ch < c.m; ++ch) {
    const uint32_t cur = rq[(int64_t)ch * kStreamTile];
    if ((cur & 0x7Fu) == kStreamNoRequest) continue;
    rq[(int64_t)ch * kStreamTile] = kStreamNoRequest;
    if (!(cur >> 7)) continue;
    const int32_t v = c.chk_var[(int64_t)ch * c.dcmax + (cur & 0x7Fu)];
    uint8_t* f = w.fl + (tile * c.n + v) * kStreamTile + col;
    *f = (uint8_t)(*f ^ 1u);
  }
}

// s ^= H f for live shots; flags shots with s != 0 and clears the fixed-point
// mark of shots whose syndrome changed.
__global__ void __launch_bounds__(256) stream_syndrome(DevCode c, StreamWS w) {
  const int32_t lane = tid_x() & 63;
  const int32_t ch = stream_row();
  const int64_t tile = bid_y();
  if (ch >= c.m || tile >= w.ctl[0]) return;
  const uint32_t live = ~ld4b(w.done + tile * kStreamTile + kSV * lane) & 0x01010101u;
  if (!live) return;
  const int32_t d = c.chk_deg[ch];
  uint32_t x4 = 0;
  for (int32_t j = 0; j < d; ++j)
    x4 ^= ld4b(w.fl + stream_at(tile, c.n, c.chk_var[(int64_t)ch * c.dcmax + j], lane));
  const int64_t so = stream_at(tile, c.m, ch, lane);
  const uint32_t flip = x4 & live;
  const uint32_t s4 = ld4b(w.s + so) ^ flip;
  st4b(w.s + so, s4);
  const uint32_t hit = s4 & live;
#pragma unroll
  for (int q = 0; q < kSV; ++q) {
    if ((hit >> (8 * q)) & 1u) w.anys[tile * kStreamTile + kSV * lane + q] = 1u;
    // a changed syndrome changes the sweep: no longer at a fixed point
    if ((flip >> (8 * q)) & 1u) w.conv[tile * kStreamTile + kSV * lane + q] = 0;
  }
}

// z ^= f and clear the requests (requests exist for live shots only).
__global__ void __launch_bounds__(256) stream_apply(DevCode c, StreamWS w) {
  const int32_t lane = tid_x() & 63;
  const int32_t v = stream_row();
  if (v >= c.n || (int32_t)bid_y() >= w.ctl[0]) return;
  const int64_t o = stream_at(bid_y(), c.n, v, lane);
  const uint32_t f4 = ld4b(w.fl + o);
  if (!f4) return;
  st4b(w.z + o, ld4b(w.z + o) ^ f4);
  st4b(w.fl + o, 0u);
}

// Per shot: t_clr at the first clear syndrome, retirement. With the exact
// shortcuts a shot also stops (frozen) when its messages were a fixed point
// at the feedback step and no active check passed Evidence: nothing was
// requested, so the syndrome is unchanged, the next round repeats this one
// exactly, and so does every later one -- the outputs are final.
__global__ void __launch_bounds__(256) stream_status(KParams kp, StreamWS w, int32_t r,
                                                     int32_t nshots) {
  const int32_t i = bid_x() * bdim_x() + tid_x();
  if (i >= nshots) return;
  w.newdone[i] = 0;
  if (w.done[i]) return;
  const bool any = w.anys[i] != 0u;
  w.anys[i] = 0u;
  const bool evid = w.evid[i] != 0;
  w.evid[i] = 0;
  if (r < 0) w.tclr[i] = any ? -1 : 0;
  else if (!any && w.tclr[i] < 0) w.tclr[i] = r + 1;
  const bool frozen = kp.skip && r >= 0 && w.conv[i] && !evid;
  if ((kp.retire && w.tclr[i] >= 0) || frozen) {
    w.done[i] = 1;
    w.newdone[i] = 1;
  }
}

// Every shot slot of the tiles: shots beyond nshots start retired.
__global__ void __launch_bounds__(256) stream_clear_shots(StreamWS w, int32_t nshots, int32_t ntot) {
  const int32_t i = bid_x() * bdim_x() + tid_x();
  if (i == 0) {
    w.ctl[0] = ntot / kStreamTile;
    w.ctl[1] = 0;
    w.ctl[2] = 0;
    w.ctl[3] = 0;
  }
  if (i >= ntot) return;
  w.sid[i] = (i < nshots) ? i : -1;
  w.anys[i] = 0u;
  w.done[i] = (i >= nshots) ? 1 : 0;
  w.newdone[i] = 0;
  w.conv[i] = 0;
  w.chg[i] = 0;
  w.evid[i] = 0;
  w.tclr[i] = -1;
}

// Beliefs of the current message state for shots that just retired
// (only_new) or for every shot not retired before (!only_new).
__global__ void __launch_bounds__(256) stream_beliefs_out(DevCode c, KParams kp, StreamWS w,
                                                          const float* __restrict__ msg,
                                                          int32_t only_new, int32_t fresh,
                                                          float* __restrict__ L, int32_t nshots) {
  const int32_t lane = tid_x() & 63;
  const int32_t v = stream_row();
  const int64_t tile = bid_y();
  if (v >= c.n || tile >= w.ctl[0]) return;
#pragma unroll 1
  for (int q = 0; q < kSV; ++q) {
    const int32_t col = kSV * lane + q;
    const int64_t i = tile * kStreamTile + col;
    if (i >= nshots) continue;
    if (only_new ? !w.newdone[i] : (w.done[i] && !w.newdone[i])) continue;
    float val;
    if (fresh) {
      val = kp.pi;
      for (int32_t qq = 0; qq < c.var_deg[v]; ++qq) val = val + 0.0f;
      val = clampf(val, kp.clamp);
    } else {
      val = stream_belief(c, msg, tile, col, v, kp.pi, kp.clamp);
    }
    L[(int64_t)w.sid[i] * c.n + v] = val;
  }
}

// Interleaved state -> caller's row-major outputs.
__global__ void __launch_bounds__(256) stream_out(DevCode c, StreamWS w, uint8_t* z, uint8_t* s,
                                                  int32_t* tclr, int32_t nshots) {
  const int64_t idx = (int64_t)bid_x() * bdim_x() + tid_x();
  const int64_t tz = (int64_t)nshots * c.n;
  const int64_t ts = (int64_t)nshots * c.m;
  if (idx < tz) {
    const int64_t i = idx / c.n;
    const int32_t v = (int32_t)(idx - i * c.n);
    z[idx] = w.z[((i / kStreamTile) * c.n + v) * kStreamTile + (i % kStreamTile)];
  } else if (idx < tz + ts) {
    const int64_t k = idx - tz;
    const int64_t i = k / c.m;
    const int32_t ch = (int32_t)(k - i * c.m);
    s[k] = w.s[((i / kStreamTile) * c.m + ch) * kStreamTile + (i % kStreamTile)];
  } else if (idx < tz + ts + nshots) {
    const int64_t i = idx - tz - ts;
    tclr[i] = w.tclr[i];
  }
}

// ---- live-shot compaction (with the exact shortcuts, over more than one
// tile). A tile sweeps while any of its shots runs, so after most shots have
// stopped the few still running are moved to the first tiles, in slot
// order, and the per-tile kernels skip every tile past them: the number of
// tiles in use is read on the device (w.ctl[0]), so the launch sequence and
// its grids stay the same and a HIP graph may hold it. w.sid maps a slot to
// its shot (the clocks' Philox words and the outputs go by shot). A shot's
// outputs are written when it stops, since its slot may then be reused, and
// those of the shots still running at the end.

// z (rows 0 .. n) and s (rows n .. n + m) of the slots that just stopped
// (only_new) or of every slot still running (!only_new) to the caller's
// row-major outputs.
__global__ void __launch_bounds__(256) stream_out_rows(DevCode c, StreamWS w, int32_t only_new, uint8_t* z,
                                                       uint8_t* s) {
  const int32_t lane = tid_x() & 63;
  const int32_t row = stream_row();
  const int64_t tile = bid_y();
  if (row >= c.n + c.m || tile >= w.ctl[0]) return;
  const int64_t b = tile * kStreamTile + kSV * lane;
  const uint32_t sel = only_new ? ld4b(w.newdone + b) : (~ld4b(w.done + b) & 0x01010101u);
  if (!sel) return;
  const bool isz = row < c.n;
  const uint32_t v4 = isz ? ld4b(w.z + stream_at(tile, c.n, row, lane)) : ld4b(w.s + stream_at(tile, c.m, row - c.n, lane));
#pragma unroll
  for (int q = 0; q < kSV; ++q) {
    if (!((sel >> (8 * q)) & 1u)) continue;
    const int64_t sh = w.sid[b + q];
    if (sh < 0) continue;
    const uint8_t x = (uint8_t)((v4 >> (8 * q)) & 0xFFu);
    if (isz)
      z[sh * c.n + row] = x;
    else
      s[sh * c.m + (row - c.n)] = x;
  }
}

// t_clr of the slots that just stopped (only_new) or of every slot still
// running (!only_new).
__global__ void __launch_bounds__(256) stream_out_tclr(StreamWS w, int32_t only_new, int32_t* tclr, int32_t ntot) {
  const int32_t i = bid_x() * bdim_x() + tid_x();
  if (i >= ntot || i >= w.ctl[0] * kStreamTile) return;
  const bool sel = only_new ? (w.newdone[i] != 0) : (w.done[i] == 0);
  const int32_t sh = w.sid[i];
  if (sel && sh >= 0) tclr[sh] = w.tclr[i];
}

// The compaction's plan, in one block: the running slots of the tiles in use
// in slot order (w.inv: new slot -> old slot), their number, the tiles they
// need, and whether to move them -- when that frees at least a quarter of
// the tiles in use, or all of them.
__global__ void __launch_bounds__(1024) stream_compact_plan(StreamWS w) {
  __shared__ int32_t part[1024];
  const int32_t ntl = w.ctl[0];
  const int32_t N = ntl * kStreamTile;
  const int32_t per = (N + 1023) / 1024;
  const int32_t b = (int32_t)tid_x() * per;
  const int32_t e = min(b + per, N);
  int32_t cnt = 0;
  for (int32_t i = b; i < e; ++i) cnt += w.done[i] ? 0 : 1;
  part[tid_x()] = cnt;
  __syncthreads();
  for (int32_t off = 1; off < 1024; off <<= 1) {  // inclusive scan
    const int32_t v = (int32_t)tid_x() >= off ? part[tid_x() - off] : 0;
    __syncthreads();
    part[tid_x()] += v;
    __syncthreads();
  }
  const int32_t total = part[1023];
  const int32_t nt = (total + kStreamTile - 1) / kStreamTile;
  const bool go = nt < ntl && (nt == 0 || 4 * nt <= 3 * ntl);
  if (go) {
    int32_t pos = part[tid_x()] - cnt;
    for (int32_t i = b; i < e; ++i)
      if (!w.done[i]) w.inv[pos++] = i;
  }
  if (tid_x() == 0) {
    w.ctl[1] = go ? 1 : 0;
    w.ctl[2] = total;
    w.ctl[3] = nt;
  }
}

// Row `row` of an array of `rows` rows per tile: new slot j (< the number of
// running shots) of the tiles after the compaction takes old slot inv[j],
// from src to dst (4-byte elements: messages).
__global__ void __launch_bounds__(256) stream_compact_f32(StreamWS w, int32_t rows, const float* __restrict__ src,
                                                          float* __restrict__ dst) {
  const int32_t lane = tid_x() & 63;
  const int32_t row = stream_row();
  const int64_t tile = bid_y();
  if (!w.ctl[1] || row >= rows || tile >= w.ctl[3]) return;
  const int32_t nlive = w.ctl[2];
  float v[kSV];
#pragma unroll
  for (int q = 0; q < kSV; ++q) {
    const int64_t j = tile * kStreamTile + kSV * lane + q;
    v[q] = 0.0f;
    if (j < nlive) {
      const int64_t i = w.inv[j];
      v[q] = src[((i / kStreamTile) * rows + row) * kStreamTile + (i % kStreamTile)];
    }
  }
  *reinterpret_cast<float4*>(dst + stream_at(tile, rows, row, lane)) = make_float4(v[0], v[1], v[2], v[3]);
}

// The same for 1-byte elements (syndrome, correction).
__global__ void __launch_bounds__(256) stream_compact_u8(StreamWS w, int32_t rows, const uint8_t* __restrict__ src,
                                                         uint8_t* __restrict__ dst) {
  const int32_t lane = tid_x() & 63;
  const int32_t row = stream_row();
  const int64_t tile = bid_y();
  if (!w.ctl[1] || row >= rows || tile >= w.ctl[3]) return;
  const int32_t nlive = w.ctl[2];
  uint32_t x = 0u;
#pragma unroll
  for (int q = 0; q < kSV; ++q) {
    const int64_t j = tile * kStreamTile + kSV * lane + q;
    if (j < nlive) {
      const int64_t i = w.inv[j];
      x |= (uint32_t)src[((i / kStreamTile) * rows + row) * kStreamTile + (i % kStreamTile)] << (8 * q);
    }
  }
  st4b(dst + stream_at(tile, rows, row, lane), x);
}

// Copies rows of the tiles after the compaction back (from -> to), and
// clears `from` when asked (the flip requests used as scratch). 16 bytes
// per lane: 4 elements of 4 bytes or 16 of 1 byte (then rows cover 4
// lanes' worth per 16 bytes: `ebytes` is the element size).
__global__ void __launch_bounds__(256) stream_compact_back(StreamWS w, int32_t rows, int32_t ebytes,
                                                           unsigned char* from, unsigned char* to, int32_t clear) {
  const int32_t lane = tid_x() & 63;
  const int32_t row = stream_row();
  const int64_t tile = bid_y();
  if (!w.ctl[1] || row >= rows || tile >= w.ctl[3]) return;
  const int64_t o = ((tile * rows + row) * kStreamTile + kSV * lane) * ebytes;
  if (ebytes == 4) {
    *reinterpret_cast<uint4*>(to + o) = *reinterpret_cast<const uint4*>(from + o);
    if (clear) *reinterpret_cast<uint4*>(from + o) = make_uint4(0u, 0u, 0u, 0u);
  } else {
    *reinterpret_cast<uint32_t*>(to + o) = *reinterpret_cast<const uint32_t*>(from + o);
    if (clear) *reinterpret_cast<uint32_t*>(from + o) = 0u;
  }
}

// Per slot, gathered into scratch (anys holds t_clr, sid2 the shot, newdone
// the fixed-point mark: all three are free at the end of a round) ...
__global__ void __launch_bounds__(256) stream_compact_slots(StreamWS w, int32_t ntot) {
  const int32_t j = bid_x() * bdim_x() + tid_x();
  if (!w.ctl[1] || j >= ntot) return;
  if (j < w.ctl[2]) {
    const int32_t i = w.inv[j];
    w.anys[j] = (uint32_t)w.tclr[i];
    w.sid2[j] = w.sid[i];
    w.newdone[j] = w.conv[i];
  } else {
    w.anys[j] = 0xFFFFFFFFu;
    w.sid2[j] = -1;
    w.newdone[j] = 0;
  }
}

// ... and put in place; the slots past the running shots are stopped.
__global__ void __launch_bounds__(256) stream_compact_slots_back(StreamWS w, int32_t ntot) {
  const int32_t j = bid_x() * bdim_x() + tid_x();
  if (!w.ctl[1] || j >= ntot) return;
  w.tclr[j] = (int32_t)w.anys[j];
  w.anys[j] = 0u;
  w.sid[j] = w.sid2[j];
  w.conv[j] = w.newdone[j];
  w.newdone[j] = 0;
  w.done[j] = (j < w.ctl[2]) ? 0 : 1;
  w.chg[j] = 0;
  w.evid[j] = 0;
}

__global__ void stream_compact_commit(StreamWS w) {
  if (tid_x() == 0 && w.ctl[1]) {
    w.ctl[0] = w.ctl[3];
    w.ctl[1] = 0;
  }
}

typedef void (*SweepFn)(DevCode, KParams, StreamWS, const float*, float*, int32_t, int32_t);
typedef void (*MovesFn)(DevCode, KParams, StreamWS, const float*, int32_t, int32_t, uint64_t);

static void stream_fns(int dcmax, SweepFn* sw, MovesFn* mv) {
  if (dcmax <= 2) {
    *sw = stream_sweep<2>;
    *mv = stream_moves<2>;
  } else if (dcmax <= 4) {
    *sw = stream_sweep<4>;
    *mv = stream_moves<4>;
  } else if (dcmax <= 6) {
    *sw = stream_sweep<6>;
    *mv = stream_moves<6>;
  } else if (dcmax <= 8) {
    *sw = stream_sweep<8>;
    *mv = stream_moves<8>;
  } else if (dcmax <= 16) {
    *sw = stream_sweep<16>;
    *mv = stream_moves<16>;
  } else {
    *sw = stream_sweep<32>;
    *mv = stream_moves<32>;
  }
}

hipError_t launch_stream(const DevCode& c, const KParams& kp, const uint8_t* e0, uint64_t shot0,
                         int32_t nshots, void* ws, uint8_t* z, uint8_t* s, int32_t* tclr, float* L,
                         hipStream_t st, const uint8_t* s0, int32_t r0) {
  if (nshots <= 0) return hipSuccess;
  SweepFn sweep_fn;
  MovesFn moves_fn;
  stream_fns(c.dcmax, &sweep_fn, &moves_fn);
  const bool seq = kp.conflict == kConflictSequential;
  StreamWS w = stream_carve(c, nshots, ws, nullptr, seq);
  const unsigned ntile = (unsigned)((nshots + kStreamTile - 1) / kStreamTile);
  const int32_t ntot = (int32_t)(ntile * kStreamTile);
  const dim3 gchk((unsigned)((c.m + kStreamRowsPerBlock - 1) / kStreamRowsPerBlock), ntile);
  const dim3 gvar((unsigned)((c.n + kStreamRowsPerBlock - 1) / kStreamRowsPerBlock), ntile);
  const dim3 blk(64 * kStreamRowsPerBlock);
  const unsigned gshot = (unsigned)((nshots + 255) / 256);
  hipLaunchKernelGGL(stream_clear_shots, dim3((unsigned)((ntot + 255) / 256)), blk, 0, st, w, nshots,
                     ntot);
  hipLaunchKernelGGL(stream_init_var, gvar, blk, 0, st, c, w);
  hipLaunchKernelGGL(stream_init_chk, gchk, blk, 0, st, c, w, e0, s0, nshots);
  hipLaunchKernelGGL(stream_status, dim3(gshot), blk, 0, st, kp, w, -1, nshots);
  // live-shot compaction: with the exact shortcuts, over more than one tile
  const bool compact = kp.skip && ntile > 1;
  const dim3 gout((unsigned)((c.n + c.m + kStreamRowsPerBlock - 1) / kStreamRowsPerBlock), ntile);
  const dim3 gmsg((unsigned)((c.m * c.dcmax + kStreamRowsPerBlock - 1) / kStreamRowsPerBlock), ntile);
  const unsigned gslot = (unsigned)((ntot + 255) / 256);
  auto out_new = [&]() {
    hipLaunchKernelGGL(stream_out_rows, gout, blk, 0, st, c, w, 1, z, s);
    hipLaunchKernelGGL(stream_out_tclr, dim3(gslot), blk, 0, st, w, 1, tclr, ntot);
  };
  int cur = 0;
  auto compaction = [&]() {
    hipLaunchKernelGGL(stream_compact_plan, dim3(1), dim3(1024), 0, st, w);
    hipLaunchKernelGGL(stream_compact_f32, gmsg, blk, 0, st, w, c.m * c.dcmax, w.msg[cur], w.msg[cur ^ 1]);
    hipLaunchKernelGGL(stream_compact_back, gmsg, blk, 0, st, w, c.m * c.dcmax, 4,
                       reinterpret_cast<unsigned char*>(w.msg[cur ^ 1]), reinterpret_cast<unsigned char*>(w.msg[cur]),
                       0);
    hipLaunchKernelGGL(stream_compact_u8, gchk, blk, 0, st, w, c.m, w.s, w.s2);
    hipLaunchKernelGGL(stream_compact_back, gchk, blk, 0, st, w, c.m, 1, w.s2, w.s, 0);
    hipLaunchKernelGGL(stream_compact_u8, gvar, blk, 0, st, w, c.n, w.z, w.fl);
    hipLaunchKernelGGL(stream_compact_back, gvar, blk, 0, st, w, c.n, 1, w.fl, w.z, 1);
    hipLaunchKernelGGL(stream_compact_slots, dim3(gslot), blk, 0, st, w, ntot);
    hipLaunchKernelGGL(stream_compact_slots_back, dim3(gslot), blk, 0, st, w, ntot);
    hipLaunchKernelGGL(stream_compact_commit, dim3(1), dim3(64), 0, st, w);
  };
  if (compact) out_new();
  bool fresh = true;
  if (L) hipLaunchKernelGGL(stream_beliefs_out, gvar, blk, 0, st, c, kp, w, w.msg[cur], 1, 1, L,
                            nshots);
  for (int32_t r = 0; r < kp.rounds; ++r) {
    for (int32_t it = 0; it < kp.iters; ++it) {
      // sweeps 7, 15, ... and the last of the round compare (never a shot's
      // first sweep, which starts from m_{v->c} = 0 and is a different map)
      const bool cmp = kp.skip && !fresh && ((it & 7) == 7 || it == kp.iters - 1);
      hipLaunchKernelGGL(sweep_fn, gchk, blk, 0, st, c, kp, w, w.msg[cur], w.msg[cur ^ 1],
                         fresh ? 1 : 0, cmp ? 1 : 0);
      if (cmp) hipLaunchKernelGGL(stream_conv, dim3((unsigned)((ntot + 255) / 256)), blk, 0, st, w, ntot);
      cur ^= 1;
      fresh = false;
    }
    hipLaunchKernelGGL(moves_fn, gchk, blk, 0, st, c, kp, w, w.msg[cur], r0 + r, fresh ? 1 : 0, shot0);
    if (seq) hipLaunchKernelGGL(stream_resolve, dim3(ntile), dim3(kStreamTile), 0, st, c, w);
    hipLaunchKernelGGL(stream_syndrome, gchk, blk, 0, st, c, w);
    hipLaunchKernelGGL(stream_apply, gvar, blk, 0, st, c, w);
    hipLaunchKernelGGL(stream_status, dim3(gshot), blk, 0, st, kp, w, r, nshots);
    if (L)
      hipLaunchKernelGGL(stream_beliefs_out, gvar, blk, 0, st, c, kp, w, w.msg[cur], 1,
                         fresh ? 1 : 0, L, nshots);
    if (compact) {
      out_new();
      if (r + 1 < kp.rounds) compaction();
    }
  }
  if (L)
    hipLaunchKernelGGL(stream_beliefs_out, gvar, blk, 0, st, c, kp, w, w.msg[cur], 0, fresh ? 1 : 0,
                       L, nshots);
  if (compact) {  // the shots still running (the others were written when they stopped)
    hipLaunchKernelGGL(stream_out_rows, gout, blk, 0, st, c, w, 0, z, s);
    hipLaunchKernelGGL(stream_out_tclr, dim3(gslot), blk, 0, st, w, 0, tclr, ntot);
  } else {
    const int64_t tot = (int64_t)nshots * (c.n + c.m + 1);
    hipLaunchKernelGGL(stream_out, dim3((unsigned)((tot + 255) / 256)), blk, 0, st, c, w, z, s, tclr,
                       nshots);
  }
  return hipGetLastError();
}

}  // namespace laim
