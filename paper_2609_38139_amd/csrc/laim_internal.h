// laim_internal.h -- shared declarations of the library's host code and
// kernel launchers (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "laim.h"

namespace laim {

// Limits of the device layout.
constexpr int kMaxCheckDegree = 32;
constexpr int kMaxQubitDegree = 16;
constexpr int kStreamTile = 256;  // shots per tile in the stream form (one wavefront, 4 per lane)

// Edge reference (c, j): the j-th qubit of check c, packed as (c << 5) | j.
__host__ __device__ inline int32_t pack_edge(int32_t c, int32_t j) { return (c << 5) | j; }
__host__ __device__ inline int32_t edge_check(int32_t e) { return e >> 5; }
__host__ __device__ inline int32_t edge_slot(int32_t e) { return e & 31; }

// Device-side view of a code. Tables are ELL-padded with -1.
struct DevCode {
  int32_t m, n, E, dcmax, dvmax, k, kw, regular;
  const int32_t* chk_var;   // [m][dcmax] qubits of check c, ascending
  const int32_t* chk_deg;   // [m]
  const int32_t* var_deg;   // [n]
  const int32_t* var_edge;  // [n][dvmax] packed edges of qubit v, ascending check
  const int32_t* partner;   // [m][dcmax][dvmax-1] packed edges of qubit chk_var[c][j]
                            // other than (c, j), ascending check
  const uint32_t* lcol;     // [n][kw] bit i of word w: qubit v in logical 32w + i
  const float* thr;         // [dcmax + 1] Evidence bound per check degree
  // 2D toric layout (null otherwise): checks i L + j, L a multiple of 4, each
  // sharing one qubit with each of its four lattice neighbours. Thread t of
  // the tiled resident variant (8 checks per thread, m / 8 threads) owns the
  // 2 x 4 tile of checks (2I + r, 4J + q), t = I L / 4 + J, as its checks
  // k = 4 r + q; in LDS check k of thread t sits at virtual index t + k m / 8
  // with its messages in lattice order (left, right, up, down neighbour).
  const int32_t* tile_chk;   // [m] check at virtual index
  const int32_t* tile_jo;    // [m][4] row slot of lattice direction g, by virtual index
  const int32_t* tile_word;  // [m][4] LDS word of message (check, row slot)
  int32_t tile_L;            // L of the 2D toric layout (0 without one)
};

// LDS word of message (check c, slot j) in the resident layout of checks of
// degree dc: a slot of a group of 64 checks spans kResSlotStride words (64
// used), so that messages of neighbouring checks in different slots fall in
// different LDS banks.
constexpr int kResSlotStride = 65;
__host__ __device__ inline int32_t resident_msg_word(int32_t dc, int32_t c, int32_t j) {
  return ((c >> 6) * dc + j) * kResSlotStride + (c & 63);
}

void set_error(const char* fmt, ...);
laim_status hip_fail(hipError_t e, const char* what);

// Parameters resolved on the host for the kernels.
struct KParams {
  int32_t bp;
  float alpha;
  float pi;       // (float) log(q / (1 - q))
  float clamp;
  int32_t iters;
  int32_t rounds;
  uint64_t mask_bound;  // floor(mask_density 2^32), 2^32 = always
  int32_t evidence;
  int32_t retire;
  uint64_t seed;
  int32_t conflict;  // kConflict*
  int32_t skip;      // 1: a group whose messages are a fixed point of the sweep skips the
                     // round's remaining (identity) sweeps
  int32_t move;      // 0: LocalMove; 1: multi-qubit move (every qubit with a positive belief)
};

// How one round's move requests combine (values of laim_decode_params.conflict).
constexpr int32_t kConflictOr = 0, kConflictXor = 1, kConflictSequential = 2;

laim_status resolve_params(const laim_decode_params* p, KParams* kp);
uint64_t bernoulli_bound(double p);

// ---- kernel launchers (laim_kernels.hip) ----
hipError_t launch_noise(const DevCode& c, uint64_t bound, uint64_t seed, uint64_t shot0,
                        int32_t nshots, uint8_t* e, hipStream_t st);
hipError_t launch_syndrome(const DevCode& c, const uint8_t* e, int32_t nshots, uint8_t* s,
                           hipStream_t st);
hipError_t launch_failure(const DevCode& c, const uint8_t* e0, const uint8_t* z, int32_t nshots,
                          uint8_t* fail, hipStream_t st);

struct ResidentShape {
  int32_t nt;    // threads per shot
  int32_t cpt;   // checks per thread
  int32_t vpt;   // qubits per thread
  int32_t spb;   // shots per block
  int32_t mpad;  // nt * cpt rounded up to a multiple of 64 (LDS holds DC * mpad messages)
  int32_t group_bytes;  // LDS bytes of one shot's group
  size_t lds;    // dynamic LDS bytes per block
  int32_t dc, dv, reg;  // kernel variant degrees (reg: exact regular variant)
  int32_t tile = 0;     // the tiled variant (2D toric layout, min-sum, 8 checks per thread)
};

// Whether the exact-degree kernels for qubit degree 2 may run: they skip the
// clamp of the qubit-side min-sum messages, which cannot bind when alpha < 1
// and |pi| / (1 - alpha) < CLAMP (then |m_{v->c}| <= |pi| + alpha max|m_{v->c}|
// keeps every message within |pi| / (1 - alpha); a 1% margin covers the
// roundings). Sum-product keeps every clamp.
inline bool reg_dv2_ok(const KParams& kp) {
  if (kp.bp != 0) return true;
  return kp.alpha < 1.0f && (kp.pi < 0.0f ? -kp.pi : kp.pi) < 0.99f * kp.clamp * (1.0f - kp.alpha);
}

// Picks / validates the resident launch shape; returns false (with an
// error text) if the code cannot run resident with it. With reg2 false the
// exact variants for qubit degree 2 are not used (the padded one is).
bool resident_shape(const DevCode& c, int bp, const laim_resident_cfg* want, ResidentShape* out,
                    int device, bool seq = false, bool reg2 = true);
size_t resident_workspace_bytes();
// sweeps[i] = iters x (rounds shot i ran), for the forms that run every sweep
hipError_t launch_sweep_count(const KParams& kp, const int32_t* tclr, int32_t nshots, int32_t* sweeps,
                              hipStream_t st);
// With s0 (start syndromes [nshots][m]) the shots start from s0 instead of
// H e0 (e0 may then be null and fail must be null); r0 numbers the first
// round for the clocks' random words.
hipError_t launch_resident(const DevCode& c, const KParams& kp, const ResidentShape& sh,
                           const uint8_t* e0, uint64_t shot0, int32_t nshots, void* ws,
                           uint8_t* z, uint8_t* s, int32_t* tclr, float* L, uint8_t* fail,
                           int32_t* sweeps, hipStream_t st, const uint8_t* s0 = nullptr,
                           int32_t r0 = 0);

// laim_decode_rounds and its variants: validation, form choice and launch
// (cfg non-null: the resident form with that launch shape).
laim_status decode_common(const laim_code* code, const laim_decode_params* params,
                          const uint8_t* e0, uint64_t shot0, int32_t nshots, void* ws,
                          size_t ws_bytes, uint8_t* z_out, uint8_t* s_out, int32_t* tclr_out,
                          float* L_out, int32_t* sweeps_out, uint8_t* fail_out, int32_t form,
                          const laim_resident_cfg* cfg, laim_stream stream);

size_t stream_workspace_bytes(const DevCode& c, int32_t nshots, bool seq);
hipError_t launch_stream(const DevCode& c, const KParams& kp, const uint8_t* e0, uint64_t shot0,
                         int32_t nshots, void* ws, uint8_t* z, uint8_t* s, int32_t* tclr, float* L,
                         hipStream_t st, const uint8_t* s0 = nullptr, int32_t r0 = 0);

// ---- multi-code kernels (batched plans and the serving loop)
// Block-uniform description of a unit: the launch shape of one code, the
// rounds to run, and whether groups resume from saved state.
struct UnitCtx {
  int32_t nt, vpt, spb, mpad, group_bytes;
  int32_t rounds;  // rounds run in this unit
  int32_t resume;  // 1: every group continues from its saved state
  int32_t events;  // 1: count flips and defects for the groups' ev_out
};

struct BatchItemDev {
  DevCode c;
  KParams kp;
  UnitCtx u;
  int32_t variant;
  const uint8_t* e0;
  uint64_t shot0;
  int32_t nshots;
  uint8_t* z;
  uint8_t* s;
  int32_t* tclr;
  uint8_t* fail;
};

// One item of a grouped resident launch (several shot ranges of one code
// and parameters in one persistent launch): shots first .. first + nshots - 1
// of the launch's shot index are this item's shots 0 .. nshots - 1.
struct GroupItemDev {
  const uint8_t* e0;
  uint64_t shot0;
  int32_t first, nshots;
  uint8_t* z;
  uint8_t* s;
  int32_t* tclr;
  uint8_t* fail;  // or null
};

struct ServerUnitDev {
  int32_t item;    // code and parameters
  int32_t first;   // first request of the unit in the request table
  int32_t count;   // requests in the unit (<= spb)
  int32_t resume;  // 0 on a request's first round
  int32_t rounds;  // rounds run: 1, or 0 for requests with a budget of no rounds
};

struct ServerReqDev {
  uint64_t shot;
  int32_t round;  // rounds already run
  int32_t pad;
  const uint8_t* e0;  // [n]
  float* msg;         // [m * dcmax]
  uint8_t* z;         // [n]
  uint8_t* s;         // [m]
  int32_t* hdr;       // [4]: t_clr, messages at a fixed point (0/1)
  int32_t* ev;        // [2]: flips, syndrome weight
  uint8_t* fail;      // [1]
};

bool batch_variant(const DevCode& c, int bp, const laim_resident_cfg* want, int device, bool seq,
                   bool reg2, UnitCtx* u, int* variant, size_t* lds, int* block);
// One persistent resident launch over the shots of several items of one
// code and parameters (items [nitems] in device memory, total shots in
// all); ws holds the shot queue (resident_workspace_bytes). With a fail
// pointer the code must have at most 128 logicals.
hipError_t launch_resident_group(const DevCode& c, const KParams& kp, const ResidentShape& sh,
                                 const GroupItemDev* items, int32_t nitems, int32_t total, void* ws,
                                 hipStream_t st);
hipError_t launch_server(int bp, const BatchItemDev* items, const ServerUnitDev* units,
                         int32_t nunits, const ServerReqDev* reqs, size_t lds, int block,
                         hipStream_t st);

// ---- continuous-time machine (laim_ctm.hip)
struct CtmParamsDev {
  int32_t bp;
  float alpha;
  float pi;
  float clamp;
  float lam;  // (float)(dt / tau)
  double dt;
  int32_t max_steps;
  int32_t evidence;
  uint64_t seed;
  int32_t skip;  // 1: steps at a fixed point of the messages are skipped
};

struct CtmShape {
  int32_t nt;    // threads per shot (one shot per block)
  int32_t cpt;   // checks per thread
  int32_t mpad;  // nt * cpt rounded up to a multiple of 64
  size_t lds;    // dynamic LDS bytes per block
  int32_t dc, dv, reg;  // kernel variant degrees
};

struct CtmArgs {
  const uint8_t* e0;
  uint64_t shot0;
  int32_t nshots;
  uint32_t* counter;  // shot queue head
  uint8_t* z;
  uint8_t* s;
  double* tclr;
  int32_t* counts;  // [nshots][2]: events, moves (or null)
  int32_t* steps;   // [nshots]: Euler steps computed (or null)
  uint8_t* fail;    // or null
  int32_t nt, mpad;
};

// Whether the continuous machine's exact kernels for qubit degree 2 may run:
// their min-sum path skips every clamp. The Euler update m + lam (F - m) with
// 0 < lam <= 1 is a convex combination of m and F, so every message stays
// within |pi| / (1 - alpha) (as for the round machine) when alpha < 1, and
// that is below CLAMP with a 1% margin for roundings.
inline bool ctm_reg_dv2_ok(const CtmParamsDev& P) {
  if (P.bp != 0) return true;
  return P.alpha < 1.0f && P.lam <= 1.0f &&
         (P.pi < 0.0f ? -P.pi : P.pi) < 0.99f * P.clamp * (1.0f - P.alpha);
}

bool ctm_shape(const DevCode& c, const CtmParamsDev& P, int32_t cpt_want, int device, CtmShape* out);
hipError_t launch_ctm(const DevCode& c, const CtmParamsDev& P, const CtmShape& sh, const uint8_t* e0,
                      uint64_t shot0, int32_t nshots, void* ws, uint8_t* z, uint8_t* s, double* tclr,
                      int32_t* counts, int32_t* steps, uint8_t* fail, hipStream_t st);

// ---- bit-centric machine (laim_bitcentric.hip)
bool bitcentric_shape(const DevCode& c, int device, int32_t* nt, size_t* lds);
hipError_t launch_bitcentric(const DevCode& c, double q, const uint8_t* e0, int32_t nshots,
                             int32_t iters, int32_t nt, size_t lds, uint8_t* z, int32_t* iclr,
                             double* L, hipStream_t st);
// chain form: bits per lane K, lanes per shot nl and shots per wavefront S
// for a chain of d bits (false if the chain is too short or too long for it)
bool bitchain_shape(int32_t d, bool periodic, int32_t* K, int32_t* nl, int32_t* S);
hipError_t launch_bitchain(int32_t d, bool periodic, int32_t K, int32_t nl, int32_t S, double q,
                           const uint8_t* e0, int32_t nshots, int32_t iters, uint8_t* z,
                           int32_t* iclr, double* L, hipStream_t st);

}  // namespace laim

// The code object behind the opaque ABI handle.
struct laim_code {
  int32_t device;
  int32_t m, n, E, dcmax, dvmax, k;
  std::vector<int32_t> h_rowptr, h_col;  // H (host copy)
  std::vector<uint8_t> logicals;         // [k][n] dense host copy
  void* dev_mem;                         // one allocation holding every table
  laim::DevCode dev;
  bool has_cfg[2];
  laim_resident_cfg cfg[2];
};
