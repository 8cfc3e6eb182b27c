// laim_probe.hip -- measurement helpers for the roofline of the decoder's
// kernels (built into liblaim_probe.so, loaded by bench.py only; not part of
// the decoder's C ABI).
//
//  - VALU issue rate per instruction class: every lane runs eight
//    independent dependency chains of one instruction, so each SIMD always
//    has an instruction ready; the rate is lane-instructions per second.
//  - LDS bandwidth: every lane reads (or writes) consecutive 4-, 8- or
//    16-byte words of a block-local LDS array, so a wavefront's access
//    covers consecutive banks without conflicts; the accesses are issued
//    eight at a time with almost no other instructions, so that neither
//    latency nor VALU work limits them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace {

constexpr int kChains = 8;

#define PROBE_BODY(ASM)                                          \
  _Pragma("unroll") for (int k = 0; k < kChains; ++k) {         \
    asm volatile(ASM : "+v"(a[k]) : "v"(b), "v"(c));            \
  }

#define PROBE_BODY_S(ASM)                                        \
  _Pragma("unroll") for (int k = 0; k < kChains; ++k) {         \
    asm volatile(ASM : "+v"(a[k]) : "v"(b), "s"(sm));           \
  }

template <int KIND>
__global__ void __launch_bounds__(256) valu_probe(float* out, int32_t iters, uint64_t sm /* a lane mask */) {
  float a[kChains];
  const float b = 1.0000001f + 1e-9f * (float)threadIdx.x, c = 1e-7f * (float)blockIdx.x;
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = 0.5f + 0.01f * (float)k + 1e-6f * (float)threadIdx.x;
  for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (KIND == 0) PROBE_BODY("v_add_f32 %0, %0, %1")
      if (KIND == 1) PROBE_BODY("v_mul_f32 %0, %0, %1")
      if (KIND == 2) PROBE_BODY("v_fma_f32 %0, %0, %1, %2")
      if (KIND == 3) PROBE_BODY("v_min3_f32 %0, %0, %1, %2")
      if (KIND == 4) PROBE_BODY("v_med3_f32 %0, %0, %1, %2")
      if (KIND == 5) PROBE_BODY("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96")
      if (KIND == 6) PROBE_BODY("v_xor_b32 %0, %0, %1")
      if (KIND == 7) PROBE_BODY("v_floor_f32 %0, %0")
      if (KIND == 8) PROBE_BODY("v_cvt_i32_f32 %0, %0")
      if (KIND == 9) PROBE_BODY("v_ldexp_f32 %0, %0, %1")
      if (KIND == 10) PROBE_BODY_S("v_cndmask_b32_e64 %0, %0, %1, %2")
      if (KIND == 11) PROBE_BODY("v_sub_f32 %0, %1, %0")
      if (KIND == 12) PROBE_BODY("v_max_f32 %0, %0, %1")
      if (KIND == 13) PROBE_BODY("v_min_f32_e64 %0, |%0|, |%1|")
      if (KIND == 14) PROBE_BODY("v_add_f32_e64 %0, %0, -%1")
      if (KIND == 15) PROBE_BODY("v_fmac_f32 %0, %1, %2")
      if (KIND == 16) PROBE_BODY("v_fmaak_f32 %0, %0, %1, 0x3e2aaaab")
      if (KIND == 17) PROBE_BODY("v_and_b32 %0, %0, %1")
      if (KIND == 18) PROBE_BODY("v_lshlrev_b32 %0, 1, %0")
      if (KIND == 19) PROBE_BODY("v_add_u32 %0, %0, %1")
      if (KIND == 20) PROBE_BODY("v_lshl_add_u32 %0, %0, 2, %1")
      if (KIND == 21) PROBE_BODY("v_bfi_b32 %0, %1, %0, %2")
      if (KIND == 22) PROBE_BODY("v_mul_f32_e64 %0, %0, %1 clamp")
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// LDS: in each step a wavefront issues kLdsPerStep reads (or writes) of
// WIDTH bytes per lane to a 32 KiB block-local array, lane l of access u at
// word base + l + 256 u, base = 64 (step mod 2): the 64 lanes touch
// consecutive words, i.e. consecutive banks, no two accesses of a step
// share a word, and every access stays inside the array (base + 63 +
// 256 (kLdsPerStep - 1) < 2048 words of 16 B). The accesses of a step are
// one asm block -- the address in one register, the access number in the
// instruction's offset field, and a wait for all of them at its end -- so
// the loop spends two VALU instructions per step and the probe measures the
// LDS, not the address arithmetic; read results are consumed by an empty
// asm statement after the wait. 32 KiB per block lets five blocks (20
// wavefronts) share a CU.
constexpr int kLdsPerStep = 8;

#define LDS_R8(OP)                                                                              \
  asm volatile(OP " %0, %8\n\t" OP " %1, %8 offset:%9\n\t" OP " %2, %8 offset:%10\n\t" OP    \
               " %3, %8 offset:%11\n\t" OP " %4, %8 offset:%12\n\t" OP " %5, %8 offset:%13\n\t" \
               OP " %6, %8 offset:%14\n\t" OP " %7, %8 offset:%15\n\ts_waitcnt lgkmcnt(0)"      \
               : "=v"(r0), "=v"(r1), "=v"(r2), "=v"(r3), "=v"(r4), "=v"(r5), "=v"(r6), "=v"(r7)   \
               : "v"(addr), "i"(1 * kStep), "i"(2 * kStep), "i"(3 * kStep), "i"(4 * kStep),       \
                 "i"(5 * kStep), "i"(6 * kStep), "i"(7 * kStep)                                  \
               : "memory")

#define LDS_W8(OP)                                                                                  \
  asm volatile(OP " %0, %1\n\t" OP " %0, %1 offset:%2\n\t" OP " %0, %1 offset:%3\n\t" OP          \
               " %0, %1 offset:%4\n\t" OP " %0, %1 offset:%5\n\t" OP " %0, %1 offset:%6\n\t" OP     \
               " %0, %1 offset:%7\n\t" OP " %0, %1 offset:%8\n\ts_waitcnt lgkmcnt(0)"               \
               :                                                                                   \
               : "v"(addr), "v"(val), "i"(1 * kStep), "i"(2 * kStep), "i"(3 * kStep),              \
                 "i"(4 * kStep), "i"(5 * kStep), "i"(6 * kStep), "i"(7 * kStep)                    \
               : "memory")

template <int WIDTH, bool WRITE>
__global__ void __launch_bounds__(256) lds_probe(float* out, int32_t iters) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<WIDTH == 4, float, typename std::conditional<WIDTH == 8, f2, f4>::type>::type
      T;
  constexpr int kBytes = 32768;
  constexpr int kStep = 256 * WIDTH;  // bytes between the accesses of a step
  static_assert(kLdsPerStep == 8, "the asm blocks issue eight accesses");
  static_assert((127 + 256 * (kLdsPerStep - 1)) * WIDTH + WIDTH <= kBytes, "every access inside the array");
  __shared__ __align__(16) f4 buf[kBytes / 16];
  const int32_t lane = threadIdx.x & 63;  // each wavefront covers words base .. base + 63 + 256 u
  for (int32_t i = threadIdx.x; i < kBytes / 16; i += blockDim.x) buf[i] = f4{(float)i, 1.0f, 2.0f, 3.0f};
  __syncthreads();
  const uint32_t buf0 = (uint32_t)(uintptr_t)buf;  // the low half of a generic LDS address is its offset
  T val;
  if constexpr (WIDTH == 4)
    val = (float)lane;
  else if constexpr (WIDTH == 8)
    val = f2{(float)lane, 1.0f};
  else
    val = f4{(float)lane, 1.0f, 2.0f, 3.0f};
  for (int32_t i = 0; i < iters; ++i) {
    const uint32_t addr = buf0 + (uint32_t)((64 * (i & 1) + lane) * WIDTH);
    if constexpr (WRITE) {
      if constexpr (WIDTH == 4) LDS_W8("ds_write_b32");
      else if constexpr (WIDTH == 8) LDS_W8("ds_write_b64");
      else LDS_W8("ds_write_b128");
    } else {
      T r0, r1, r2, r3, r4, r5, r6, r7;
      if constexpr (WIDTH == 4) LDS_R8("ds_read_b32");
      else if constexpr (WIDTH == 8) LDS_R8("ds_read_b64");
      else LDS_R8("ds_read_b128");
      asm volatile("" : : "v"(r0), "v"(r1), "v"(r2), "v"(r3), "v"(r4), "v"(r5), "v"(r6), "v"(r7));
    }
  }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = reinterpret_cast<float*>(buf)[threadIdx.x];
}

// ds_write2_b32 with the two dwords 65 words apart (the resident decode
// kernels' message writes): per step eight such writes per lane, each to
// its own address register (word base + lane + 256 u), every word inside
// the 32 KiB array (base + 63 + 256 * 7 + 65 < 8192 words).
__global__ void __launch_bounds__(256) lds_write2_probe(float* out, int32_t iters) {
  constexpr int kBytes = 32768;
  static_assert((127 + 256 * 7 + 65) * 4 + 4 <= kBytes, "every access inside the array");
  __shared__ __align__(16) float buf[kBytes / 4];
  const int32_t lane = threadIdx.x & 63;
  for (int32_t i = threadIdx.x; i < kBytes / 4; i += blockDim.x) buf[i] = (float)i;
  __syncthreads();
  const uint32_t buf0 = (uint32_t)(uintptr_t)buf;
  const float va = (float)lane, vb = 1.0f;
  for (int32_t i = 0; i < iters; ++i) {
    const uint32_t a0 = buf0 + (uint32_t)((64 * (i & 1) + lane) * 4);
    asm volatile(
        "ds_write2_b32 %0, %8, %9 offset1:65\n\t"
        "ds_write2_b32 %1, %8, %9 offset1:65\n\t"
        "ds_write2_b32 %2, %8, %9 offset1:65\n\t"
        "ds_write2_b32 %3, %8, %9 offset1:65\n\t"
        "ds_write2_b32 %4, %8, %9 offset1:65\n\t"
        "ds_write2_b32 %5, %8, %9 offset1:65\n\t"
        "ds_write2_b32 %6, %8, %9 offset1:65\n\t"
        "ds_write2_b32 %7, %8, %9 offset1:65\n\t"
        "s_waitcnt lgkmcnt(0)"
        :
        : "v"(a0), "v"(a0 + 1024u), "v"(a0 + 2048u), "v"(a0 + 3072u), "v"(a0 + 4096u), "v"(a0 + 5120u),
          "v"(a0 + 6144u), "v"(a0 + 7168u), "v"(va), "v"(vb)
        : "memory");
  }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = buf[threadIdx.x];
}

typedef void (*ProbeFn)(float*, int32_t);
typedef void (*ValuFn)(float*, int32_t, uint64_t);

const ValuFn kValu[] = {valu_probe<0>,  valu_probe<1>,  valu_probe<2>,  valu_probe<3>,
                         valu_probe<4>,  valu_probe<5>,  valu_probe<6>,  valu_probe<7>,
                         valu_probe<8>,  valu_probe<9>,  valu_probe<10>, valu_probe<11>,
                         valu_probe<12>, valu_probe<13>, valu_probe<14>, valu_probe<15>,
                         valu_probe<16>, valu_probe<17>, valu_probe<18>, valu_probe<19>,
                         valu_probe<20>, valu_probe<21>, valu_probe<22>};
const ProbeFn kLds[] = {lds_probe<4, false>, lds_probe<8, false>, lds_probe<16, false>,
                        lds_probe<4, true>,  lds_probe<8, true>,  lds_probe<16, true>,
                        lds_write2_probe};

}  // namespace

extern "C" {

// Number of VALU probe kinds (instruction classes), and their names.
int32_t laim_probe_valu_kinds(void) { return (int32_t)(sizeof(kValu) / sizeof(kValu[0])); }

const char* laim_probe_valu_name(int32_t kind) {
  static const char* names[] = {"v_add_f32",       "v_mul_f32",       "v_fma_f32",
                                "v_min3_f32",      "v_med3_f32",      "v_bitop3_b32",
                                "v_xor_b32",       "v_floor_f32",     "v_cvt_i32_f32",
                                "v_ldexp_f32",     "v_cndmask_b32_e64", "v_sub_f32",
                                "v_max_f32",       "v_min_f32_e64 |a| |b|", "v_add_f32_e64 -b",
                                "v_fmac_f32",      "v_fmaak_f32",     "v_and_b32",
                                "v_lshlrev_b32",   "v_add_u32",       "v_lshl_add_u32",
                                "v_bfi_b32",       "v_mul_f32_e64 clamp"};
  return (kind >= 0 && kind < laim_probe_valu_kinds()) ? names[kind] : "";
}

// Runs VALU probe `kind` on `blocks` blocks of 256 threads (out: device
// float [blocks * 256]); returns the kernel time in ms (HIP events), or a
// negative value on error. Lane-instructions executed: blocks * 256 * iters
// * 64.
double laim_probe_valu(int32_t kind, int32_t blocks, int32_t iters, float* out) {
  if (kind < 0 || kind >= laim_probe_valu_kinds() || blocks < 1 || iters < 1 || !out) return -1.0;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  const uint64_t mask = 0x5555555555555555ull;
  hipLaunchKernelGGL(kValu[kind], dim3(blocks), dim3(256), 0, 0, out, iters, mask);  // warm-up
  (void)hipEventRecord(a, 0);
  hipLaunchKernelGGL(kValu[kind], dim3(blocks), dim3(256), 0, 0, out, iters, mask);
  (void)hipEventRecord(b, 0);
  float ms = -3.0f;
  if (hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return hipGetLastError() == hipSuccess ? (double)ms : -4.0;
}

// Accesses per lane and step of the LDS probe.
int32_t laim_probe_lds_per_step(void) { return kLdsPerStep; }

// LDS probe: mode 0..2 reads of 4, 8, 16 bytes per lane, 3..5 writes, 6
// ds_write2_b32 (8 bytes per lane, two dwords 65 words apart).
// Bytes moved: blocks * 256 * iters * laim_probe_lds_per_step() * width.
// Returns ms as above.
double laim_probe_lds(int32_t mode, int32_t blocks, int32_t iters, float* out) {
  if (mode < 0 || mode > 6 || blocks < 1 || iters < 1 || !out) return -1.0;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  hipLaunchKernelGGL(kLds[mode], dim3(blocks), dim3(256), 0, 0, out, iters);
  (void)hipEventRecord(a, 0);
  hipLaunchKernelGGL(kLds[mode], dim3(blocks), dim3(256), 0, 0, out, iters);
  (void)hipEventRecord(b, 0);
  float ms = -3.0f;
  if (hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return hipGetLastError() == hipSuccess ? (double)ms : -4.0;
}

}  // extern "C"
