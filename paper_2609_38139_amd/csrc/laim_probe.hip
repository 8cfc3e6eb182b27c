// laim_probe.hip -- measurement helpers for the roofline of the decoder's
// kernels (built into liblaim_probe.so, loaded by bench.py only; not part of
// the decoder's C ABI).
//
//  - VALU issue rate per instruction class: every lane runs eight
//    independent dependency chains of one instruction, so each SIMD always
//    has an instruction ready; the rate is lane-instructions per second.
//  - LDS bandwidth: every lane reads (or writes) consecutive 4-, 8- or
//    16-byte words of a block-local LDS array, so a wavefront's access
//    covers consecutive banks without conflicts.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// LDS: in each step a lane reads (or writes) 16 distinct words of WIDTH
// bytes of a 64 KiB block-local array, word lane + 256 u (+ a shift that
// depends on the step, so nothing is hoisted out of the loop, and no two
// accesses of a step share a word, so none is merged); the 64 lanes of a
// wavefront touch consecutive words, i.e. consecutive banks.
template <int WIDTH, bool WRITE>
__global__ void __launch_bounds__(256) lds_probe(float* out, int32_t iters) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  constexpr int kBytes = 65536;
  constexpr int kWords = kBytes / WIDTH;  // per block, >= 16 x 256
  __shared__ __align__(16) f4 buf[kBytes / 16];
  const int32_t lane = threadIdx.x;
  for (int32_t i = lane; i < kBytes / 16; i += blockDim.x) buf[i] = f4{(float)i, 1.0f, 2.0f, 3.0f};
  __syncthreads();
  float acc = 0.0f;
  for (int32_t i = 0; i < iters; ++i) {
    const int32_t sh = (64 * i) & (kWords - 1);  // repeats only after kWords / 64 steps
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int32_t w = (lane + 256 * u + sh) & (kWords - 1);
      if (WIDTH == 4) {
        float* p = reinterpret_cast<float*>(buf) + w;
        if (WRITE)
          *p = acc + (float)u;
        else
          acc += *p;
      } else if (WIDTH == 8) {
        f2* p = reinterpret_cast<f2*>(buf) + w;
        if (WRITE) {
          *p = f2{acc, (float)u};
        } else {
          const f2 v = *p;
          acc += v.x + v.y;
        }
      } else {
        f4* p = buf + w;
        if (WRITE) {
          *p = f4{acc, (float)u, acc, (float)i};
        } else {
          const f4 v = *p;
          acc += (v.x + v.y) + (v.z + v.w);
        }
      }
    }
    if (WRITE) acc += 1.0f;
  }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc + reinterpret_cast<float*>(buf)[lane];
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
                        lds_probe<4, true>,  lds_probe<8, true>,  lds_probe<16, true>};

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

// LDS probe: mode 0..2 reads of 4, 8, 16 bytes per lane, 3..5 writes.
// Bytes moved: blocks * 256 * iters * 16 * width. Returns ms as above.
double laim_probe_lds(int32_t mode, int32_t blocks, int32_t iters, float* out) {
  if (mode < 0 || mode > 5 || blocks < 1 || iters < 1 || !out) return -1.0;
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
