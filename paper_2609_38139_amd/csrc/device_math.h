// device_math.h -- device-side primitives of the decoder: the counter-based
// generator behind every random draw, and the FP32 arithmetic of the BP
// check rule (BP-LLR2). Compiled with -ffp-contract=off: every expression
// below is one IEEE operation per arithmetic operator (fmaf one fused
// operation), evaluated in the order written, so results are reproducible
// bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace laim {

// Work-item and work-group indices, the work-group size, and the high half
// of a 32-bit product, from the compiler's builtins. The kernels are built
// with IEEE mode off (-mno-amdgpu-ieee); the device library behind
// threadIdx, blockIdx, blockDim and __umulhi is not, so its accessors would
// not be inlined (their floating-point modes differ) and every use would be
// a function call.
__device__ __forceinline__ uint32_t tid_x() { return __builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ uint32_t bid_x() { return __builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ uint32_t bid_y() { return __builtin_amdgcn_workgroup_id_y(); }
__device__ __forceinline__ uint32_t bdim_x() { return __builtin_amdgcn_workgroup_size_x(); }
__device__ __forceinline__ uint32_t mulhi_u32(uint32_t a, uint32_t b) {
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
// easy as 1, 2, 3", SC'11). Ten rounds of the 4x32 S-box: the products of
// words 0 and 2 with the two round multipliers are split into halves; the
// high halves are mixed into words 1 and 3 together with the round key;
// the round key advances by the two Weyl constants after each round.
struct Philox4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t a = 0xD2511F53u * c0;                  // low half of M0 * c0
    const uint32_t ah = mulhi_u32(0xD2511F53u, c0);        // high half
    const uint32_t b = 0xCD9E8D57u * c2;
    const uint32_t bh = mulhi_u32(0xCD9E8D57u, c2);
    const uint32_t n0 = bh ^ c1 ^ k0;
    const uint32_t n2 = ah ^ c3 ^ k1;
    c0 = n0;
    c1 = b;
    c2 = n2;
    c3 = a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Philox4{c0, c1, c2, c3};
}

// Bernoulli event "w < bound" with a 64-bit bound (bound = 2^32 means always).
__device__ __forceinline__ bool below(uint32_t w, uint64_t bound) { return (uint64_t)w < bound; }

__device__ __forceinline__ float clampf(float x, float c) { return fminf(fmaxf(x, -c), c); }

// Smallest of three (exact; the compiler forms one v_min3_f32).
__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }

// min(|a|, |b|, |c|) as a single v_min3_f32. Written as an asm statement so
// that the compiler cannot split several of them into two-input minima
// shared between results, which costs one more instruction per four.
// Exact, and equal to min3f(fabsf(a), fabsf(b), fabsf(c)) for non-NaN input.
__device__ __forceinline__ float min3_abs(float a, float b, float c) {
  float r;
  asm("v_min3_f32 %0, |%1|, |%2|, |%3|" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// e^{-a} for a >= 0, by Cody-Waite reduction -a = k ln2 + r (ln2 split into
// a head with 16 significant bits, so k*head is exact, and a tail), the
// degree-7 Taylor polynomial of e^r in Horner form with one fused
// multiply-add (v_fma_f32, a single rounding) per step, and a 2^k scale
// built in the exponent field. Arguments above 80 (and +inf) give 0. The
// evaluation has no branch: an argument above 80 is evaluated as 80 and the
// result then replaced by 0, so every lane runs the same instructions and
// the results for a <= 80 are those of the plain sequence.
__device__ __forceinline__ float exp_neg(float a) {
  const bool big = !(a <= 80.0f);
  const float ln2_hi = __uint_as_float(0x3F317200u);
  const float ln2_lo = (float)(0.69314718055994530942 - 0.693145751953125);
  const float log2e = (float)1.44269504088896340736;
  const float x = -(big ? 80.0f : a);
  const float kf = floorf(fmaf(x, log2e, 0.5f));
  const float r = fmaf(-kf, ln2_lo, fmaf(-kf, ln2_hi, x));
  float p = 1.0f / 5040.0f;
  p = fmaf(p, r, 1.0f / 720.0f);
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  const int k = (int)kf;
  const float v = p * __uint_as_float((uint32_t)(k + 127) << 23);
  return big ? 0.0f : v;
}

// log(1 + u) for u in [0, 1] as u Q(u), Q the degree-9 polynomial that
// interpolates log(1 + u)/u at the 10 Chebyshev nodes of [0, 1] (computed in
// high precision, coefficients rounded to FP32), in Horner form with one
// fused multiply-add per step: no division, under 3 ulp of relative error.
__device__ __forceinline__ float log1p_unit(float u) {
  float q = -0x1.a04acap-9f;
  q = fmaf(q, u, 0x1.402f4cp-6f);
  q = fmaf(q, u, -0x1.cdd008p-5f);
  q = fmaf(q, u, 0x1.afdde8p-4f);
  q = fmaf(q, u, -0x1.38b908p-3f);
  q = fmaf(q, u, 0x1.92b430p-3f);
  q = fmaf(q, u, -0x1.ff0254p-3f);
  q = fmaf(q, u, 0x1.554bd6p-2f);
  q = fmaf(q, u, -0x1.ffffb8p-2f);
  q = fmaf(q, u, 1.0f);
  return u * q;
}

// log(1 + e^{-y}), y >= 0.
__device__ __forceinline__ float softplus_neg(float y) { return log1p_unit(exp_neg(y)); }

// a [+] b = 2 atanh(tanh(a/2) tanh(b/2)) (the two-input sum-product check
// rule; Hagenauer, Offer, Papke 1996), through its exact rewriting on the
// magnitudes |a| [+] |b| = min + log(1 + e^{-(|a|+|b|)}) - log(1 + e^{-||a|-|b||}),
// a negative rounding set to +0, and the sign sg(a) sg(b) with sg(x) = -1
// iff x < 0 for a nonzero result (a zero result is +0).
__device__ __forceinline__ float boxplus(float a, float b) {
  const float aa = fabsf(a);
  const float ab = fabsf(b);
  const float mn = (ab < aa) ? ab : aa;
  const float d = (aa < ab) ? (ab - aa) : (aa - ab);
  float mag = (mn + softplus_neg(aa + ab)) - softplus_neg(d);
  if (mag < 0.0f) mag = 0.0f;
  const bool neg = (a < 0.0f) != (b < 0.0f);
  return (neg && mag > 0.0f) ? -mag : mag;
}

// The sum-product check rule's box-plus of all inputs but one, for every
// output: acc[j] = F_{j-1} [+] B_{j+1} with the ascending prefix folds
// F_k = F_{k-1} [+] x_k and the suffix folds B_k = x_k [+] B_{k+1}; an
// empty side is dropped ((+inf) [+] y is y with -0 made +0, i.e. y + 0).
// Inputs x[0 .. deg); deg = DC when REG. 3 (deg - 2) box-plus steps.
template <int DC, bool REG>
__device__ __forceinline__ void boxplus_others(const float* x, int32_t deg, float* acc) {
  float F[DC], B[DC];
  if (REG) {
    F[0] = x[0] + 0.0f;
#pragma unroll
    for (int k = 1; k < DC - 1; ++k) F[k] = boxplus(F[k - 1], x[k]);
    B[DC - 1] = x[DC - 1] + 0.0f;
#pragma unroll
    for (int k = DC - 2; k >= 1; --k) B[k] = boxplus(x[k], B[k + 1]);
    acc[0] = B[1];
    acc[DC - 1] = F[DC - 2];
#pragma unroll
    for (int j = 1; j < DC - 1; ++j) acc[j] = boxplus(F[j - 1], B[j + 1]);
  } else {
    F[0] = x[0] + 0.0f;
#pragma unroll
    for (int k = 1; k < DC; ++k) F[k] = (k < deg) ? boxplus(F[k - 1], x[k]) : F[k - 1];
    B[DC - 1] = (DC - 1 < deg) ? x[DC - 1] + 0.0f : __builtin_inff();
#pragma unroll
    for (int k = DC - 2; k >= 0; --k)
      B[k] = (k >= deg) ? __builtin_inff() : (k == deg - 1 ? x[k] + 0.0f : boxplus(x[k], B[k + 1]));
#pragma unroll
    for (int j = 0; j < DC; ++j) {
      if (j >= deg) continue;
      if (j == 0)
        acc[j] = (deg >= 2) ? B[1] : __builtin_inff();
      else if (j == deg - 1)
        acc[j] = F[j - 1];
      else
        acc[j] = boxplus(F[j - 1], B[j + 1]);
    }
  }
}

}  // namespace laim
