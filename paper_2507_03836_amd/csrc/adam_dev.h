// The Adam update of one parameter, shared by the dense sweep and the deferred
// (lazy) update kernels so that both apply bit-identical arithmetic.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <math.h>
#include <stdint.h>

#include "fhash.h"

namespace fh {

// FP32 constants of one step.  step_size = lr / (1 - b1^t) and
// inv_bc2_sqrt = 1 / sqrt(1 - b2^t) are formed in double on the host.
struct AdamK {
  float step_size, b1, omb1, b2, omb2, eps, inv_bc2_sqrt, gscale;
};

// Host: the constants of a step from its descriptor.
inline AdamK make_adam_k(const fhash_adam_desc* o) {
  AdamK k;
  const double bc1 = 1.0 - pow(o->beta1, (double)o->step);
  const double bc2 = 1.0 - pow(o->beta2, (double)o->step);
  k.step_size = (float)(o->lr / bc1);
  k.inv_bc2_sqrt = (float)(1.0 / sqrt(bc2));
  k.b1 = (float)o->beta1;
  k.omb1 = (float)(1.0 - o->beta1);
  k.b2 = (float)o->beta2;
  k.omb2 = (float)(1.0 - o->beta2);
  k.eps = (float)o->eps;
  k.gscale = (float)o->grad_scale;
  return k;
}

// Float offset of the moment of parameter a: a itself, or, when the moments
// are stored in runs of 16 separated by 16-float gaps (paired: m runs
// alternate with v runs, v = m + 16; with parameters: m runs follow the
// parameters' runs, v runs the gradients'), 32 (a / 16) + a % 16.
template <bool PAIRED>
__host__ __device__ __forceinline__ int64_t moment_off(int64_t a) {
  if constexpr (PAIRED)
    return ((a >> 4) << 5) + (a & 15);
  else
    return a;
}

#ifdef __HIPCC__
// One Adam step (PyTorch semantics, bias-corrected, no weight decay) with
// every rounding spelled out and contraction off, so that every kernel that
// inlines it computes the same bits:
//   gs = g * gscale;  m = b1 m + (1-b1) gs;  v = b2 v + (1-b2) gs^2;
//   p = fma(-step_size, m * (1 / (sqrt(v) * inv_bc2_sqrt + eps)), p).
// The square root and the reciprocal are the hardware's (v_sqrt_f32,
// v_rcp_f32: within 1 ulp, deterministic); the quotient is not correctly
// rounded, which stays far inside the FP32 tolerance against the FP64 update.
__device__ __forceinline__ void adam1(const AdamK& k, float g, float& p, float& m, float& v) {
#pragma clang fp contract(off)
  const float gs = g * k.gscale;
  m = __fmaf_rn(k.b1, m, k.omb1 * gs);
  v = __fmaf_rn(k.b2, v, (k.omb2 * gs) * gs);
  const float denom = __fmaf_rn(__builtin_amdgcn_sqrtf(v), k.inv_bc2_sqrt, k.eps);
  p = __fmaf_rn(-k.step_size, m * __builtin_amdgcn_rcpf(denom), p);
}

// adam1 with g = +0 and a finite gscale: gs is a zero, so (1-b1) gs and
// (1-b2) gs^2 are zeros and the two fused multiply-adds reduce to the plain
// products fl(b1 m) and fl(b2 v) (m and v are never -0: both start at +0, and
// an fma returns -0 only from two -0 terms).  Same bits as adam1(k, +0, ...).
__device__ __forceinline__ void adam0(const AdamK& k, float& p, float& m, float& v) {
#pragma clang fp contract(off)
  m = k.b1 * m;
  v = k.b2 * v;
  const float denom = __fmaf_rn(__builtin_amdgcn_sqrtf(v), k.inv_bc2_sqrt, k.eps);
  p = __fmaf_rn(-k.step_size, m * __builtin_amdgcn_rcpf(denom), p);
}

__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void store_shadow(void* sh, int dt, int64_t i, float x) {
  if (dt == FHASH_F16)
    reinterpret_cast<__half*>(sh)[i] = __float2half_rn(x);
  else
    reinterpret_cast<uint16_t*>(sh)[i] = to_bf16_rne(x);
}
#endif

}  // namespace fh
