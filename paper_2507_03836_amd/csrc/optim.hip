// Dense Adam step with loss-scale unscaling, overflow skip, low-precision
// shadow write and gradient zeroing; finite check; casts; FP64 reductions.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "adam_dev.h"
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void adam4(const AdamK& k, const f4v g, f4v& p, f4v& m, f4v& v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float pc = p[c], mc = m[c], vc = v[c];
    adam1(k, g[c], pc, mc, vc);
    p[c] = pc;
    m[c] = mc;
    v[c] = vc;
  }
}

__device__ __forceinline__ void store_shadow4(void* shadow, int sdt, int64_t i, const f4v pp) {
  uint2 raw;
  if (sdt == FHASH_F16) {
    __half2 a = __floats2half2_rn(pp[0], pp[1]), b = __floats2half2_rn(pp[2], pp[3]);
    raw.x = *reinterpret_cast<uint32_t*>(&a);
    raw.y = *reinterpret_cast<uint32_t*>(&b);
  } else {
    raw.x = (uint32_t)to_bf16_rne(pp[0]) | ((uint32_t)to_bf16_rne(pp[1]) << 16);
    raw.y = (uint32_t)to_bf16_rne(pp[2]) | ((uint32_t)to_bf16_rne(pp[3]) << 16);
  }
  // streamed like the other arrays: a non-temporal 8-byte store
  const uint64_t word = (uint64_t)raw.x | ((uint64_t)raw.y << 32);
  __builtin_nontemporal_store(word, reinterpret_cast<uint64_t*>(shadow) + i);
}

// Streaming sweep: every array is touched once, so loads and stores bypass the
// caches' retention (non-temporal) and each thread keeps two float4 groups in
// flight.  The gradient is reset only where it is nonzero.
// Gradient read of the float4 group at logical index f (a multiple of 4)
// under touched-segment tracking: a group that lies inside [tb, te) is read
// only when its segment is flagged (otherwise the gradient is zero there); a
// group that opens a segment in the range clears its flag after the read.
// The 4 groups of a segment are 4 consecutive lanes of one wave, so all of
// them have read the flag before the clearing store.
__device__ __forceinline__ void tracked_load(const float* __restrict__ g, int64_t f, int64_t pm,
                                             uint8_t* __restrict__ touch, int64_t tb, int64_t te,
                                             f4v& out) {
  const f4v* g4 = reinterpret_cast<const f4v*>(g + run_off(f, pm));
  if (touch == nullptr || f < tb || f >= te) {
    out = __builtin_nontemporal_load(g4);
    return;
  }
  const int64_t seg = f / FHASH_TOUCH_FLOATS;
  if (f + 4 <= te && touch[seg] == 0) {
    out = (f4v){0.0f, 0.0f, 0.0f, 0.0f};
  } else {
    out = __builtin_nontemporal_load(g4);
  }
  if ((f % FHASH_TOUCH_FLOATS) == 0) touch[seg] = 0;
}

// The parameters [first, first + n) of the vector (first: a multiple of 4).
// p, g, m, v and shadow point at the vector's start; parameter a sits at
// p / g + run_off(a, pm) (pm = ~15: parameters and gradients in runs of 16,
// interleaved with m and v), at m / v + moment_off<PAIRED>(a) and at
// shadow[a].
template <bool PAIRED>
__global__ void __launch_bounds__(256)
    adam_kernel(AdamK k, float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                float* __restrict__ v, void* __restrict__ shadow, int sdt, int64_t n,
                int64_t first, int64_t pm, const int32_t* __restrict__ found_inf,
                uint8_t* __restrict__ touch, int64_t tb, int64_t te) {
  const bool skip = (found_inf != nullptr) && (*found_inf != 0);
  const int64_t n4 = n >> 2;
  const int64_t S = (int64_t)gridDim.x * blockDim.x;
  auto p4 = [&](int64_t i) { return reinterpret_cast<f4v*>(p + run_off(first + 4 * i, pm)); };
  auto g4 = [&](int64_t i) { return reinterpret_cast<f4v*>(g + run_off(first + 4 * i, pm)); };
  auto m4 = [&](int64_t i) { return reinterpret_cast<f4v*>(m + moment_off<PAIRED>(first + 4 * i)); };
  auto v4 = [&](int64_t i) { return reinterpret_cast<f4v*>(v + moment_off<PAIRED>(first + 4 * i)); };
  const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += 2 * S) {
    const int64_t j = i + S;
    const bool two = j < n4;
    f4v g0, g1 = zero;
    tracked_load(g, first + 4 * i, pm, touch, tb, te, g0);
    if (two) tracked_load(g, first + 4 * j, pm, touch, tb, te, g1);
    if (!skip) {
      f4v p0 = __builtin_nontemporal_load(p4(i)), m0 = __builtin_nontemporal_load(m4(i));
      f4v v0 = __builtin_nontemporal_load(v4(i));
      f4v p1 = zero, m1 = zero, v1 = zero;
      if (two) {
        p1 = __builtin_nontemporal_load(p4(j));
        m1 = __builtin_nontemporal_load(m4(j));
        v1 = __builtin_nontemporal_load(v4(j));
      }
      adam4(k, g0, p0, m0, v0);
      __builtin_nontemporal_store(p0, p4(i));
      __builtin_nontemporal_store(m0, m4(i));
      __builtin_nontemporal_store(v0, v4(i));
      if (shadow != nullptr) store_shadow4(shadow, sdt, first / 4 + i, p0);
      if (two) {
        adam4(k, g1, p1, m1, v1);
        __builtin_nontemporal_store(p1, p4(j));
        __builtin_nontemporal_store(m1, m4(j));
        __builtin_nontemporal_store(v1, v4(j));
        if (shadow != nullptr) store_shadow4(shadow, sdt, first / 4 + j, p1);
      }
    }
    if (g0[0] != 0.0f || g0[1] != 0.0f || g0[2] != 0.0f || g0[3] != 0.0f)
      __builtin_nontemporal_store(zero, g4(i));
    if (two && (g1[0] != 0.0f || g1[1] != 0.0f || g1[2] != 0.0f || g1[3] != 0.0f))
      __builtin_nontemporal_store(zero, g4(j));
  }
  // Tail (n not a multiple of 4).
  const int64_t t = (n4 << 2) + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n && t < (n4 << 2) + 4) {
    const int64_t a = first + t, po = run_off(a, pm);
    const float gg = g[po];
    if (!skip) {
      const int64_t mo = moment_off<PAIRED>(a);
      float pp = p[po], mm = m[mo], vv = v[mo];
      adam1(k, gg, pp, mm, vv);
      p[po] = pp;
      m[mo] = mm;
      v[mo] = vv;
      if (shadow != nullptr) store_shadow(shadow, sdt, a, pp);
    }
    if (gg != 0.0f) g[po] = 0.0f;
  }
}

__global__ void __launch_bounds__(256)
    check_finite_kernel(const float* __restrict__ g, int64_t n, int32_t* __restrict__ found) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(g[i]);
  bad = __syncthreads_or(bad);
  if (bad && threadIdx.x == 0) atomicOr(found, 1);
}

__global__ void __launch_bounds__(256)
    cast_kernel(const float* __restrict__ src, void* __restrict__ dst, int dt, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    store_shadow(dst, dt, i, src[i]);
}

__device__ __forceinline__ double block_sum_double(double v) {
  __shared__ double sh[16];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

__global__ void __launch_bounds__(256)
    sq_err_kernel(const float* __restrict__ y, const float* __restrict__ v, int64_t n,
                  double* __restrict__ sum) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double r = (double)y[i] - (double)v[i];
    acc += r * r;
  }
  const double tot = block_sum_double(acc);
  if (threadIdx.x == 0) unsafeAtomicAdd(sum, tot);
}

__global__ void __launch_bounds__(256)
    mse_grad_kernel(const float* __restrict__ y, const float* __restrict__ v, int64_t n,
                    float coef, float* __restrict__ dy, double* __restrict__ sum) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[i] - v[i];
    dy[i] = coef * r;
    acc += (double)r * (double)r;
  }
  if (sum != nullptr) {
    const double tot = block_sum_double(acc);
    if (threadIdx.x == 0) unsafeAtomicAdd(sum, tot);
  }
}

// d_params[p] += sum_w part[w][p]: 16 columns x 16 row groups per block, fixed
// summation order (deterministic).
__global__ void __launch_bounds__(256)
    reduce_partials_kernel(const float* __restrict__ part, int64_t nwav, int64_t P,
                           float* __restrict__ d_params) {
  __shared__ float sh[16][17];
  const int col = threadIdx.x & 15, rg = threadIdx.x >> 4;
  const int64_t p = blockIdx.x * 16 + col;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  if (p < P) {
    int64_t w = rg;
    for (; w + 48 < nwav; w += 64) {
      a0 += part[w * P + p];
      a1 += part[(w + 16) * P + p];
      a2 += part[(w + 32) * P + p];
      a3 += part[(w + 48) * P + p];
    }
    for (; w < nwav; w += 16) a0 += part[w * P + p];
  }
  sh[rg][col] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (rg == 0 && p < P) {
    float s = 0.f;
    for (int r = 0; r < 16; ++r) s += sh[r][col];
    d_params[p] += s;
  }
}

inline unsigned blocks_for(int64_t n, int64_t per_thread) {
  int64_t b = (n / per_thread + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_adam(const fhash_adam_desc* o, float* p, float* g, float* m, float* v,
                       void* shadow, fhash_dtype sdt, int64_t n, int64_t first,
                       const int32_t* found_inf, const fhash_touch* touch, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const AdamK k = make_adam_k(o);
  // Two float4 groups per thread per iteration; a deep grid keeps every CU's
  // memory pipeline full (measured best on MI355X: ~128K workgroups).
  int64_t b = (n / 8 + 255) / 256;
  if (b > 131072) b = 131072;
  if (b < 1) b = 1;
  uint8_t* tf = touch ? touch->flags : nullptr;
  const int64_t tb = touch ? touch->begin : 0, te = touch ? touch->end : 0;
  // moments with parameters: p, g (and m, v) in runs of 16; paired: m, v only
  const int64_t pm = o->moments == FHASH_MOMENTS_WITH_PARAMS ? ~(int64_t)15 : 0;
  if (o->moments != FHASH_MOMENTS_SEPARATE)
    hipLaunchKernelGGL(adam_kernel<true>, dim3((unsigned)b), dim3(256), 0, st, k, p, g, m, v,
                       shadow, (int)sdt, n, first, pm, found_inf, tf, tb, te);
  else
    hipLaunchKernelGGL(adam_kernel<false>, dim3((unsigned)b), dim3(256), 0, st, k, p, g, m, v,
                       shadow, (int)sdt, n, first, pm, found_inf, tf, tb, te);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* part, int64_t nwav, int64_t P, float* d_params,
                                  hipStream_t st) {
  if (P == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((P + 15) / 16)), dim3(256), 0, st,
                     part, nwav, P, d_params);
  return hipGetLastError();
}

hipError_t launch_check_finite(const float* g, int64_t n, int32_t* found, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3(blocks_for(n, 4)), dim3(256), 0, st, g, n, found);
  return hipGetLastError();
}

hipError_t launch_cast(const float* src, void* dst, fhash_dtype dt, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_kernel, dim3(blocks_for(n, 4)), dim3(256), 0, st, src, dst, (int)dt, n);
  return hipGetLastError();
}

hipError_t launch_sq_err(const float* y, const float* v, int64_t n, double* sum, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(sq_err_kernel, dim3(blocks_for(n, 8)), dim3(256), 0, st, y, v, n, sum);
  return hipGetLastError();
}

hipError_t launch_mse_grad(const float* y, const float* v, int64_t n, float coef, float* dy,
                           double* sum, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks_for(n, 8)), dim3(256), 0, st, y, v, n, coef, dy,
                     sum);
  return hipGetLastError();
}

}  // namespace fh
