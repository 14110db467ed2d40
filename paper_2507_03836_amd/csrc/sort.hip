// Sort training samples by a 4D Morton key of their positions (positions
// quantised to 256 cells per axis, bits interleaved x, y, z, t), so that samples
// of the same cells are neighbours: the gathers reuse cache lines and the
// scatter-add can combine equal slots of neighbouring lanes before its atomics.
// The order changes neither the MSE loss (a mean) nor its gradient (a sum).
//
// Stable LSD radix sort, 4 passes of 8-bit digits over 1024-element tiles:
// per-tile digit histograms -> an exclusive scan of every digit's row of tile
// counts (one workgroup per digit) and the digits' totals -> a scatter that
// adds the digit's base (the totals' exclusive prefix, formed in LDS by every
// workgroup), in which each wave ranks equal digits with 8 ballots and waves
// are ordered through LDS, so every pass is stable.
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

constexpr int kTile = 1024;

__device__ __forceinline__ uint32_t spread4(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) r |= ((v >> i) & 1u) << (4 * i);
  return r;
}

__device__ __forceinline__ uint32_t q8(float p) {
  p = fminf(fmaxf(p, 0.0f), 1.0f);
  const int q = (int)(p * 256.0f);
  return (uint32_t)(q > 255 ? 255 : q);
}

__global__ void __launch_bounds__(256)
    keys_kernel(const float4* __restrict__ pos, int64_t n, uint32_t* __restrict__ key,
                uint32_t* __restrict__ val) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float4 p = pos[i];
    key[i] = spread4(q8(p.x)) | (spread4(q8(p.y)) << 1) | (spread4(q8(p.z)) << 2) |
             (spread4(q8(p.w)) << 3);
    val[i] = (uint32_t)i;
  }
}

__global__ void __launch_bounds__(kTile)
    hist_kernel(const uint32_t* __restrict__ key, int64_t n, int shift, int64_t nb,
                uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  if (threadIdx.x < 256) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)kTile + threadIdx.x;
  if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  __syncthreads();
  if (threadIdx.x < 256) hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of one digit's row of tile counts, hist[d * nb + 0 .. nb),
// in place (workgroup d, 1024 threads, 1024 entries per round with a carry);
// the row's total goes to tot[d].
__global__ void __launch_bounds__(1024)
    row_scan_kernel(uint32_t* __restrict__ hist, int64_t nb, uint32_t* __restrict__ tot) {
  __shared__ uint32_t wsum[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t* row = hist + (int64_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (int64_t r0 = 0; r0 < nb; r0 += 1024) {
    const int64_t i = r0 + threadIdx.x;
    const uint32_t v = i < nb ? row[i] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      before += w < wid ? wsum[w] : 0u;
      all += wsum[w];
    }
    if (i < nb) row[i] = carry + before + x - v;
    carry += all;
    __syncthreads();  // wsum is rewritten by the next round
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kTile)
    scatter_kernel(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                   uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n, int shift,
                   int64_t nb, const uint32_t* __restrict__ off, const uint32_t* __restrict__ tot) {
  __shared__ uint32_t cnt[kTile / 64][256];
  __shared__ uint32_t base[256];
  for (int e = threadIdx.x; e < (kTile / 64) * 256; e += kTile) (&cnt[0][0])[e] = 0;
  if (threadIdx.x < 64) {
    // digit bases: the exclusive prefix of the 256 digit totals, 4 per lane
    uint32_t t[4], s4 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      t[j] = tot[4 * threadIdx.x + j];
      s4 += t[j];
    }
    uint32_t x = s4;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if ((int)threadIdx.x >= o) x += y;
    }
    uint32_t run = x - s4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      base[4 * threadIdx.x + j] = run;
      run += t[j];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = blockIdx.x * (int64_t)kTile + threadIdx.x;
  const bool valid = i < n;
  const uint32_t k = valid ? kin[i] : 0u;
  const uint32_t d = (k >> shift) & 255u;
  uint64_t eq = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bb = __ballot(valid && ((d >> b) & 1u));
    eq &= ((d >> b) & 1u) ? bb : ~bb;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t rank = (uint32_t)__popcll(eq & lt);
  if (valid && (eq & lt) == 0ull) cnt[w][d] = (uint32_t)__popcll(eq);
  __syncthreads();
  if (threadIdx.x < 256) {
    uint32_t run = 0;
    for (int ww = 0; ww < kTile / 64; ++ww) {
      const uint32_t c = cnt[ww][threadIdx.x];
      cnt[ww][threadIdx.x] = run;
      run += c;
    }
  }
  __syncthreads();
  if (valid) {
    const uint32_t p = base[d] + off[d * nb + blockIdx.x] + cnt[w][d] + rank;
    kout[p] = k;
    vout[p] = vin[i];
  }
}

__global__ void __launch_bounds__(256)
    permute_kernel(const float4* __restrict__ pin, const float* __restrict__ tin,
                   const uint32_t* __restrict__ idx, int64_t n, float4* __restrict__ pout,
                   float* __restrict__ tout) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t j = idx[i];
    pout[i] = pin[j];
    if (tout != nullptr) tout[i] = tin[j];
  }
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

inline unsigned grid256(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

size_t sort_ws_bytes(int64_t n) {
  const int64_t nb = (n + kTile - 1) / kTile;
  return 4 * al(n * 4) + al(nb * 256 * 4) + al(256 * 4) + al(n * 16) + al(n * 4);
}

hipError_t launch_sort_samples(float* pos, float* target, int64_t n, void* ws, hipStream_t st) {
  if (n <= 1) return hipSuccess;
  const int64_t nb = (n + kTile - 1) / kTile;
  char* p = static_cast<char*>(ws);
  uint32_t* k0 = reinterpret_cast<uint32_t*>(p);
  p += al(n * 4);
  uint32_t* v0 = reinterpret_cast<uint32_t*>(p);
  p += al(n * 4);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(p);
  p += al(n * 4);
  uint32_t* v1 = reinterpret_cast<uint32_t*>(p);
  p += al(n * 4);
  uint32_t* hist = reinterpret_cast<uint32_t*>(p);
  p += al(nb * 256 * 4);
  uint32_t* tot = reinterpret_cast<uint32_t*>(p);
  p += al(256 * 4);
  float4* pcopy = reinterpret_cast<float4*>(p);
  p += al(n * 16);
  float* tcopy = reinterpret_cast<float*>(p);
  hipLaunchKernelGGL(keys_kernel, dim3(grid256(n)), dim3(256), 0, st,
                     reinterpret_cast<const float4*>(pos), n, k0, v0);
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)nb), dim3(kTile), 0, st, k0, n, shift, nb,
                       hist);
    hipLaunchKernelGGL(row_scan_kernel, dim3(256), dim3(1024), 0, st, hist, nb, tot);
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)nb), dim3(kTile), 0, st, k0, v0, k1, v1, n,
                       shift, nb, hist, tot);
    uint32_t* t = k0;
    k0 = k1;
    k1 = t;
    t = v0;
    v0 = v1;
    v1 = t;
  }
  hipError_t e = hipMemcpyAsync(pcopy, pos, n * 16, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  if (target != nullptr) {
    e = hipMemcpyAsync(tcopy, target, n * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(permute_kernel, dim3(grid256(n)), dim3(256), 0, st, pcopy,
                     target ? tcopy : nullptr, v0, n, reinterpret_cast<float4*>(pos), target);
  return hipGetLastError();
}

}  // namespace fh
