// Device version of the seeded synthetic-input generator (same definitions as
// synth.c, evaluated in FP64 on the GPU) for production-shape volumes that are
// too large to generate on the host: the field, its min-max normalisation, the
// gradient-magnitude attribute and the order statistic that sets the feature
// threshold value.  Inputs only: the feature mask, its dilation and the
// coreset are computed from these by the method's own calls.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

namespace {

__device__ __forceinline__ uint64_t sm64(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double vn_lattice(uint64_t seed, int64_t X, int64_t Y, int64_t Z,
                                             int64_t T) {
  uint64_t h = seed;
  h ^= sm64((uint64_t)X * 0x8CB92BA72F3D8DD7ull);
  h = sm64(h ^ ((uint64_t)Y * 0xD6E8FEB86659FD93ull));
  h = sm64(h ^ ((uint64_t)Z * 0xA0761D6478BD642Full));
  h = sm64(h ^ ((uint64_t)T * 0xE7037ED1A0B428DBull));
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double smooth(double u) { return u * u * (3.0 - 2.0 * u); }

__device__ double value_noise4(uint64_t seed, double x, double y, double z, double t) {
  const double q[4] = {x, y, z, t};
  int64_t b[4];
  double w[4];
  for (int d = 0; d < 4; ++d) {
    const double fl = floor(q[d]);
    b[d] = (int64_t)fl;
    w[d] = smooth(q[d] - fl);
  }
  double acc = 0.0;
  for (int c = 0; c < 16; ++c) {
    double wc = 1.0;
    for (int d = 0; d < 4; ++d) wc *= ((c >> d) & 1) ? w[d] : 1.0 - w[d];
    acc += wc * vn_lattice(seed, b[0] + (c & 1), b[1] + ((c >> 1) & 1), b[2] + ((c >> 2) & 1),
                           b[3] + ((c >> 3) & 1));
  }
  return acc;
}

__global__ void field_kernel(int64_t Sx, int64_t Sy, int64_t Sz, int64_t T,
                             const double* __restrict__ blobs, int n_blobs, double turb,
                             uint64_t nseed, int clip01, float* __restrict__ out) {
  const int64_t N = Sx * Sy * Sz * T;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q % Sx, j = (q / Sx) % Sy, k = (q / (Sx * Sy)) % Sz, n = q / (Sx * Sy * Sz);
    const double x = (double)i / (double)(Sx - 1), y = (double)j / (double)(Sy - 1);
    const double z = (double)k / (double)(Sz - 1);
    const double t = T > 1 ? (double)n / (double)(T - 1) : 0.0;
    double f = 0.0;
    for (int b = 0; b < n_blobs; ++b) {
      const double* o = blobs + 8 * b;
      const double dx = x - (o[0] + n * o[5]), dy = y - (o[1] + n * o[6]);
      const double dz = z - (o[2] + n * o[7]);
      f += o[4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * o[3] * o[3]));
    }
    if (turb != 0.0) {
      double s = 1.0;
      for (int oc = 0; oc < 3; ++oc) {
        const double m = (double)(1 << oc);
        f += turb * s * value_noise4(nseed + (uint64_t)oc, 8.0 * x * m, 8.0 * y * m, 8.0 * z * m,
                                     4.0 * t * m);
        s *= 0.5;
      }
    }
    if (clip01) f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    out[q] = (float)f;
  }
}

__global__ void minmax_kernel(const float* __restrict__ f, int64_t N, unsigned* __restrict__ mm) {
  float lo = 3.4e38f, hi = -3.4e38f;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N;
       q += (int64_t)gridDim.x * blockDim.x) {
    lo = fminf(lo, f[q]);
    hi = fmaxf(hi, f[q]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, 64));
    hi = fmaxf(hi, __shfl_xor(hi, off, 64));
  }
  // order-preserving integer keys of floats
  auto key = [](float v) {
    unsigned u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  };
  if ((threadIdx.x & 63) == 0) {
    atomicMin(mm, key(lo));
    atomicMax(mm + 1, key(hi));
  }
}

__global__ void normalise_kernel(float* __restrict__ f, int64_t N, const unsigned* __restrict__ mm) {
  auto val = [](unsigned k) {
    unsigned u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
  };
  const double lo = val(mm[0]), hi = val(mm[1]);
  const double inv = hi > lo ? 1.0 / (hi - lo) : 0.0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N;
       q += (int64_t)gridDim.x * blockDim.x)
    f[q] = (float)(((double)f[q] - lo) * inv);
}

__global__ void grad_kernel(int64_t Sx, int64_t Sy, int64_t Sz, int64_t T,
                            const float* __restrict__ f, float* __restrict__ g) {
  const int64_t N = Sx * Sy * Sz * T;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx[3] = {q % Sx, (q / Sx) % Sy, (q / (Sx * Sy)) % Sz};
    const int64_t ext[3] = {Sx, Sy, Sz}, stride[3] = {1, Sx, Sx * Sy};
    double g2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      double gd;
      if (ext[d] < 2) gd = 0.0;
      else if (idx[d] == 0) gd = (double)f[q + stride[d]] - f[q];
      else if (idx[d] == ext[d] - 1) gd = (double)f[q] - f[q - stride[d]];
      else gd = 0.5 * ((double)f[q + stride[d]] - f[q - stride[d]]);
      g2 += gd * gd;
    }
    g[q] = (float)sqrt(g2);
  }
}

// Histogram of 12-bit digits of non-negative float bit patterns whose higher
// bits equal `prefix` (radix select, 3 passes: bits 31..20, 19..8, 7..0).
__global__ void hist_kernel(const float* __restrict__ v, int64_t N, int shift, unsigned pmask,
                            unsigned prefix, unsigned long long* __restrict__ hist, int nbins) {
  __shared__ unsigned h[4096];
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N;
       q += (int64_t)gridDim.x * blockDim.x) {
    const unsigned u = __float_as_uint(v[q]);
    if ((u & pmask) == prefix) atomicAdd(&h[(u >> shift) & (nbins - 1)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], (unsigned long long)h[b]);
}

inline unsigned nblk(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

extern "C" {

int sy_gpu_field(const int64_t* dims, const double* blobs_dev, int n_blobs, double turb,
                 uint64_t nseed, int clip01, float* out, void* stream) {
  const int64_t N = dims[0] * dims[1] * dims[2] * dims[3];
  hipLaunchKernelGGL(field_kernel, dim3(nblk(N)), dim3(256), 0, (hipStream_t)stream, dims[0],
                     dims[1], dims[2], dims[3], blobs_dev, n_blobs, turb, nseed, clip01, out);
  return (int)hipGetLastError();
}

int sy_gpu_normalise(float* f, int64_t N, unsigned* mm_dev, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  unsigned init[2] = {0xffffffffu, 0u};
  hipMemcpyAsync(mm_dev, init, sizeof(init), hipMemcpyHostToDevice, st);
  hipLaunchKernelGGL(minmax_kernel, dim3(nblk(N)), dim3(256), 0, st, f, N, mm_dev);
  hipLaunchKernelGGL(normalise_kernel, dim3(nblk(N)), dim3(256), 0, st, f, N, mm_dev);
  return (int)hipStreamSynchronize(st);
}

int sy_gpu_grad_mag(const int64_t* dims, const float* f, float* g, void* stream) {
  const int64_t N = dims[0] * dims[1] * dims[2] * dims[3];
  hipLaunchKernelGGL(grad_kernel, dim3(nblk(N)), dim3(256), 0, (hipStream_t)stream, dims[0],
                     dims[1], dims[2], dims[3], f, g);
  return (int)hipGetLastError();
}

// Order statistic of rank `rank` (0-based, ascending) of non-negative floats.
int sy_gpu_select(const float* v, int64_t N, int64_t rank, unsigned long long* hist_dev,
                  float* out, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int shifts[3] = {20, 8, 0}, bins[3] = {4096, 4096, 256};
  unsigned prefix = 0, pmask = 0;
  int64_t r = rank;
  unsigned long long h[4096];
  for (int p = 0; p < 3; ++p) {
    hipMemsetAsync(hist_dev, 0, sizeof(unsigned long long) * bins[p], st);
    hipLaunchKernelGGL(hist_kernel, dim3(nblk(N) > 4096 ? 4096 : nblk(N)), dim3(256), 0, st, v, N,
                       shifts[p], pmask, prefix, hist_dev, bins[p]);
    hipMemcpyAsync(h, hist_dev, sizeof(unsigned long long) * bins[p], hipMemcpyDeviceToHost, st);
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    int b = 0;
    for (; b < bins[p]; ++b) {
      if ((int64_t)h[b] > r) break;
      r -= (int64_t)h[b];
    }
    if (b == bins[p]) return -2;
    prefix |= (unsigned)b << shifts[p];
    pmask |= (unsigned)(bins[p] - 1) << shifts[p];
  }
  float fv;
  memcpy(&fv, &prefix, sizeof(fv));
  *out = fv;
  return 0;
}

}  // extern "C"
