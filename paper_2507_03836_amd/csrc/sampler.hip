// Training sampler: Philox4x32-10 counter-based draws -> coreset voxel -> FP32
// position and label (Sec. 3.1, time-step concatenation).  The time coordinate
// of a frame is n / (T - 1), or frame_t[n] when the caller gives a frame-time
// table (key-frame training, Sec. 3.2.2).  The spatial coordinates are those of
// the whole volume, or of the feature bounding box (Sec. 3.1, position
// translation and scaling) when the caller gives one.
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, multipliers 0xD2511F53 /
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

__global__ void __launch_bounds__(256)
    sample_kernel(uint64_t seed, uint64_t step, int64_t n, const uint64_t* __restrict__ coreset,
                  uint64_t M, int64_t Sx, int64_t Sy, int64_t Sz, int64_t St,
                  const float* __restrict__ field, const float* __restrict__ frame_t,
                  int4 box_lo, int4 box_ext, float4* __restrict__ pos,
                  float* __restrict__ target) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint4 ctr = make_uint4((uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)step,
                                 (uint32_t)(step >> 32));
    const uint4 o = philox10(ctr, make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const uint64_t r = ((uint64_t)o.y << 32) | o.x;
    const uint64_t id = __umul64hi(r, M);
    const uint64_t lin = coreset ? coreset[id] : id;
    const uint64_t x = lin % (uint64_t)Sx;
    const uint64_t y = (lin / (uint64_t)Sx) % (uint64_t)Sy;
    const uint64_t z = (lin / ((uint64_t)Sx * Sy)) % (uint64_t)Sz;
    const uint64_t t = lin / ((uint64_t)Sx * Sy * Sz);
    float4 p;
    p.x = __fdiv_rn((float)((int64_t)x - box_lo.x), (float)box_ext.x);
    p.y = __fdiv_rn((float)((int64_t)y - box_lo.y), (float)box_ext.y);
    p.z = __fdiv_rn((float)((int64_t)z - box_lo.z), (float)box_ext.z);
    p.w = frame_t ? frame_t[t] : __fdiv_rn((float)t, (float)(St - 1));
    pos[i] = p;
    target[i] = field[lin];
  }
}

}  // namespace

hipError_t launch_sample(uint64_t seed, uint64_t step, int64_t n, const uint64_t* coreset,
                         uint64_t M, const int64_t* dims, const float* field,
                         const float* frame_t, const int32_t* box, float* pos, float* target,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  // spatial frame: the whole volume [0, S - 1], or the box [lo, hi] (inclusive)
  int4 lo = make_int4(0, 0, 0, 0);
  int4 ext = make_int4((int)(dims[0] - 1), (int)(dims[1] - 1), (int)(dims[2] - 1), 0);
  if (box != nullptr) {
    lo = make_int4(box[0], box[1], box[2], 0);
    ext = make_int4(box[3] - box[0], box[4] - box[1], box[5] - box[2], 0);
  }
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)b), dim3(256), 0, st, seed, step, n, coreset, M,
                     dims[0], dims[1], dims[2], dims[3], field, frame_t, lo, ext,
                     reinterpret_cast<float4*>(pos), target);
  return hipGetLastError();
}

}  // namespace fh
