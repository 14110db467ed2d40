// Multi-resolution tesseract encoding (Sec. 3.2.4): per level, locate the 4D cell,
// look up the 16 corner slots through the per-level hash and blend the corner
// embeddings with quadrilinear weights; and its adjoint (scatter-add).
//
// One thread per sample, levels in a wave-uniform loop (level constants come from
// the kernel arguments, i.e. scalar registers).  The 16 corners are visited as 8
// pairs (corner_pair): in the rows order the vertex rows (dy, dz, dt) of an x-pair
// (x, x+1), one directory entry serving both vertices unless x sits on bit 63 of
// a word; in the brick order pairs along an axis that keeps both in one brick.
#include "encode_dev.h"
#include "kernels.h"

namespace fh {

namespace {

template <int F, typename T>
__global__ void __launch_bounds__(256)
    encode_fwd_kernel(GridDev g, const float4* __restrict__ pos, int64_t n,
                      const T* __restrict__ table, float* __restrict__ enc) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float4 p = pos[s];
  float* out = enc + s * (int64_t)g.L * F;
  for (int l = 0; l < g.L; ++l) {
    const LevelDev& d = g.lv[l];
    if (d.brick)
      encode_level<F, T, true>(d, g.dir, g.active != 0, p, table, out + l * F, g.tmask);
    else
      encode_level<F, T, false>(d, g.dir, g.active != 0, p, table, out + l * F, g.tmask);
  }
}

// 2F threads per sample (pair element x feature), see scatter_level_lane.
template <int F>
__global__ void __launch_bounds__(256)
    encode_bwd_kernel(GridDev g, const float4* __restrict__ pos, int64_t n,
                      const float* __restrict__ d_enc, float* __restrict__ d_table) {
  constexpr int Q = 2 * F;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t s = t / Q;
  if (s >= n) return;
  const int r = (int)(t % Q), e = r / F, f = r % F;
  const float4 p = pos[s];
  const float* gin = d_enc + s * (int64_t)g.L * F;
  for (int l = 0; l < g.L; ++l) {
    if (g.lv[l].brick)
      scatter_level_lane<F, true>(g.lv[l], g.dir, g.active != 0, p, e, f, gin[l * F + f],
                                  d_table, g.touch, g.touch_begin, g.gmask);
    else
      scatter_level_lane<F, false>(g.lv[l], g.dir, g.active != 0, p, e, f, gin[l * F + f],
                                   d_table, g.touch, g.touch_begin, g.gmask);
  }
}

// Instrumentation: per (sample, level) the directory entries and table rows the
// 8 corner pairs of its cell touch (corner_pair: rows layout, pair r = the
// x-pair of row (dy, dz, dt) = (r & 1, r >> 1 & 1, r >> 2); bricks, pairs along
// pair_axis).
__global__ void __launch_bounds__(256)
    corner_rows_kernel(GridDev g, const float4* __restrict__ pos, int64_t n,
                       long long* __restrict__ out_dir, long long* __restrict__ out_slot) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * g.L) return;
  const int64_t s = t / g.L;
  const int l = (int)(t % g.L);
  const LevelDev& d = g.lv[l];
  const float4 p = pos[s];
  int ix, iy, iz, it;
  float fx, fy, fz, ft;
  locate(p.x, d.rx, d.sx, ix, fx);
  locate(p.y, d.ry, d.sy, iy, fy);
  locate(p.z, d.rz, d.sz, iz, fz);
  locate(p.w, d.rt, d.st, it, ft);
  const bool active = g.active != 0 && d.hash_bits == 0;
  const int a = d.brick ? pair_axis<true>(ix, iy, iz, it) : 0;
  for (int r = 0; r < 8; ++r) {
    float wr;
    int64_t s0, s1;
    bool v0, v1;
    if (d.brick)
      corner_pair<true>(d, g.dir, g.active != 0, ix, iy, iz, it, fx, fy, fz, ft, a, r, s0, s1,
                        v0, v1, wr);
    else
      corner_pair<false>(d, g.dir, g.active != 0, ix, iy, iz, it, fx, fy, fz, ft, a, r, s0, s1,
                         v0, v1, wr);
    const int64_t o = (t * 8 + r) * 2;
    long long w0 = -1, w1 = -1;
    if (active) {
      int ox = 0, oy = r & 1, oz = (r >> 1) & 1, ot = r >> 2;
      if (d.brick) pair_offsets(r, a, ox, oy, oz, ot);
      int64_t e0, e1;
      int b0, b1;
      // the entries of the pair's first corner and of its x neighbour (the
      // second corner shares the first one's entry unless the pair is along x)
      if (d.brick)
        pair_entries<true>(d, it + ot, iz + oz, iy + oy, ix + ox, e0, e1, b0, b1);
      else
        pair_entries<false>(d, it + ot, iz + oz, iy + oy, ix + ox, e0, e1, b0, b1);
      w0 = e0;
      if (a == 0 && e1 != e0) w1 = e1;
    }
    out_dir[o] = w0;
    out_dir[o + 1] = w1;
    out_slot[o] = v0 ? s0 : -1;
    out_slot[o + 1] = v1 ? s1 : -1;
  }
}

template <int F>
hipError_t launch_fwd_t(const GridDev& g, const float* pos, int64_t n, const void* table,
                        fhash_dtype dt, float* enc, hipStream_t st) {
  const int T = 256;
  const int64_t blocks = (n + T - 1) / T;
  if (dt == FHASH_F32)
    hipLaunchKernelGGL((encode_fwd_kernel<F, float>), dim3((unsigned)blocks), dim3(T), 0, st, g,
                       reinterpret_cast<const float4*>(pos), n,
                       reinterpret_cast<const float*>(table), enc);
  else
    hipLaunchKernelGGL((encode_fwd_kernel<F, __half>), dim3((unsigned)blocks), dim3(T), 0, st, g,
                       reinterpret_cast<const float4*>(pos), n,
                       reinterpret_cast<const __half*>(table), enc);
  return hipGetLastError();
}

template <int F>
hipError_t launch_bwd_t(const GridDev& g, const float* pos, int64_t n, const float* d_enc,
                        float* d_table, hipStream_t st) {
  const int T = 256;
  const int64_t blocks = (n * 2 * F + T - 1) / T;
  hipLaunchKernelGGL((encode_bwd_kernel<F>), dim3((unsigned)blocks), dim3(T), 0, st, g,
                     reinterpret_cast<const float4*>(pos), n, d_enc, d_table);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_encode_fwd(const GridDev& g, const float* pos, int64_t n, const void* table,
                             fhash_dtype dt, float* enc, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (g.F) {
    case 1: return launch_fwd_t<1>(g, pos, n, table, dt, enc, st);
    case 2: return launch_fwd_t<2>(g, pos, n, table, dt, enc, st);
    case 4: return launch_fwd_t<4>(g, pos, n, table, dt, enc, st);
    case 8: return launch_fwd_t<8>(g, pos, n, table, dt, enc, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_corner_rows(const GridDev& g, const float* pos, int64_t n, int64_t* out_dir,
                              int64_t* out_slot, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n * g.L + 255) / 256;
  hipLaunchKernelGGL(corner_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, g,
                     reinterpret_cast<const float4*>(pos), n,
                     reinterpret_cast<long long*>(out_dir), reinterpret_cast<long long*>(out_slot));
  return hipGetLastError();
}

hipError_t launch_encode_bwd(const GridDev& g, const float* pos, int64_t n, const float* d_enc,
                             float* d_table, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (g.F) {
    case 1: return launch_bwd_t<1>(g, pos, n, d_enc, d_table, st);
    case 2: return launch_bwd_t<2>(g, pos, n, d_enc, d_table, st);
    case 4: return launch_bwd_t<4>(g, pos, n, d_enc, d_table, st);
    case 8: return launch_bwd_t<8>(g, pos, n, d_enc, d_table, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fh
