// Scatter-add of the coarsest levels' encoding gradient through LDS
// (FHASH_COARSE_LDS).  The fused backward leaves the gradient of the encoding
// of levels 0 .. g.coarse - 1 in dxc ([level][sample][feature]) instead of
// adding it into the table; this kernel adds it.  Each workgroup takes one
// level and a contiguous chunk of the batch (neighbours in space when the batch is
// sorted), finds the box of the level's vertices its samples touch, sums the
// 16 corner contributions of every sample into an LDS image of that box, and
// adds the box into the table gradient with one atomic per touched vertex and
// feature.  At the coarse levels a vertex collects the contributions of many
// samples, so the memory-side atomic requests, which bound the scatter, drop
// from one per sample, corner and instruction to one per vertex and chunk.  A
// chunk whose box does not fit the LDS image is retried in kParts parts, and a
// part that still does not fit adds its samples directly.
// The sum over samples is the adjoint of the quadrilinear blend (Sec. 3.2.3),
// reordered: the same result up to FP32 summation order.
#include <climits>

#include "common.h"
#include "encode_dev.h"
#include "kernels.h"

namespace fh {

namespace {

constexpr int kThreads = 1024;  // 16 waves: the loops below wait on L2 latency
constexpr int kChunk = 2048;    // samples per workgroup
constexpr int kUnroll = 4;      // independent loads in flight per thread
constexpr int kParts = 4;       // a chunk whose box does not fit is retried in 4 parts
constexpr int kCap = 16000;   // floats of the LDS image (with the reduction slots, under 64 KiB)

// Slot of vertex (x, y, z, t) of a rows-ordered level: dense, hashed, or
// through the rank directory (valid = false for an inactive vertex).  Reads
// only the directory entry that holds x.
__device__ __forceinline__ int64_t vertex_slot(const LevelDev& d, const ulonglong2* dir,
                                               bool active, int t, int z, int y, int x,
                                               bool& valid) {
  if (d.hash_bits) {
    const uint32_t yzt = (uint32_t)y * 2654435761u ^ (uint32_t)z * 805459861u ^
                         (uint32_t)t * 3674653429u;
    const uint32_t mask = (d.hash_bits >= 32) ? 0xffffffffu : ((1u << d.hash_bits) - 1u);
    valid = true;
    return d.slot_off + spatial_hash((uint32_t)x, yzt, mask);
  }
  if (!active) {
    valid = true;
    return d.slot_off + ((int64_t)(t * d.rz + z) * d.ry + y) * d.rx + x;
  }
  const int32_t tz = t * d.rz + z;
  const ulonglong2 e = dir[d.dir_off + (int64_t)((tz * d.wv + (x >> 6)) * d.ry + y)];
  return entry_slot(e, x & 63, d.slot_off, valid);
}

template <int F>
__global__ void __launch_bounds__(kThreads)
    coarse_scatter_kernel(GridDev g, const float4* __restrict__ pos, int64_t n,
                          const float* __restrict__ dxc, float* __restrict__ d_table) {
  extern __shared__ float acc[];  // kCap floats
  __shared__ int red[8][kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  const int cnt = (int)((n - c0) < kChunk ? (n - c0) : kChunk);
  const bool active = g.active != 0;
  {
    const int l = blockIdx.y;  // one level per workgroup row of the grid
    const LevelDev& d = g.lv[l];
    const float* gl = dxc + (int64_t)l * n * F;
    int nparts = 1;
    for (int part = 0; part < nparts; ++part) {
    // samples s0 .. s0 + bn - 1: the chunk, or one of its parts
    const int b0 = (int)((int64_t)cnt * part / nparts);
    const int bn = (int)((int64_t)cnt * (part + 1) / nparts) - b0;
    const int64_t s0 = c0 + b0;
    if (bn == 0) continue;  // a part of a chunk shorter than kParts samples
    // the cells the range's samples fall in: per-axis minimum and maximum
    int lo[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX}, hi[4] = {-1, -1, -1, -1};
    for (int i = tid; i < bn; i += kThreads) {
      const float4 p = pos[s0 + i];
      int c[4];
      float f;
      locate(p.x, d.rx, d.sx, c[0], f);
      locate(p.y, d.ry, d.sy, c[1], f);
      locate(p.z, d.rz, d.sz, c[2], f);
      locate(p.w, d.rt, d.st, c[3], f);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        lo[k] = min(lo[k], c[k]);
        hi[k] = max(hi[k], c[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      for (int o = 32; o > 0; o >>= 1) {
        lo[k] = min(lo[k], __shfl_xor(lo[k], o, 64));
        hi[k] = max(hi[k], __shfl_xor(hi[k], o, 64));
      }
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        red[k][wid] = lo[k];
        red[4 + k][wid] = hi[k];
      }
    __syncthreads();
    int blo[4], ext[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int a = red[k][0], b = red[4 + k][0];
      for (int w = 1; w < kThreads / 64; ++w) {
        a = min(a, red[k][w]);
        b = max(b, red[4 + k][w]);
      }
      blo[k] = a;
      ext[k] = b - a + 2;  // vertices a .. b + 1
    }
    __syncthreads();  // red is rewritten by the next level
    const int64_t V = (int64_t)ext[0] * ext[1] * ext[2] * ext[3];
    if (V * F <= kCap) {
      for (int i = tid; i < (int)V * F; i += kThreads) acc[i] = 0.0f;
      __syncthreads();
      // lane group of 16: one corner per lane (bits x, y, z, t), the group
      // walking a contiguous run of the range's samples and summing in
      // registers while its vertex stays the same (neighbours in a sorted batch
      // often share the cell), so an LDS atomic is issued per change of vertex
      const int cr = tid & 15;
      const int ox = cr & 1, oy = (cr >> 1) & 1, oz = (cr >> 2) & 1, ot = (cr >> 3) & 1;
      constexpr int kGroups = kThreads / 16;
      const int per = (bn + kGroups - 1) / kGroups;
      const int ib = (tid >> 4) * per, ie = min(bn, ib + per);
      int cur = -1;
      float run[F];
#pragma unroll
      for (int k = 0; k < F; ++k) run[k] = 0.0f;
      for (int i0 = ib; i0 < ie; i0 += kUnroll) {
        float4 pu[kUnroll];
        float gu[kUnroll][F];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int i = i0 + u;
          pu[u] = i < ie ? pos[s0 + i] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
          for (int k = 0; k < F; ++k) gu[u][k] = i < ie ? gl[(s0 + i) * F + k] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (i0 + u >= ie) break;
          int cx, cy, cz, ct;
          float fx, fy, fz, ft;
          locate(pu[u].x, d.rx, d.sx, cx, fx);
          locate(pu[u].y, d.ry, d.sy, cy, fy);
          locate(pu[u].z, d.rz, d.sz, cz, fz);
          locate(pu[u].w, d.rt, d.st, ct, ft);
          const float w = ((ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy)) *
                          ((oz ? fz : 1.0f - fz) * (ot ? ft : 1.0f - ft));
          const int li = (((ct + ot - blo[3]) * ext[2] + (cz + oz - blo[2])) * ext[1] +
                          (cy + oy - blo[1])) * ext[0] + (cx + ox - blo[0]);
          if (li != cur) {
            if (cur >= 0)
#pragma unroll
              for (int k = 0; k < F; ++k) atomicAdd(&acc[cur * F + k], run[k]);
            cur = li;
#pragma unroll
            for (int k = 0; k < F; ++k) run[k] = 0.0f;
          }
#pragma unroll
          for (int k = 0; k < F; ++k) run[k] += w * gu[u][k];
        }
      }
      if (cur >= 0)
#pragma unroll
        for (int k = 0; k < F; ++k) atomicAdd(&acc[cur * F + k], run[k]);
      __syncthreads();
      // the box into the table: x fastest, so neighbouring lanes add into
      // neighbouring slots of a vertex row; kUnroll directory loads in flight
      for (int v0 = tid; v0 < (int)V; v0 += kThreads * kUnroll) {
        float val[kUnroll][F];
        int64_t sv[kUnroll];
        bool add[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int v = v0 + u * kThreads;
          bool any = false;
#pragma unroll
          for (int k = 0; k < F; ++k) {
            val[u][k] = v < (int)V ? acc[v * F + k] : 0.0f;
            any = any || val[u][k] != 0.0f;
          }
          add[u] = false;
          sv[u] = 0;
          if (any) {
            int r = v;
            const int x = blo[0] + r % ext[0];
            r /= ext[0];
            const int y = blo[1] + r % ext[1];
            r /= ext[1];
            const int z = blo[2] + r % ext[2];
            const int t = blo[3] + r / ext[2];
            sv[u] = vertex_slot(d, g.dir, active, t, z, y, x, add[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (add[u]) {
#pragma unroll
            for (int k = 0; k < F; ++k)
              unsafeAtomicAdd(d_table + run_off(sv[u] * F, g.gmask) + k, val[u][k]);
            mark_touched(g.touch, g.touch_begin, sv[u] * F);
          }
      }
      __syncthreads();  // the next range clears acc
    } else if (nparts == 1) {
      nparts = kParts;  // the same decision in every thread: retry in parts
      part = -1;
    } else {
      // straight into the table, one lane per sample, corner and feature, so
      // that the lanes of an atomic instruction cover both rows of a corner
      // pair and every feature (one request per pair and sample)
      constexpr int Q = 16 * F;
      const int k = tid % F, cr = (tid / F) & 15;
      const int ox = cr & 1, oy = (cr >> 1) & 1, oz = (cr >> 2) & 1, ot = (cr >> 3) & 1;
      for (int i = tid / Q; i < bn; i += kThreads / Q) {
        const float4 p = pos[s0 + i];
        int cx, cy, cz, ct;
        float fx, fy, fz, ft;
        locate(p.x, d.rx, d.sx, cx, fx);
        locate(p.y, d.ry, d.sy, cy, fy);
        locate(p.z, d.rz, d.sz, cz, fz);
        locate(p.w, d.rt, d.st, ct, ft);
        const float w = ((ox ? fx : 1.0f - fx) * (oy ? fy : 1.0f - fy)) *
                        ((oz ? fz : 1.0f - fz) * (ot ? ft : 1.0f - ft));
        bool valid;
        const int64_t sl = vertex_slot(d, g.dir, active, ct + ot, cz + oz, cy + oy, cx + ox, valid);
        if (valid) {
          unsafeAtomicAdd(d_table + run_off(sl * F, g.gmask) + k, w * gl[(s0 + i) * F + k]);
          if (k == 0) mark_touched(g.touch, g.touch_begin, sl * F);
        }
      }
    }
    }
  }
}

template <int F>
hipError_t launch_f(const GridDev& g, const float* pos, int64_t n, float* d_table,
                    hipStream_t st) {
  const int64_t blocks = (n + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(coarse_scatter_kernel<F>, dim3((unsigned)blocks, (unsigned)g.coarse),
                     dim3(kThreads),
                     kCap * sizeof(float), st, g, reinterpret_cast<const float4*>(pos), n,
                     g.dxc, d_table);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_coarse_scatter(const GridDev& g, const float* pos, int64_t n, float* d_table,
                                 hipStream_t st) {
  if (g.coarse <= 0 || n == 0) return hipSuccess;
  switch (g.F) {
    case 1: return launch_f<1>(g, pos, n, d_table, st);
    case 2: return launch_f<2>(g, pos, n, d_table, st);
    case 4: return launch_f<4>(g, pos, n, d_table, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fh
