// Deferred (lazy) dense Adam over the large table levels.
//
// The dense update touches every parameter at every step; at the fine levels
// a step's samples read a few percent of the table, and everywhere else the
// gradient is zero, so the step there is a fixed function of (p, m, v) and the
// step's constants.  Here no step is applied when it happens.  Each segment
// of FHASH_LAZY_FLOATS floats records the last step it has received (`done`)
// and the step it was last enrolled in (`stamp`), the constants of every step
// are kept, and just before the segment is read again its missing steps are
// replayed with adam1 (the dense sweep's own arithmetic): the step it was
// enrolled in with its gradient (which then is reset), every other one with a
// zero gradient.  Values read after the catch-up are the dense sweep's values,
// bit for bit.
//
// State word per segment: {done, stamp}.  Prepare for step S+1 stores S+1
// into stamp (atomic max; the first claimer appends {segment, old stamp} to
// the step's list), then replays steps done+1..S of the new list entries; the
// step's gradient is written by the caller's backward.  The step call only
// records the constants (and whether found_inf skipped the step), runs the
// dense update outside the range and empties the list; the gradient step of an
// enrolled segment is applied by its next catch-up or by the flush.
#include "adam_dev.h"
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

constexpr int kSeg = FHASH_LAZY_FLOATS;
static_assert(kSeg == 16, "one segment per 16 lanes");
constexpr int kChunk = 1024;  // list entries a workgroup sorts by gap in LDS
constexpr int kBins = 32;

// Per-step record: {step_size, inv_bc2_sqrt, gscale, skipped (0 or 1)}.
__device__ __forceinline__ AdamK step_k(const float4 c, const AdamK& base) {
  AdamK k = base;
  k.step_size = c.x;
  k.inv_bc2_sqrt = c.y;
  k.gscale = c.z;
  return k;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t y = (uint32_t)__shfl_xor((int)x, o, 64);
    x = y < x ? y : x;
  }
  return __builtin_amdgcn_readfirstlane(x);
}

// Wave-wide exclusive prefix sum of a per-lane count (64 lanes).
__device__ __forceinline__ int wave_excl_scan(int x, int& total) {
  const int lane = threadIdx.x & 63;
  int s = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(s, o, 64);
    if (lane >= o) s += y;
  }
  total = __shfl(s, 63, 64);
  return s - x;
}

// Bring one parameter per lane from step `done` to step `upto`.  `pend` (0:
// none) is the step whose gradient `gg` is still to be applied; every other
// missing step has a zero gradient.  A parameter with m = v = +0 and no
// pending gradient is a fixed point of the replay (m, v stay +0 and
// p - step_size * (+0 * 1/eps) == p) and is marked inactive by the caller.
// The loop runs over steps in wave-uniform order, so each step's constants
// are one uniform load; lanes whose segment starts later wait.
__device__ __forceinline__ void replay(const float4* __restrict__ rec, const AdamK& base,
                                       bool active, uint32_t done, uint32_t pend, uint32_t upto,
                                       float gg, float& p, float& m, float& v) {
  const uint32_t j0 = wave_min_u32(active ? done + 1 : 0xffffffffu);
  for (uint32_t j = j0; j <= upto; ++j) {
    const float4 c = rec[j];
    if (active && j > done && c.w == 0.0f) adam1(step_k(c, base), j == pend ? gg : 0.0f, p, m, v);
  }
}

// Catch-up of one segment by its 16 lanes (`sub`): loads, replay, stores,
// gradient reset and the state's `done`.  stale: done < upto.
__device__ __forceinline__ void catch_up_lanes(
    uint32_t seg, uint32_t done, uint32_t pend, bool stale, int sub, const float4* rec,
    const AdamK& base, float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
    float* __restrict__ v, void* __restrict__ shadow, int sdt, int64_t begin, int64_t end,
    uint32_t upto) {
  const int64_t f = begin + (int64_t)seg * kSeg + sub;
  // a segment never stepped (done == 0, nothing pending) holds m = v = 0
  const bool work = stale && f < end && !(pend == 0 && done == 0);
  float pp = 0.f, mm = 0.f, vv = 0.f, gg = 0.f;
  if (work) {
    pp = p[f];
    mm = m[f];
    vv = v[f];
    if (pend != 0) gg = g[f];
  }
  const bool active = work && (pend != 0 || (__float_as_uint(mm) | __float_as_uint(vv)) != 0u);
  replay(rec, base, active, done, pend, upto, gg, pp, mm, vv);
  if (active) {
    p[f] = pp;
    m[f] = mm;
    v[f] = vv;
    if (shadow != nullptr) store_shadow(shadow, sdt, f, pp);
  }
  if (work && pend != 0 && gg != 0.0f) g[f] = 0.0f;
}

// Every segment of [begin, end) that the forward or backward of a sample reads
// or writes at the levels [l0, l1): the corner row pairs of its cell, exactly
// as the encoding visits them.  Newly claimed segments are appended to the
// list as {segment, previous stamp}, one counter atomic per wave and level.
__global__ void __launch_bounds__(256)
    lazy_mark_kernel(GridDev g, int l0, int l1, const float4* __restrict__ pos, int64_t n,
                     uint2* __restrict__ state, uint2* __restrict__ list,
                     unsigned long long* __restrict__ count, int64_t begin, int64_t end,
                     uint32_t target) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int F = g.F;
  // the loop bound is wave-uniform: every lane takes part in the appends
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < n;
    const float4 p = live ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int l = l0; l < l1; ++l) {
      const LevelDev& d = g.lv[l];
      int ix, iy, iz, it;
      float fx, fy, fz, ft;
      locate(p.x, d.rx, d.sx, ix, fx);
      locate(p.y, d.ry, d.sy, iy, fy);
      locate(p.z, d.rz, d.sz, iz, fz);
      locate(p.w, d.rt, d.st, it, ft);
      uint32_t cand[16], prev[16];
      uint32_t won = 0;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int dy = r & 1, dz = (r >> 1) & 1, dt = (r >> 2) & 1;
        const int32_t tz = (it + dt) * d.rz + (iz + dz);
        int64_t s0, s1;
        bool v0, v1;
        row_pair_slots(d, g.dir, g.active != 0, tz, iy + dy, ix, s0, s1, v0, v1);
        cand[2 * r] = cand[2 * r + 1] = 0;
        prev[2 * r] = prev[2 * r + 1] = 0;
        if (live && (v0 || v1)) {
          // valid slots of a pair are consecutive: one float run of F or 2F
          int64_t lo = (v0 ? s0 : s1) * F, hi = (v1 ? s1 : s0) * F + F - 1;
          lo = lo < begin ? begin : lo;
          hi = hi >= end ? end - 1 : hi;
          if (lo <= hi) {
            const uint32_t a = (uint32_t)((lo - begin) / kSeg), b = (uint32_t)((hi - begin) / kSeg);
            cand[2 * r] = a;
            cand[2 * r + 1] = b;
            uint32_t* sa = reinterpret_cast<uint32_t*>(state + a) + 1;
            const uint32_t oa = atomicMax(sa, target);
            prev[2 * r] = oa;
            if (oa < target) won |= 1u << (2 * r);
            if (b != a) {
              uint32_t* sb = reinterpret_cast<uint32_t*>(state + b) + 1;
              const uint32_t ob = atomicMax(sb, target);
              prev[2 * r + 1] = ob;
              if (ob < target) won |= 1u << (2 * r + 1);
            }
          }
        }
      }
      int total;
      const int off = wave_excl_scan(__popc(won), total);
      if (total == 0) continue;
      unsigned long long at = 0;
      if ((threadIdx.x & 63) == 0) at = atomicAdd(count, (unsigned long long)total);
      at = __shfl(at, 0, 64) + off;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (won & (1u << c)) list[at++] = make_uint2(cand[c], prev[c]);
    }
  }
}

__device__ __forceinline__ int gap_bin(uint32_t gap) {  // gap >= 1
  if (gap < 16) return (int)gap;
  const int k = 31 - __clz(gap);          // >= 4
  const int half = (gap >> (k - 1)) & 1;  // gaps within one bin differ by < 1.5x
  const int b = 16 + 2 * (k - 4) + half;
  return b < kBins ? b : kBins - 1;
}

// Catch-up of the list entries [ctr[1], ctr[0]) to step `upto`.  Each
// workgroup takes chunks of kChunk entries, sorts them by the number of steps
// to replay (counting sort in LDS) and runs them 16 at a time, so that the
// four segments of a wave replay about as many steps.
__global__ void __launch_bounds__(256)
    lazy_catchup_kernel(const uint2* __restrict__ list, const unsigned long long* ctr,
                        uint2* __restrict__ state, const float4* __restrict__ rec, AdamK base,
                        float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, void* __restrict__ shadow, int sdt, int64_t begin,
                        int64_t end, uint32_t upto) {
  __shared__ uint4 srt[kChunk];
  __shared__ int hist[kBins], boff[kBins];
  const int64_t lo = (int64_t)ctr[1], hi = (int64_t)ctr[0];
  const int sub = threadIdx.x & (kSeg - 1);
  for (int64_t c0 = lo + (int64_t)blockIdx.x * kChunk; c0 < hi; c0 += (int64_t)gridDim.x * kChunk) {
    const int nloc = (int)((hi - c0) < kChunk ? (hi - c0) : kChunk);
    if (threadIdx.x < kBins) hist[threadIdx.x] = 0;
    __syncthreads();
    uint4 ent[kChunk / 256];
    int bin[kChunk / 256], rank[kChunk / 256];
#pragma unroll
    for (int k = 0; k < kChunk / 256; ++k) {
      const int i = threadIdx.x + k * 256;
      bin[k] = -1;
      if (i < nloc) {
        const uint2 e = list[c0 + i];
        const uint32_t done = state[e.x].x;
        const uint32_t pend = e.y > done ? e.y : 0u;  // enrolled step not yet applied
        ent[k] = make_uint4(e.x, done, pend, 0u);
        bin[k] = (done >= upto || (pend == 0 && done == 0)) ? 0 : gap_bin(upto - done);
        rank[k] = atomicAdd(&hist[bin[k]], 1);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int s = 0;
      for (int b = 0; b < kBins; ++b) {
        boff[b] = s;
        s += hist[b];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kChunk / 256; ++k)
      if (bin[k] >= 0) srt[boff[bin[k]] + rank[k]] = ent[k];
    __syncthreads();
    for (int r0 = 0; r0 < nloc; r0 += 256 / kSeg) {
      const int e = r0 + (int)(threadIdx.x / kSeg);
      const uint4 en = e < nloc ? srt[e] : make_uint4(0u, upto, 0u, 0u);
      const bool stale = e < nloc && en.y < upto;
      catch_up_lanes(en.x, en.y, en.z, stale, sub, rec, base, p, g, m, v, shadow, sdt, begin,
                     end, upto);
      if (stale && sub == 0) state[en.x].x = upto;
    }
    __syncthreads();  // srt and hist are reused by the next chunk
  }
}

// Every segment up to step `upto` (a pass over all state words).  A segment
// enrolled in the open step (stamp == upto + 1) keeps its stamp.
__global__ void __launch_bounds__(256)
    lazy_flush_kernel(int64_t nseg, uint2* __restrict__ state, const float4* __restrict__ rec,
                      AdamK base, float* __restrict__ p, float* __restrict__ g,
                      float* __restrict__ m, float* __restrict__ v, void* __restrict__ shadow,
                      int sdt, int64_t begin, int64_t end, uint32_t upto) {
  const int sub = threadIdx.x & (kSeg - 1);
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kSeg);
  // wave-uniform trip count: every lane reaches the replay's shuffles
  const int64_t first = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSeg;
  const int64_t wave_first = first - (threadIdx.x & 63) / kSeg;
  for (int64_t base_seg = wave_first; base_seg < nseg; base_seg += groups) {
    const int64_t seg = base_seg + (threadIdx.x & 63) / kSeg;
    const bool in = seg < nseg;
    const uint2 st = in ? state[seg] : make_uint2(upto, upto);
    const uint32_t pend = (st.y > st.x && st.y <= upto) ? st.y : 0u;
    const bool stale = in && st.x < upto;
    catch_up_lanes((uint32_t)seg, st.x, pend, stale, sub, rec, base, p, g, m, v, shadow, sdt,
                   begin, end, upto);
    if (stale && sub == 0) state[seg] = make_uint2(upto, st.y > upto ? st.y : upto);
  }
}

__global__ void lazy_record_kernel(float4* rec, int64_t t, float step_size, float inv_bc2_sqrt,
                                   float gscale, const int32_t* found_inf) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const float skipped = (found_inf != nullptr && *found_inf != 0) ? 1.0f : 0.0f;
    rec[t] = make_float4(step_size, inv_bc2_sqrt, gscale, skipped);
  }
}

// ctr[1] = ctr[0] (entries caught up), or both = 0 (list emptied).
__global__ void lazy_counters_kernel(unsigned long long* ctr, int empty) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (empty) {
      ctr[0] = 0ull;
      ctr[1] = 0ull;
    } else {
      ctr[1] = ctr[0];
    }
  }
}

__global__ void __launch_bounds__(256) lazy_zero_kernel(uint4* __restrict__ w, int64_t n16) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = make_uint4(0u, 0u, 0u, 0u);
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct LazyWs {
  uint2* state;
  uint2* list;
  unsigned long long* ctr;  // [0] entries, [1] entries caught up
  float4* rec;
};

LazyWs carve(const fhash_lazy* lz) {
  const int64_t nseg = lazy_num_segments(lz->end - lz->begin);
  char* b = reinterpret_cast<char*>(lz->ws);
  LazyWs w;
  w.state = reinterpret_cast<uint2*>(b);
  b += align256((size_t)nseg * 8);
  w.list = reinterpret_cast<uint2*>(b);
  b += align256((size_t)nseg * 8);
  w.ctr = reinterpret_cast<unsigned long long*>(b);
  b += 256;
  w.rec = reinterpret_cast<float4*>(b);
  return w;
}

AdamK lazy_base(const fhash_lazy* lz) {
  fhash_adam_desc o{};
  o.lr = 1.0;
  o.beta1 = lz->beta1;
  o.beta2 = lz->beta2;
  o.eps = lz->eps;
  o.step = 1;
  o.grad_scale = 1.0;
  return make_adam_k(&o);
}

// Fixed grid for the list kernels (the list length is only known on the
// device): grid-strided over chunks.
constexpr unsigned kListBlocks = 2048;

}  // namespace

int64_t lazy_num_segments(int64_t range_floats) { return (range_floats + kSeg - 1) / kSeg; }

size_t lazy_ws_bytes(int64_t range_floats, int64_t max_steps) {
  const int64_t nseg = lazy_num_segments(range_floats);
  return 2 * align256((size_t)nseg * 8) + 256 + align256((size_t)(max_steps + 1) * 16);
}

hipError_t launch_lazy_init(const fhash_lazy* lz, hipStream_t st) {
  const int64_t bytes =
      (int64_t)lazy_ws_bytes(lz->end - lz->begin, lz->max_steps);  // a multiple of 16
  const int64_t n16 = bytes / 16;
  int64_t b = (n16 + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(lazy_zero_kernel, dim3((unsigned)b), dim3(256), 0, st,
                     reinterpret_cast<uint4*>(lz->ws), n16);
  return hipGetLastError();
}

hipError_t launch_lazy_prepare(const GridDev& g, int l0, int l1, const float* pos, int64_t n,
                               const fhash_lazy* lz, float* p, float* gr, float* m, float* v,
                               void* shadow, fhash_dtype sdt, hipStream_t st) {
  const LazyWs w = carve(lz);
  const uint32_t S = (uint32_t)lz->steps;
  if (n > 0 && l0 < l1) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(lazy_mark_kernel, dim3((unsigned)b), dim3(256), 0, st, g, l0, l1,
                       reinterpret_cast<const float4*>(pos), n, w.state, w.list, w.ctr,
                       lz->begin, lz->end, S + 1);
  }
  hipLaunchKernelGGL(lazy_catchup_kernel, dim3(kListBlocks), dim3(256), 0, st, w.list, w.ctr,
                     w.state, w.rec, lazy_base(lz), p, gr, m, v, shadow, (int)sdt, lz->begin,
                     lz->end, S);
  hipLaunchKernelGGL(lazy_counters_kernel, dim3(1), dim3(64), 0, st, w.ctr, 0);
  return hipGetLastError();
}

hipError_t launch_lazy_step(const fhash_adam_desc* o, const fhash_lazy* lz, const int32_t* found_inf,
                            hipStream_t st) {
  const LazyWs w = carve(lz);
  const AdamK k = make_adam_k(o);
  hipLaunchKernelGGL(lazy_record_kernel, dim3(1), dim3(64), 0, st, w.rec, lz->steps + 1,
                     k.step_size, k.inv_bc2_sqrt, k.gscale, found_inf);
  hipLaunchKernelGGL(lazy_counters_kernel, dim3(1), dim3(64), 0, st, w.ctr, 1);
  return hipGetLastError();
}

hipError_t launch_lazy_flush(const fhash_lazy* lz, float* p, float* gr, float* m, float* v,
                             void* shadow, fhash_dtype sdt, hipStream_t st) {
  const LazyWs w = carve(lz);
  const int64_t nseg = lazy_num_segments(lz->end - lz->begin);
  if (nseg == 0 || lz->steps == 0) return hipSuccess;
  int64_t b = (nseg * kSeg + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(lazy_flush_kernel, dim3((unsigned)b), dim3(256), 0, st, nseg, w.state, w.rec,
                     lazy_base(lz), p, gr, m, v, shadow, (int)sdt, lz->begin, lz->end,
                     (uint32_t)lz->steps);
  return hipGetLastError();
}

}  // namespace fh
