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
// step's gradient is written by the caller's backward; every catch-up empties
// the list.  The step call only records the constants (and whether found_inf
// skipped the step) and runs the dense update outside the range; the gradient
// step of an enrolled segment is applied by its next catch-up or by the flush
// (which lists every segment behind the last step and catches them up).
#include "adam_dev.h"
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

constexpr int kSeg = FHASH_LAZY_FLOATS;
static_assert(kSeg == 16, "segments of 16 floats");
constexpr int kChunk = 512;  // list entries a workgroup sorts by gap in LDS
constexpr int kBins = 32;

// Per-step record: {step_size, inv_bc2_sqrt, gscale, kind}; kind 0: a step
// whose zero-gradient form is adam0 (finite gscale), 1: skipped (found_inf),
// 2: applied with a non-finite gscale (zero-gradient form: adam1 itself).
constexpr float kStep = 0.0f, kSkipped = 1.0f, kOddScale = 2.0f;

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

// Four parameters per lane (a float4), four lanes per segment.
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kLanesPerSeg = kSeg / 4;

__device__ __forceinline__ void adam1_4(const AdamK& k, f4v g, f4v& p, f4v& m, f4v& v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float pc = p[c], mc = m[c], vc = v[c];
    adam1(k, g[c], pc, mc, vc);
    p[c] = pc, m[c] = mc, v[c] = vc;
  }
}

__device__ __forceinline__ void adam0_4(const AdamK& k, f4v& p, f4v& m, f4v& v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float pc = p[c], mc = m[c], vc = v[c];
    adam0(k, pc, mc, vc);
    p[c] = pc, m[c] = mc, v[c] = vc;
  }
}

// Bring a lane's four parameters from step `done` to step `upto`.  `pend`
// (0: none; else done + 1) is the step whose gradient `g` is still to be
// applied; every other missing step has a zero gradient.  Parameters with
// m = v = +0 and no pending gradient are fixed points of such steps (m, v stay
// +0 and fma(-step_size, +0, p) == p), so a lane whose four are all of that
// kind is marked inactive by the caller.  The zero-gradient steps run in
// wave-uniform order, so each step's record is one uniform load; lanes whose
// segment starts later wait.
template <bool ODD>
__device__ __forceinline__ void replay(const float4* __restrict__ rec, const AdamK& base,
                                       bool active, uint32_t done, uint32_t pend, uint32_t upto,
                                       f4v g, f4v& p, f4v& m, f4v& v) {
  if (active && pend != 0) {
    const float4 c = rec[pend];
    if (c.w != kSkipped) adam1_4(step_k(c, base), g, p, m, v);
    done = pend;
  }
  const uint32_t j0 = wave_min_u32(active ? done + 1 : 0xffffffffu);
  for (uint32_t j = j0; j <= upto; ++j) {
    const float4 c = rec[j];
    if (c.w == kStep) {
      if (active && j > done) adam0_4(step_k(c, base), p, m, v);
    } else if (ODD && c.w == kOddScale) {
      if (active && j > done) adam1_4(step_k(c, base), (f4v){0.f, 0.f, 0.f, 0.f}, p, m, v);
    }
  }
}

// Catch-up of one segment by its 4 lanes (`sub`), in two parts so that the
// loads of the next segments are in flight while these replay.
struct Lane {
  int64_t f;  // first of the lane's four floats
  uint32_t seg, done, pend;
  bool stale, work;
  f4v p, m, v, g;
};

// Loads.  stale: done < upto.  A segment never stepped (done == 0, nothing
// pending) holds m = v = 0 and needs no loads.  begin is a multiple of 16 and
// end of 4, so a lane's four floats are all inside the range or all outside.
template <bool PAIRED>
__device__ __forceinline__ Lane load_lanes(uint32_t seg, uint32_t done, uint32_t pend, bool stale,
                                           int sub, const float* __restrict__ p,
                                           const float* __restrict__ g,
                                           const float* __restrict__ m,
                                           const float* __restrict__ v, int64_t begin,
                                           int64_t end) {
  Lane L;
  L.seg = seg;
  L.done = done;
  L.pend = pend;
  L.stale = stale;
  L.f = begin + (int64_t)seg * kSeg + 4 * sub;
  L.work = stale && L.f < end && !(pend == 0 && done == 0);
  const f4v z = {0.f, 0.f, 0.f, 0.f};
  L.p = L.m = L.v = L.g = z;
  if (L.work) {
    L.p = *reinterpret_cast<const f4v*>(p + L.f);
    L.m = *reinterpret_cast<const f4v*>(m + moment_off<PAIRED>(L.f));
    L.v = *reinterpret_cast<const f4v*>(v + moment_off<PAIRED>(L.f));
    if (pend != 0) L.g = *reinterpret_cast<const f4v*>(g + L.f);
  }
  return L;
}

// The four shadow values of a lane in one 8-byte store (f: a multiple of 4).
__device__ __forceinline__ void store_shadow_group(void* shadow, int sdt, int64_t f, const f4v x) {
  uint32_t lo, hi;
  if (sdt == FHASH_F16) {
    const __half2 a = __floats2half2_rn(x[0], x[1]), b = __floats2half2_rn(x[2], x[3]);
    lo = *reinterpret_cast<const uint32_t*>(&a);
    hi = *reinterpret_cast<const uint32_t*>(&b);
  } else {
    lo = (uint32_t)to_bf16_rne(x[0]) | ((uint32_t)to_bf16_rne(x[1]) << 16);
    hi = (uint32_t)to_bf16_rne(x[2]) | ((uint32_t)to_bf16_rne(x[3]) << 16);
  }
  reinterpret_cast<uint2*>(shadow)[f / 4] = make_uint2(lo, hi);
}

__device__ __forceinline__ bool nonzero_state(const f4v m, const f4v v) {
  uint32_t b = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) b |= __float_as_uint(m[c]) | __float_as_uint(v[c]);
  return b != 0u;
}

// Replay, stores, gradient reset.  ODD: some recorded step has a non-finite
// gscale (its zero-gradient form is adam1).
template <bool ODD, bool PAIRED>
__device__ __forceinline__ bool finish_lanes(Lane L, const float4* rec, const AdamK& base,
                                             float* __restrict__ p, float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v,
                                             void* __restrict__ shadow, int sdt, uint32_t upto) {
  const bool active = L.work && (L.pend != 0 || nonzero_state(L.m, L.v));
  replay<ODD>(rec, base, active, L.done, L.pend, upto, L.g, L.p, L.m, L.v);
  if (active) {
    *reinterpret_cast<f4v*>(p + L.f) = L.p;
    *reinterpret_cast<f4v*>(m + moment_off<PAIRED>(L.f)) = L.m;
    *reinterpret_cast<f4v*>(v + moment_off<PAIRED>(L.f)) = L.v;
    if (shadow != nullptr) store_shadow_group(shadow, sdt, L.f, L.p);
  }
  if (L.work && L.pend != 0 && (L.g[0] != 0.f || L.g[1] != 0.f || L.g[2] != 0.f || L.g[3] != 0.f))
    *reinterpret_cast<f4v*>(g + L.f) = (f4v){0.f, 0.f, 0.f, 0.f};
  return active;
}

// Every segment of [begin, end) that the forward or backward of a sample reads
// or writes at the levels [l0, l1): the corner row pairs of its cell, exactly
// as the encoding visits them.  Newly claimed segments are appended to the
// list as {segment, previous stamp}, one counter atomic per wave and level.
__global__ void __launch_bounds__(256)
    lazy_mark_kernel(GridDev g, int l0, int l1, const float4* __restrict__ pos, int64_t n,
                     uint2* __restrict__ state, uint2* __restrict__ list,
                     unsigned long long* __restrict__ count, int64_t begin, int64_t end,
                     uint32_t target, unsigned long long cap) {
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
      const int ax = d.brick ? pair_axis<true>(ix, iy, iz, it) : 0;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float wr;
        int64_t s0, s1;
        bool v0, v1;
        if (d.brick)
          corner_pair<true>(d, g.dir, g.active != 0, ix, iy, iz, it, fx, fy, fz, ft, ax, r, s0,
                            s1, v0, v1, wr);
        else
          corner_pair<false>(d, g.dir, g.active != 0, ix, iy, iz, it, fx, fy, fz, ft, ax, r, s0,
                             s1, v0, v1, wr);
        cand[2 * r] = cand[2 * r + 1] = 0;
        prev[2 * r] = prev[2 * r + 1] = 0;
        if (live && (v0 || v1)) {
          // F divides 16 and begin is a multiple of 16, so the F floats of a slot
          // lie in one segment; the two slots of a pair are neighbouring rows,
          // rows of one brick, or two hashed rows
          const int64_t fa = (v0 ? s0 : s1) * F, fb = (v1 ? s1 : s0) * F;
          const bool ina = fa >= begin && fa < end, inb = fb >= begin && fb < end;
          const uint32_t a = ina ? (uint32_t)((fa - begin) / kSeg) : 0u;
          const uint32_t b = inb ? (uint32_t)((fb - begin) / kSeg) : 0u;
          cand[2 * r] = a;
          cand[2 * r + 1] = b;
          if (ina) {
            uint32_t* sa = reinterpret_cast<uint32_t*>(state + a) + 1;
            const uint32_t oa = atomicMax(sa, target);
            prev[2 * r] = oa;
            if (oa < target) won |= 1u << (2 * r);
          }
          if (inb && !(ina && b == a)) {
            uint32_t* sb = reinterpret_cast<uint32_t*>(state + b) + 1;
            const uint32_t ob = atomicMax(sb, target);
            prev[2 * r + 1] = ob;
            if (ob < target) won |= 1u << (2 * r + 1);
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
        if (won & (1u << c)) {
          // the bound always holds: the list has one entry per segment, and a
          // segment is listed at most once between two catch-ups
          if (at < cap) list[at] = make_uint2(cand[c], prev[c]);
          ++at;
        }
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

// Catch-up of the list entries [ctr[1], ctr[0]) to step `upto`; ctr[2..5]
// accumulate the segments caught up, those that loaded data, those with a
// pending gradient and the segment-steps replayed (workload statistics).  Each
// workgroup takes chunks of kChunk entries, sorts them by the number of steps
// to replay (counting sort in LDS) and runs them 16 at a time, so that the
// four segments of a wave replay about as many steps.
template <bool ODD, bool PAIRED>
__global__ void __launch_bounds__(256)
    lazy_catchup_kernel(const uint2* __restrict__ list, unsigned long long* ctr,
                        uint2* __restrict__ state, const float4* __restrict__ rec, AdamK base,
                        float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, void* __restrict__ shadow, int sdt, int64_t begin,
                        int64_t end, uint32_t upto, int64_t cap) {
  __shared__ uint4 srt[kChunk];
  __shared__ int hist[kBins], boff[kBins];
  __shared__ unsigned long long tally[4];
  if (threadIdx.x < 4) tally[threadIdx.x] = 0ull;
  unsigned long long n_stale = 0, n_work = 0, n_pend = 0, n_steps = 0;
  const int64_t lo = (int64_t)ctr[1];
  const int64_t hi = (int64_t)ctr[0] < cap ? (int64_t)ctr[0] : cap;
  const int sub = threadIdx.x & (kLanesPerSeg - 1);
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
    // software-pipelined rounds of 64 segments: load round r+1, replay round r
    auto fetch = [&](int r0) {
      const int e = r0 + (int)(threadIdx.x / kLanesPerSeg);
      const uint4 en = e < nloc ? srt[e] : make_uint4(0u, upto, 0u, 0u);
      return load_lanes<PAIRED>(en.x, en.y, en.z, e < nloc && en.y < upto, sub, p, g, m, v,
                                begin, end);
    };
    Lane cur = fetch(0);
    for (int r0 = 0; r0 < nloc; r0 += 256 / kLanesPerSeg) {
      const Lane nxt = fetch(r0 + 256 / kLanesPerSeg);
      const bool active =
          finish_lanes<ODD, PAIRED>(cur, rec, base, p, g, m, v, shadow, sdt, upto);
      if (cur.stale && sub == 0) {
        state[cur.seg].x = upto;
        n_stale += 1;
        n_work += cur.work;
        n_pend += cur.work && cur.pend != 0;
        if (active) n_steps += upto - cur.done;
      }
      cur = nxt;
    }
    __syncthreads();  // srt and hist are reused by the next chunk
  }
  if (n_stale) {
    atomicAdd(&tally[0], n_stale);
    atomicAdd(&tally[1], n_work);
    atomicAdd(&tally[2], n_pend);
    atomicAdd(&tally[3], n_steps);
  }
  __syncthreads();
  if (threadIdx.x < 4 && tally[threadIdx.x] != 0ull) atomicAdd(&ctr[2 + threadIdx.x], tally[threadIdx.x]);
}

// Flush, first part: append every segment behind step `upto` that was ever
// enrolled to the list as {segment, stamp} (its stamp <= upto: a segment
// enrolled in the open step is already at upto).  A workgroup takes 4096 segments (16 per thread, coalesced),
// ranks its stale ones with a workgroup scan and reserves their list entries
// with one counter atomic.
constexpr int kCompactPerThread = 16;

__global__ void __launch_bounds__(256)
    lazy_compact_kernel(int64_t nseg, const uint2* __restrict__ state, uint2* __restrict__ list,
                        unsigned long long* __restrict__ count, uint32_t upto) {
  // runs on an empty list (the flush catches up first): at most nseg entries
  __shared__ int wave_total[4];
  __shared__ unsigned long long block_base;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t tile = 256 * kCompactPerThread;
  for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < nseg; t0 += (int64_t)gridDim.x * tile) {
    uint32_t mask = 0, stamp[kCompactPerThread];
#pragma unroll
    for (int k = 0; k < kCompactPerThread; ++k) {
      const int64_t seg = t0 + k * 256 + threadIdx.x;
      const uint2 st = seg < nseg ? state[seg] : make_uint2(upto, upto);
      stamp[k] = st.y;
      // never enrolled (done == stamp == 0): m = v = 0 and p is a fixed point of
      // every missed step, so its state already is the dense state at any step
      if (st.x < upto && (st.x | st.y) != 0u) mask |= 1u << k;
    }
    int wtot;
    const int off = wave_excl_scan(__popc(mask), wtot);
    if (lane == 0) wave_total[wid] = wtot;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int tot = wave_total[0] + wave_total[1] + wave_total[2] + wave_total[3];
      block_base = tot ? atomicAdd(count, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    unsigned long long at = block_base + off;
    for (int w = 0; w < wid; ++w) at += wave_total[w];
#pragma unroll
    for (int k = 0; k < kCompactPerThread; ++k)
      if (mask & (1u << k)) {
        if (at < (unsigned long long)nseg)
          list[at] = make_uint2((uint32_t)(t0 + k * 256 + threadIdx.x), stamp[k]);
        ++at;
      }
    __syncthreads();  // wave_total and block_base are reused by the next tile
  }
}

__global__ void lazy_record_kernel(float4* rec, int64_t t, float step_size, float inv_bc2_sqrt,
                                   float gscale, const int32_t* found_inf) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const bool skipped = found_inf != nullptr && *found_inf != 0;
    const float kind = skipped ? kSkipped : (isfinite(gscale) ? kStep : kOddScale);
    rec[t] = make_float4(step_size, inv_bc2_sqrt, gscale, kind);
  }
}

// Empty the list (after a catch-up every entry has been consumed).
__global__ void lazy_empty_list_kernel(unsigned long long* ctr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctr[0] = 0ull;
    ctr[1] = 0ull;
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

// Catch up the listed segments to step `steps`, then empty the list.
void launch_catch_up(const fhash_lazy* lz, const LazyWs& w, float* p, float* gr, float* m,
                     float* v, void* shadow, fhash_dtype sdt, hipStream_t st) {
  const int64_t nseg = lazy_num_segments(lz->end - lz->begin);
  const bool odd = (lz->flags & 1) != 0;
  auto kern = odd ? (lz->moments == FHASH_MOMENTS_PAIRED ? lazy_catchup_kernel<true, true>
                                                         : lazy_catchup_kernel<true, false>)
                  : (lz->moments == FHASH_MOMENTS_PAIRED ? lazy_catchup_kernel<false, true>
                                                         : lazy_catchup_kernel<false, false>);
  hipLaunchKernelGGL(kern, dim3(kListBlocks), dim3(256), 0, st, w.list, w.ctr, w.state, w.rec,
                     lazy_base(lz), p, gr, m, v, shadow, (int)sdt, lz->begin, lz->end,
                     (uint32_t)lz->steps, nseg);
  hipLaunchKernelGGL(lazy_empty_list_kernel, dim3(1), dim3(64), 0, st, w.ctr);
}

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
                               void* shadow, fhash_dtype sdt, uint32_t phases, hipStream_t st) {
  const LazyWs w = carve(lz);
  const uint32_t S = (uint32_t)lz->steps;
  const int64_t nseg = lazy_num_segments(lz->end - lz->begin);
  if ((phases & FHASH_LAZY_MARK) && n > 0 && l0 < l1) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(lazy_mark_kernel, dim3((unsigned)b), dim3(256), 0, st, g, l0, l1,
                       reinterpret_cast<const float4*>(pos), n, w.state, w.list, w.ctr,
                       lz->begin, lz->end, S + 1, (unsigned long long)nseg);
  }
  if (phases & FHASH_LAZY_CATCH_UP) launch_catch_up(lz, w, p, gr, m, v, shadow, sdt, st);
  return hipGetLastError();
}

hipError_t launch_lazy_step(const fhash_adam_desc* o, const fhash_lazy* lz, const int32_t* found_inf,
                            hipStream_t st) {
  const LazyWs w = carve(lz);
  const AdamK k = make_adam_k(o);
  hipLaunchKernelGGL(lazy_record_kernel, dim3(1), dim3(64), 0, st, w.rec, lz->steps + 1,
                     k.step_size, k.inv_bc2_sqrt, k.gscale, found_inf);
  return hipGetLastError();
}

hipError_t lazy_read_stats(const fhash_lazy* lz, int64_t* out, hipStream_t st) {
  const LazyWs w = carve(lz);
  unsigned long long h[4];
  hipError_t e = hipMemcpyAsync(h, w.ctr + 2, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess)
    for (int i = 0; i < 4; ++i) out[i] = (int64_t)h[i];
  return e;
}

hipError_t launch_lazy_flush(const fhash_lazy* lz, float* p, float* gr, float* m, float* v,
                             void* shadow, fhash_dtype sdt, hipStream_t st) {
  const LazyWs w = carve(lz);
  const int64_t nseg = lazy_num_segments(lz->end - lz->begin);
  if (nseg == 0 || lz->steps == 0) return hipSuccess;
  // segments marked without their catch-up first: the list is then empty
  launch_catch_up(lz, w, p, gr, m, v, shadow, sdt, st);
  int64_t b = (nseg + 256 * kCompactPerThread - 1) / (256 * kCompactPerThread);
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(lazy_compact_kernel, dim3((unsigned)b), dim3(256), 0, st, nseg, w.state,
                     w.list, w.ctr, (uint32_t)lz->steps);
  launch_catch_up(lz, w, p, gr, m, v, shadow, sdt, st);
  return hipGetLastError();
}

}  // namespace fh
