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
// State word per segment: {done, stamp}, and one claim flag byte.  The mark
// of prepare for step S+1 sets the flag of every segment the samples touch
// (a plain byte store: every claimer writes the same value, so no atomics are
// needed).  The catch-up scans the flags in segment order, clears them, and
// for each flagged segment not yet enrolled in S+1 replays steps done+1..S
// (the enrolled step `stamp` with its gradient) and stores {S, S+1}; the
// step's gradient is written by the caller's backward.  The step call only
// records the constants (and whether found_inf skipped the step) and runs the
// dense update outside the range; the gradient step of an enrolled segment is
// applied by its next catch-up or by the flush (which flags every segment
// behind the last step and catches them up, keeping their stamps).
#include "adam_dev.h"
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

constexpr int kSeg = FHASH_LAZY_FLOATS;
static_assert(kSeg == 16, "segments of 16 floats");
constexpr int kChunk = 512;  // flagged segments a workgroup sorts by gap in LDS
constexpr int kBins = 64;
constexpr int kTile = 2048;  // claim flags a workgroup scans per pass (8 per thread)

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
  uint32_t seg, done, pend, stamp;  // stamp: the segment's new stamp (0: state unchanged)
  bool stale, work;
  f4v p, m, v, g;
};

// Loads.  stale: done < upto.  A segment never stepped (done == 0, nothing
// pending) holds m = v = 0 and needs no loads.  begin is a multiple of 16 and
// end of 4, so a lane's four floats are all inside the range or all outside.
// Parameter / gradient float a sits at p / g + run_off(a, pm).
template <bool PAIRED>
__device__ __forceinline__ Lane load_lanes(uint32_t seg, uint32_t done, uint32_t pend,
                                           uint32_t stamp, bool stale, int sub,
                                           const float* __restrict__ p,
                                           const float* __restrict__ g,
                                           const float* __restrict__ m,
                                           const float* __restrict__ v, int64_t pm,
                                           int64_t begin, int64_t end) {
  Lane L;
  L.seg = seg;
  L.done = done;
  L.pend = pend;
  L.stamp = stamp;
  L.stale = stale;
  L.f = begin + (int64_t)seg * kSeg + 4 * sub;
  L.work = stale && L.f < end && !(pend == 0 && done == 0);
  const f4v z = {0.f, 0.f, 0.f, 0.f};
  L.p = L.m = L.v = L.g = z;
  if (L.work) {
    L.p = *reinterpret_cast<const f4v*>(p + run_off(L.f, pm));
    L.m = *reinterpret_cast<const f4v*>(m + moment_off<PAIRED>(L.f));
    L.v = *reinterpret_cast<const f4v*>(v + moment_off<PAIRED>(L.f));
    if (pend != 0) L.g = *reinterpret_cast<const f4v*>(g + run_off(L.f, pm));
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
                                             int64_t pm, void* __restrict__ shadow, int sdt,
                                             uint32_t upto) {
  const bool active = L.work && (L.pend != 0 || nonzero_state(L.m, L.v));
  replay<ODD>(rec, base, active, L.done, L.pend, upto, L.g, L.p, L.m, L.v);
  if (active) {
    *reinterpret_cast<f4v*>(p + run_off(L.f, pm)) = L.p;
    *reinterpret_cast<f4v*>(m + moment_off<PAIRED>(L.f)) = L.m;
    *reinterpret_cast<f4v*>(v + moment_off<PAIRED>(L.f)) = L.v;
    if (shadow != nullptr) store_shadow_group(shadow, sdt, L.f, L.p);
  }
  if (L.work && L.pend != 0 && (L.g[0] != 0.f || L.g[1] != 0.f || L.g[2] != 0.f || L.g[3] != 0.f))
    *reinterpret_cast<f4v*>(g + run_off(L.f, pm)) = (f4v){0.f, 0.f, 0.f, 0.f};
  return active;
}

// Every segment of [begin, end) that the forward or backward of a sample reads
// or writes at the levels [l0, l1): the corner row pairs of its cell, exactly
// as the encoding visits them, gets its claim flag set.
__global__ void __launch_bounds__(256)
    lazy_mark_kernel(GridDev g, int l0, int l1, const float4* __restrict__ pos, int64_t n,
                     uint8_t* __restrict__ flags, int64_t begin, int64_t end) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int F = g.F;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float4 p = pos[i];
    for (int l = l0; l < l1; ++l) {
      const LevelDev& d = g.lv[l];
      int ix, iy, iz, it;
      float fx, fy, fz, ft;
      locate(p.x, d.rx, d.sx, ix, fx);
      locate(p.y, d.ry, d.sy, iy, fy);
      locate(p.z, d.rz, d.sz, iz, fz);
      locate(p.w, d.rt, d.st, it, ft);
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
        if (v0 || v1) {
          // F divides 16 and begin is a multiple of 16, so the F floats of a slot
          // lie in one segment; the two slots of a pair are neighbouring rows,
          // rows of one brick, or two hashed rows
          const int64_t fa = (v0 ? s0 : s1) * F, fb = (v1 ? s1 : s0) * F;
          const bool ina = fa >= begin && fa < end, inb = fb >= begin && fb < end;
          const int64_t a = (fa - begin) / kSeg, b = (fb - begin) / kSeg;
          if (ina) flags[a] = 1;
          if (inb && !(ina && b == a)) flags[b] = 1;
        }
      }
    }
  }
}

__device__ __forceinline__ int gap_bin(uint32_t gap) {  // gap >= 1
  if (gap < 16) return (int)gap;
  const int k = 31 - __clz(gap);             // >= 4
  const int quarter = (gap >> (k - 2)) & 3;  // gaps within one bin differ by < 1.25x
  const int b = 16 + 4 * (k - 4) + quarter;
  return b < kBins ? b : kBins - 1;
}

// Catch-up of the flagged segments to step `upto`; ctr[0] hands out the groups
// of tiles (zero at launch); ctr[2..5] accumulate the
// segments caught up, those that loaded data, those with a pending gradient
// and the segment-steps replayed (workload statistics).  target: the stamp
// the caught-up segments take (the step being prepared), or 0 to keep their
// stamps (the flush); with target != 0 a flagged segment already stamped
// target was caught up by an earlier prepare of the same step and is left as
// it is.  Each workgroup scans tiles of kTile flags (clearing them), collects
// the flagged segments in LDS in segment order, and takes them in chunks of
// at most kChunk: a counting sort in LDS by the number of steps to replay,
// then rounds of 64 segments, so that the four segments of a wave replay about
// as many steps.  The flag array is padded with zeros to whole tiles.
template <bool ODD, bool PAIRED>
__global__ void __launch_bounds__(256)
    lazy_catchup_kernel(uint8_t* __restrict__ flags, int64_t nseg, unsigned long long* ctr,
                        uint2* __restrict__ state, const float4* __restrict__ rec, AdamK base,
                        float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, int64_t pm, void* __restrict__ shadow, int sdt,
                        int64_t begin, int64_t end, uint32_t upto, uint32_t target, int group) {
  // flagged segments not yet caught up: fewer than kChunk carried over plus
  // at most one tile's worth
  __shared__ uint32_t ids[kTile + kChunk];
  __shared__ uint4 srt[kChunk];
  __shared__ int hist[kBins], boff[kBins];
  __shared__ int wave_total[4];
  __shared__ unsigned long long tally[4];
  if (threadIdx.x < 4) tally[threadIdx.x] = 0ull;
  unsigned long long n_stale = 0, n_work = 0, n_pend = 0, n_steps = 0;
  const int sub = threadIdx.x & (kLanesPerSeg - 1);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __shared__ int64_t next_first;
  int cnt = 0;  // entries in ids (the same in every thread)
  // groups of `group` consecutive tiles, each claimed by the next workgroup
  // free (counter ctr[0], zero at launch): a chunk's segments are mostly
  // neighbours in memory, and the work follows the flags' density
  const int64_t ntiles = (nseg + kTile - 1) / kTile;
  int64_t first = 0;
  for (int64_t it = 0;; ++it) {
    if (it % group == 0) {
      // thread 0 writes next_first again only after the scan's barriers of
      // this group's first tile, which every thread reaches after reading it
      if (threadIdx.x == 0) next_first = (int64_t)atomicAdd(&ctr[0], 1ull) * group;
      __syncthreads();
      first = next_first;
    }
    const int64_t tile = first + it % group;
    const bool more = first < ntiles;  // workgroup-uniform
    const int64_t t0 = tile * kTile;
    if (more && tile < ntiles) {
      // the flags of segments t0 + 8 threadIdx.x .. + 7
      uint2* fw = reinterpret_cast<uint2*>(flags + t0) + threadIdx.x;
      const uint2 w = *fw;
      uint32_t bits = 0;
      if ((w.x | w.y) != 0u) {
        *fw = make_uint2(0u, 0u);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          bits |= ((w.x >> (8 * k)) & 0xffu) ? 1u << k : 0u;
          bits |= ((w.y >> (8 * k)) & 0xffu) ? 1u << (k + 4) : 0u;
        }
      }
      int wtot;
      const int off = wave_excl_scan(__popc(bits), wtot);
      if (lane == 0) wave_total[wid] = wtot;
      __syncthreads();
      int at = cnt + off, total = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        at += q < wid ? wave_total[q] : 0;
        total += wave_total[q];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (bits & (1u << k)) ids[at++] = (uint32_t)(t0 + 8 * threadIdx.x + k);
      cnt += total;
      __syncthreads();  // ids written; wave_total may be reused
    }
    // full chunks (the fuller the chunk, the closer the replay lengths its
    // sort puts into one wave); at the end the rest
    int c0 = 0;
    while (cnt - c0 >= kChunk || (!more && cnt - c0 > 0)) {
      const int nloc = cnt - c0 < kChunk ? cnt - c0 : kChunk;
      if (threadIdx.x < kBins) hist[threadIdx.x] = 0;
      __syncthreads();
      uint4 ent[kChunk / 256];
      int bin[kChunk / 256], rank[kChunk / 256];
#pragma unroll
      for (int k = 0; k < kChunk / 256; ++k) {
        const int i = threadIdx.x + k * 256;
        bin[k] = -1;
        if (i < nloc) {
          const uint32_t seg = ids[c0 + i];
          const uint2 st = state[seg];
          const uint32_t done = st.x;
          if (target == 0u || st.y < target) {
            // enrolled step not yet applied (stamps never pass upto here)
            const uint32_t pend = st.y > done && st.y <= upto ? st.y : 0u;
            ent[k] = make_uint4(seg, done, pend, target != 0u ? target : st.y);
            bin[k] = (done >= upto || (pend == 0 && done == 0)) ? 0 : gap_bin(upto - done);
          } else {  // enrolled in this step already: nothing to do
            ent[k] = make_uint4(seg, upto, 0u, 0u);
            bin[k] = 0;
          }
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
        return load_lanes<PAIRED>(en.x, en.y, en.z, en.w, e < nloc && en.y < upto, sub, p, g, m,
                                  v, pm, begin, end);
      };
      Lane cur = fetch(0);
      for (int r0 = 0; r0 < nloc; r0 += 256 / kLanesPerSeg) {
        const Lane nxt = fetch(r0 + 256 / kLanesPerSeg);
        const bool active =
            finish_lanes<ODD, PAIRED>(cur, rec, base, p, g, m, v, pm, shadow, sdt, upto);
        if (sub == 0 && cur.stamp != 0u)
          state[cur.seg] = make_uint2(cur.stale ? upto : cur.done, cur.stamp);
        if (cur.stale && sub == 0) {
          n_stale += 1;
          n_work += cur.work;
          n_pend += cur.work && cur.pend != 0;
          if (active) n_steps += upto - cur.done;
        }
        cur = nxt;
      }
      c0 += nloc;
      __syncthreads();  // srt and hist are reused by the next chunk
    }
    if (!more) break;
    if (c0 > 0) {
      // carry the rest (fewer than kChunk) to the front
      const int rest = cnt - c0;
      uint32_t keep[kChunk / 256];
#pragma unroll
      for (int k = 0; k < kChunk / 256; ++k) {
        const int i = threadIdx.x + k * 256;
        keep[k] = i < rest ? ids[c0 + i] : 0u;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kChunk / 256; ++k) {
        const int i = threadIdx.x + k * 256;
        if (i < rest) ids[i] = keep[k];
      }
      __syncthreads();
      cnt = rest;
    }
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

// Flush, first part: flag every segment behind step `upto` that was ever
// enrolled (a segment enrolled in the open step is already at upto); 8
// segments per thread, one 8-byte flag store.
__global__ void __launch_bounds__(256)
    lazy_flag_stale_kernel(int64_t nseg, const uint2* __restrict__ state,
                           uint8_t* __restrict__ flags, uint32_t upto) {
  for (int64_t s0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8; s0 < nseg;
       s0 += (int64_t)gridDim.x * blockDim.x * 8) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint2 st = s0 + k < nseg ? state[s0 + k] : make_uint2(upto, upto);
      // never enrolled (done == stamp == 0): m = v = 0 and p is a fixed point of
      // every missed step, so its state already is the dense state at any step
      if (st.x < upto && (st.x | st.y) != 0u) {
        if (k < 4)
          lo |= 1u << (8 * k);
        else
          hi |= 1u << (8 * (k - 4));
      }
    }
    if (lo | hi) *reinterpret_cast<uint2*>(flags + s0) = make_uint2(lo, hi);
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

// Zero the catch-up's group counter (a fill kernel, not a memset node, so that
// the launch sequence can be captured in a graph).
__global__ void lazy_reset_groups_kernel(unsigned long long* ctr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr[0] = 0ull;
}

__global__ void __launch_bounds__(256) lazy_zero_kernel(uint4* __restrict__ w, int64_t n16) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = make_uint4(0u, 0u, 0u, 0u);
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct LazyWs {
  uint2* state;
  uint8_t* flags;           // one per segment, zero-padded to whole tiles
  unsigned long long* ctr;  // [0] next group of flag tiles, [2..5] workload statistics
  float4* rec;
};

inline int64_t flag_bytes(int64_t nseg) { return (nseg + kTile - 1) / kTile * kTile; }

LazyWs carve(const fhash_lazy* lz) {
  const int64_t nseg = lazy_num_segments(lz->end - lz->begin);
  char* b = reinterpret_cast<char*>(lz->ws);
  LazyWs w;
  w.state = reinterpret_cast<uint2*>(b);
  b += align256((size_t)nseg * 8);
  w.flags = reinterpret_cast<uint8_t*>(b);
  b += align256((size_t)flag_bytes(nseg));
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

// Grid of the catch-up: grid-strided over tiles of flags.
constexpr int64_t kCatchUpBlocks = 2048;

// Catch up the flagged segments to step `steps` (stamping them `target`, or
// keeping their stamps when 0) and clear the flags.  expected: about how many
// flags are set (0: unknown, dense); it sizes the groups of tiles so that a
// group holds about one chunk.
void launch_catch_up(const fhash_lazy* lz, const LazyWs& w, uint32_t target, int64_t expected,
                     float* p, float* gr, float* m, float* v, void* shadow, fhash_dtype sdt,
                     hipStream_t st) {
  const int64_t nseg = lazy_num_segments(lz->end - lz->begin);
  if (nseg == 0) return;
  const int64_t ntiles = flag_bytes(nseg) / kTile;
  int64_t group = 1;
  if (expected > 0 && expected < nseg) {
    group = (2 * (int64_t)kChunk * nseg + kTile * expected) / (2 * (int64_t)kTile * expected);
    group = group < 1 ? 1 : (group > 64 ? 64 : group);
  }
  int64_t blocks = (ntiles + group - 1) / group;
  if (blocks > kCatchUpBlocks) blocks = kCatchUpBlocks;
  const bool odd = (lz->flags & 1) != 0;
  const bool runs = lz->moments != FHASH_MOMENTS_SEPARATE;  // m, v in runs of 16
  auto kern = odd ? (runs ? lazy_catchup_kernel<true, true> : lazy_catchup_kernel<true, false>)
                  : (runs ? lazy_catchup_kernel<false, true> : lazy_catchup_kernel<false, false>);
  const int64_t pm = lz->moments == FHASH_MOMENTS_WITH_PARAMS ? ~(int64_t)15 : 0;
  hipLaunchKernelGGL(lazy_reset_groups_kernel, dim3(1), dim3(64), 0, st, w.ctr);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, w.flags, nseg, w.ctr,
                     w.state, w.rec, lazy_base(lz), p, gr, m, v, pm, shadow, (int)sdt, lz->begin,
                     lz->end, (uint32_t)lz->steps, target, (int)group);
}

}  // namespace

int64_t lazy_num_segments(int64_t range_floats) { return (range_floats + kSeg - 1) / kSeg; }

size_t lazy_ws_bytes(int64_t range_floats, int64_t max_steps) {
  const int64_t nseg = lazy_num_segments(range_floats);
  return align256((size_t)nseg * 8) + align256((size_t)flag_bytes(nseg)) + 256 +
         align256((size_t)(max_steps + 1) * 16);
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
  if ((phases & FHASH_LAZY_MARK) && n > 0 && l0 < l1) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(lazy_mark_kernel, dim3((unsigned)b), dim3(256), 0, st, g, l0, l1,
                       reinterpret_cast<const float4*>(pos), n, w.flags, lz->begin, lz->end);
  }
  // at most 9 segments per sample and level (8 row pairs, one may straddle)
  const int64_t expected = n * (int64_t)(l1 > l0 ? l1 - l0 : 0) * 9;
  if (phases & FHASH_LAZY_CATCH_UP)
    launch_catch_up(lz, w, S + 1, expected, p, gr, m, v, shadow, sdt, st);
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
  // segments marked without their catch-up first (enrolled in the open step);
  // then every flag is clear
  launch_catch_up(lz, w, (uint32_t)lz->steps + 1, 0, p, gr, m, v, shadow, sdt, st);
  int64_t b = (nseg + 256 * 8 - 1) / (256 * 8);
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(lazy_flag_stale_kernel, dim3((unsigned)b), dim3(256), 0, st, nseg, w.state,
                     w.flags, (uint32_t)lz->steps);
  launch_catch_up(lz, w, 0u, 0, p, gr, m, v, shadow, sdt, st);
  return hipGetLastError();
}

}  // namespace fh
