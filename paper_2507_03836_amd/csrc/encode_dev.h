// Device-side building blocks of the tesseract encoding, shared by the
// standalone encoding kernels and the fused encoding + MLP kernels.
#pragma once
#include <hip/hip_fp16.h>

#include "common.h"

namespace fh {

// The F values of a table row whose first element is at offset e.
template <int F, typename T>
struct RowLoad;

template <>
struct RowLoad<1, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t e, float* o) { o[0] = t[e]; }
};
template <>
struct RowLoad<2, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t e, float* o) {
    const float2 v = *reinterpret_cast<const float2*>(t + e);
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct RowLoad<4, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t e, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(t + e);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct RowLoad<8, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t e, float* o) {
    const float4 a = *reinterpret_cast<const float4*>(t + e);
    const float4 b = *reinterpret_cast<const float4*>(t + e + 4);
    o[0] = a.x, o[1] = a.y, o[2] = a.z, o[3] = a.w;
    o[4] = b.x, o[5] = b.y, o[6] = b.z, o[7] = b.w;
  }
};
template <>
struct RowLoad<1, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t e, float* o) {
    o[0] = __half2float(t[e]);
  }
};
template <>
struct RowLoad<2, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t e, float* o) {
    const __half2 v = *reinterpret_cast<const __half2*>(t + e);
    const float2 f = __half22float2(v);
    o[0] = f.x;
    o[1] = f.y;
  }
};
template <>
struct RowLoad<4, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t e, float* o) {
    const uint2 raw = *reinterpret_cast<const uint2*>(t + e);
    const __half2* h = reinterpret_cast<const __half2*>(&raw);
    const float2 a = __half22float2(h[0]), b = __half22float2(h[1]);
    o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
  }
};
template <>
struct RowLoad<8, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t e, float* o) {
    const uint4 raw = *reinterpret_cast<const uint4*>(t + e);
    const __half2* h = reinterpret_cast<const __half2*>(&raw);
    for (int i = 0; i < 4; ++i) {
      const float2 a = __half22float2(h[i]);
      o[2 * i] = a.x;
      o[2 * i + 1] = a.y;
    }
  }
};

// Forward of one level for one sample: out[k] = sum_c w_c E[slot_c][k].
// Invalid (inactive) corners get weight 0 and read row 0, so every load is
// unconditional and the 8 directory / 16 table loads overlap in flight.
// Requires a table with at least one row.  tmask: the table's run mask
// (run_off; F divides 16, so a row never straddles a run).
template <int F, typename T, bool BRICK = false>
__device__ __forceinline__ void encode_level(const LevelDev& d, const ulonglong2* dir, bool active,
                                             const float4 p, const T* __restrict__ table,
                                             float* out, int64_t tmask) {
  int ix, iy, iz, it;
  float fx, fy, fz, ft;
  locate(p.x, d.rx, d.sx, ix, fx);
  locate(p.y, d.ry, d.sy, iy, fy);
  locate(p.z, d.rz, d.sz, iz, fz);
  locate(p.w, d.rt, d.st, it, ft);
  float acc[F];
#pragma unroll
  for (int k = 0; k < F; ++k) acc[k] = 0.0f;
  const int a = pair_axis<BRICK>(ix, iy, iz, it);
  const float fa = pair_frac(a, fx, fy, fz, ft);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    float wr;
    int64_t s0, s1;
    bool v0, v1;
    corner_pair<BRICK>(d, dir, active, ix, iy, iz, it, fx, fy, fz, ft, a, r, s0, s1, v0, v1, wr);
    float e0[F], e1[F];
    RowLoad<F, T>::load(table, run_off((v0 ? s0 : 0) * F, tmask), e0);
    RowLoad<F, T>::load(table, run_off((v1 ? s1 : 0) * F, tmask), e1);
    const float w0 = v0 ? wr * (1.0f - fa) : 0.0f;
    const float w1 = v1 ? wr * fa : 0.0f;
#pragma unroll
    for (int k = 0; k < F; ++k) acc[k] += w0 * e0[k] + w1 * e1[k];
  }
#pragma unroll
  for (int k = 0; k < F; ++k) out[k] = acc[k];
}

// Touched-segment flag of a gradient write at float index fidx: the segment of
// FHASH_TOUCH_FLOATS floats that holds it is flagged (a plain byte store; all
// writers store the same value).  Only floats at or after `tbeg` are tracked.
__device__ __forceinline__ void mark_touched(uint8_t* touch, int64_t tbeg, int64_t fidx) {
  if (touch != nullptr && fidx >= tbeg) touch[fidx / FHASH_TOUCH_FLOATS] = 1;
}

// Adjoint of encode_level: d_table[slot_c][k] += w_c g[k] with FP32 hardware
// atomics (no return value).  Weights are recomputed from the position.
// gmask: the gradient's run mask (run_off); touch flags index the logical
// floats.
template <int F, bool BRICK = false>
__device__ __forceinline__ void scatter_level(const LevelDev& d, const ulonglong2* dir,
                                              bool active, const float4 p, const float* g,
                                              float* __restrict__ d_table, uint8_t* touch,
                                              int64_t tbeg, int64_t gmask) {
  int ix, iy, iz, it;
  float fx, fy, fz, ft;
  locate(p.x, d.rx, d.sx, ix, fx);
  locate(p.y, d.ry, d.sy, iy, fy);
  locate(p.z, d.rz, d.sz, iz, fz);
  locate(p.w, d.rt, d.st, it, ft);
  const int a = pair_axis<BRICK>(ix, iy, iz, it);
  const float fa = pair_frac(a, fx, fy, fz, ft);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    float wr;
    int64_t s0, s1;
    bool v0, v1;
    corner_pair<BRICK>(d, dir, active, ix, iy, iz, it, fx, fy, fz, ft, a, r, s0, s1, v0, v1, wr);
    const float w0 = wr * (1.0f - fa), w1 = wr * fa;
    if (v0) {
#pragma unroll
      for (int k = 0; k < F; ++k) unsafeAtomicAdd(d_table + run_off(s0 * F, gmask) + k, w0 * g[k]);
      mark_touched(touch, tbeg, s0 * F);
    }
    if (v1) {
#pragma unroll
      for (int k = 0; k < F; ++k) unsafeAtomicAdd(d_table + run_off(s1 * F, gmask) + k, w1 * g[k]);
      mark_touched(touch, tbeg, s1 * F);
    }
  }
}

// One lane's share of a level's scatter-add.  The lane owns pair element e
// (the first or second corner of every corner pair, corner_pair) and feature f
// of one sample: 2F consecutive lanes own one sample, so the 2F atomics they
// issue together hit the two slots of one pair (8F contiguous bytes in the
// rows layout and for x pairs inside a brick; 4F-byte halves a few rows apart
// inside one brick otherwise).  Atomics of one
// instruction that fall in the same 64-byte segment are performed as one
// memory transaction, which is what bounds the scatter on gfx950.
template <int F, bool BRICK = false>
__device__ __forceinline__ void scatter_level_lane(const LevelDev& d, const ulonglong2* dir,
                                                   bool active, const float4 p, int e, int f,
                                                   float gval, float* __restrict__ d_table,
                                                   uint8_t* touch, int64_t tbeg, int64_t gmask) {
  int ix, iy, iz, it;
  float fx, fy, fz, ft;
  locate(p.x, d.rx, d.sx, ix, fx);
  locate(p.y, d.ry, d.sy, iy, fy);
  locate(p.z, d.rz, d.sz, iz, fz);
  locate(p.w, d.rt, d.st, it, ft);
  const int a = pair_axis<BRICK>(ix, iy, iz, it);
  const float fa = pair_frac(a, fx, fy, fz, ft);
  const float wx = e ? fa : 1.0f - fa;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    float wr;
    int64_t s0, s1;
    bool v0, v1;
    corner_pair<BRICK>(d, dir, active, ix, iy, iz, it, fx, fy, fz, ft, a, r, s0, s1, v0, v1, wr);
    const int64_t s = e ? s1 : s0;
    if (e ? v1 : v0) {
      unsafeAtomicAdd(d_table + run_off(s * F, gmask) + f, wr * wx * gval);
      if (f == 0) mark_touched(touch, tbeg, s * F);  // F divides the segment: one flag per slot
    }
  }
}

// scatter_level_lane for a batch in cell order (fhash_sort_samples): a pass
// of the scatter holds one level for W / 2F samples (the W lanes that share
// the level: 64, or 32 at F = 1), and at the coarse levels neighbouring
// samples often all fall on the same vertex.  Lanes that add into the same
// float of one chunk cannot share a memory request, so a corner that every
// sample of the pass hits on one slot is summed across the samples first
// (xor shuffles) and added by the first sample's lanes alone; any other corner
// is added lane by lane.  Every lane of the W-lane group calls it (a sample
// that is not valid passes valid = false and adds nothing).
template <int F, bool BRICK = false>
__device__ __forceinline__ void scatter_level_lane_merge(const LevelDev& d, const ulonglong2* dir,
                                                         bool active, const float4 p, bool valid,
                                                         int e, int f, float gval,
                                                         float* __restrict__ d_table,
                                                         uint8_t* touch, int64_t tbeg,
                                                         int64_t gmask) {
  constexpr int Q = 2 * F;
  constexpr int W = (16 * Q < 64) ? 16 * Q : 64;
  const int lane = threadIdx.x & 63;
  const int base = lane & ~(W - 1);
  const int lead = base + (lane & (Q - 1));  // the same (e, f) lane of the first sample
  const uint64_t group = (W == 64) ? ~0ull : (((1ull << W) - 1) << base);
  int ix, iy, iz, it;
  float fx, fy, fz, ft;
  locate(p.x, d.rx, d.sx, ix, fx);
  locate(p.y, d.ry, d.sy, iy, fy);
  locate(p.z, d.rz, d.sz, iz, fz);
  locate(p.w, d.rt, d.st, it, ft);
  const int a = pair_axis<BRICK>(ix, iy, iz, it);
  const float fa = pair_frac(a, fx, fy, fz, ft);
  const float wx = e ? fa : 1.0f - fa;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    float wr;
    int64_t s0, s1;
    bool v0, v1;
    corner_pair<BRICK>(d, dir, active, ix, iy, iz, it, fx, fy, fz, ft, a, r, s0, s1, v0, v1, wr);
    const int64_t s = (valid && (e ? v1 : v0)) ? (e ? s1 : s0) : -1;
    float val = (s >= 0) ? wr * wx * gval : 0.0f;
    const int64_t s_lead = __shfl(s, lead, 64);
    const bool same = s_lead >= 0 && (s < 0 || s == s_lead);
    if ((__ballot(same) & group) == group) {
#pragma unroll
      for (int o = Q; o < W; o <<= 1) val += __shfl_xor(val, o, 64);
      if (lane == lead) {
        unsafeAtomicAdd(d_table + run_off(s_lead * F, gmask) + f, val);
        if (f == 0) mark_touched(touch, tbeg, s_lead * F);
      }
    } else if (s >= 0) {
      unsafeAtomicAdd(d_table + run_off(s * F, gmask) + f, val);
      if (f == 0) mark_touched(touch, tbeg, s * F);
    }
  }
}

}  // namespace fh
