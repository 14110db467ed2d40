// Device-side building blocks of the tesseract encoding, shared by the
// standalone encoding kernels and the fused encoding + MLP kernels.
#pragma once
#include <hip/hip_fp16.h>

#include "common.h"

namespace fh {

template <int F, typename T>
struct RowLoad;

template <>
struct RowLoad<1, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t s, float* o) { o[0] = t[s]; }
};
template <>
struct RowLoad<2, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t s, float* o) {
    const float2 v = *reinterpret_cast<const float2*>(t + 2 * s);
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct RowLoad<4, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t s, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(t + 4 * s);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct RowLoad<8, float> {
  static __device__ __forceinline__ void load(const float* t, int64_t s, float* o) {
    const float4 a = *reinterpret_cast<const float4*>(t + 8 * s);
    const float4 b = *reinterpret_cast<const float4*>(t + 8 * s + 4);
    o[0] = a.x, o[1] = a.y, o[2] = a.z, o[3] = a.w;
    o[4] = b.x, o[5] = b.y, o[6] = b.z, o[7] = b.w;
  }
};
template <>
struct RowLoad<1, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t s, float* o) {
    o[0] = __half2float(t[s]);
  }
};
template <>
struct RowLoad<2, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t s, float* o) {
    const __half2 v = *reinterpret_cast<const __half2*>(t + 2 * s);
    const float2 f = __half22float2(v);
    o[0] = f.x;
    o[1] = f.y;
  }
};
template <>
struct RowLoad<4, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t s, float* o) {
    const uint2 raw = *reinterpret_cast<const uint2*>(t + 4 * s);
    const __half2* h = reinterpret_cast<const __half2*>(&raw);
    const float2 a = __half22float2(h[0]), b = __half22float2(h[1]);
    o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
  }
};
template <>
struct RowLoad<8, __half> {
  static __device__ __forceinline__ void load(const __half* t, int64_t s, float* o) {
    const uint4 raw = *reinterpret_cast<const uint4*>(t + 8 * s);
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
// Requires a table with at least one row.
template <int F, typename T>
__device__ __forceinline__ void encode_level(const LevelDev& d, const ulonglong2* dir, bool active,
                                             const float4 p, const T* __restrict__ table,
                                             float* out) {
  int ix, iy, iz, it;
  float fx, fy, fz, ft;
  locate(p.x, d.rx, d.sx, ix, fx);
  locate(p.y, d.ry, d.sy, iy, fy);
  locate(p.z, d.rz, d.sz, iz, fz);
  locate(p.w, d.rt, d.st, it, ft);
  float acc[F];
#pragma unroll
  for (int k = 0; k < F; ++k) acc[k] = 0.0f;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int dy = r & 1, dz = (r >> 1) & 1, dt = (r >> 2) & 1;
    const int64_t row = ((int64_t)(it + dt) * d.rz + (iz + dz)) * d.ry + (iy + dy);
    const float wr = (dy ? fy : 1.0f - fy) * (dz ? fz : 1.0f - fz) * (dt ? ft : 1.0f - ft);
    int64_t s0, s1;
    bool v0, v1;
    row_pair_slots(d, dir, active, row, ix, s0, s1, v0, v1);
    float e0[F], e1[F];
    RowLoad<F, T>::load(table, v0 ? s0 : 0, e0);
    RowLoad<F, T>::load(table, v1 ? s1 : 0, e1);
    const float w0 = v0 ? wr * (1.0f - fx) : 0.0f;
    const float w1 = v1 ? wr * fx : 0.0f;
#pragma unroll
    for (int k = 0; k < F; ++k) acc[k] += w0 * e0[k] + w1 * e1[k];
  }
#pragma unroll
  for (int k = 0; k < F; ++k) out[k] = acc[k];
}

// Adjoint of encode_level: d_table[slot_c][k] += w_c g[k] with FP32 hardware
// atomics (no return value).  Weights are recomputed from the position.
template <int F>
__device__ __forceinline__ void scatter_level(const LevelDev& d, const ulonglong2* dir,
                                              bool active, const float4 p, const float* g,
                                              float* __restrict__ d_table) {
  int ix, iy, iz, it;
  float fx, fy, fz, ft;
  locate(p.x, d.rx, d.sx, ix, fx);
  locate(p.y, d.ry, d.sy, iy, fy);
  locate(p.z, d.rz, d.sz, iz, fz);
  locate(p.w, d.rt, d.st, it, ft);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int dy = r & 1, dz = (r >> 1) & 1, dt = (r >> 2) & 1;
    const int64_t row = ((int64_t)(it + dt) * d.rz + (iz + dz)) * d.ry + (iy + dy);
    const float wr = (dy ? fy : 1.0f - fy) * (dz ? fz : 1.0f - fz) * (dt ? ft : 1.0f - ft);
    int64_t s0, s1;
    bool v0, v1;
    row_pair_slots(d, dir, active, row, ix, s0, s1, v0, v1);
    const float w0 = wr * (1.0f - fx), w1 = wr * fx;
    if (v0) {
#pragma unroll
      for (int k = 0; k < F; ++k) unsafeAtomicAdd(d_table + s0 * F + k, w0 * g[k]);
    }
    if (v1) {
#pragma unroll
      for (int k = 0; k < F; ++k) unsafeAtomicAdd(d_table + s1 * F + k, w1 * g[k]);
    }
  }
}

}  // namespace fh
