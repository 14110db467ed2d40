// Internal definitions shared by the HIP kernels and the C-ABI layer of libfhash.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fhash.h"

namespace fh {

// Per-level constants, passed by value in kernel arguments (wave-uniform loads).
struct LevelDev {
  int32_t rx, ry, rz, rt;  // vertex counts
  float sx, sy, sz, st;    // (float)(R - 1), the FP32 scale of cell location
  int32_t wv;              // directory words per vertex row: ceil(rx / 64); bricks:
                           // words per brick row, ceil(ceil(rx / 2) / 4)
  int32_t hash_bits;       // 0, or b: the level's vertices hash into 2^b rows
  int64_t slot_off;        // first table row of the level
  int64_t dir_off;         // first directory entry of the level
  int32_t brick;           // 1: slots ranked in 2^4-vertex bricks
  int32_t by;              // brick rows per (bt, bz): ceil(ry / 2)
};
static_assert(sizeof(LevelDev) == 64, "LevelDev layout");

struct GridDev {
  LevelDev lv[FHASH_MAX_LEVELS];
  const ulonglong2* dir;  // {bits, rank-before-word}; NULL when dense
  int32_t L, F;
  int32_t active;
  uint32_t dedup;  // bit l: combine equal slots of neighbouring lanes before level l's atomics
  uint8_t* touch;  // touched-segment flags of the table gradient (NULL: not tracked)
  int64_t touch_begin;  // first tracked float (a multiple of FHASH_TOUCH_FLOATS)
  // run masks of the table read and of the table gradient (run_off): 0, dense;
  // ~15, the paired layout (16 values, then 16 floats of the other array)
  int64_t tmask, gmask;
  // levels 0 .. coarse - 1: the fused backward leaves their encoding gradient
  // in dxc ([level][sample][feature], nsamp samples) for the LDS scatter
  int32_t coarse;
  float* dxc;
  int64_t nsamp;
};

// Float offset of element i of a vector stored in runs of 16 values separated
// by 16-float gaps (mask ~15), or densely (mask 0): i + 16 floor(i / 16).
__host__ __device__ __forceinline__ int64_t run_off(int64_t i, int64_t mask) {
  return i + (i & mask);
}

// Fill a GridDev from a public index descriptor (host).
inline void make_grid_dev(const fhash_index* idx, GridDev* g) {
  const fhash_grid_desc& gd = idx->grid;
  g->L = gd.n_levels;
  g->F = gd.n_features;
  g->active = idx->active;
  g->dir = reinterpret_cast<const ulonglong2*>(idx->dir);
  g->dedup = 0;
  g->touch = nullptr;
  g->touch_begin = 0;
  g->tmask = 0;
  g->gmask = 0;
  g->coarse = 0;
  g->dxc = nullptr;
  g->nsamp = 0;
  for (int l = 0; l < FHASH_MAX_LEVELS; ++l) {
    LevelDev& d = g->lv[l];
    if (l < gd.n_levels) {
      d.rx = gd.res[l][0];
      d.ry = gd.res[l][1];
      d.rz = gd.res[l][2];
      d.rt = gd.res[l][3];
      d.sx = (float)(d.rx - 1);
      d.sy = (float)(d.ry - 1);
      d.sz = (float)(d.rz - 1);
      d.st = (float)(d.rt - 1);
      d.brick = gd.layout == FHASH_LAYOUT_BRICKS ? 1 : 0;
      d.wv = d.brick ? ((d.rx + 1) / 2 + 3) / 4 : (d.rx + 63) / 64;
      d.by = (d.ry + 1) / 2;
      d.slot_off = idx->slot_offset[l];
      d.dir_off = idx->dir_offset[l];
      const double nv = (double)d.rx * d.ry * d.rz * d.rt;
      d.hash_bits = (idx->hash_bits > 0 && nv > (double)(1ll << idx->hash_bits)) ? idx->hash_bits : 0;
    } else {
      d = LevelDev{};
    }
  }
}

#ifdef __HIPCC__
// Cell location along one dimension (Sec. 3.2.4 steps 1-2).  Clamp to [0,1]
// (NaN -> 0 via IEEE maxNum), one FP32 multiply, floor, clamp to R-2, exact
// fraction.  __fmul_rn / __fsub_rn keep the compiler from contracting.
__device__ __forceinline__ void locate(float p, int R, float s, int& cell, float& frac) {
  p = fminf(fmaxf(p, 0.0f), 1.0f);
  float u = __fmul_rn(p, s);
  int i = (int)floorf(u);
  i = min(i, R - 2);
  cell = i;
  frac = __fsub_rn(u, (float)i);
}

// Row of vertex (x, y, z, t) in a hashed level (see fhash_hash_index).
__device__ __forceinline__ uint32_t spatial_hash(uint32_t x, uint32_t yzt, uint32_t mask) {
  return (x ^ yzt) & mask;
}

// Rank-directory lookup: slot of bit b of entry e (valid iff the bit is set).
__device__ __forceinline__ int64_t entry_slot(const ulonglong2& e, int b, int64_t slot_off,
                                              bool& valid) {
  valid = (e.x >> b) & 1ull;
  const uint64_t below = (b == 0) ? 0ull : (e.x & ((1ull << b) - 1ull));
  return slot_off + (int64_t)e.y + __popcll(below);
}

// Directory entries holding vertices x and x+1 of vertex row (t, z, y) of an
// active level (w1 = w0 when both sit in one entry).  Rows layout: entries
// ((t*Rz + z)*Wv + word)*Ry + y (rows y and y+1 of a cell are neighbours);
// bricks: ((bt*Bz + bz)*Wb + word)*By + by.  Bit positions in b0, b1.  Row,
// word and entry indices are 32-bit: the host rejects levels with 2^31
// directory entries or more.
// BRICK: the index's slot order (rows false, bricks true), a compile-time
// choice so that each order's kernels carry only their own arithmetic.
template <bool BRICK>
__device__ __forceinline__ void pair_entries(const LevelDev& d, int32_t t, int32_t z, int32_t y,
                                             int x, int64_t& w0, int64_t& w1, int& b0, int& b1) {
  if constexpr (BRICK) {
    const int inner = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((t & 1) << 3);
    const int bit0 = (x >> 1) * 16 + inner;
    // x odd: x + 1 is the first x of the next brick, 15 bits further on
    const int bit1 = (x & 1) ? bit0 + 15 : bit0 + 1;
    const int32_t btz = (t >> 1) * ((d.rz + 1) >> 1) + (z >> 1);
    w0 = d.dir_off + (int64_t)((btz * d.wv + (bit0 >> 6)) * d.by + (y >> 1));
    w1 = ((bit1 >> 6) == (bit0 >> 6)) ? w0 : w0 + d.by;
    b0 = bit0 & 63;
    b1 = bit1 & 63;
  } else {
    const int32_t tz = t * d.rz + z;
    w0 = d.dir_off + (int64_t)((tz * d.wv + (x >> 6)) * d.ry + y);
    w1 = ((x & 63) == 63) ? w0 + d.ry : w0;
    b0 = x & 63;
    b1 = (x + 1) & 63;
  }
}

// Brick layout: the 16 corners of a cell are taken as 8 pairs along one axis
// a, the first axis (x, y, z, t) whose cell index is even, so that both
// corners of every pair lie in one brick (neighbouring rows, or rows 2^a apart
// inside it) and a pair's atomics stay one memory transaction; x when every
// index is odd (pairs then straddle two bricks).  Rows layout: a = 0, pairs
// along x (the vertex rows of the F-Hash order).
template <bool BRICK>
__device__ __forceinline__ int pair_axis(int cx, int cy, int cz, int ct) {
  if constexpr (!BRICK) return 0;
  return !(cx & 1) ? 0 : !(cy & 1) ? 1 : !(cz & 1) ? 2 : !(ct & 1) ? 3 : 0;
}

// Offsets of corner pair r (0..7) of a cell paired along axis a: the other
// three axes, in increasing order, take bits 0, 1, 2 of r (the pair's own
// axis is 0 for its first corner, 1 for its second).
__device__ __forceinline__ void pair_offsets(int r, int a, int& ox, int& oy, int& oz, int& ot) {
  ox = a == 0 ? 0 : (r & 1);
  oy = a == 1 ? 0 : (a == 0 ? (r & 1) : ((r >> 1) & 1));
  oz = a == 2 ? 0 : (a == 3 ? ((r >> 2) & 1) : ((r >> 1) & 1));
  ot = a == 3 ? 0 : ((r >> 2) & 1);
}

// Slots of the vertex pair (x, x+1) on vertex row (t, z, y) of a level.
// Dense: the F-Hash equation; hashed: the spatial hash; active: ranks in the
// directory (rows or bricks layout, see pair_entries).
template <bool BRICK = false>
__device__ __forceinline__ void row_pair_slots(const LevelDev& d, const ulonglong2* dir,
                                               bool active, int32_t t, int32_t z, int32_t y, int x,
                                               int64_t& s0, int64_t& s1, bool& v0, bool& v1) {
  if (d.hash_bits) {
    const uint32_t yzt = (uint32_t)y * 2654435761u ^ (uint32_t)z * 805459861u ^
                         (uint32_t)t * 3674653429u;
    const uint32_t mask = (d.hash_bits >= 32) ? 0xffffffffu : ((1u << d.hash_bits) - 1u);
    s0 = d.slot_off + spatial_hash((uint32_t)x, yzt, mask);
    s1 = d.slot_off + spatial_hash((uint32_t)x + 1u, yzt, mask);
    v0 = v1 = true;
    return;
  }
  if (!active) {
    s0 = d.slot_off + ((int64_t)(t * d.rz + z) * d.ry + y) * d.rx + x;
    s1 = s0 + 1;
    v0 = v1 = true;
    return;
  }
  int64_t w0, w1;
  int b0, b1;
  pair_entries<BRICK>(d, t, z, y, x, w0, w1, b0, b1);
  const ulonglong2 e = dir[w0];
  s0 = entry_slot(e, b0, d.slot_off, v0);
  if (w1 == w0) {
    if (b1 == b0 + 1) {  // neighbouring bits: the next slot
      v1 = (e.x >> b1) & 1ull;
      s1 = s0 + (v0 ? 1 : 0);
    } else {
      s1 = entry_slot(e, b1, d.slot_off, v1);
    }
  } else {
    s1 = entry_slot(dir[w1], b1, d.slot_off, v1);
  }
}

// Corner pair r of the cell (cx, cy, cz, ct) with in-cell fractions (fx, fy,
// fz, ft), paired along axis a (pair_axis): the two slots and validities and
// the product wr of the three other axes' weights (the pair's own weights are
// wr (1 - f_a) and wr f_a, f_a = pair_frac).  Rows layout: the x-pair of row
// (dy, dz, dt) = bits of r, exactly as the vertex rows are visited.
template <bool BRICK>
__device__ __forceinline__ void corner_pair(const LevelDev& d, const ulonglong2* dir, bool active,
                                            int cx, int cy, int cz, int ct, float fx, float fy,
                                            float fz, float ft, int a, int r, int64_t& s0,
                                            int64_t& s1, bool& v0, bool& v1, float& wr) {
  if constexpr (!BRICK) {
    const int dy = r & 1, dz = (r >> 1) & 1, dt = (r >> 2) & 1;
    wr = (dy ? fy : 1.0f - fy) * (dz ? fz : 1.0f - fz) * (dt ? ft : 1.0f - ft);
    row_pair_slots<false>(d, dir, active, ct + dt, cz + dz, cy + dy, cx, s0, s1, v0, v1);
    return;
  }
  int ox, oy, oz, ot;
  pair_offsets(r, a, ox, oy, oz, ot);
  const float gx = a == 0 ? 1.0f : (ox ? fx : 1.0f - fx);
  const float gy = a == 1 ? 1.0f : (oy ? fy : 1.0f - fy);
  const float gz = a == 2 ? 1.0f : (oz ? fz : 1.0f - fz);
  const float gt = a == 3 ? 1.0f : (ot ? ft : 1.0f - ft);
  wr = ((gx * gy) * gz) * gt;
  const int x = cx + ox, y = cy + oy, z = cz + oz, t = ct + ot;
  if (a == 0) {  // x pair (neighbouring rows, or the next brick when x is odd)
    row_pair_slots<true>(d, dir, active, t, z, y, x, s0, s1, v0, v1);
    return;
  }
  // the pair's axis has an even index: both corners in one brick, inner bits
  // 2^a apart, so in one directory word
  const int inner = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((t & 1) << 3);
  const int bit0 = (x >> 1) * 16 + inner;
  const int32_t btz = (t >> 1) * ((d.rz + 1) >> 1) + (z >> 1);
  const ulonglong2 e =
      dir[d.dir_off + (int64_t)((btz * d.wv + (bit0 >> 6)) * d.by + (y >> 1))];
  s0 = entry_slot(e, bit0 & 63, d.slot_off, v0);
  s1 = entry_slot(e, (bit0 & 63) + (1 << a), d.slot_off, v1);
}

__device__ __forceinline__ float pair_frac(int a, float fx, float fy, float fz, float ft) {
  return a == 0 ? fx : a == 1 ? fy : a == 2 ? fz : ft;
}
#endif

}  // namespace fh
