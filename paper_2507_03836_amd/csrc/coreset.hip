// Feature-based coreset selection on the GPU (Sec. 3.1): feature extraction
// into voxel mask bits, feature dilation, per-frame bounding boxes and their
// temporal fusion (the FBB), the Morton-ordered occupancy grid, and the list
// of coreset voxels that the training sampler draws from.
//
// Every kernel works on the mask's 64-voxel words ([T][Sz][Sy][W], W =
// ceil(Sx/64)), so a word is one wave's ballot in the extraction pass and one
// thread's unit of work everywhere else: a dilation or a cell-crossing test
// is a handful of shifts, ANDs and ORs over neighbouring words.
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

constexpr int kBlock = 256;
constexpr int kWordsPerThread = 16;                  // coreset count / emit
constexpr int64_t kChunk = (int64_t)kBlock * kWordsPerThread;

__device__ __forceinline__ uint64_t valid_bits(int64_t Sx, int64_t w) {
  const int64_t left = Sx - 64 * w;  // voxels of this word inside the row
  return left >= 64 ? ~0ull : left <= 0 ? 0ull : ((1ull << left) - 1ull);
}

// Pass 1: one wave per word; lane b decides voxel x = 64 w + b and the wave's
// ballot is the word.  Interval: lo < v <= hi.  Sign (isosurface pass 1):
// v >= lo.  A wave takes kUnroll consecutive words per iteration and issues
// their loads before the ballots, so each wave keeps 1 KiB of reads in flight.
constexpr int kUnroll = 4;
__global__ void __launch_bounds__(kBlock)
    classify_kernel(const float* __restrict__ field, int64_t Sx, int64_t W, int64_t n_words,
                    int kind, float lo, float hi, uint64_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t step = (int64_t)gridDim.x * (kBlock / 64) * kUnroll;
  for (int64_t q0 = (blockIdx.x * (int64_t)(kBlock / 64) + (threadIdx.x >> 6)) * kUnroll;
       q0 < n_words; q0 += step) {
    float v[kUnroll];
    bool in[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t q = q0 + u;
      const int64_t row = q / W, w = q - row * W;
      const int64_t x = 64 * w + lane;
      in[u] = q < n_words && x < Sx;
      v[u] = in[u] ? __builtin_nontemporal_load(field + row * Sx + x) : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool p = in[u] && (kind == FHASH_FEATURE_INTERVAL ? (v[u] > lo && v[u] <= hi)
                                                              : (v[u] >= lo));
      const uint64_t b = __ballot(p);
      if (lane == 0 && q0 + u < n_words) out[q0 + u] = b;
    }
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Bits 0..15 of x moved to bits 0, 4, 8, ..., 60.
__device__ __forceinline__ uint64_t spread4(uint64_t x) {
  x &= 0xFFFFull;
  x = (x | (x << 24)) & 0x000000FF000000FFull;
  x = (x | (x << 12)) & 0x000F000F000F000Full;
  x = (x | (x << 6)) & 0x0303030303030303ull;
  x = (x | (x << 3)) & 0x1111111111111111ull;
  return x;
}

// Pass 1 for rows of a multiple of 4 voxels on a 16-byte aligned field: a wave
// takes a segment of 4 words (256 voxels) of one row, lane l loads voxels
// 4l..4l+3 as one float4, and four ballots (one per component) hold the
// segment's bits; word k of the segment is bits 16k..16k+15 of the four
// ballots interleaved, which lane k assembles and stores.
__global__ void __launch_bounds__(kBlock)
    classify4_kernel(const float* __restrict__ field, int64_t Sx, int64_t W, int64_t n_seg,
                     int kind, float lo, float hi, uint64_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t SW = (W + 3) / 4;
  const int64_t step = (int64_t)gridDim.x * (kBlock / 64) * kUnroll;
  for (int64_t q0 = (blockIdx.x * (int64_t)(kBlock / 64) + (threadIdx.x >> 6)) * kUnroll;
       q0 < n_seg; q0 += step) {
    f32x4 v[kUnroll];
    bool in[kUnroll];
    int64_t row[kUnroll], sw[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t q = q0 + u;
      row[u] = q / SW;
      sw[u] = q - row[u] * SW;
      const int64_t x = 256 * sw[u] + 4 * lane;
      in[u] = q < n_seg && x < Sx;
      v[u] = in[u] ? __builtin_nontemporal_load(
                         reinterpret_cast<const f32x4*>(field + row[u] * Sx + x))
                   : f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const f32x4 a = v[u];
      bool p0, p1, p2, p3;
      if (kind == FHASH_FEATURE_INTERVAL) {
        p0 = a.x > lo && a.x <= hi;
        p1 = a.y > lo && a.y <= hi;
        p2 = a.z > lo && a.z <= hi;
        p3 = a.w > lo && a.w <= hi;
      } else {
        p0 = a.x >= lo;
        p1 = a.y >= lo;
        p2 = a.z >= lo;
        p3 = a.w >= lo;
      }
      const uint64_t b0 = __ballot(in[u] && p0), b1 = __ballot(in[u] && p1);
      const uint64_t b2 = __ballot(in[u] && p2), b3 = __ballot(in[u] && p3);
      const int64_t w = 4 * sw[u] + lane;
      if (lane < 4 && q0 + u < n_seg && w < W) {
        const int sh = 16 * lane;
        out[row[u] * W + w] = spread4(b0 >> sh) | (spread4(b1 >> sh) << 1) |
                              (spread4(b2 >> sh) << 2) | (spread4(b3 >> sh) << 3);
      }
    }
  }
}

// Cells of x-row (z, y) pairs crossed by the isosurface, for the 64 cells
// cx = 64 w .. 64 w + 63 of cell row (cz, cy): some corner at or above the
// level and some below it.  sign = pass-1 bits (padding bits zero).
__device__ __forceinline__ uint64_t crossed_cells(const uint64_t* __restrict__ sign, int64_t Sx,
                                                  int64_t Sy, int64_t W, int64_t frame_row0,
                                                  int64_t cz, int64_t cy, int64_t w) {
  uint64_t all = ~0ull, any = 0;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const uint64_t* r = sign + ((frame_row0 + (cz + dz) * Sy + (cy + dy)) * W);
      const uint64_t s = r[w];
      const uint64_t nx = w + 1 < W ? r[w + 1] : 0ull;
      const uint64_t s1 = (s >> 1) | (nx << 63);  // corner x + 1
      all &= s & s1;
      any |= s | s1;
    }
  // cells exist for cx <= Sx - 2
  return (any & ~all) & valid_bits(Sx - 1, w);
}

// Pass 2 of the isosurface feature: a voxel belongs to the feature iff it is a
// corner of a crossed cell, i.e. cell (x or x-1, y or y-1, z or z-1) is crossed.
// One workgroup per (t, z) slice (blockIdx.x = t Sz + z): the words of a
// slice are indexed in 32 bits (Sy W < 2^31, checked by the host).
__global__ void __launch_bounds__(kBlock)
    iso_kernel(const uint64_t* __restrict__ sign, int64_t Sx, int64_t Sy, int64_t Sz, int64_t W,
               uint64_t* __restrict__ out) {
  const int64_t slice = blockIdx.x;
  const int64_t z = slice % Sz;
  const int64_t frame_row0 = (slice - z) * Sy;
  const uint32_t per_slice = (uint32_t)(Sy * W), Wu = (uint32_t)W;
  for (uint32_t i = threadIdx.x; i < per_slice; i += kBlock) {
    const int64_t y = i / Wu, w = i - (uint32_t)y * Wu;
    const int64_t q = slice * per_slice + i;
    uint64_t f = 0;
    for (int64_t cz = z - 1; cz <= z; ++cz) {
      if (cz < 0 || cz > Sz - 2) continue;
      for (int64_t cy = y - 1; cy <= y; ++cy) {
        if (cy < 0 || cy > Sy - 2) continue;
        const uint64_t c = crossed_cells(sign, Sx, Sy, W, frame_row0, cz, cy, w);
        const uint64_t cp = w > 0 ? crossed_cells(sign, Sx, Sy, W, frame_row0, cz, cy, w - 1) : 0;
        f |= c | (c << 1) | (cp >> 63);
      }
    }
    out[q] = f & valid_bits(Sx, w);
  }
}

// Cube dilation of radius r (0 <= r <= 63) inside each frame: a voxel is set
// iff some set voxel lies within r along each of x, y and z.
// One workgroup per (t, z) slice, as the isosurface pass.
__global__ void __launch_bounds__(kBlock)
    dilate_kernel(const uint64_t* __restrict__ in, int64_t Sx, int64_t Sy, int64_t Sz, int64_t W,
                  int r, uint64_t* __restrict__ out) {
  const int64_t slice = blockIdx.x;
  const int64_t z = slice % Sz;
  const int64_t frame_row0 = (slice - z) * Sy;
  const uint32_t per_slice = (uint32_t)(Sy * W), Wu = (uint32_t)W;
  for (uint32_t i = threadIdx.x; i < per_slice; i += kBlock) {
    const int64_t y = i / Wu, w = i - (uint32_t)y * Wu;
    const int64_t q = slice * per_slice + i;
    uint64_t f = 0;
    const int64_t z0 = z - r < 0 ? 0 : z - r, z1 = z + r > Sz - 1 ? Sz - 1 : z + r;
    const int64_t y0 = y - r < 0 ? 0 : y - r, y1 = y + r > Sy - 1 ? Sy - 1 : y + r;
    for (int64_t c = z0; c <= z1; ++c)
      for (int64_t b = y0; b <= y1; ++b) {
        const uint64_t* rw = in + (frame_row0 + c * Sy + b) * W;
        const uint64_t s = rw[w];
        const uint64_t pv = w > 0 ? rw[w - 1] : 0ull;
        const uint64_t nx = w + 1 < W ? rw[w + 1] : 0ull;
        uint64_t d = s;
        for (int k = 1; k <= r; ++k) {
          d |= (s << k) | (pv >> (64 - k));  // set voxel k to the left
          d |= (s >> k) | (nx << (64 - k));  // set voxel k to the right
        }
        f |= d;
      }
    out[q] = f & valid_bits(Sx, w);
  }
}

// The same dilation, separable inside a workgroup: pass 1 ORs the x-dilated
// rows of the z window into an LDS copy of the slice ((2r+1) x 3 word loads
// per word), pass 2 ORs the y window out of LDS, so a word costs 6r + 3 global
// loads instead of 3 (2r+1)^2.  Used when a slice fits kDilateLdsWords.
constexpr int kDilateLdsWords = 8192;  // 64 KiB of LDS
__global__ void __launch_bounds__(kBlock)
    dilate_lds_kernel(const uint64_t* __restrict__ in, int64_t Sx, int64_t Sy, int64_t Sz,
                      int64_t W, int r, uint64_t* __restrict__ out) {
  extern __shared__ uint64_t zx[];  // [Sy][W]
  const int64_t slice = blockIdx.x;
  const int64_t z = slice % Sz;
  const int64_t frame_row0 = (slice - z) * Sy;
  const uint32_t per_slice = (uint32_t)(Sy * W), Wu = (uint32_t)W;
  const int64_t z0 = z - r < 0 ? 0 : z - r, z1 = z + r > Sz - 1 ? Sz - 1 : z + r;
  for (uint32_t i = threadIdx.x; i < per_slice; i += kBlock) {
    const int64_t y = i / Wu, w = i - (uint32_t)y * Wu;
    uint64_t f = 0;
    for (int64_t c = z0; c <= z1; ++c) {
      const uint64_t* rw = in + (frame_row0 + c * Sy + y) * W;
      const uint64_t s = rw[w];
      const uint64_t pv = w > 0 ? rw[w - 1] : 0ull;
      const uint64_t nx = w + 1 < W ? rw[w + 1] : 0ull;
      uint64_t d = s;
      for (int k = 1; k <= r; ++k) {
        d |= (s << k) | (pv >> (64 - k));
        d |= (s >> k) | (nx << (64 - k));
      }
      f |= d;
    }
    zx[i] = f;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < per_slice; i += kBlock) {
    const int64_t y = i / Wu, w = i - (uint32_t)y * Wu;
    const int64_t y0 = y - r < 0 ? 0 : y - r, y1 = y + r > Sy - 1 ? Sy - 1 : y + r;
    uint64_t f = 0;
    for (int64_t b = y0; b <= y1; ++b) f |= zx[b * W + w];
    out[slice * per_slice + i] = f & valid_bits(Sx, w);
  }
}

__global__ void box_init_kernel(int32_t* box, int64_t rows, int32_t Sx, int32_t Sy, int32_t Sz) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < rows) {
    box[6 * i + 0] = Sx;
    box[6 * i + 1] = Sy;
    box[6 * i + 2] = Sz;
    box[6 * i + 3] = -1;
    box[6 * i + 4] = -1;
    box[6 * i + 5] = -1;
  }
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Per-frame bounding boxes: one workgroup per (t, z) slice reduces its words
// and issues at most 6 atomics, all to frame row t (the fused row T is formed
// afterwards by fuse_boxes_kernel).
__global__ void __launch_bounds__(kBlock)
    box_kernel(const uint64_t* __restrict__ bits, int64_t Sx, int64_t Sy, int64_t Sz, int64_t W,
               int64_t T, int32_t* __restrict__ box) {
  const int64_t slice = blockIdx.x;
  const int64_t z = slice % Sz, t = slice / Sz;
  const uint32_t per_slice = (uint32_t)(Sy * W), Wu = (uint32_t)W;
  const uint64_t* fb = bits + slice * per_slice;
  int mn[3] = {(int)Sx, (int)Sy, (int)Sz}, mx[3] = {-1, -1, -1};
  for (uint32_t i = threadIdx.x; i < per_slice; i += kBlock) {
    const uint32_t y = i / Wu, w = i - y * Wu;
    const uint64_t b = fb[i] & valid_bits(Sx, w);
    if (b == 0) continue;
    const int x0 = (int)(64 * w + __builtin_ctzll(b));
    const int x1 = (int)(64 * w + 63 - __builtin_clzll(b));
    mn[0] = min(mn[0], x0);
    mx[0] = max(mx[0], x1);
    mn[1] = min(mn[1], (int)y);
    mx[1] = max(mx[1], (int)y);
    mn[2] = (int)z;
    mx[2] = (int)z;
  }
  __shared__ int red[kBlock / 64][6];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int a = wave_min(mn[d]), b = wave_max(mx[d]);
    if (lane == 0) {
      red[wid][d] = a;
      red[wid][3 + d] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int d = threadIdx.x;
    int v = red[0][d];
    for (int k = 1; k < kBlock / 64; ++k) v = d < 3 ? min(v, red[k][d]) : max(v, red[k][d]);
    // A plain read first: the stored bound only moves towards the answer, so
    // when it is already at least as tight, the atomic cannot change it.
    int* dst = &box[6 * t + d];
    const int cur = __atomic_load_n(dst, __ATOMIC_RELAXED);
    if (d < 3 ? v < cur : v > cur) {
      if (d < 3)
        atomicMin(dst, v);
      else
        atomicMax(dst, v);
    }
  }
}

// Temporal fusion: row T = the smallest box containing rows 0..T-1 (empty
// rows carry (Sx, Sy, Sz, -1, -1, -1) and so never widen it).
__global__ void __launch_bounds__(64) fuse_boxes_kernel(int32_t* box, int64_t T) {
  const int lane = threadIdx.x;
  int v[6];
  for (int d = 0; d < 6; ++d) v[d] = box[6 * T + d];  // the empty box
  for (int64_t k = lane; k < T; k += 64)
    for (int d = 0; d < 6; ++d) v[d] = d < 3 ? min(v[d], box[6 * k + d]) : max(v[d], box[6 * k + d]);
  for (int d = 0; d < 6; ++d) {
    const int r = d < 3 ? wave_min(v[d]) : wave_max(v[d]);
    if (lane == 0) box[6 * T + d] = r;
  }
}

// Occupancy grid: one word per 4x4x4 brick, bricks row-major (bx fastest),
// voxel (lx, ly, lz) of a brick at bit lx0 | ly0<<1 | lz0<<2 | lx1<<3 | ly1<<4 |
// lz1<<5 (Morton order inside the brick).  Voxels outside the volume are 0.
// One workgroup per (t, bz) slab of bricks (blockIdx.x = t Bz + bz).  A thread
// takes one mask word w of one brick row by: it loads the word from each of
// the brick row's 16 voxel rows (4 z x 4 y) once and writes the 16 bricks
// bx = 16 w .. 16 w + 15 that those words cover.
__global__ void __launch_bounds__(kBlock)
    morton_kernel(const uint64_t* __restrict__ bits, int64_t Sx, int64_t Sy, int64_t Sz, int64_t W,
                  int64_t Bx, int64_t By, int64_t Bz, uint64_t* __restrict__ occ) {
  const int64_t slab = blockIdx.x;
  const int64_t bz = slab % Bz, t = slab / Bz;
  const uint32_t per_slab = (uint32_t)(By * W), Wu = (uint32_t)W;
  for (uint32_t i = threadIdx.x; i < per_slab; i += kBlock) {
    const int64_t by = i / Wu, w = i - (uint32_t)by * Wu;
    const uint64_t valid = valid_bits(Sx, w);
    uint64_t r[4][4];
#pragma unroll
    for (int lz = 0; lz < 4; ++lz)
#pragma unroll
      for (int ly = 0; ly < 4; ++ly) {
        const int64_t z = 4 * bz + lz, y = 4 * by + ly;
        r[lz][ly] = (z < Sz && y < Sy) ? bits[((t * Sz + z) * Sy + y) * W + w] & valid : 0ull;
      }
    uint64_t* dst = occ + (slab * By + by) * Bx;
    for (int j = 0; j < 16; ++j) {
      const int64_t bx = 16 * w + j;
      if (bx >= Bx) break;
      uint64_t o = 0;
#pragma unroll
      for (int lz = 0; lz < 4; ++lz)
#pragma unroll
        for (int ly = 0; ly < 4; ++ly) {
          const uint64_t nib = (r[lz][ly] >> (4 * j)) & 0xFull;  // voxels lx = 0..3
          // lx bit 0 -> Morton bit 0, lx bit 1 -> Morton bit 3
          const uint64_t xs = (nib & 0x3ull) | ((nib & 0xCull) << 6);
          const int base = ((ly & 1) << 1) | ((lz & 1) << 2) | ((ly >> 1) << 4) | ((lz >> 1) << 5);
          o |= xs << base;
        }
      dst[bx] = o;
    }
  }
}

// Coreset, step 1: set voxels per chunk of kChunk words.
__global__ void __launch_bounds__(kBlock)
    chunk_count_kernel(const uint64_t* __restrict__ bits, int64_t Sx, int64_t W, int64_t n_words,
                       int64_t* __restrict__ chunk) {
  const int64_t base = blockIdx.x * kChunk;
  int64_t c = 0;
  for (int k = 0; k < kWordsPerThread; ++k) {
    const int64_t q = base + (int64_t)k * kBlock + threadIdx.x;
    if (q < n_words) c += __popcll(bits[q] & valid_bits(Sx, q % W));
  }
  __shared__ int64_t red[kBlock];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) chunk[blockIdx.x] = red[0];
}

// Step 2: exclusive scan of the chunk counts in one workgroup; chunk[n] = total.
__global__ void __launch_bounds__(1024) chunk_scan_kernel(int64_t* chunk, int64_t n) {
  __shared__ int64_t s[1024];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < n; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < n ? chunk[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan
      const int64_t a = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < n) chunk[i] = carry + s[threadIdx.x] - v;
    const int64_t tot = s[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) chunk[n] = carry;
}

// Step 3: write the linear ids of the set voxels in increasing order.  Each
// wave owns a quarter of its workgroup's chunk; it takes 64 words at a time
// (one per lane), scans their counts across the wave, and then writes the ids
// of one word after another with all 64 lanes, so every store instruction
// writes up to 64 consecutive ids.
__global__ void __launch_bounds__(kBlock)
    chunk_emit_kernel(const uint64_t* __restrict__ bits, int64_t Sx, int64_t W, int64_t n_words,
                      const int64_t* __restrict__ chunk, uint64_t* __restrict__ ids,
                      int64_t id_base) {
  constexpr int kWaves = kBlock / 64;
  constexpr int64_t kPerWave = kChunk / kWaves;  // 1024 words, 16 groups of 64
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t w0 = blockIdx.x * kChunk + wid * kPerWave;
  int c = 0;
  for (int g = 0; g < (int)(kPerWave / 64); ++g) {
    const int64_t q = w0 + g * 64 + lane;
    if (q < n_words) c += __popcll(bits[q] & valid_bits(Sx, q % W));
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  __shared__ int64_t wave_total[kWaves];
  if (lane == 0) wave_total[wid] = c;
  __syncthreads();
  int64_t at = chunk[blockIdx.x];
  for (int k = 0; k < wid; ++k) at += wave_total[k];
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));  // lanes under this one
  for (int g = 0; g < (int)(kPerWave / 64); ++g) {
    const int64_t q = w0 + g * 64 + lane;
    uint64_t b = 0;
    int64_t id0 = 0;
    if (q < n_words) {
      const int64_t row = q / W, w = q - row * W;
      b = bits[q] & valid_bits(Sx, w);
      id0 = id_base + row * Sx + 64 * w;
    }
    const int pc = __popcll(b);
    int incl = pc;  // inclusive scan of the counts over the lanes
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    const int excl = incl - pc;
    uint64_t any = __ballot(b != 0);
    while (any) {
      const int k = __builtin_ctzll(any);
      any &= any - 1;
      const uint64_t bk = __shfl(b, k);
      const int64_t ik = __shfl(id0, k);
      const int ek = __shfl(excl, k);
      if ((bk >> lane) & 1ull) ids[at + ek + __popcll(bk & below)] = (uint64_t)(ik + lane);
    }
    at += __shfl(incl, 63);
  }
}

unsigned grid_for(int64_t items, int64_t per_block) {
  const int64_t g = (items + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : g > 65536 ? 65536 : g);
}

}  // namespace

int64_t mask_words(const int64_t* dims) { return dims[3] * dims[2] * dims[1] * ((dims[0] + 63) / 64); }

size_t feature_ws_bytes(const int64_t* dims, int kind) {
  return kind == FHASH_FEATURE_ISOSURFACE ? (size_t)mask_words(dims) * 8 : 0;
}

// Extraction pass into `out`: the float4 form when every row starts 16-byte aligned.
static void classify(const float* field, const int64_t* dims, int64_t W, int64_t n, int kind, float lo,
              float hi, uint64_t* out, hipStream_t st) {
  if (dims[0] % 4 == 0 && (reinterpret_cast<uintptr_t>(field) & 15u) == 0) {
    const int64_t n_seg = dims[3] * dims[2] * dims[1] * ((W + 3) / 4);
    classify4_kernel<<<grid_for(n_seg, kBlock / 64 * kUnroll), kBlock, 0, st>>>(
        field, dims[0], W, n_seg, kind, lo, hi, out);
  } else {
    classify_kernel<<<grid_for(n, kBlock / 64 * kUnroll), kBlock, 0, st>>>(field, dims[0], W, n,
                                                                            kind, lo, hi, out);
  }
}

hipError_t launch_feature_mask(const float* field, const int64_t* dims, int kind, float lo,
                               float hi, uint64_t* bits, void* ws, hipStream_t st) {
  const int64_t W = (dims[0] + 63) / 64, n = mask_words(dims);
  if (kind == FHASH_FEATURE_INTERVAL) {
    classify(field, dims, W, n, kind, lo, hi, bits, st);
    return hipGetLastError();
  }
  uint64_t* sign = static_cast<uint64_t*>(ws);
  classify(field, dims, W, n, kind, lo, hi, sign, st);
  iso_kernel<<<(unsigned)(dims[3] * dims[2]), kBlock, 0, st>>>(sign, dims[0], dims[1], dims[2], W,
                                                               bits);
  return hipGetLastError();
}

hipError_t launch_dilate_mask(const uint64_t* in, const int64_t* dims, int r, uint64_t* out,
                              hipStream_t st) {
  const int64_t W = (dims[0] + 63) / 64, n = mask_words(dims);
  (void)n;
  if (dims[1] * W <= kDilateLdsWords) {
    dilate_lds_kernel<<<(unsigned)(dims[3] * dims[2]), kBlock, (size_t)(dims[1] * W) * 8, st>>>(
        in, dims[0], dims[1], dims[2], W, r, out);
  } else {
    dilate_kernel<<<(unsigned)(dims[3] * dims[2]), kBlock, 0, st>>>(in, dims[0], dims[1], dims[2],
                                                                    W, r, out);
  }
  return hipGetLastError();
}

hipError_t launch_feature_boxes(const uint64_t* bits, const int64_t* dims, int32_t* box,
                                hipStream_t st) {
  const int64_t W = (dims[0] + 63) / 64, T = dims[3];
  box_init_kernel<<<grid_for(T + 1, kBlock), kBlock, 0, st>>>(box, T + 1, (int32_t)dims[0],
                                                               (int32_t)dims[1], (int32_t)dims[2]);
  box_kernel<<<(unsigned)(T * dims[2]), kBlock, 0, st>>>(bits, dims[0], dims[1], dims[2], W, T, box);
  fuse_boxes_kernel<<<1, 64, 0, st>>>(box, T);
  return hipGetLastError();
}

int64_t occupancy_words(const int64_t* dims) {
  return dims[3] * ((dims[2] + 3) / 4) * ((dims[1] + 3) / 4) * ((dims[0] + 3) / 4);
}

hipError_t launch_occupancy_morton(const uint64_t* bits, const int64_t* dims, uint64_t* occ,
                                   hipStream_t st) {
  const int64_t W = (dims[0] + 63) / 64;
  const int64_t Bx = (dims[0] + 3) / 4, By = (dims[1] + 3) / 4, Bz = (dims[2] + 3) / 4;
  morton_kernel<<<(unsigned)(dims[3] * Bz), kBlock, 0, st>>>(bits, dims[0], dims[1], dims[2], W, Bx,
                                                             By, Bz, occ);
  return hipGetLastError();
}

size_t coreset_ws_bytes(const int64_t* dims) {
  const int64_t chunks = (mask_words(dims) + kChunk - 1) / kChunk;
  return (size_t)(chunks + 1) * sizeof(int64_t);
}

hipError_t launch_coreset(const uint64_t* bits, const int64_t* dims, void* ws, uint64_t* ids,
                          int64_t capacity, int64_t* count, hipStream_t st) {
  const int64_t W = (dims[0] + 63) / 64, n = mask_words(dims);
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  if (chunks > 0x7fffffffLL) return hipErrorInvalidValue;
  int64_t* chunk = static_cast<int64_t*>(ws);
  chunk_count_kernel<<<(unsigned)chunks, kBlock, 0, st>>>(bits, dims[0], W, n, chunk);
  chunk_scan_kernel<<<1, 1024, 0, st>>>(chunk, chunks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(count, chunk + chunks, sizeof(int64_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (ids == nullptr || *count > capacity) return hipSuccess;
  chunk_emit_kernel<<<(unsigned)chunks, kBlock, 0, st>>>(bits, dims[0], W, n, chunk, ids, 0);
  return hipGetLastError();
}

// Coreset of a subset of the frames (key-frame training, Sec. 3.2.2): the
// count / scan / emit passes of launch_coreset run on each listed frame's
// mask words, the ids of a frame offset by its first voxel id and written
// after those of the frames before it.  Frames must be increasing.
size_t coreset_frames_ws_bytes(const int64_t* dims) {
  const int64_t frame_words = dims[2] * dims[1] * ((dims[0] + 63) / 64);
  return (size_t)((frame_words + kChunk - 1) / kChunk + 1) * sizeof(int64_t);
}

hipError_t launch_coreset_frames(const uint64_t* bits, const int64_t* dims, const int32_t* frames,
                                 int32_t n_frames, void* ws, uint64_t* ids, int64_t capacity,
                                 int64_t* count, hipStream_t st) {
  const int64_t W = (dims[0] + 63) / 64, fw = dims[2] * dims[1] * W;
  const int64_t fvox = dims[0] * dims[1] * dims[2];
  const int64_t chunks = (fw + kChunk - 1) / kChunk;
  if (chunks > 0x7fffffffLL) return hipErrorInvalidValue;
  int64_t* chunk = static_cast<int64_t*>(ws);
  int64_t total = 0;
  for (int32_t k = 0; k < n_frames; ++k) {
    const uint64_t* fb = bits + (int64_t)frames[k] * fw;
    chunk_count_kernel<<<(unsigned)chunks, kBlock, 0, st>>>(fb, dims[0], W, fw, chunk);
    chunk_scan_kernel<<<1, 1024, 0, st>>>(chunk, chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t c = 0;
    e = hipMemcpyAsync(&c, chunk + chunks, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (ids != nullptr && total + c <= capacity) {
      chunk_emit_kernel<<<(unsigned)chunks, kBlock, 0, st>>>(fb, dims[0], W, fw, chunk,
                                                             ids + total, frames[k] * fvox);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    total += c;
  }
  *count = total;
  return hipSuccess;
}

}  // namespace fh
