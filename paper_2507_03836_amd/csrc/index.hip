// Index build: voxel feature mask -> per-level active cells -> active vertices ->
// rank directory (the collision-free per-level hash, Sec. 3.2.3 / Sec. 3.1).
//
// A level's active cells are found with separable OR-reductions of the bit mask
// along t, z, y (whole 64-bit words) and a final bit-range test along x; the
// active vertices are the separable 1-step dilation of the active cells along
// t, z, y, x.  The directory stores, for every 64-vertex word of a row-padded
// vertex bitmap, the bits and the number of active vertices before the word
// (exclusive prefix sum of popcounts in F-Hash linearisation order).  Row
// padding bits are zero, so ranks equal ranks in the unpadded order.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

__device__ __forceinline__ void voxel_range(int64_t c, int64_t S, int64_t R, int64_t& lo,
                                            int64_t& hi) {
  // Voxels i with c <= i(R-1)/(S-1) <= c+1 (closed cell box).
  const int64_t d = S - 1, r = R - 1;
  lo = (c * d + r - 1) / r;
  hi = ((c + 1) * d) / r;
  if (hi > S - 1) hi = S - 1;
}

// out[o][c][q] = OR over voxels s of cell c of in[o][s][q].
__global__ void or_reduce_axis_kernel(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                      int64_t outer, int64_t S, int64_t C, int64_t inner,
                                      int64_t R) {
  const int64_t total = outer * C * inner;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e % inner;
    const int64_t c = (e / inner) % C;
    const int64_t o = e / (inner * C);
    int64_t lo, hi;
    voxel_range(c, S, R, lo, hi);
    uint64_t acc = 0;
    const uint64_t* src = in + (o * S) * inner + q;
    for (int64_t s = lo; s <= hi; ++s) acc |= src[s * inner];
    out[e] = acc;
  }
}

// Cell bits along x: bit cx of row r = any voxel bit in the x-range of cell cx.
__global__ void cells_x_kernel(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                               int64_t rows, int64_t Wm, int64_t Wc, int64_t Sx, int64_t Rx) {
  const int64_t total = rows * Wc;
  const int64_t Cx = Rx - 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = e % Wc, r = e / Wc;
    const uint64_t* row = in + r * Wm;
    uint64_t bits = 0;
    for (int b = 0; b < 64; ++b) {
      const int64_t cx = w * 64 + b;
      if (cx >= Cx) break;
      int64_t lo, hi;
      voxel_range(cx, Sx, Rx, lo, hi);
      bool any = false;
      for (int64_t wi = lo >> 6; wi <= (hi >> 6) && !any; ++wi) {
        uint64_t m = row[wi];
        const int64_t b0 = wi * 64;
        if (lo > b0) m &= ~0ull << (lo - b0);
        if (hi < b0 + 63) m &= (1ull << (hi - b0 + 1)) - 1ull;
        any = m != 0;
      }
      if (any) bits |= 1ull << b;
    }
    out[e] = bits;
  }
}

// Vertex dilation along one axis: out[o][v][q] = in[o][v-1][q] | in[o][v][q],
// where in has C = R-1 cells along the axis and out has R vertices.
__global__ void dilate_axis_kernel(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                   int64_t outer, int64_t C, int64_t inner) {
  const int64_t R = C + 1;
  const int64_t total = outer * R * inner;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e % inner;
    const int64_t v = (e / inner) % R;
    const int64_t o = e / (inner * R);
    const uint64_t* src = in + o * C * inner + q;
    uint64_t acc = 0;
    if (v < C) acc |= src[v * inner];
    if (v > 0) acc |= src[(v - 1) * inner];
    out[e] = acc;
  }
}

// Vertex bits along x (vertex x active iff cell x or cell x-1 active), written
// into the directory's bit words.
__global__ void vert_x_kernel(const uint64_t* __restrict__ in, ulonglong2* __restrict__ dir,
                              int64_t rows, int64_t Wc, int64_t Wv) {
  const int64_t total = rows * Wv;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = e % Wv, r = e / Wv;
    const uint64_t* row = in + r * Wc;
    const uint64_t cur = (w < Wc) ? row[w] : 0ull;
    const uint64_t prev = (w > 0 && w - 1 < Wc) ? row[w - 1] : 0ull;
    ulonglong2 ent;
    ent.x = cur | (cur << 1) | (prev >> 63);
    ent.y = 0;
    dir[e] = ent;
  }
}

// Store order of the directory: the entries of one x word for all y of a
// (t, z) row block are adjacent, index ((t*Rz + z)*Wv + w)*Ry + y, so the
// y and y+1 rows of a cell read neighbouring 16-byte entries (one line).
// Ranks are computed in F-Hash order first (row-major, src) and then moved.
__global__ void dir_interleave_kernel(const ulonglong2* __restrict__ src,
                                      ulonglong2* __restrict__ dst, int64_t rows, int64_t ry,
                                      int64_t wv) {
  const int64_t total = rows * wv;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = e % wv, row = e / wv;
    const int64_t tz = row / ry, y = row % ry;
    dst[(tz * wv + w) * ry + y] = src[e];
  }
}

// Brick order (layout FHASH_LAYOUT_BRICKS): word w of brick row (bt, bz, by)
// holds bricks bx = 4w .. 4w+3, brick q at bits 16q .. 16q+15, vertex inner
// index (x%2) | (y%2)<<1 | (z%2)<<2 | (t%2)<<3.  Built from the row-major
// vertex bits (rows (t, z, y) of wv words): the 8 x bits 8w .. 8w+7 of each of
// the brick row's 8 vertex rows lie in one row word.  Output in brick-linear
// order (((bt*Bz + bz)*By + by)*Wb + w), ranks still to be written.
__global__ void brickify_kernel(const ulonglong2* __restrict__ rows, ulonglong2* __restrict__ out,
                                int64_t rx, int64_t ry, int64_t rz, int64_t rt, int64_t wv,
                                int64_t wb, int64_t by_n, int64_t bz_n, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = e % wb, row = e / wb;
    const int64_t by = row % by_n, bz = (row / by_n) % bz_n, bt = row / (by_n * bz_n);
    uint64_t bits = 0;
    for (int c = 0; c < 8; ++c) {  // (y%2, z%2, t%2) of the vertex row
      const int64_t y = 2 * by + (c & 1), z = 2 * bz + ((c >> 1) & 1), t = 2 * bt + (c >> 2);
      if (y >= ry || z >= rz || t >= rt) continue;
      const int64_t x0 = 8 * w;  // x bits 8w .. 8w+7 (x >= rx reads the row's zero padding)
      if (x0 >= rx) continue;
      const uint64_t xb = (rows[((t * rz + z) * ry + y) * wv + (x0 >> 6)].x >> (x0 & 63)) & 0xFFull;
      for (int q = 0; q < 4; ++q)
        for (int ix = 0; ix < 2; ++ix)
          if ((xb >> (2 * q + ix)) & 1ull) bits |= 1ull << (16 * q + (ix | (c << 1)));
    }
    ulonglong2 ent;
    ent.x = bits;
    ent.y = 0;
    out[e] = ent;
  }
}

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 8;
constexpr int64_t kScanBlockWords = kScanThreads * kScanPerThread;

__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* sh,
                                                         uint64_t& total) {
  // Inclusive scan inside each wave, then across waves (<= 16 waves).
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) {
      uint64_t t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[16] = run;
  }
  __syncthreads();
  total = sh[16];
  const uint64_t res = sh[wid] + x - v;
  __syncthreads();
  return res;
}

__global__ void __launch_bounds__(kScanThreads)
    popc_block_sums_kernel(const ulonglong2* __restrict__ dir, int64_t words,
                           uint64_t* __restrict__ partial) {
  __shared__ uint64_t sh[17];
  const int64_t base = blockIdx.x * kScanBlockWords + threadIdx.x * (int64_t)kScanPerThread;
  uint64_t s = 0;
  for (int i = 0; i < kScanPerThread; ++i)
    if (base + i < words) s += __popcll(dir[base + i].x);
  uint64_t total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of the block partials in one workgroup; *count = total.
__global__ void __launch_bounds__(1024)
    scan_partials_kernel(uint64_t* __restrict__ partial, int64_t nb, uint64_t* __restrict__ count) {
  __shared__ uint64_t sh[17];
  const int64_t per = (nb + blockDim.x - 1) / blockDim.x;
  const int64_t b0 = threadIdx.x * per;
  uint64_t s = 0;
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) s += partial[b0 + i];
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, sh, total);
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) {
      uint64_t t = partial[b0 + i];
      partial[b0 + i] = run;
      run += t;
    }
  if (threadIdx.x == 0) *count = total;
}

__global__ void __launch_bounds__(kScanThreads)
    write_ranks_kernel(ulonglong2* __restrict__ dir, int64_t words,
                       const uint64_t* __restrict__ partial) {
  __shared__ uint64_t sh[17];
  const int64_t base = blockIdx.x * kScanBlockWords + threadIdx.x * (int64_t)kScanPerThread;
  uint64_t pc[kScanPerThread];
  uint64_t s = 0;
  for (int i = 0; i < kScanPerThread; ++i) {
    pc[i] = (base + i < words) ? (uint64_t)__popcll(dir[base + i].x) : 0ull;
    s += pc[i];
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, sh, total) + partial[blockIdx.x];
  for (int i = 0; i < kScanPerThread; ++i)
    if (base + i < words) {
      dir[base + i].y = run;
      run += pc[i];
    }
}

inline int grid_for(int64_t total, int threads) {
  int64_t b = (total + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

struct LevelSizes {
  int64_t Ct, Cz, Cy, Cx, Wm, Wc, Wv;
  int64_t A, B, Cb, cell, D1, D2, D3, words, nb;
  int64_t Bx, By, Bz, Bt, Wb, bwords, bnb;  // brick layout
};

LevelSizes level_sizes(const int32_t* r, const int64_t* dims) {
  LevelSizes s;
  const int64_t Sx = dims[0], Sy = dims[1], Sz = dims[2];
  s.Cx = r[0] - 1;
  s.Cy = r[1] - 1;
  s.Cz = r[2] - 1;
  s.Ct = r[3] - 1;
  s.Wm = (Sx + 63) / 64;
  s.Wc = (s.Cx + 63) / 64;
  s.Wv = ((int64_t)r[0] + 63) / 64;
  s.A = s.Ct * Sz * Sy * s.Wm;
  s.B = s.Ct * s.Cz * Sy * s.Wm;
  s.Cb = s.Ct * s.Cz * s.Cy * s.Wm;
  s.cell = s.Ct * s.Cz * s.Cy * s.Wc;
  s.D1 = (int64_t)r[3] * s.Cz * s.Cy * s.Wc;
  s.D2 = (int64_t)r[3] * r[2] * s.Cy * s.Wc;
  s.D3 = (int64_t)r[3] * r[2] * r[1] * s.Wc;
  s.words = (int64_t)r[3] * r[2] * r[1] * s.Wv;
  s.nb = (s.words + kScanBlockWords - 1) / kScanBlockWords;
  s.Bx = ((int64_t)r[0] + 1) / 2;
  s.By = ((int64_t)r[1] + 1) / 2;
  s.Bz = ((int64_t)r[2] + 1) / 2;
  s.Bt = ((int64_t)r[3] + 1) / 2;
  s.Wb = (s.Bx + 3) / 4;
  s.bwords = s.Bt * s.Bz * s.By * s.Wb;
  s.bnb = (s.bwords + kScanBlockWords - 1) / kScanBlockWords;
  return s;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int64_t index_dir_words(const fhash_grid_desc* g, int l) {
  const int32_t* r = g->res[l];
  if (g->layout == FHASH_LAYOUT_BRICKS)
    return (((int64_t)r[3] + 1) / 2) * (((int64_t)r[2] + 1) / 2) * (((int64_t)r[1] + 1) / 2) *
           ((((int64_t)r[0] + 1) / 2 + 3) / 4);
  return (int64_t)r[3] * r[2] * r[1] * (((int64_t)r[0] + 63) / 64);
}

size_t index_workspace_bytes(const fhash_grid_desc* g, const int64_t* dims) {
  int64_t b0 = 1, b1 = 1, nb = 1;
  for (int l = 0; l < g->n_levels; ++l) {
    LevelSizes s = level_sizes(g->res[l], dims);
    b0 = std::max(b0, std::max(std::max(s.A, s.Cb), std::max(s.D1, s.D3)));
    b1 = std::max(b1, std::max(std::max(s.B, s.cell), s.D2));
    nb = std::max(nb, s.nb);
  }
  int64_t words = 1, bwords = 1;
  for (int l = 0; l < g->n_levels; ++l) {
    LevelSizes ls = level_sizes(g->res[l], dims);
    words = std::max(words, ls.words);
    bwords = std::max(bwords, ls.bwords);
    nb = std::max(nb, ls.bnb);
  }
  const bool bricks = g->layout == FHASH_LAYOUT_BRICKS;
  return align256(b0 * 8) + align256(b1 * 8) + align256(nb * 8) + align256(8 * FHASH_MAX_LEVELS) +
         align256(words * 16) + (bricks ? align256(bwords * 16) : 0);
}

hipError_t launch_build_index(const fhash_grid_desc* g, const uint64_t* mask,
                              const int64_t* dims, ulonglong2* dir, const int64_t* dir_off,
                              void* ws, uint64_t* counts_host, hipStream_t st) {
  const bool bricks = g->layout == FHASH_LAYOUT_BRICKS;
  int64_t b0 = 1, b1 = 1, nbmax = 1, wmax = 1;
  for (int l = 0; l < g->n_levels; ++l) {
    LevelSizes s = level_sizes(g->res[l], dims);
    b0 = std::max(b0, std::max(std::max(s.A, s.Cb), std::max(s.D1, s.D3)));
    b1 = std::max(b1, std::max(std::max(s.B, s.cell), s.D2));
    nbmax = std::max(nbmax, std::max(s.nb, s.bnb));
    wmax = std::max(wmax, s.words);
  }
  char* p = static_cast<char*>(ws);
  uint64_t* buf0 = reinterpret_cast<uint64_t*>(p);
  p += align256(b0 * 8);
  uint64_t* buf1 = reinterpret_cast<uint64_t*>(p);
  p += align256(b1 * 8);
  uint64_t* partial = reinterpret_cast<uint64_t*>(p);
  p += align256(nbmax * 8);
  uint64_t* counts = reinterpret_cast<uint64_t*>(p);
  p += align256(8 * FHASH_MAX_LEVELS);
  ulonglong2* rowmajor = reinterpret_cast<ulonglong2*>(p);  // one level's directory, F-Hash order
  p += align256(wmax * 16);
  ulonglong2* bricked = reinterpret_cast<ulonglong2*>(p);   // brick-linear order (bricks only)

  const int T = 256;
  const int64_t Sx = dims[0], Sy = dims[1], Sz = dims[2], St = dims[3];
  for (int l = 0; l < g->n_levels; ++l) {
    const int32_t* r = g->res[l];
    LevelSizes s = level_sizes(r, dims);
    // Active cells: reduce t, z, y over whole words, then x over bit ranges.
    hipLaunchKernelGGL(or_reduce_axis_kernel, dim3(grid_for(s.A, T)), dim3(T), 0, st, mask, buf0,
                       (int64_t)1, St, s.Ct, Sz * Sy * s.Wm, (int64_t)r[3]);
    hipLaunchKernelGGL(or_reduce_axis_kernel, dim3(grid_for(s.B, T)), dim3(T), 0, st, buf0, buf1,
                       s.Ct, Sz, s.Cz, Sy * s.Wm, (int64_t)r[2]);
    hipLaunchKernelGGL(or_reduce_axis_kernel, dim3(grid_for(s.Cb, T)), dim3(T), 0, st, buf1, buf0,
                       s.Ct * s.Cz, Sy, s.Cy, s.Wm, (int64_t)r[1]);
    hipLaunchKernelGGL(cells_x_kernel, dim3(grid_for(s.cell, T)), dim3(T), 0, st, buf0, buf1,
                       s.Ct * s.Cz * s.Cy, s.Wm, s.Wc, Sx, (int64_t)r[0]);
    // Active vertices: corners of active cells (dilate by one step per axis).
    hipLaunchKernelGGL(dilate_axis_kernel, dim3(grid_for(s.D1, T)), dim3(T), 0, st, buf1, buf0,
                       (int64_t)1, s.Ct, s.Cz * s.Cy * s.Wc);
    hipLaunchKernelGGL(dilate_axis_kernel, dim3(grid_for(s.D2, T)), dim3(T), 0, st, buf0, buf1,
                       (int64_t)r[3], s.Cz, s.Cy * s.Wc);
    hipLaunchKernelGGL(dilate_axis_kernel, dim3(grid_for(s.D3, T)), dim3(T), 0, st, buf1, buf0,
                       (int64_t)r[3] * r[2], s.Cy, s.Wc);
    ulonglong2* d = rowmajor;
    hipLaunchKernelGGL(vert_x_kernel, dim3(grid_for(s.words, T)), dim3(T), 0, st, buf0, d,
                       (int64_t)r[3] * r[2] * r[1], s.Wc, s.Wv);
    // Order of the ranks: F-Hash rows, or bricks (then the words are regrouped first).
    int64_t words = s.words, nb = s.nb, nrows = (int64_t)r[3] * r[2] * r[1], ry = r[1],
            wv = s.Wv;
    if (bricks) {
      hipLaunchKernelGGL(brickify_kernel, dim3(grid_for(s.bwords, T)), dim3(T), 0, st, rowmajor,
                         bricked, (int64_t)r[0], (int64_t)r[1], (int64_t)r[2], (int64_t)r[3],
                         s.Wv, s.Wb, s.By, s.Bz, s.bwords);
      d = bricked;
      words = s.bwords;
      nb = s.bnb;
      nrows = s.Bt * s.Bz * s.By;
      ry = s.By;
      wv = s.Wb;
    }
    // Ranks: exclusive prefix sum of popcounts.
    hipLaunchKernelGGL(popc_block_sums_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st,
                       d, words, partial);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, st, partial, nb,
                       counts + l);
    hipLaunchKernelGGL(write_ranks_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, d,
                       words, partial);
    hipLaunchKernelGGL(dir_interleave_kernel, dim3(grid_for(words, T)), dim3(T), 0, st, d,
                       dir + dir_off[l], nrows, ry, wv);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(counts_host, counts, sizeof(uint64_t) * g->n_levels, hipMemcpyDeviceToHost,
                     st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace fh
