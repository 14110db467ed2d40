// Ray-marching renderer with the adaptive marching pace (Sec. 3.3, Algorithm 1).
//
// Per request: rays are set up once (pinhole camera, slab test against the
// volume box in voxel units) and the occupancy of every voxel cell at the
// render time t is folded into one bit grid (a cell is occupied iff one of its
// 8 corner voxels is in the feature mask at floor(t) or ceil(t)).  Then, while
// rays are alive, every alive ray walks its lattice s_k = s_near + (k+1/2) ds
// and emits up to `pace` occupied samples (pace = clamp(rays / alive, 1, 64)
// as in Algorithm 1); the samples of all rays are decoded in one batch by the
// fused encoding + MLP kernel; each ray composites its samples front to back
// and dies at opacity >= alpha_stop or at the end of its lattice.  The pace
// only changes which samples share a batch: every sample's value is computed
// independently, and each ray composites in lattice order, so the image does
// not depend on the pace.  Ray and sample positions use explicit IEEE FP32
// operations (no contraction) so that they are reproducible bit for bit.
#include "common.h"
#include "kernels.h"

namespace fh {

namespace {

struct alignas(16) Ray {
  float ox, oy, oz, dx;
  float dy, dz, s0, s1;
  float cr, cg, cb, ca;
  int32_t k, pixel, off, cnt;  // cnt: samples of this iteration; bit 30 = lattice exhausted
};
static_assert(sizeof(Ray) == 64, "Ray layout");

constexpr int32_t kExhausted = 1 << 30;

__device__ __forceinline__ float fmul(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ float fadd(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ float fsub(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ float fdiv(float a, float b) { return __fdiv_rn(a, b); }

__global__ void __launch_bounds__(256)
    init_rays_kernel(fhash_view v, int W, int H, float bx, float by, float bz, Ray* __restrict__ rays,
                     int32_t* __restrict__ alive, int32_t* __restrict__ n_alive,
                     float* __restrict__ rgba) {
  const int64_t NR = (int64_t)W * H;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < NR;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int px = (int)(r % W), py = (int)(r / W);
    const float u = fmul(fmul(fsub(fdiv(fmul(2.0f, fadd((float)px, 0.5f)), (float)W), 1.0f),
                              v.tan_half_fovy),
                         v.aspect);
    const float w = fmul(fsub(1.0f, fdiv(fmul(2.0f, fadd((float)py, 0.5f)), (float)H)),
                         v.tan_half_fovy);
    float d[3];
    for (int k = 0; k < 3; ++k) d[k] = fadd(fadd(v.fwd[k], fmul(u, v.right[k])), fmul(w, v.up[k]));
    const float nrm = __fsqrt_rn(fadd(fadd(fmul(d[0], d[0]), fmul(d[1], d[1])), fmul(d[2], d[2])));
    const float dir[3] = {fdiv(d[0], nrm), fdiv(d[1], nrm), fdiv(d[2], nrm)};
    const float org[3] = {v.eye[0], v.eye[1], v.eye[2]};
    const float hi_b[3] = {bx, by, bz};
    float lo = 0.0f, hi = 3.0e38f;
    for (int k = 0; k < 3; ++k) {
      const float a = fdiv(fsub(0.0f, org[k]), dir[k]);
      const float b = fdiv(fsub(hi_b[k], org[k]), dir[k]);
      const float mn = a < b ? a : b, mx = a < b ? b : a;
      if (mn > lo) lo = mn;
      if (mx < hi) hi = mx;
    }
    Ray ray;
    ray.ox = org[0], ray.oy = org[1], ray.oz = org[2];
    ray.dx = dir[0], ray.dy = dir[1], ray.dz = dir[2];
    ray.s0 = lo, ray.s1 = hi;
    ray.cr = ray.cg = ray.cb = ray.ca = 0.0f;
    ray.k = 0;
    ray.pixel = (int32_t)r;
    ray.off = 0;
    ray.cnt = 0;
    rays[r] = ray;
    reinterpret_cast<float4*>(rgba)[r] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lo < hi) {
      const int32_t slot = atomicAdd(n_alive, 1);
      alive[slot] = (int32_t)r;
    }
  }
}

// Occupancy of voxel cells at time t: bit cx of cell row (cz, cy).
__global__ void occupancy_kernel(const uint64_t* __restrict__ mask, int64_t Sx, int64_t Sy,
                                 int64_t Sz, int64_t St, int t0, int t1,
                                 uint64_t* __restrict__ occ) {
  const int64_t Wm = (Sx + 63) / 64, Wc = (Sx - 1 + 63) / 64;
  const int64_t rows = (Sz - 1) * (Sy - 1);
  const int64_t total = rows * Wc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = e % Wc, row = e / Wc;
    const int64_t cy = row % (Sy - 1), cz = row / (Sy - 1);
    uint64_t cur = 0, nxt = 0;
    for (int n = t0; n <= t1; ++n)
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy) {
          const uint64_t* src = mask + (((int64_t)n * Sz + cz + dz) * Sy + cy + dy) * Wm;
          cur |= src[w];
          if (w + 1 < Wm) nxt |= src[w + 1];
        }
    // cell cx occupied iff voxel x = cx or cx + 1 is set in the OR row
    uint64_t bits = cur | (cur >> 1) | (nxt << 63);
    const int64_t valid = (Sx - 1) - w * 64;
    if (valid < 64) bits &= (1ull << valid) - 1ull;
    occ[e] = bits;
  }
}

// The same cell bits from the coreset's occupancy grid (one word per 4x4x4
// brick, bricks [T][Bz][By][Bx], voxel (lx, ly, lz) of a brick at bit
// lx0 | ly0<<1 | lz0<<2 | lx1<<3 | ly1<<4 | lz1<<5): voxel row (z, y) over
// x in [64w, 64w + 68) is gathered from 17 bricks, 4 bits each.
__device__ __forceinline__ uint64_t brick_row_bits(uint64_t b, int ly, int lz) {
  const int base = (ly & 1) << 1 | (lz & 1) << 2 | (ly >> 1) << 4 | (lz >> 1) << 5;
  return ((b >> base) & 3ull) | (((b >> (base + 8)) & 3ull) << 2);
}

__global__ void occupancy_grid_cells_kernel(const uint64_t* __restrict__ grid, int64_t Sx,
                                            int64_t Sy, int64_t Sz, int t0, int t1,
                                            uint64_t* __restrict__ occ) {
  const int64_t Wc = (Sx - 1 + 63) / 64;
  const int64_t Bx = (Sx + 3) / 4, By = (Sy + 3) / 4, Bz = (Sz + 3) / 4;
  const int64_t rows = (Sz - 1) * (Sy - 1);
  const int64_t total = rows * Wc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = e % Wc, row = e / Wc;
    const int64_t cy = row % (Sy - 1), cz = row / (Sy - 1);
    uint64_t cur = 0, nxt = 0;
    // voxel rows y in {cy, cy+1}, z in {cz, cz+1}: one or two brick rows per
    // axis; each brick word is loaded once for the rows it holds
    const int64_t zb0 = cz >> 2, zb1 = (cz + 1) >> 2, yb0 = cy >> 2, yb1 = (cy + 1) >> 2;
    for (int n = t0; n <= t1; ++n)
      for (int64_t zb = zb0; zb <= zb1; ++zb)
        for (int64_t yb = yb0; yb <= yb1; ++yb) {
          const uint64_t* src = grid + ((n * Bz + zb) * By + yb) * Bx;
          for (int b = 0; b <= 16; ++b) {
            const int64_t bx = 16 * w + b;
            if (bx >= Bx) break;
            const uint64_t word = src[bx];
            uint64_t r = 0;
            for (int dz = 0; dz < 2; ++dz)
              for (int dy = 0; dy < 2; ++dy)
                if (((cz + dz) >> 2) == zb && ((cy + dy) >> 2) == yb)
                  r |= brick_row_bits(word, (int)((cy + dy) & 3), (int)((cz + dz) & 3));
            if (b < 16)
              cur |= r << (4 * b);
            else
              nxt |= r;
          }
        }
    uint64_t bits = cur | (cur >> 1) | (nxt << 63);
    const int64_t valid = (Sx - 1) - w * 64;
    if (valid < 64) bits &= (1ull << valid) - 1ull;
    occ[e] = bits;
  }
}

struct MarchArgs {
  const uint64_t* occ;
  int64_t Sx, Sy, Sz;
  int64_t Wc;
  float fx, fy, fz;        // (float)(S - 1)
  float tn;                // t / (T - 1)
  float ds;
  int32_t max_steps;
  int32_t pace;
};

// Cell of a coordinate: floor clamped to [0, S-2].  Sample positions lie in
// the volume box up to rounding, so the conversion stays in range.
template <typename I>
__device__ __forceinline__ I cell_of(float p, int64_t S) {
  I i = (I)floorf(p);
  i = i < 0 ? 0 : i;
  return i > (I)(S - 2) ? (I)(S - 2) : i;
}

// Occupancy bit of the cell holding (px, py, pz).  I: index type of the bit
// grid (32-bit whenever every word index fits, which the host checks).  The
// caller's one-word cache (w_idx, w_val) skips the load while consecutive
// samples stay in the same 64-cell word (w_idx starts at -1).
template <typename I>
__device__ __forceinline__ bool occupied(const MarchArgs& a, float px, float py, float pz,
                                         I& w_idx, uint64_t& w_val) {
  const I cx = cell_of<I>(px, a.Sx), cy = cell_of<I>(py, a.Sy), cz = cell_of<I>(pz, a.Sz);
  const I word = (cz * (I)(a.Sy - 1) + cy) * (I)a.Wc + (cx >> 6);
  if (word != w_idx) {
    w_idx = word;
    w_val = a.occ[word];
  }
  return (w_val >> (cx & 63)) & 1ull;
}

// Walk an alive ray's lattice from its cursor, emitting up to `pace` occupied
// samples: pass 0 counts, a wave-wide reservation gives each ray a contiguous
// output range (offset out_base + the reservation), pass 1 writes the model
// inputs.  Every lane of the wave calls it (act = false for idle lanes).
// Returns the ray's sample count (0 when idle).
template <typename I>
__device__ __forceinline__ int32_t march_one(const MarchArgs& a, Ray* __restrict__ rays,
                                             int32_t rid, bool act, float4* __restrict__ out,
                                             int32_t* __restrict__ counter, int64_t out_base) {
  Ray ray;
  int32_t k_end = 0, cnt = 0;
  bool exh = false;
  I w_idx = -1;
  uint64_t w_val = 0;
  if (act) {
    ray = rays[rid];
    int32_t k = ray.k;
    while (cnt < a.pace) {
      if (k >= a.max_steps) {
        exh = true;
        break;
      }
      const float sk = __fmaf_rn(fadd((float)k, 0.5f), a.ds, ray.s0);
      if (!(sk < ray.s1)) {
        exh = true;
        break;
      }
      const float px = __fmaf_rn(sk, ray.dx, ray.ox);
      const float py = __fmaf_rn(sk, ray.dy, ray.oy);
      const float pz = __fmaf_rn(sk, ray.dz, ray.oz);
      if (occupied<I>(a, px, py, pz, w_idx, w_val)) ++cnt;
      ++k;
    }
    k_end = k;
  }
  // wave-wide exclusive scan of counts and one reservation per wave
  const int lane = threadIdx.x & 63;
  int32_t incl = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int32_t tot = __shfl(incl, 63, 64);
  int32_t base = 0;
  if (lane == 63 && tot > 0) base = atomicAdd(counter, tot);
  base = __shfl(base, 63, 64);
  if (!act) return 0;
  const int64_t off = out_base + base + incl - cnt;
  int32_t k = ray.k, w = 0;
  w_idx = -1;
  while (w < cnt) {
    const float sk = __fmaf_rn(fadd((float)k, 0.5f), a.ds, ray.s0);
    const float px = __fmaf_rn(sk, ray.dx, ray.ox);
    const float py = __fmaf_rn(sk, ray.dy, ray.oy);
    const float pz = __fmaf_rn(sk, ray.dz, ray.oz);
    if (occupied<I>(a, px, py, pz, w_idx, w_val)) {
      out[off + w] = make_float4(fdiv(px, a.fx), fdiv(py, a.fy), fdiv(pz, a.fz), a.tn);
      ++w;
    }
    ++k;
  }
  Ray* rp = rays + rid;
  rp->k = k_end;
  rp->off = (int32_t)off;
  rp->cnt = cnt | (exh ? kExhausted : 0);
  return cnt;
}

template <typename I>
__global__ void __launch_bounds__(256)
    march_kernel(MarchArgs a, Ray* __restrict__ rays, const int32_t* __restrict__ alive,
                 int32_t n_alive, float4* __restrict__ out, int32_t* __restrict__ counter) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = i < n_alive;
  march_one<I>(a, rays, act ? alive[i] : 0, act, out, counter, 0);
}

// Several requests in one launch: request r owns the alive rays
// [first_r, first_r + n_alive_r) of the launch's index space, with first_r a
// multiple of 64 so that every wave serves one request (its arguments are
// then wave-uniform, and so are the addresses of its counter atomics).
constexpr int kBatchMax = FHASH_RENDER_BATCH_MAX;

struct BatchMarchReq {
  Ray* rays;
  const int32_t* alive;
  const uint64_t* occ;
  int32_t first, n_alive, pace, Wc;
  int32_t Sx, Sy, Sz, pad;
  float fx, fy, fz, tn;
};

struct BatchMarchArgs {
  BatchMarchReq q[kBatchMax];
  int32_t n, total, max_steps;
  float ds;
  int64_t out_base;
};

// Request of the wave holding launch index i (wave-uniform, in an SGPR).
template <typename Q>
__device__ __forceinline__ int wave_request(const Q* q, int32_t n, int64_t i) {
  const int64_t w0 = i & ~(int64_t)63;
  int r = 0;
  while (r + 1 < n && w0 >= q[r + 1].first) ++r;
  return __builtin_amdgcn_readfirstlane(r);
}

// counts[0]: sample counter of the launch; counts[1 + r]: samples of request r.
template <typename I>
__global__ void __launch_bounds__(256)
    march_batch_kernel(BatchMarchArgs A, float4* __restrict__ out, int32_t* __restrict__ counts) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int r = wave_request(A.q, A.n, i);
  const BatchMarchReq& q = A.q[r];
  const int64_t j = i - q.first;
  const bool act = j < q.n_alive;
  MarchArgs a;
  a.occ = q.occ;
  a.Sx = q.Sx;
  a.Sy = q.Sy;
  a.Sz = q.Sz;
  a.Wc = q.Wc;
  a.fx = q.fx;
  a.fy = q.fy;
  a.fz = q.fz;
  a.tn = q.tn;
  a.ds = A.ds;
  a.max_steps = A.max_steps;
  a.pace = q.pace;
  int32_t t = march_one<I>(a, q.rays, act ? q.alive[j] : 0, act, out, counts, A.out_base);
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if ((threadIdx.x & 63) == 0 && t > 0) atomicAdd(&counts[1 + r], t);
}

__device__ __forceinline__ float4 tf_lookup(const float4* __restrict__ tf, float v) {
  v = fminf(fmaxf(v, 0.0f), 1.0f);
  const float x = v * 255.0f;
  int i = (int)floorf(x);
  i = i > 254 ? 254 : i;
  const float f = x - (float)i;
  const float4 a = tf[i], b = tf[i + 1];
  return make_float4((1.0f - f) * a.x + f * b.x, (1.0f - f) * a.y + f * b.y,
                     (1.0f - f) * a.z + f * b.z, (1.0f - f) * a.w + f * b.w);
}

// Composite the last march's samples of ray rid; a ray still alive afterwards
// is appended to `next` (one counter atomic per wave).  Every lane of the wave
// calls it (act = false for idle lanes).
__device__ __forceinline__ void composite_one(Ray* __restrict__ rays, int32_t rid, bool act,
                                              const float* __restrict__ y,
                                              const float4* __restrict__ tf, float alpha_stop,
                                              float4* __restrict__ rgba,
                                              int32_t* __restrict__ next,
                                              int32_t* __restrict__ n_next) {
  bool keep = false;
  if (act) {
    Ray ray = rays[rid];
    const int32_t cnt = ray.cnt & (kExhausted - 1);
    bool dead = (ray.cnt & kExhausted) != 0;
    float cr = ray.cr, cg = ray.cg, cb = ray.cb, A = ray.ca;
    for (int32_t j = 0; j < cnt; ++j) {
      const float4 c = tf_lookup(tf, y[ray.off + j]);
      const float t = (1.0f - A) * c.w;
      cr += t * c.x;
      cg += t * c.y;
      cb += t * c.z;
      A += t;
      if (A >= alpha_stop) {
        dead = true;
        break;
      }
    }
    Ray* rp = rays + rid;
    rp->cr = cr, rp->cg = cg, rp->cb = cb, rp->ca = A;
    if (dead)
      rgba[ray.pixel] = make_float4(cr, cg, cb, A);
    keep = !dead;
  }
  const uint64_t m = __ballot(keep);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)m) - 1;
  int32_t base = 0;
  if (lane == leader) base = atomicAdd(n_next, __popcll(m));
  base = __shfl(base, leader, 64);
  if (keep) next[base + __popcll(m & ((1ull << lane) - 1ull))] = rid;
}

__global__ void __launch_bounds__(256)
    composite_kernel(Ray* __restrict__ rays, const int32_t* __restrict__ alive, int32_t n_alive,
                     const float* __restrict__ y, const float4* __restrict__ tf, float alpha_stop,
                     float4* __restrict__ rgba, int32_t* __restrict__ next,
                     int32_t* __restrict__ n_next) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = i < n_alive;
  composite_one(rays, act ? alive[i] : 0, act, y, tf, alpha_stop, rgba, next, n_next);
}

struct BatchCompReq {
  Ray* rays;
  const int32_t* alive;
  int32_t* next;
  const float4* tf;
  float4* rgba;
  int32_t first, n_alive;
};

struct BatchCompArgs {
  BatchCompReq q[kBatchMax];
  int32_t n, total;
  float alpha_stop;
};

// counts[1 + r]: rays of request r still alive (the next list's length).
__global__ void __launch_bounds__(256)
    composite_batch_kernel(BatchCompArgs A, const float* __restrict__ y,
                           int32_t* __restrict__ counts) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int r = wave_request(A.q, A.n, i);
  const BatchCompReq& q = A.q[r];
  const int64_t j = i - q.first;
  const bool act = j < q.n_alive;
  composite_one(q.rays, act ? q.alive[j] : 0, act, y, q.tf, A.alpha_stop, q.rgba, q.next,
                &counts[1 + r]);
}

// One thread per alive ray (the kernels have no grid-stride loop): at most
// 2^30 rays, i.e. 2^22 blocks, well inside the grid limit.
inline unsigned blocks_exact(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : b);
}

inline unsigned blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

// Workspace: rays[NR], alive lists 2 x [NR], counters[4], occupancy bits.
size_t render_ws_bytes(int64_t NR, const int64_t* dims) {
  const int64_t Wc = (dims[0] - 1 + 63) / 64;
  const int64_t occ = (dims[2] - 1) * (dims[1] - 1) * Wc;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return al(NR * sizeof(Ray)) + 2 * al(NR * 4) + al(64) + al(occ * 8);
}

struct RenderWs {
  Ray* rays;
  int32_t* alive[2];
  int32_t* counters;  // [0] n_alive of list 0, [1] of list 1, [2] sample counter
  uint64_t* occ;
};

static RenderWs carve(void* ws, int64_t NR) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* p = static_cast<char*>(ws);
  RenderWs w;
  w.rays = reinterpret_cast<Ray*>(p);
  p += al(NR * sizeof(Ray));
  w.alive[0] = reinterpret_cast<int32_t*>(p);
  p += al(NR * 4);
  w.alive[1] = reinterpret_cast<int32_t*>(p);
  p += al(NR * 4);
  w.counters = reinterpret_cast<int32_t*>(p);
  p += al(64);
  w.occ = reinterpret_cast<uint64_t*>(p);
  return w;
}

hipError_t launch_render_begin(const fhash_view* v, int W, int H, const uint64_t* mask,
                               bool brick_grid, const int64_t* dims, float t, void* ws,
                               int32_t* n_alive_host, float* rgba, hipStream_t st) {
  const int64_t NR = (int64_t)W * H;
  RenderWs w = carve(ws, NR);
  int t0 = (int)floorf(t), t1 = (int)ceilf(t);
  t0 = t0 < 0 ? 0 : (t0 > dims[3] - 1 ? (int)dims[3] - 1 : t0);
  t1 = t1 < 0 ? 0 : (t1 > dims[3] - 1 ? (int)dims[3] - 1 : t1);
  hipError_t e = hipMemsetAsync(w.counters, 0, 64, st);
  if (e != hipSuccess) return e;
  const int64_t Wc = (dims[0] - 1 + 63) / 64;
  if (brick_grid)
    hipLaunchKernelGGL(occupancy_grid_cells_kernel, dim3(blocks((dims[2] - 1) * (dims[1] - 1) * Wc)),
                       dim3(256), 0, st, mask, dims[0], dims[1], dims[2], t0, t1, w.occ);
  else
    hipLaunchKernelGGL(occupancy_kernel, dim3(blocks((dims[2] - 1) * (dims[1] - 1) * Wc)),
                       dim3(256), 0, st, mask, dims[0], dims[1], dims[2], dims[3], t0, t1, w.occ);
  hipLaunchKernelGGL(init_rays_kernel, dim3(blocks(NR)), dim3(256), 0, st, *v, W, H,
                     (float)(dims[0] - 1), (float)(dims[1] - 1), (float)(dims[2] - 1), w.rays,
                     w.alive[0], w.counters, rgba);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(n_alive_host, w.counters, 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t launch_render_march(void* ws, int W, int H, const int64_t* dims, float t01, float ds,
                               int32_t max_steps, int32_t pace, int cur, int32_t n_alive,
                               float* pos_out, int32_t* n_samples_host, hipStream_t st) {
  const int64_t NR = (int64_t)W * H;
  RenderWs w = carve(ws, NR);
  MarchArgs a;
  a.occ = w.occ;
  a.Sx = dims[0];
  a.Sy = dims[1];
  a.Sz = dims[2];
  a.Wc = (dims[0] - 1 + 63) / 64;
  a.fx = (float)(dims[0] - 1);
  a.fy = (float)(dims[1] - 1);
  a.fz = (float)(dims[2] - 1);
  a.tn = t01;
  a.ds = ds;
  a.max_steps = max_steps;
  a.pace = pace;
  hipError_t e = hipMemsetAsync(w.counters + 2, 0, 4, st);
  if (e != hipSuccess) return e;
  if (n_alive > 0) {
    float4* out = reinterpret_cast<float4*>(pos_out);
    if ((dims[2] - 1) * (dims[1] - 1) * a.Wc < ((int64_t)1 << 31))
      hipLaunchKernelGGL(march_kernel<int32_t>, dim3(blocks_exact(n_alive)), dim3(256), 0, st, a,
                         w.rays, w.alive[cur], n_alive, out, w.counters + 2);
    else
      hipLaunchKernelGGL(march_kernel<int64_t>, dim3(blocks_exact(n_alive)), dim3(256), 0, st, a,
                         w.rays, w.alive[cur], n_alive, out, w.counters + 2);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(n_samples_host, w.counters + 2, 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t launch_render_composite(void* ws, int W, int H, int cur, int32_t n_alive,
                                   const float* y, const float* tf, float alpha_stop, float* rgba,
                                   int32_t* n_alive_host, hipStream_t st) {
  const int64_t NR = (int64_t)W * H;
  RenderWs w = carve(ws, NR);
  const int nxt = 1 - cur;
  hipError_t e = hipMemsetAsync(w.counters + nxt, 0, 4, st);
  if (e != hipSuccess) return e;
  if (n_alive > 0)
    hipLaunchKernelGGL(composite_kernel, dim3(blocks_exact(n_alive)), dim3(256), 0, st, w.rays,
                       w.alive[cur], n_alive, y, reinterpret_cast<const float4*>(tf), alpha_stop,
                       reinterpret_cast<float4*>(rgba), w.alive[nxt], w.counters + nxt);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(n_alive_host, w.counters + nxt, 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t launch_render_march_batch(const RenderBatch* b, int32_t n, float ds, int32_t max_steps,
                                     float* pos, int64_t out_base, int32_t* counts_dev,
                                     int32_t* counts_host, hipStream_t st) {
  BatchMarchArgs A{};
  A.n = n;
  A.ds = ds;
  A.max_steps = max_steps;
  A.out_base = out_base;
  int32_t total = 0;
  bool wide = false;
  for (int32_t r = 0; r < n; ++r) {
    const int64_t* dims = b[r].dims;
    const int64_t NR = (int64_t)b[r].W * b[r].H;
    RenderWs w = carve(b[r].ws, NR);
    BatchMarchReq& q = A.q[r];
    q.rays = w.rays;
    q.alive = w.alive[b[r].cur];
    q.occ = w.occ;
    q.first = total;
    q.n_alive = b[r].n_alive;
    q.pace = b[r].pace;
    q.Wc = (int32_t)((dims[0] - 1 + 63) / 64);
    q.Sx = (int32_t)dims[0];
    q.Sy = (int32_t)dims[1];
    q.Sz = (int32_t)dims[2];
    q.fx = (float)(dims[0] - 1);
    q.fy = (float)(dims[1] - 1);
    q.fz = (float)(dims[2] - 1);
    q.tn = b[r].t01;
    total += (b[r].n_alive + 63) & ~63;
    if ((dims[2] - 1) * (dims[1] - 1) * (int64_t)q.Wc >= ((int64_t)1 << 31)) wide = true;
  }
  A.total = total;
  hipError_t e = hipMemsetAsync(counts_dev, 0, (size_t)(1 + n) * 4, st);
  if (e != hipSuccess) return e;
  if (total > 0) {
    float4* out = reinterpret_cast<float4*>(pos);
    if (wide)
      hipLaunchKernelGGL(march_batch_kernel<int64_t>, dim3(blocks_exact(total)), dim3(256), 0, st,
                         A, out, counts_dev);
    else
      hipLaunchKernelGGL(march_batch_kernel<int32_t>, dim3(blocks_exact(total)), dim3(256), 0, st,
                         A, out, counts_dev);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(counts_host, counts_dev, (size_t)(1 + n) * 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t launch_render_composite_batch(const RenderBatch* b, int32_t n, const float* y,
                                         float alpha_stop, int32_t* counts_dev,
                                         int32_t* counts_host, hipStream_t st) {
  BatchCompArgs A{};
  A.n = n;
  A.alpha_stop = alpha_stop;
  int32_t total = 0;
  for (int32_t r = 0; r < n; ++r) {
    const int64_t NR = (int64_t)b[r].W * b[r].H;
    RenderWs w = carve(b[r].ws, NR);
    BatchCompReq& q = A.q[r];
    q.rays = w.rays;
    q.alive = w.alive[b[r].cur];
    q.next = w.alive[1 - b[r].cur];
    q.tf = reinterpret_cast<const float4*>(b[r].tf);
    q.rgba = reinterpret_cast<float4*>(b[r].rgba);
    q.first = total;
    q.n_alive = b[r].n_alive;
    total += (b[r].n_alive + 63) & ~63;
  }
  A.total = total;
  hipError_t e = hipMemsetAsync(counts_dev, 0, (size_t)(1 + n) * 4, st);
  if (e != hipSuccess) return e;
  if (total > 0)
    hipLaunchKernelGGL(composite_batch_kernel, dim3(blocks_exact(total)), dim3(256), 0, st, A, y,
                       counts_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(counts_host, counts_dev, (size_t)(1 + n) * 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace fh
