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
// output range, pass 1 writes the model inputs.
template <typename I>
__global__ void __launch_bounds__(256)
    march_kernel(MarchArgs a, Ray* __restrict__ rays, const int32_t* __restrict__ alive,
                 int32_t n_alive, float4* __restrict__ out, int32_t* __restrict__ counter) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = i < n_alive;
  Ray ray;
  int32_t k_end = 0, cnt = 0;
  bool exh = false;
  I w_idx = -1;
  uint64_t w_val = 0;
  if (act) {
    ray = rays[alive[i]];
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
  if (!act) return;
  const int32_t off = base + incl - cnt;
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
  Ray* rp = rays + alive[i];
  rp->k = k_end;
  rp->off = off;
  rp->cnt = cnt | (exh ? kExhausted : 0);
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

__global__ void __launch_bounds__(256)
    composite_kernel(Ray* __restrict__ rays, const int32_t* __restrict__ alive, int32_t n_alive,
                     const float* __restrict__ y, const float4* __restrict__ tf, float alpha_stop,
                     float4* __restrict__ rgba, int32_t* __restrict__ next,
                     int32_t* __restrict__ n_next) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_alive) return;
  const int32_t rid = alive[i];
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
  if (dead) {
    rgba[ray.pixel] = make_float4(cr, cg, cb, A);
  } else {
    const int32_t s = atomicAdd(n_next, 1);
    next[s] = rid;
  }
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
                               const int64_t* dims, float t, void* ws, int32_t* n_alive_host,
                               float* rgba, hipStream_t st) {
  const int64_t NR = (int64_t)W * H;
  RenderWs w = carve(ws, NR);
  int t0 = (int)floorf(t), t1 = (int)ceilf(t);
  t0 = t0 < 0 ? 0 : (t0 > dims[3] - 1 ? (int)dims[3] - 1 : t0);
  t1 = t1 < 0 ? 0 : (t1 > dims[3] - 1 ? (int)dims[3] - 1 : t1);
  hipError_t e = hipMemsetAsync(w.counters, 0, 64, st);
  if (e != hipSuccess) return e;
  const int64_t Wc = (dims[0] - 1 + 63) / 64;
  hipLaunchKernelGGL(occupancy_kernel, dim3(blocks((dims[2] - 1) * (dims[1] - 1) * Wc)), dim3(256),
                     0, st, mask, dims[0], dims[1], dims[2], dims[3], t0, t1, w.occ);
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

}  // namespace fh
