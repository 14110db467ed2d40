// Scattered-access ceiling of the chip, the bound that the gather and the
// scatter-add of the fine levels run against (random rows of tables far larger
// than L2 and the last-level cache): rates of
//   - random 128-byte line reads (8 lanes read 16 B each of one line),
//   - random 16-byte reads (every lane a different line),
//   - random 16-byte atomic groups (4 lanes add one float each into 16
//     consecutive bytes, as 2F lanes scatter one x-pair of a row pair),
// over a 24 GiB buffer, at 64K to 4M threads; then atomics against the bytes
// one instruction puts into a line and the footprint, a read followed by an
// atomic into the same line or another, random byte stores against returning
// atomics (claim flags), and the deferred Adam update's per-segment traffic in
// two state layouts.  Not part of the library.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

// splitmix64 finaliser: the random line of draw (g, k)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void line_read(const float4* __restrict__ buf, uint64_t nlines, int iters,
                          float* __restrict__ sink) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t g = t / 8;
  const int l = (int)(t % 8);
  float acc = 0.f;
  for (int k = 0; k < iters; ++k) {
    const uint64_t line = mix64(g * 131 + k) % nlines;
    const float4 v = buf[line * 8 + l];
    acc += v.x + v.y + v.z + v.w;
  }
  if (acc == 12345.f) sink[0] = acc;  // keeps the loads; never true on a zeroed buffer
}

__global__ void word_read(const float4* __restrict__ buf, uint64_t nlines, int iters,
                          float* __restrict__ sink) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  float acc = 0.f;
  for (int k = 0; k < iters; ++k) {
    const uint64_t r = mix64(t * 131 + k);
    const float4 v = buf[(r % nlines) * 8 + (r >> 60) % 8];
    acc += v.x + v.y + v.z + v.w;
  }
  if (acc == 12345.f) sink[0] = acc;
}

__global__ void group_atomic(float* __restrict__ buf, uint64_t nlines, int iters) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t g = t / 4;
  const int l = (int)(t % 4);
  for (int k = 0; k < iters; ++k) {
    const uint64_t r = mix64(g * 131 + k);
    unsafeAtomicAdd(buf + (r % nlines) * 32 + ((r >> 60) % 8) * 4 + l, 1.0f);
  }
}

// W lanes add one float each into W consecutive floats of one random line
// (W divides 32): how the atomic rate depends on the bytes an instruction puts
// into one line.
__global__ void wide_atomic(float* __restrict__ buf, uint64_t nlines, int iters, int W) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t g = t / W;
  const int l = (int)(t % W);
  for (int k = 0; k < iters; ++k) {
    const uint64_t r = mix64(g * 131 + k);
    unsafeAtomicAdd(buf + (r % nlines) * 32 + ((r >> 59) % (32 / W)) * W + l, 1.0f);
  }
}

// Gather then scatter, as the fused training step does per row: 4 lanes read
// 16 bytes of the first half of a random line, then add (the read value + 1)
// into 16 bytes of the second half of the same line (same = 1) or of another
// random line (same = 0).
__global__ void read_then_atomic(float* __restrict__ buf, uint64_t nlines, int iters, int same) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t g = t / 4;
  const int l = (int)(t % 4);
  for (int k = 0; k < iters; ++k) {
    const uint64_t r = mix64(g * 131 + k);
    const uint64_t a = r % nlines;
    const uint64_t b = same ? a : mix64(r) % nlines;
    const int q = (int)((r >> 60) % 4) * 4;
    const float v = buf[a * 32 + q + l];
    unsafeAtomicAdd(buf + b * 32 + 16 + q + l, v + 1.0f);
  }
}

// Random one-byte stores (the deferred update's claim flags).
__global__ void byte_store(uint8_t* __restrict__ buf, uint64_t n, int iters) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  for (int k = 0; k < iters; ++k) buf[mix64(t * 131 + k) % n] = 1;
}

// Random returning atomic max on the upper half of 8-byte words (a claim by
// stamp).
__global__ void ret_atomic_max(uint32_t* __restrict__ buf, uint64_t nwords, int iters,
                               uint32_t* __restrict__ sink) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (int k = 0; k < iters; ++k)
    acc += atomicMax(buf + 2 * (mix64(t * 131 + k) % nwords) + 1, (uint32_t)k + 1);
  if (acc == 0xdeadbeefu) sink[0] = acc;
}

// A deferred Adam update of random 16-float segments, 4 lanes per segment:
// read p, g, m, v, write p, m, v and a zero g.  LINES == 3: p and g in arrays of
// their own, m and v paired in one line; LINES == 2: p with m in one line, g
// with v in another, the [g | v] array DELTA floats after the end of the
// [p | m] array; LINES == 1: [p | m | g | v], the two lines of a segment
// adjacent.  nseg segments of 256 bytes of state in buf (+ DELTA floats).
template <int LINES, int DELTA = 0>
__global__ void seg_update(float* __restrict__ buf, uint64_t nseg, int iters) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t s0 = t / 4;
  const int sub = (int)(t % 4);
  for (int k = 0; k < iters; ++k) {
    const uint64_t seg = mix64(s0 * 131 + k) % nseg;
    float *pp, *gp, *mp, *vp;
    if (LINES == 3) {
      pp = buf + seg * 16 + 4 * sub;
      gp = buf + nseg * 16 + seg * 16 + 4 * sub;
      mp = buf + nseg * 32 + seg * 32 + 4 * sub;
      vp = mp + 16;
    } else if (LINES == 2) {
      pp = buf + seg * 32 + 4 * sub;
      mp = pp + 16;
      gp = buf + nseg * 32 + DELTA + seg * 32 + 4 * sub;
      vp = gp + 16;
    } else {
      pp = buf + seg * 64 + 4 * sub;
      mp = pp + 16;
      gp = pp + 32;
      vp = pp + 48;
    }
    f4 p = *(f4*)pp, g = *(f4*)gp, m = *(f4*)mp, v = *(f4*)vp;
    m = m * 0.9f + g;
    v = v * 0.999f + g * g;
    p = p - m * 0.001f;
    *(f4*)pp = p;
    *(f4*)gp = (f4){0.f, 0.f, 0.f, 0.f};
    *(f4*)mp = m;
    *(f4*)vp = v;
  }
}

bool ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return false;
}

}  // namespace

int main() {
  const uint64_t bytes = 24ull << 30;
  const uint64_t nlines = bytes / 128;
  float* buf = nullptr;
  float* sink = nullptr;
  const uint64_t slack = 1ull << 20;  // room for the shifted [g | v] array
  if (!ok(hipMalloc(&buf, bytes + slack), "hipMalloc") || !ok(hipMalloc(&sink, 16), "hipMalloc") ||
      !ok(hipMemset(buf, 0, bytes + slack), "hipMemset"))
    return 1;
  hipEvent_t a, b;
  if (!ok(hipEventCreate(&a), "event") || !ok(hipEventCreate(&b), "event")) return 1;
  const int iters = 64;
  for (int kthreads : {64, 256, 1024, 4096}) {
    const uint64_t threads = (uint64_t)kthreads * 1024;
    const unsigned blocks = (unsigned)(threads / 256);
    float ms[3] = {0, 0, 0};
    for (int rep = 0; rep < 2; ++rep) {  // the second repetition is reported
      for (int kind = 0; kind < 3; ++kind) {
        hipEventRecord(a);
        if (kind == 0)
          hipLaunchKernelGGL(line_read, dim3(blocks), dim3(256), 0, 0, (const float4*)buf, nlines,
                             iters, sink);
        else if (kind == 1)
          hipLaunchKernelGGL(word_read, dim3(blocks), dim3(256), 0, 0, (const float4*)buf, nlines,
                             iters, sink);
        else
          hipLaunchKernelGGL(group_atomic, dim3(blocks), dim3(256), 0, 0, buf, nlines, iters);
        hipEventRecord(b);
        if (!ok(hipEventSynchronize(b), "kernel")) return 1;
        hipEventElapsedTime(&ms[kind], a, b);
      }
    }
    const double lines = threads / 8.0 * iters, words = threads * (double)iters,
                 groups = threads / 4.0 * iters;
    std::printf("threads %5dK: 128-B line reads %.2f G/s (%.0f GB/s of lines); 16-B reads "
                "%.2f G/s (%.0f GB/s as 128-B lines); 16-B atomic groups %.2f G/s (%.0f GB/s "
                "as 128-B read + write)\n",
                kthreads, lines / ms[0] / 1e6, lines * 128 / ms[0] / 1e6, words / ms[1] / 1e6,
                words * 128 / ms[1] / 1e6, groups / ms[2] / 1e6, groups * 256 / ms[2] / 1e6);
    std::fflush(stdout);
  }
  // atomic rate against the bytes per line per instruction and the footprint
  // (4 MiB: one XCD's L2; 128 MiB: inside the last-level cache; 24 GiB), and
  // against a read of the same line just before; 4M threads
  {
    const uint64_t threads = 4096ull * 1024;
    const unsigned blocks = (unsigned)(threads / 256);
    for (int W : {1, 4, 16, 32}) {
      for (uint64_t foot : {(uint64_t)4 << 20, (uint64_t)128 << 20, bytes}) {
        const uint64_t nl = foot / 128;
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          hipEventRecord(a);
          hipLaunchKernelGGL(wide_atomic, dim3(blocks), dim3(256), 0, 0, buf, nl, iters, W);
          hipEventRecord(b);
          if (!ok(hipEventSynchronize(b), "kernel")) return 1;
          hipEventElapsedTime(&ms, a, b);
        }
        const double groups = threads / (double)W * iters;
        std::printf("atomics: %2d lanes per line, footprint %8.0f MiB: %.2f G lines/s, "
                    "%.1f G lane-atomics/s\n",
                    W, foot / 1048576.0, groups / ms / 1e6, threads * (double)iters / ms / 1e6);
        std::fflush(stdout);
      }
    }
    for (int same : {0, 1}) {
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(a);
        hipLaunchKernelGGL(read_then_atomic, dim3(blocks), dim3(256), 0, 0, buf, nlines, iters,
                           same);
        hipEventRecord(b);
        if (!ok(hipEventSynchronize(b), "kernel")) return 1;
        hipEventElapsedTime(&ms, a, b);
      }
      const double groups = threads / 4.0 * iters;
      std::printf("16-B read then 16-B atomic group into %s line: %.2f G pairs/s\n",
                  same ? "the same" : "another", groups / ms / 1e6);
      std::fflush(stdout);
    }
    // claim flags: byte stores against returning atomics on state words
    const int it2 = 32;
    for (uint64_t foot : {(uint64_t)64 << 20, (uint64_t)512 << 20, (uint64_t)4 << 30}) {
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(a);
        hipLaunchKernelGGL(byte_store, dim3(blocks), dim3(256), 0, 0,
                           reinterpret_cast<uint8_t*>(buf), foot, it2);
        hipEventRecord(b);
        if (!ok(hipEventSynchronize(b), "kernel")) return 1;
        hipEventElapsedTime(&ms, a, b);
      }
      std::printf("random byte stores over %5.0f MiB: %.2f G/s\n", foot / 1048576.0,
                  threads * (double)it2 / ms / 1e6);
      std::fflush(stdout);
    }
    for (uint64_t foot : {(uint64_t)64 << 20, (uint64_t)4 << 30}) {
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(a);
        hipLaunchKernelGGL(ret_atomic_max, dim3(blocks), dim3(256), 0, 0,
                           reinterpret_cast<uint32_t*>(buf), foot / 8, it2,
                           reinterpret_cast<uint32_t*>(sink));
        hipEventRecord(b);
        if (!ok(hipEventSynchronize(b), "kernel")) return 1;
        hipEventElapsedTime(&ms, a, b);
      }
      std::printf("returning atomic max on 8-byte words over %5.0f MiB: %.2f G/s\n",
                  foot / 1048576.0, threads * (double)it2 / ms / 1e6);
      std::fflush(stdout);
    }
    // the deferred update's segment traffic in two state layouts
    const uint64_t nseg = bytes / 256;
    const char* names[5] = {"p | g | m+v lines", "p+m | g+v lines",
                            "p+m | g+v lines, g+v array 4 KiB further",
                            "p+m | g+v lines, g+v array 96 KiB further",
                            "p+m+g+v, the two lines adjacent"};
    for (int kind = 0; kind < 5; ++kind) {
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        hipEventRecord(a);
        if (kind == 0)
          hipLaunchKernelGGL(seg_update<3>, dim3(blocks), dim3(256), 0, 0, buf, nseg, it2);
        else if (kind == 1)
          hipLaunchKernelGGL(seg_update<2>, dim3(blocks), dim3(256), 0, 0, buf, nseg, it2);
        else if (kind == 2)
          hipLaunchKernelGGL((seg_update<2, 1024>), dim3(blocks), dim3(256), 0, 0, buf, nseg, it2);
        else if (kind == 3)
          hipLaunchKernelGGL((seg_update<2, 24576>), dim3(blocks), dim3(256), 0, 0, buf, nseg,
                             it2);
        else
          hipLaunchKernelGGL(seg_update<1>, dim3(blocks), dim3(256), 0, 0, buf, nseg, it2);
        hipEventRecord(b);
        if (!ok(hipEventSynchronize(b), "kernel")) return 1;
        hipEventElapsedTime(&ms, a, b);
      }
      std::printf("segment update (p, g, m, v read; p, m, v, g written), %s: %.2f G "
                  "segments/s\n",
                  names[kind], threads / 4.0 * it2 / ms / 1e6);
      std::fflush(stdout);
    }
  }
  return 0;
}
