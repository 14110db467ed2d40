// Standalone decoder kernels (FP32 MFMA): forward, and backward with per-wave
// gradient partials reduced deterministically by a second kernel.
#include "kernels.h"
#include "mlp_dev.h"

namespace fh {

namespace {

constexpr int kWaves = 4;  // waves per workgroup

template <int INP>
__device__ __forceinline__ void load_input_b(const float* __restrict__ x, int64_t smp, bool valid,
                                             int in_w, float (&xb)[INP / 16][4]) {
  const int lane = threadIdx.x & 63, g = lane >> 4;
#pragma unroll
  for (int a = 0; a < INP / 16; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = 16 * a + 4 * g + i;
      xb[a][i] = (valid && c < in_w) ? x[smp * in_w + c] : 0.0f;
    }
}

template <int INP, int H, int NH>
__global__ void __launch_bounds__(64 * kWaves)
    mlp_fwd_kernel(const float* __restrict__ params, const float* __restrict__ x, int64_t n,
                   int in_w, float* __restrict__ y) {
  using S = MlpShape<INP, H, NH>;
  __shared__ __attribute__((aligned(16))) float lds[S::WFLOATS];
  load_weights_lds<INP, H, NH>(lds, params, in_w);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, s = lane & 15;
  const int64_t nblk = (n + 15) / 16;
  const int64_t nwav = (int64_t)gridDim.x * kWaves;
  for (int64_t b = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); b < nblk; b += nwav) {
    const int64_t smp = b * 16 + s;
    const bool valid = smp < n;
    float xb[S::INB][4];
    load_input_b<INP>(x, smp, valid, in_w, xb);
    float hs[NH][S::HB][4];
    const float yv = mlp_block_fwd<INP, H, NH>(lds, xb, hs);
    if (g == 0 && valid) y[smp] = yv;
  }
}

template <int INP, int H, int NH>
__global__ void __launch_bounds__(64 * kWaves)
    mlp_bwd_kernel(const float* __restrict__ params, const float* __restrict__ x,
                   const float* __restrict__ dy, int64_t n, int in_w, float* __restrict__ dx,
                   float* __restrict__ part, int64_t P) {
  using S = MlpShape<INP, H, NH>;
  constexpr int WS = mlp_wave_scratch<INP, H, NH>();
  __shared__ __attribute__((aligned(16))) float lds[S::WFLOATS + kWaves * WS];
  load_weights_lds<INP, H, NH>(lds, params, in_w);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, s = lane & 15;
  const int wib = threadIdx.x >> 6;
  float* scratch = lds + S::WFLOATS + wib * WS;
  const int64_t nblk = (n + 15) / 16;
  const int64_t nwav = (int64_t)gridDim.x * kWaves;
  const int64_t wave = (int64_t)blockIdx.x * kWaves + wib;
  MlpGrad<INP, H, NH> gr;
  gr.zero();
  for (int64_t b = wave; b < nblk; b += nwav) {
    const int64_t smp = b * 16 + s;
    const bool valid = smp < n;
    float xb[S::INB][4];
    load_input_b<INP>(x, smp, valid, in_w, xb);
    mlp_stage_input<INP, H, NH>(scratch, xb);
    float hs[NH][S::HB][4];
    mlp_block_fwd<INP, H, NH>(lds, xb, hs);
    const float dyv = valid ? dy[smp] : 0.0f;
    float dxb[S::INB][4];
    mlp_block_bwd<INP, H, NH>(lds, scratch, hs, dyv, gr, dxb);
    if (dx != nullptr && valid) {
#pragma unroll
      for (int a = 0; a < S::INB; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * a + 4 * g + i;
          if (c < in_w) dx[smp * in_w + c] = dxb[a][i];
        }
    }
  }
  mlp_write_partial<INP, H, NH>(gr, in_w, part + wave * P);
}

inline int64_t bwd_waves(int64_t n) {
  int64_t nblk = (n + 15) / 16;
  int64_t w = nblk < 1024 ? nblk : 1024;
  w = ((w + kWaves - 1) / kWaves) * kWaves;
  return w < kWaves ? kWaves : w;
}

template <int INP, int H, int NH>
hipError_t fwd_t(const float* params, const float* x, int64_t n, int in_w, float* y,
                 hipStream_t st) {
  int64_t nblk = (n + 15) / 16;
  int64_t wg = (nblk + kWaves - 1) / kWaves;
  if (wg > 2048) wg = 2048;
  hipLaunchKernelGGL((mlp_fwd_kernel<INP, H, NH>), dim3((unsigned)wg), dim3(64 * kWaves), 0, st,
                     params, x, n, in_w, y);
  return hipGetLastError();
}

template <int INP, int H, int NH>
hipError_t bwd_t(const float* params, const float* x, const float* dy, int64_t n, int in_w,
                 float* d_params, float* dx, float* part, int64_t P, hipStream_t st) {
  const int64_t nw = bwd_waves(n);
  hipLaunchKernelGGL((mlp_bwd_kernel<INP, H, NH>), dim3((unsigned)(nw / kWaves)),
                     dim3(64 * kWaves), 0, st, params, x, dy, n, in_w, dx, part, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(part, nw, P, d_params, st);
}

}  // namespace

bool mlp_supported(int in_w, int H, int NH) {
  return in_w >= 1 && in_w <= 64 && (H == 32 || H == 64) && NH >= 1 && NH <= 3;
}

size_t mlp_bwd_ws_bytes(int64_t n, int64_t P) { return (size_t)bwd_waves(n) * (size_t)P * 4; }

#define FH_MLP_DISPATCH(CALL)                                            \
  do {                                                                   \
    const int inp = ((in_w + 15) / 16) * 16;                             \
    switch (inp * 1000 + H * 10 + NH) {                                  \
      case 16321: return CALL(16, 32, 1);                                \
      case 16322: return CALL(16, 32, 2);                                \
      case 16323: return CALL(16, 32, 3);                                \
      case 16641: return CALL(16, 64, 1);                                \
      case 16642: return CALL(16, 64, 2);                                \
      case 16643: return CALL(16, 64, 3);                                \
      case 32321: return CALL(32, 32, 1);                                \
      case 32322: return CALL(32, 32, 2);                                \
      case 32323: return CALL(32, 32, 3);                                \
      case 32641: return CALL(32, 64, 1);                                \
      case 32642: return CALL(32, 64, 2);                                \
      case 32643: return CALL(32, 64, 3);                                \
      case 48321: return CALL(48, 32, 1);                                \
      case 48322: return CALL(48, 32, 2);                                \
      case 48323: return CALL(48, 32, 3);                                \
      case 48641: return CALL(48, 64, 1);                                \
      case 48642: return CALL(48, 64, 2);                                \
      case 48643: return CALL(48, 64, 3);                                \
      case 64321: return CALL(64, 32, 1);                                \
      case 64322: return CALL(64, 32, 2);                                \
      case 64323: return CALL(64, 32, 3);                                \
      case 64641: return CALL(64, 64, 1);                                \
      case 64642: return CALL(64, 64, 2);                                \
      case 64643: return CALL(64, 64, 3);                                \
    }                                                                    \
    return hipErrorInvalidValue;                                         \
  } while (0)

hipError_t launch_mlp_fwd(int in_w, int H, int NH, const float* params, const float* x, int64_t n,
                          float* y, hipStream_t st) {
  if (n == 0) return hipSuccess;
#define FH_CALL_FWD(A, B, C) fwd_t<A, B, C>(params, x, n, in_w, y, st)
  FH_MLP_DISPATCH(FH_CALL_FWD);
#undef FH_CALL_FWD
}

hipError_t launch_mlp_bwd(int in_w, int H, int NH, const float* params, const float* x,
                          const float* dy, int64_t n, float* d_params, float* dx, void* ws,
                          int64_t P, hipStream_t st) {
  if (n == 0) return hipSuccess;
  float* part = static_cast<float*>(ws);
#define FH_CALL_BWD(A, B, C) bwd_t<A, B, C>(params, x, dy, n, in_w, d_params, dx, part, P, st)
  FH_MLP_DISPATCH(FH_CALL_BWD);
#undef FH_CALL_BWD
}

}  // namespace fh
