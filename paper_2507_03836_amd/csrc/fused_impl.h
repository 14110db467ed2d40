// Fused tesseract encoding + MLP decoder (forward, backward, and forward + MSE
// + backward in one pass).
//
// A wave processes blocks of 16 samples.  Lane l = 16 g + s owns sample s of
// the block and the embedding features 16 a + 4 g + i of it -- exactly the
// features its MFMA B-operand registers carry -- so each lane gathers the
// levels behind those features itself (4/F levels per 16-feature block), the
// encoding lands directly in MLP input registers, and the encoding gradient
// that the MLP backward leaves in the same registers is scattered by the same
// lane for the same levels.  Corner weights are recomputed, never stored.
#pragma once
#include <type_traits>

#include "encode_dev.h"
#include "kernels.h"
#include "mlp_dev.h"
#include "mlp_train_dev.h"

namespace fh {

namespace fused_detail {

// Waves per workgroup: eight in every mode.  The forward keeps only the
// decoder weights in LDS; the backward modes also hold the workgroup's
// gradient image and per-wave tiles.  MODE_FWD16: the forward with a 16-bit
// MFMA decoder (inference).
enum { MODE_FWD = 0, MODE_BWD = 1, MODE_TRAIN = 2, MODE_FWD16 = 3 };
constexpr bool is_forward(int mode) { return mode == MODE_FWD || mode == MODE_FWD16; }
constexpr int waves_per_block(int mode) { return (void)mode, 8; }

struct FusedArgs {
  const float4* pos;
  const float* target;  // MODE_TRAIN
  const float* dy;      // MODE_BWD
  int64_t n;
  const void* table;
  const float* params;
  float* y;        // MODE_FWD
  float* d_table;  // MODE_BWD / TRAIN
  float* part;     // per-workgroup parameter-gradient partials
  double* loss_sum;
  int64_t P;
  float coef;  // dL/dy = coef * (y - target)
  int in_w;    // L * F
};

template <int F, typename T, int INP, bool BRICK>
__device__ __forceinline__ void gather_block(const GridDev& g, const LevelDev* lv, float4 p,
                                             bool valid, const T* table,
                                             float (&xb)[INP / 16][4]) {
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  constexpr int LPB = 4 / F;  // levels per lane per 16-feature block
#pragma unroll
  for (int a = 0; a < INP / 16; ++a)
#pragma unroll
    for (int j = 0; j < LPB; ++j) {
      const int l = (16 * a + 4 * grp) / F + j;
      float e[F];
      if (valid && l < g.L) {
        encode_level<F, T, BRICK>(lv[l], g.dir, g.active != 0, p, table, e, g.tmask);
      } else {
#pragma unroll
        for (int k = 0; k < F; ++k) e[k] = 0.0f;
      }
#pragma unroll
      for (int k = 0; k < F; ++k) xb[a][j * F + k] = e[k];
    }
}

// Scatter of a block's encoding gradient, redistributed so that 2F
// consecutive lanes own one (sample, level): pass k of 2F gives lane q the
// sample-level held by lane k * (64 / 2F) + q / 2F, whose position and
// gradient arrive by shuffles.  Levels flagged in g.dedup (sorted batches,
// coarse levels) sum a corner across the samples of the pass first when they
// all share its slot (scatter_level_lane_merge).  Levels below g.coarse are
// not added here: their gradient goes to g.dxc for the LDS scatter
// (coarse.hip).
template <int F, int INP, bool BRICK>
__device__ __forceinline__ void scatter_block(const GridDev& g, const LevelDev* lv, float4 p,
                                              bool valid, int64_t smp,
                                              const float (&dx)[INP / 16][4], float* d_table) {
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  constexpr int LPB = 4 / F;
  constexpr int Q = 2 * F, PER = 64 / Q;
  const int r = lane % Q, e = r / F, f = r % F;
  if (g.coarse > 0 && valid) {
#pragma unroll
    for (int a = 0; a < INP / 16; ++a)
#pragma unroll
      for (int j = 0; j < LPB; ++j) {
        const int l = (16 * a + 4 * grp) / F + j;  // this lane group's level
        if (l < g.coarse)
#pragma unroll
          for (int q = 0; q < F; ++q)
            g.dxc[((int64_t)l * g.nsamp + smp) * F + q] = dx[a][j * F + q];
      }
  }
#pragma unroll
  for (int a = 0; a < INP / 16; ++a)
#pragma unroll
    for (int j = 0; j < LPB; ++j) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int m = k * PER + lane / Q;  // source lane (= sample-level)
        const int src_grp = m >> 4;
        const int ls = (16 * a + 4 * src_grp) / F + j;
        float gsrc[F];
#pragma unroll
        for (int q = 0; q < F; ++q) gsrc[q] = __shfl(dx[a][j * F + q], m, 64);
        float4 ps;
        ps.x = __shfl(p.x, m, 64);
        ps.y = __shfl(p.y, m, 64);
        ps.z = __shfl(p.z, m, 64);
        ps.w = __shfl(p.w, m, 64);
        const bool vs = __shfl((int)valid, m, 64) != 0;
        float gval = gsrc[0];
#pragma unroll
        for (int q = 1; q < F; ++q)
          if (f == q) gval = gsrc[q];
        if (ls < g.L && ls >= g.coarse) {
          if ((g.dedup >> ls) & 1u)
            scatter_level_lane_merge<F, BRICK>(lv[ls], g.dir, g.active != 0, ps, vs, e, f, gval,
                                               d_table, g.touch, g.touch_begin, g.gmask);
          else if (vs)
            scatter_level_lane<F, BRICK>(lv[ls], g.dir, g.active != 0, ps, e, f, gval, d_table,
                                         g.touch, g.touch_begin, g.gmask);
        }
      }
    }
}

// One workgroup per CU in the backward modes: the decoder weights, the FP32
// gradient image of the workgroup (mlp_train_dev.h) and eight waves' tiles
// share its LDS.  D is the decoder arithmetic: float (FP32 MFMA) or a 16-bit
// type (_Float16 / __bf16 MFMA with FP32 accumulation); the FP32-decoder
// forward is MODE_FWD, the 16-bit one MODE_FWD16.
template <int MODE, int F, typename T, int INP, int H, int NH, typename D, bool BRICK>
__global__ void __launch_bounds__(64 * waves_per_block(MODE))
    __attribute__((amdgpu_waves_per_eu(is_forward(MODE) ? 1 : 2)))
    fused_kernel(GridDev g, FusedArgs A) {
  constexpr int kWaves = waves_per_block(MODE);
  constexpr bool FWD = is_forward(MODE);
  constexpr bool D32 = std::is_same<D, float>::value;
  using S = MlpShape<INP, H, NH>;
  using G = GradLds<INP, H, NH>;
  constexpr int WFL = (MODE == MODE_FWD16) ? MlpShapeH<INP, H, NH>::TOTAL_FLOATS
                      : D32               ? S::WFLOATS
                                          : MlpShapeT<INP, H, NH>::TOTAL_FLOATS;
  constexpr int GFL = FWD ? 0 : G::FLOATS;
  constexpr int WS = FWD ? 0
                     : D32 ? train_wave_scratch_f32<INP, H, NH>()
                           : train_wave_scratch_t<INP, H, NH>();
  __shared__ __attribute__((aligned(16))) float lds[WFL + GFL + kWaves * WS + 1];
  __shared__ LevelDev lv[FHASH_MAX_LEVELS];
  if constexpr (MODE == MODE_FWD16)
    load_weights_lds_h<INP, H, NH, D>(lds, A.params, A.in_w);
  else if constexpr (D32)
    load_weights_lds<INP, H, NH>(lds, A.params, A.in_w);
  else
    load_weights_lds_t<INP, H, NH, D>(lds, A.params, A.in_w);
  float* grad = lds + WFL;
  if constexpr (!FWD) grad_lds_zero<INP, H, NH>(grad);
  for (int e = threadIdx.x; e < FHASH_MAX_LEVELS; e += blockDim.x) lv[e] = g.lv[e];
  __syncthreads();
  const T* table = reinterpret_cast<const T*>(A.table);
  const int lane = threadIdx.x & 63, grp = lane >> 4, s = lane & 15;
  const int wib = threadIdx.x >> 6;
  float* scratch = lds + WFL + GFL + wib * WS;
  const int64_t nblk = (A.n + 15) / 16;
  const int64_t nwav = (int64_t)gridDim.x * kWaves;
  const int64_t wave = (int64_t)blockIdx.x * kWaves + wib;
  double loss = 0.0;
  for (int64_t b = wave; b < nblk; b += nwav) {
    // Keep the decoder weights in LDS rather than in registers across blocks:
    // the compiler would otherwise hoist every layer's weight fragments out of
    // this loop (64 registers per 64x64 layer) and cut the waves per SIMD.
    __asm__ volatile("" ::: "memory");
    const int64_t smp = b * 16 + s;
    const bool valid = smp < A.n;
    const float4 p = valid ? A.pos[smp] : make_float4(0.f, 0.f, 0.f, 0.f);
    float xb[S::INB][4];
    gather_block<F, T, INP, BRICK>(g, lv, p, valid, table, xb);
    float hs[NH][S::HB][4];
    float yv;
    if constexpr (MODE == MODE_FWD16)
      yv = mlp_block_fwd_h<INP, H, NH, D>(lds, xb);
    else if constexpr (D32)
      yv = mlp_block_fwd<INP, H, NH>(lds, xb, hs);
    else
      yv = mlp_block_fwd_t<INP, H, NH, D>(lds, xb, hs);
    if constexpr (FWD) {
      if (grp == 0 && valid) A.y[smp] = yv;
      continue;
    } else {
      float dyv = 0.0f;
      if (MODE == MODE_BWD) {
        dyv = valid ? A.dy[smp] : 0.0f;
      } else {
        const float r = valid ? yv - A.target[smp] : 0.0f;
        dyv = A.coef * r;
        if (grp == 0) loss += (double)r * (double)r;
      }
      float dxb[S::INB][4];
      if constexpr (D32)
        mlp_block_bwd_lds<INP, H, NH>(lds, grad, scratch, xb, hs, dyv, dxb);
      else
        mlp_block_bwd_t<INP, H, NH, D>(lds, grad, reinterpret_cast<D*>(scratch), xb, hs, dyv,
                                       dxb);
      scatter_block<F, INP, BRICK>(g, lv, p, valid, smp, dxb, A.d_table);
    }
  }
  if constexpr (!FWD) {
    __syncthreads();
    grad_lds_write<INP, H, NH>(grad, A.in_w, A.part + (int64_t)blockIdx.x * A.P);
    if (MODE == MODE_TRAIN && A.loss_sum != nullptr) {
      for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
      if (lane == 0) unsafeAtomicAdd(A.loss_sum, loss);
    }
  }
}

inline int64_t fused_waves(int64_t n, int mode) {
  const int kWaves = waves_per_block(mode);
  int64_t nblk = (n + 15) / 16;
  int64_t cap = is_forward(mode) ? 8192 : 2048;
  int64_t w = nblk < cap ? nblk : cap;
  w = ((w + kWaves - 1) / kWaves) * kWaves;
  return w < kWaves ? kWaves : w;
}

// Workgroups of a launch (= decoder-gradient partials of a backward launch).
inline int64_t fused_blocks(int64_t n, int mode) {
  return fused_waves(n, mode) / waves_per_block(mode);
}

// The brick slot order is built for the production decoder shapes only
// (32 inputs, hidden width 64, 2 or 3 hidden layers, F = 2 or 4); the host
// rejects other shapes on a brick-ordered index.
template <int F, int INP, int H, int NH>
constexpr bool brick_shape() {
  return (F == 2 || F == 4) && INP == 32 && H == 64 && (NH == 2 || NH == 3);
}

template <int MODE, int F, typename T, int INP, int H, int NH, typename D>
hipError_t fused_t(const GridDev& g, FusedArgs A, float* d_params, hipStream_t st) {
  constexpr int kWaves = waves_per_block(MODE);
  const int64_t nb = fused_blocks(A.n, MODE);
  if (g.lv[0].brick) {
    if constexpr (brick_shape<F, INP, H, NH>())
      hipLaunchKernelGGL((fused_kernel<MODE, F, T, INP, H, NH, D, true>), dim3((unsigned)nb),
                         dim3(64 * kWaves), 0, st, g, A);
    else
      return hipErrorNotSupported;
  } else {
    hipLaunchKernelGGL((fused_kernel<MODE, F, T, INP, H, NH, D, false>), dim3((unsigned)nb),
                       dim3(64 * kWaves), 0, st, g, A);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || is_forward(MODE)) return e;
  if (g.coarse > 0) {
    e = launch_coarse_scatter(g, reinterpret_cast<const float*>(A.pos), A.n, A.d_table, st);
    if (e != hipSuccess) return e;
  }
  return launch_reduce_partials(A.part, nb, A.P, d_params, st);
}

template <int MODE, int F, typename T, typename D>
hipError_t fused_shape(const GridDev& g, int H, int NH, FusedArgs A, float* d_params,
                       hipStream_t st) {
  const int inp = ((A.in_w + 15) / 16) * 16;
  switch (inp * 1000 + H * 10 + NH) {
#define FH_C(I, HH, N) \
  case I * 1000 + HH * 10 + N: return fused_t<MODE, F, T, I, HH, N, D>(g, A, d_params, st);
    FH_C(16, 32, 1) FH_C(16, 32, 2) FH_C(16, 32, 3)
    FH_C(16, 64, 1) FH_C(16, 64, 2) FH_C(16, 64, 3)
    FH_C(32, 32, 1) FH_C(32, 32, 2) FH_C(32, 32, 3)
    FH_C(32, 64, 1) FH_C(32, 64, 2) FH_C(32, 64, 3)
#undef FH_C
  }
  return hipErrorInvalidValue;
}

// Every feature count, FP32 or FP16 table, decoder arithmetic D.
template <int MODE, typename D>
hipError_t fused_dispatch(const GridDev& g, int H, int NH, fhash_dtype tdt, FusedArgs A,
                          float* d_params, hipStream_t st) {
  if (A.n == 0) return hipSuccess;
  if (tdt == FHASH_F32) {
    switch (g.F) {
      case 1: return fused_shape<MODE, 1, float, D>(g, H, NH, A, d_params, st);
      case 2: return fused_shape<MODE, 2, float, D>(g, H, NH, A, d_params, st);
      case 4: return fused_shape<MODE, 4, float, D>(g, H, NH, A, d_params, st);
    }
  } else {
    switch (g.F) {
      case 1: return fused_shape<MODE, 1, __half, D>(g, H, NH, A, d_params, st);
      case 2: return fused_shape<MODE, 2, __half, D>(g, H, NH, A, d_params, st);
      case 4: return fused_shape<MODE, 4, __half, D>(g, H, NH, A, d_params, st);
    }
  }
  return hipErrorInvalidValue;
}

// Two features per level only (the production configurations).
template <int MODE, typename D>
hipError_t fused_dispatch_f2(const GridDev& g, int H, int NH, fhash_dtype tdt, FusedArgs A,
                             float* d_params, hipStream_t st) {
  if (A.n == 0) return hipSuccess;
  if (g.F != 2) return hipErrorInvalidValue;
  if (tdt == FHASH_F32) return fused_shape<MODE, 2, float, D>(g, H, NH, A, d_params, st);
  return fused_shape<MODE, 2, __half, D>(g, H, NH, A, d_params, st);
}

}  // namespace fused_detail

}  // namespace fh
