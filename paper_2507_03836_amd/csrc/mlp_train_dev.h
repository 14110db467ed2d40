// Decoder backward for the fused training kernels: parameter gradients are
// accumulated per workgroup in LDS instead of per-wave registers.
//
// The register engine (mlp_dev.h, MlpGrad) keeps a wave's whole decoder
// gradient in registers across sample blocks: 145 registers per lane for a
// 32-64-64-1 decoder, 225 for 32-64-64-64-1, which caps the fused training
// kernel at one or two waves per SIMD (and spills at 32-64-64-1).  Here each
// 16-sample block computes its weight-gradient tiles with MFMA into transient
// registers and adds them (ds_add_f32) into one FP32 gradient image per
// workgroup; biases are summed over the block's 16 sample lanes first.  At the
// end the workgroup writes its image as one partial of the packed parameter
// vector.  Summation order across the waves of a workgroup is not fixed.
//
// Two decoder arithmetics share the layout:
//  - FP32: v_mfma_f32_16x16x4_f32, weights FP32 in LDS (the image of
//    mlp_dev.h), FP32 transposition tiles;
//  - 16-bit (FP16 or BF16): v_mfma_f32_16x16x16_{f16,bf16} with FP32
//    accumulation.  Weights and every hidden-layer input are rounded to the
//    16-bit type (RNE), biases, the output layer and all accumulations stay
//    FP32.  The backward contracts with rounded deltas and a rounded,
//    transposed copy of each weight matrix, so every A operand is one 8-byte
//    LDS read.  A block's 16 samples are one K step of the weight-gradient
//    MFMA.
#pragma once
#include "mlp_dev.h"

namespace fh {

__device__ __forceinline__ void lds_add(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// FP32 gradient image of a workgroup in LDS (row strides padded against bank
// conflicts of the tile adds).
template <int INP, int H, int NH>
struct GradLds {
  static constexpr int LD0 = INP + 4;
  static constexpr int LDH = H + 4;
  static constexpr int W0 = 0;
  static constexpr int B0 = W0 + H * LD0;
  static constexpr int WK = B0 + H;
  static constexpr int WKSTRIDE = H * LDH + H;
  static constexpr int WOUT = WK + (NH - 1) * WKSTRIDE;
  static constexpr int BOUT = WOUT + H;
  static constexpr int FLOATS = (BOUT + 1 + 3) / 4 * 4;
};

template <int INP, int H, int NH>
__device__ void grad_lds_zero(float* g) {
  for (int e = threadIdx.x; e < GradLds<INP, H, NH>::FLOATS; e += blockDim.x) g[e] = 0.0f;
}

// The workgroup's image in the packed parameter layout (W_k[out][in] then b_k;
// W0 has in_w columns).  Whole workgroup, after a barrier.
template <int INP, int H, int NH>
__device__ void grad_lds_write(const float* g, int in_w, float* __restrict__ part) {
  using G = GradLds<INP, H, NH>;
  for (int e = threadIdx.x; e < H * in_w; e += blockDim.x)
    part[e] = g[G::W0 + (e / in_w) * G::LD0 + e % in_w];
  float* p = part + H * in_w;
  for (int e = threadIdx.x; e < H; e += blockDim.x) p[e] = g[G::B0 + e];
  p += H;
  for (int k = 1; k < NH; ++k) {
    const float* gk = g + G::WK + (k - 1) * G::WKSTRIDE;
    for (int e = threadIdx.x; e < H * H; e += blockDim.x) p[e] = gk[(e / H) * G::LDH + e % H];
    p += H * H;
    for (int e = threadIdx.x; e < H; e += blockDim.x) p[e] = gk[H * G::LDH + e];
    p += H;
  }
  for (int e = threadIdx.x; e < H; e += blockDim.x) p[e] = g[G::WOUT + e];
  if (threadIdx.x == 0) p[H] = g[G::BOUT];
}

// g[16 a + 4 grp + i] += sum over the block's 16 samples of v[a][i] (lane
// 16 grp + s holds sample s).  After the sums every lane of a group holds all
// NB * 4 of them; lane s of the group adds value s, so one LDS add instruction
// covers a group's values.
template <int NB>
__device__ __forceinline__ void bias_add(float* g, const float (&v)[NB][4]) {
  static_assert(NB * 4 <= 16, "at most 16 features per lane group");
  const int lane = threadIdx.x & 63, grp = lane >> 4, s = lane & 15;
  float mine = 0.0f;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float t = sum16(v[a][i]);
      if (s == 4 * a + i) mine = t;
    }
  if (s < NB * 4) lds_add(&g[16 * (s >> 2) + 4 * grp + (s & 3)], mine);
}

// Output layer y = wout . h + bout: gradients of wout and bout, and the delta
// of the last hidden layer.  wout: FP32 in LDS.
template <int HB>
__device__ __forceinline__ void out_layer_bwd(const float* wout, const float (&h)[HB][4], float dy,
                                              float* g_wout, float* g_bout,
                                              float (&delta)[HB][4]) {
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  float dwo[HB][4];
#pragma unroll
  for (int a = 0; a < HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dwo[a][i] = dy * h[a][i];
      delta[a][i] = (h[a][i] > 0.0f) ? wout[16 * a + 4 * grp + i] * dy : 0.0f;
    }
  bias_add<HB>(g_wout, dwo);
  const float sdy = sum16(dy);
  if (lane == 0) lds_add(g_bout, sdy);
}

// ------------------------------------------------------------------- FP32
// Weight gradient of one block: g[(16 ob + r) * ld + 16 ib + c] += sum over the
// 16 samples of delta[16 ob + r] x input[16 ib + c], from the two transposed
// FP32 tiles ([rows][17]).  Output lane (grp, n): rows 16 ob + 4 grp + i,
// column 16 ib + n.
template <int OB, int IB>
__device__ __forceinline__ void dw_lds_f32(const float* dtile, const float* itile, float* g,
                                           int ld) {
  const int lane = threadIdx.x & 63, grp = lane >> 4, m = lane & 15;
  f4v acc[OB][IB];
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) acc[ob][ib] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float a[OB], b[IB];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) a[ob] = dtile[(16 * ob + m) * 17 + 4 * j + grp];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) b[ib] = itile[(16 * ib + m) * 17 + 4 * j + grp];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob)
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) acc[ob][ib] = mfma4(a[ob], b[ib], acc[ob][ib]);
  }
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int ib = 0; ib < IB; ++ib)
#pragma unroll
      for (int i = 0; i < 4; ++i) lds_add(&g[(16 * ob + 4 * grp + i) * ld + 16 * ib + m], acc[ob][ib][i]);
}

// Backward of one block through the FP32 decoder (weights: the LDS image of
// load_weights_lds), gradients added to the workgroup image `grad`.  xb: the
// block input (B layout); hs: hidden activations of the forward; scratch: the
// wave's two [TROWS][17] tiles.  Returns dx = dL/dx (C layout).
template <int INP, int H, int NH>
__device__ __forceinline__ void mlp_block_bwd_lds(const float* lds, float* grad, float* scratch,
                                                  const float (&xb)[INP / 16][4],
                                                  const float (&hs)[NH][H / 16][4], float dy,
                                                  float (&dx)[INP / 16][4]) {
  using S = MlpShape<INP, H, NH>;
  using G = GradLds<INP, H, NH>;
  float* dtile = scratch;
  float* htile = scratch + S::TILE;
  float delta[S::HB][4];
  out_layer_bwd<S::HB>(lds + S::WOUT, hs[NH - 1], dy, grad + G::WOUT, grad + G::BOUT, delta);
#pragma unroll
  for (int k = NH - 1; k >= 1; --k) {
    const float* wk = lds + S::WK + (k - 1) * S::WKSTRIDE;
    float* gk = grad + G::WK + (k - 1) * G::WKSTRIDE;
    bias_add<S::HB>(gk + H * G::LDH, delta);
    wave_lds_fence();
    tile_store<S::HB>(dtile, delta);
    tile_store<S::HB>(htile, hs[k - 1]);
    wave_lds_fence();
    dw_lds_f32<S::HB, S::HB>(dtile, htile, gk, G::LDH);
    float dprev[S::HB][4];
    bwd_data<S::HB, S::HB>(wk, S::LDH, delta, dprev);
#pragma unroll
    for (int a = 0; a < S::HB; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) delta[a][i] = (hs[k - 1][a][i] > 0.0f) ? dprev[a][i] : 0.0f;
  }
  bias_add<S::HB>(grad + G::B0, delta);
  wave_lds_fence();
  tile_store<S::HB>(dtile, delta);
  tile_store<S::INB>(htile, xb);
  wave_lds_fence();
  dw_lds_f32<S::HB, S::INB>(dtile, htile, grad + G::W0, G::LD0);
  bwd_data<S::HB, S::INB>(lds + S::W0, S::LD0, delta, dx);
  wave_lds_fence();
}

// Per-wave scratch floats of the FP32 engine: two transposition tiles.
template <int INP, int H, int NH>
constexpr int train_wave_scratch_f32() {
  return 2 * MlpShape<INP, H, NH>::TILE;
}

// ------------------------------------------------------------------ 16-bit
// LDS image of the 16-bit training decoder: FP32 biases and output layer, then
// the rounded weight matrices and their transposes (rows padded by 8 elements).
template <int INP, int H, int NH>
struct MlpShapeT {
  static constexpr int INB = INP / 16;
  static constexpr int HB = H / 16;
  static constexpr int B0 = 0;
  static constexpr int BK = B0 + H;
  static constexpr int WOUT = BK + (NH - 1) * H;
  static constexpr int BOUT = WOUT + H;
  static constexpr int FLOATS = (BOUT + 1 + 3) / 4 * 4;
  // 16-bit part, offsets in elements from the end of the float part
  static constexpr int LD0 = INP + 8;  // W0 rows
  static constexpr int LDH = H + 8;    // W_k rows, and rows of every transpose
  static constexpr int W0 = 0;
  static constexpr int WK = W0 + H * LD0;
  static constexpr int W0T = WK + (NH - 1) * H * LDH;  // [INP][LDH]
  static constexpr int WKT = W0T + INP * LDH;          // per k: [H][LDH]
  static constexpr int ELEMS = WKT + (NH - 1) * H * LDH;
  static constexpr int TOTAL_FLOATS = FLOATS + (ELEMS + 1) / 2 + 4;
  // transposition tile of a wave: [rows][TS] 16-bit elements (8-byte reads of
  // 4 consecutive samples)
  static constexpr int TS = 20;
  static constexpr int TROWS = (H > INP ? H : INP);
  static constexpr int TILE = TROWS * TS;
};

template <int INP, int H, int NH, typename T>
__device__ void load_weights_lds_t(float* lds, const float* __restrict__ params, int in_w) {
  using S = MlpShapeT<INP, H, NH>;
  T* wh = reinterpret_cast<T*>(lds + S::FLOATS);
  for (int e = threadIdx.x; e < H * INP; e += blockDim.x) {
    const int o = e / INP, i = e % INP;
    const T w = (T)((i < in_w) ? params[o * in_w + i] : 0.0f);
    wh[S::W0 + o * S::LD0 + i] = w;
    wh[S::W0T + i * S::LDH + o] = w;
  }
  const float* p = params + H * in_w;
  for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::B0 + e] = p[e];
  p += H;
  for (int k = 1; k < NH; ++k) {
    T* wk = wh + S::WK + (k - 1) * H * S::LDH;
    T* wt = wh + S::WKT + (k - 1) * H * S::LDH;
    for (int e = threadIdx.x; e < H * H; e += blockDim.x) {
      const T w = (T)p[e];
      wk[(e / H) * S::LDH + e % H] = w;
      wt[(e % H) * S::LDH + e / H] = w;
    }
    p += H * H;
    for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::BK + (k - 1) * H + e] = p[e];
    p += H;
  }
  for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::WOUT + e] = p[e];
  if (threadIdx.x == 0) lds[S::BOUT] = p[H];
}

// Forward of one block through the 16-bit decoder, keeping the (FP32) hidden
// activations for the backward; the output layer is an FP32 dot product.
template <int INP, int H, int NH, typename T>
__device__ __forceinline__ float mlp_block_fwd_t(const float* lds, const float (&xb)[INP / 16][4],
                                                 float (&hs)[NH][H / 16][4]) {
  using S = MlpShapeT<INP, H, NH>;
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  const T* wh = reinterpret_cast<const T*>(lds + S::FLOATS);
  fwd_layer_t<T, S::INB, S::HB>(wh + S::W0, S::LD0, lds + S::B0, xb, hs[0]);
#pragma unroll
  for (int k = 1; k < NH; ++k)
    fwd_layer_t<T, S::HB, S::HB>(wh + S::WK + (k - 1) * H * S::LDH, S::LDH,
                                 lds + S::BK + (k - 1) * H, hs[k - 1], hs[k]);
  float y = 0.0f;
#pragma unroll
  for (int a = 0; a < S::HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) y += lds[S::WOUT + 16 * a + 4 * grp + i] * hs[NH - 1][a][i];
  return sum_groups(y) + lds[S::BOUT];
}

// dprev = W^T round(delta): A operand from the rounded transpose WT ([in][ldt]).
template <typename T, int OB, int IB>
__device__ __forceinline__ void bwd_data_t(const T* WT, int ldt, const float (&delta)[OB][4],
                                           float (&dprev)[IB][4]) {
  using V = typename Vec4T<T>::type;
  const int lane = threadIdx.x & 63, grp = lane >> 4, m = lane & 15;
  V bin[OB];
#pragma unroll
  for (int a = 0; a < OB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) bin[a][i] = (T)delta[a][i];
  f4v c[IB];
#pragma unroll
  for (int ib = 0; ib < IB; ++ib) c[ib] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int a = 0; a < OB; ++a)
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
      const V w = *reinterpret_cast<const V*>(WT + (16 * ib + m) * ldt + 16 * a + 4 * grp);
      c[ib] = mfma16t<T>(w, bin[a], c[ib]);
    }
#pragma unroll
  for (int ib = 0; ib < IB; ++ib)
#pragma unroll
    for (int i = 0; i < 4; ++i) dprev[ib][i] = c[ib][i];
}

// Register block (C layout) rounded and transposed into a [rows][TS] tile.
template <typename T, int NB, int TS>
__device__ __forceinline__ void tile_store_t(T* tile, const float (&v)[NB][4]) {
  const int lane = threadIdx.x & 63, grp = lane >> 4, s = lane & 15;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) tile[(16 * a + 4 * grp + i) * TS + s] = (T)v[a][i];
}

// Weight gradient of one block from two rounded tiles: one MFMA per 16x16
// output block (K = the 16 samples).  A lane (grp, m): delta row 16 ob + m,
// samples 4 grp..4 grp+3; B lane (grp, n): input row 16 ib + n, same samples.
template <typename T, int OB, int IB, int TS>
__device__ __forceinline__ void dw_lds_t(const T* dtile, const T* itile, float* g, int ld) {
  using V = typename Vec4T<T>::type;
  const int lane = threadIdx.x & 63, grp = lane >> 4, m = lane & 15;
  V a[OB], b[IB];
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
    a[ob] = *reinterpret_cast<const V*>(dtile + (16 * ob + m) * TS + 4 * grp);
#pragma unroll
  for (int ib = 0; ib < IB; ++ib)
    b[ib] = *reinterpret_cast<const V*>(itile + (16 * ib + m) * TS + 4 * grp);
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
      const f4v acc = mfma16t<T>(a[ob], b[ib], f4v{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
      for (int i = 0; i < 4; ++i) lds_add(&g[(16 * ob + 4 * grp + i) * ld + 16 * ib + m], acc[i]);
    }
}

// Backward of one block through the 16-bit decoder (LDS image of
// load_weights_lds_t); scratch: the wave's two 16-bit tiles.
template <int INP, int H, int NH, typename T>
__device__ __forceinline__ void mlp_block_bwd_t(const float* lds, float* grad, T* scratch,
                                                const float (&xb)[INP / 16][4],
                                                const float (&hs)[NH][H / 16][4], float dy,
                                                float (&dx)[INP / 16][4]) {
  using S = MlpShapeT<INP, H, NH>;
  using G = GradLds<INP, H, NH>;
  const T* wh = reinterpret_cast<const T*>(lds + S::FLOATS);
  T* dtile = scratch;
  T* htile = scratch + S::TILE;
  float delta[S::HB][4];
  out_layer_bwd<S::HB>(lds + S::WOUT, hs[NH - 1], dy, grad + G::WOUT, grad + G::BOUT, delta);
#pragma unroll
  for (int k = NH - 1; k >= 1; --k) {
    float* gk = grad + G::WK + (k - 1) * G::WKSTRIDE;
    bias_add<S::HB>(gk + H * G::LDH, delta);
    wave_lds_fence();
    tile_store_t<T, S::HB, S::TS>(dtile, delta);
    tile_store_t<T, S::HB, S::TS>(htile, hs[k - 1]);
    wave_lds_fence();
    dw_lds_t<T, S::HB, S::HB, S::TS>(dtile, htile, gk, G::LDH);
    float dprev[S::HB][4];
    bwd_data_t<T, S::HB, S::HB>(wh + S::WKT + (k - 1) * H * S::LDH, S::LDH, delta, dprev);
#pragma unroll
    for (int a = 0; a < S::HB; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) delta[a][i] = (hs[k - 1][a][i] > 0.0f) ? dprev[a][i] : 0.0f;
  }
  bias_add<S::HB>(grad + G::B0, delta);
  wave_lds_fence();
  tile_store_t<T, S::HB, S::TS>(dtile, delta);
  tile_store_t<T, S::INB, S::TS>(htile, xb);
  wave_lds_fence();
  dw_lds_t<T, S::HB, S::INB, S::TS>(dtile, htile, grad + G::W0, G::LD0);
  bwd_data_t<T, S::HB, S::INB>(wh + S::W0T, S::LDH, delta, dx);
  wave_lds_fence();
}

// Per-wave scratch floats of the 16-bit engine: two 16-bit tiles.
template <int INP, int H, int NH>
constexpr int train_wave_scratch_t() {
  return MlpShapeT<INP, H, NH>::TILE;  // 2 tiles x TILE elements x 2 bytes = TILE floats
}

}  // namespace fh
