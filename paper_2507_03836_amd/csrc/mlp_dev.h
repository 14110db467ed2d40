// Device-side MLP engine on FP32 MFMA (v_mfma_f32_16x16x4_f32), shared by the
// standalone MLP kernels and the fused encoding + MLP kernels.
//
// A wave processes samples in blocks of 16.  Activations are kept transposed
// (features x samples) in the MFMA accumulator layout: lane l = 16 g + s holds,
// for sample s of the block, features 16 a + 4 g + i in register [a][i]
// (a = 16-feature block, i = 0..3).  Because a contraction may visit its K
// index in any order, that same register layout is directly the B operand of
// the next layer (K step (a, i): lane group g supplies feature 16 a + 4 g + i),
// so layers chain in registers with no data movement; the A operand (weights)
// is read from LDS in the matching permuted order.  Weight gradients contract
// over samples, so the wave transposes delta and the layer input through a
// small per-wave LDS tile and runs one more MFMA per 16x16 output block.
#pragma once
#include "common.h"

namespace fh {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Shape of a decoder: input padded to INP (multiple of 16), NH hidden layers of
// width H (multiple of 16), scalar output.
template <int INP, int H, int NH>
struct MlpShape {
  static constexpr int INB = INP / 16;
  static constexpr int HB = H / 16;
  static constexpr int LD0 = INP + 4;  // LDS row stride of W0 (floats)
  static constexpr int LDH = H + 4;    // LDS row stride of the hidden W_k
  // LDS weight image offsets (floats)
  static constexpr int W0 = 0;
  static constexpr int B0 = W0 + H * LD0;
  static constexpr int WK = B0 + H;                        // W_k, k = 1..NH-1
  static constexpr int WKSTRIDE = H * LDH + H;             // W_k then b_k
  static constexpr int WOUT = WK + (NH - 1) * WKSTRIDE;    // output weights [H]
  static constexpr int BOUT = WOUT + H;                    // output bias
  static constexpr int WFLOATS = BOUT + 4;
  // Per-wave transpose tile: [rows][17] for delta and for the layer input.
  static constexpr int TROWS = (H > INP ? H : INP);
  static constexpr int TILE = TROWS * 17;
  static constexpr int SCRATCH = 2 * TILE;
};

// Copy the packed parameter vector into the LDS weight image (zero-padding the
// input columns of W0 beyond in_w).  Whole workgroup; caller syncs.
template <int INP, int H, int NH>
__device__ void load_weights_lds(float* lds, const float* __restrict__ params, int in_w) {
  using S = MlpShape<INP, H, NH>;
  for (int e = threadIdx.x; e < H * INP; e += blockDim.x) {
    const int o = e / INP, i = e % INP;
    lds[S::W0 + o * S::LD0 + i] = (i < in_w) ? params[o * in_w + i] : 0.0f;
  }
  const float* p = params + H * in_w;
  for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::B0 + e] = p[e];
  p += H;
  for (int k = 1; k < NH; ++k) {
    float* wk = lds + S::WK + (k - 1) * S::WKSTRIDE;
    for (int e = threadIdx.x; e < H * H; e += blockDim.x) wk[(e / H) * S::LDH + e % H] = p[e];
    p += H * H;
    for (int e = threadIdx.x; e < H; e += blockDim.x) wk[H * S::LDH + e] = p[e];
    p += H;
  }
  for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::WOUT + e] = p[e];
  if (threadIdx.x == 0) lds[S::BOUT] = p[H];
}

// out = act(W in + b) for one 16-sample block.  W is [HB*16][ld] in LDS.
template <int INB, int HB>
__device__ __forceinline__ void fwd_layer(const float* W, int ld, const float* b,
                                          const float (&in)[INB][4], float (&out)[HB][4],
                                          bool relu) {
  const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
  f4v c[HB];
#pragma unroll
  for (int ob = 0; ob < HB; ++ob)
#pragma unroll
    for (int i = 0; i < 4; ++i) c[ob][i] = b[16 * ob + 4 * g + i];
#pragma unroll
  for (int a = 0; a < INB; ++a)
#pragma unroll
    for (int ob = 0; ob < HB; ++ob) {
      const float4 w = *reinterpret_cast<const float4*>(W + (16 * ob + m) * ld + 16 * a + 4 * g);
      c[ob] = mfma4(w.x, in[a][0], c[ob]);
      c[ob] = mfma4(w.y, in[a][1], c[ob]);
      c[ob] = mfma4(w.z, in[a][2], c[ob]);
      c[ob] = mfma4(w.w, in[a][3], c[ob]);
    }
#pragma unroll
  for (int ob = 0; ob < HB; ++ob)
#pragma unroll
    for (int i = 0; i < 4; ++i) out[ob][i] = relu ? fmaxf(c[ob][i], 0.0f) : c[ob][i];
}

// dprev = W^T delta for one block (no activation mask).  W is [OB*16][ld].
template <int OB, int IB>
__device__ __forceinline__ void bwd_data(const float* W, int ld, const float (&delta)[OB][4],
                                         float (&dprev)[IB][4]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
  f4v c[IB];
#pragma unroll
  for (int ib = 0; ib < IB; ++ib) c[ib] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int a = 0; a < OB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) {
        const float w = W[(16 * a + 4 * g + i) * ld + 16 * ib + m];
        c[ib] = mfma4(w, delta[a][i], c[ib]);
      }
#pragma unroll
  for (int ib = 0; ib < IB; ++ib)
#pragma unroll
    for (int i = 0; i < 4; ++i) dprev[ib][i] = c[ib][i];
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Write a register block (C layout) transposed into a per-wave [rows][17] tile.
template <int NB>
__device__ __forceinline__ void tile_store(float* tile, const float (&v)[NB][4]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, s = lane & 15;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) tile[(16 * a + 4 * g + i) * 17 + s] = v[a][i];
}

// acc[ob][ib] += delta[16ob + .][:] x input[16ib + .][:]^T over the 16 samples
// held in the two transposed tiles.  Output lane (g, n): rows 16 ob + 4 g + i,
// column 16 ib + n.
template <int OB, int IB>
__device__ __forceinline__ void dw_accumulate(const float* dtile, const float* itile,
                                              f4v (&acc)[OB][IB]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float a[OB], b[IB];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) a[ob] = dtile[(16 * ob + m) * 17 + 4 * j + g];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) b[ib] = itile[(16 * ib + m) * 17 + 4 * j + g];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob)
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) acc[ob][ib] = mfma4(a[ob], b[ib], acc[ob][ib]);
  }
}

// Sum over the 16 sample lanes of a lane group (xor butterfly within 16 lanes).
__device__ __forceinline__ float sum16(float v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}
// Sum over the 4 lane groups (same sample column).
__device__ __forceinline__ float sum_groups(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Gradient accumulators of one wave.
template <int INP, int H, int NH>
struct MlpGrad {
  using S = MlpShape<INP, H, NH>;
  f4v dw0[S::HB][S::INB];
  f4v dwk[NH > 1 ? NH - 1 : 1][S::HB][S::HB];
  float db[NH][S::HB][4];
  float dwout[S::HB][4];
  float dbout;

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < S::HB; ++a) {
#pragma unroll
      for (int b = 0; b < S::INB; ++b) dw0[a][b] = f4v{0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < (NH > 1 ? NH - 1 : 1); ++k)
#pragma unroll
        for (int b = 0; b < S::HB; ++b) dwk[k][a][b] = f4v{0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dwout[a][i] = 0.0f;
#pragma unroll
        for (int k = 0; k < NH; ++k) db[k][a][i] = 0.0f;
      }
    }
    dbout = 0.0f;
  }
};

// Forward of one 16-sample block: hidden activations hs[k] and output y (every
// lane of a sample column holds y of its sample).
template <int INP, int H, int NH>
__device__ __forceinline__ float mlp_block_fwd(const float* lds, const float (&xb)[INP / 16][4],
                                               float (&hs)[NH][H / 16][4]) {
  using S = MlpShape<INP, H, NH>;
  const int lane = threadIdx.x & 63, g = lane >> 4;
  fwd_layer<S::INB, S::HB>(lds + S::W0, S::LD0, lds + S::B0, xb, hs[0], true);
#pragma unroll
  for (int k = 1; k < NH; ++k) {
    const float* wk = lds + S::WK + (k - 1) * S::WKSTRIDE;
    fwd_layer<S::HB, S::HB>(wk, S::LDH, wk + H * S::LDH, hs[k - 1], hs[k], true);
  }
  float y = 0.0f;
#pragma unroll
  for (int a = 0; a < S::HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) y += lds[S::WOUT + 16 * a + 4 * g + i] * hs[NH - 1][a][i];
  return sum_groups(y) + lds[S::BOUT];
}

// ---------------------------------------------------------------------------
// 16-bit decoder (FP16 or BF16 operands, v_mfma_f32_16x16x16_{f16,bf16} with
// FP32 accumulation).  Same register layout as the FP32 engine: the
// accumulator of a layer holds, in lane 16 g + s, features 16 a + 4 g + i of
// sample s, and those 4 values rounded to the 16-bit type are exactly the B
// operand of a 16-deep K block of the next layer (B lane (g, s) supplies
// k = 4 g + i); the A operand of that block is the 4 consecutive rounded
// weights W[16 ob + m][16 a + 4 g .. + 3] (one 8-byte LDS read).  One
// instruction covers what four FP32 16x16x4 steps did.
template <typename T>
struct Vec4T;
template <>
struct Vec4T<_Float16> {
  typedef _Float16 type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4T<__bf16> {
  typedef __bf16 type __attribute__((ext_vector_type(4)));
};

template <typename T>
__device__ __forceinline__ f4v mfma16t(typename Vec4T<T>::type a, typename Vec4T<T>::type b,
                                       f4v c);
template <>
__device__ __forceinline__ f4v mfma16t<_Float16>(Vec4T<_Float16>::type a,
                                                 Vec4T<_Float16>::type b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f4v mfma16t<__bf16>(Vec4T<__bf16>::type a, Vec4T<__bf16>::type b,
                                               f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// LDS image of the 16-bit inference decoder: FP32 biases and output layer
// first, then the rounded weight matrices (rows padded by 8 elements against
// bank conflicts).
template <int INP, int H, int NH>
struct MlpShapeH {
  static constexpr int INB = INP / 16;
  static constexpr int HB = H / 16;
  // float part
  static constexpr int B0 = 0;                      // b_0 [H]
  static constexpr int BK = B0 + H;                 // b_k [NH-1][H]
  static constexpr int WOUT = BK + (NH - 1) * H;    // output weights [H]
  static constexpr int BOUT = WOUT + H;             // output bias
  static constexpr int FLOATS = (BOUT + 1 + 3) / 4 * 4;
  // 16-bit part (offsets in elements, from the end of the float part)
  static constexpr int LD0 = INP + 8;
  static constexpr int LDH = H + 8;
  static constexpr int W0 = 0;
  static constexpr int WK = W0 + H * LD0;
  static constexpr int HALVES = WK + (NH - 1) * H * LDH;
  static constexpr int TOTAL_FLOATS = FLOATS + (HALVES + 1) / 2 + 4;
};

// Round the packed FP32 parameters into the 16-bit LDS image (RNE; W0 columns
// beyond in_w are zero).  Whole workgroup; caller syncs.
template <int INP, int H, int NH, typename T>
__device__ void load_weights_lds_h(float* lds, const float* __restrict__ params, int in_w) {
  using S = MlpShapeH<INP, H, NH>;
  T* wh = reinterpret_cast<T*>(lds + S::FLOATS);
  for (int e = threadIdx.x; e < H * INP; e += blockDim.x) {
    const int o = e / INP, i = e % INP;
    wh[S::W0 + o * S::LD0 + i] = (T)((i < in_w) ? params[o * in_w + i] : 0.0f);
  }
  const float* p = params + H * in_w;
  for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::B0 + e] = p[e];
  p += H;
  for (int k = 1; k < NH; ++k) {
    T* wk = wh + S::WK + (k - 1) * H * S::LDH;
    for (int e = threadIdx.x; e < H * H; e += blockDim.x) wk[(e / H) * S::LDH + e % H] = (T)p[e];
    p += H * H;
    for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::BK + (k - 1) * H + e] = p[e];
    p += H;
  }
  for (int e = threadIdx.x; e < H; e += blockDim.x) lds[S::WOUT + e] = p[e];
  if (threadIdx.x == 0) lds[S::BOUT] = p[H];
}

// out = relu(W round(in) + b) with 16-bit operands and FP32 accumulation.
template <typename T, int INB, int HB>
__device__ __forceinline__ void fwd_layer_t(const T* W, int ld, const float* b,
                                            const float (&in)[INB][4], float (&out)[HB][4]) {
  using V = typename Vec4T<T>::type;
  const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
  V bin[INB];
#pragma unroll
  for (int a = 0; a < INB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) bin[a][i] = (T)in[a][i];
  f4v c[HB];
#pragma unroll
  for (int ob = 0; ob < HB; ++ob)
#pragma unroll
    for (int i = 0; i < 4; ++i) c[ob][i] = b[16 * ob + 4 * g + i];
#pragma unroll
  for (int a = 0; a < INB; ++a)
#pragma unroll
    for (int ob = 0; ob < HB; ++ob) {
      const V w = *reinterpret_cast<const V*>(W + (16 * ob + m) * ld + 16 * a + 4 * g);
      c[ob] = mfma16t<T>(w, bin[a], c[ob]);
    }
#pragma unroll
  for (int ob = 0; ob < HB; ++ob)
#pragma unroll
    for (int i = 0; i < 4; ++i) out[ob][i] = fmaxf(c[ob][i], 0.0f);
}

// Forward of one 16-sample block through the 16-bit decoder; the output layer
// (a dot product of width H) runs in FP32 on the FP32 hidden activations.
template <int INP, int H, int NH, typename T>
__device__ __forceinline__ float mlp_block_fwd_h(const float* lds, const float (&xb)[INP / 16][4]) {
  using S = MlpShapeH<INP, H, NH>;
  const int lane = threadIdx.x & 63, g = lane >> 4;
  const T* wh = reinterpret_cast<const T*>(lds + S::FLOATS);
  float h[S::HB][4];
  fwd_layer_t<T, S::INB, S::HB>(wh + S::W0, S::LD0, lds + S::B0, xb, h);
#pragma unroll
  for (int k = 1; k < NH; ++k) {
    float h2[S::HB][4];
    fwd_layer_t<T, S::HB, S::HB>(wh + S::WK + (k - 1) * H * S::LDH, S::LDH,
                                 lds + S::BK + (k - 1) * H, h, h2);
#pragma unroll
    for (int a = 0; a < S::HB; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) h[a][i] = h2[a][i];
  }
  float y = 0.0f;
#pragma unroll
  for (int a = 0; a < S::HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) y += lds[S::WOUT + 16 * a + 4 * g + i] * h[a][i];
  return sum_groups(y) + lds[S::BOUT];
}

// Backward of one block given dy (per sample column, 0 for padding samples),
// the block input xb (B layout), its transposed copy in xtile (per-wave LDS,
// [INP][17], written by the caller) and the hidden activations.  Accumulates
// the parameter gradients into gr and returns dx (C layout) in dx.
template <int INP, int H, int NH>
__device__ __forceinline__ void mlp_block_bwd(const float* lds, float* scratch,
                                              const float (&hs)[NH][H / 16][4], float dy,
                                              MlpGrad<INP, H, NH>& gr, float (&dx)[INP / 16][4]) {
  using S = MlpShape<INP, H, NH>;
  const int lane = threadIdx.x & 63, g = lane >> 4;
  float* dtile = scratch;
  float* htile = scratch + S::TILE;
  float delta[S::HB][4];
  // Output layer: y = wout . h_{NH-1} + bout.
#pragma unroll
  for (int a = 0; a < S::HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float h = hs[NH - 1][a][i];
      gr.dwout[a][i] += dy * h;
      delta[a][i] = (h > 0.0f) ? lds[S::WOUT + 16 * a + 4 * g + i] * dy : 0.0f;
    }
  if (g == 0) gr.dbout += dy;
  // Hidden-to-hidden layers, last to first.
#pragma unroll
  for (int k = NH - 1; k >= 1; --k) {
    const float* wk = lds + S::WK + (k - 1) * S::WKSTRIDE;
#pragma unroll
    for (int a = 0; a < S::HB; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) gr.db[k][a][i] += delta[a][i];
    wave_lds_fence();
    tile_store<S::HB>(dtile, delta);
    tile_store<S::HB>(htile, hs[k - 1]);
    wave_lds_fence();
    dw_accumulate<S::HB, S::HB>(dtile, htile, gr.dwk[k - 1]);
    float dprev[S::HB][4];
    bwd_data<S::HB, S::HB>(wk, S::LDH, delta, dprev);
#pragma unroll
    for (int a = 0; a < S::HB; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) delta[a][i] = (hs[k - 1][a][i] > 0.0f) ? dprev[a][i] : 0.0f;
  }
  // First layer: input x (its transposed tile was written to htile by the caller
  // via mlp_stage_input), weights W0.
#pragma unroll
  for (int a = 0; a < S::HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) gr.db[0][a][i] += delta[a][i];
  wave_lds_fence();
  tile_store<S::HB>(dtile, delta);
  wave_lds_fence();
  dw_accumulate<S::HB, S::INB>(dtile, scratch + 2 * S::TILE, gr.dw0);
  bwd_data<S::HB, S::INB>(lds + S::W0, S::LD0, delta, dx);
  wave_lds_fence();
}

// Store the block input transposed into the per-wave input tile (used by the
// first-layer weight gradient).
template <int INP, int H, int NH>
__device__ __forceinline__ void mlp_stage_input(float* scratch, const float (&xb)[INP / 16][4]) {
  using S = MlpShape<INP, H, NH>;
  wave_lds_fence();
  tile_store<S::INB>(scratch + 2 * S::TILE, xb);
  wave_lds_fence();
}

// Per-wave scratch floats: delta tile, hidden tile, input tile.
template <int INP, int H, int NH>
constexpr int mlp_wave_scratch() {
  using S = MlpShape<INP, H, NH>;
  return 2 * S::TILE + INP * 17;
}

// Reduce the per-lane sample partials and write this wave's gradient into
// part (packed parameter layout, length P).
template <int INP, int H, int NH>
__device__ void mlp_write_partial(const MlpGrad<INP, H, NH>& gr, int in_w, float* part) {
  using S = MlpShape<INP, H, NH>;
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  // W0 [H][in_w]
#pragma unroll
  for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
    for (int ib = 0; ib < S::INB; ++ib)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 16 * ob + 4 * g + i, c = 16 * ib + n;
        if (c < in_w) part[o * in_w + c] = gr.dw0[ob][ib][i];
      }
  float* p = part + H * in_w;
#pragma unroll
  for (int a = 0; a < S::HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float v = sum16(gr.db[0][a][i]);
      if (n == 0) p[16 * a + 4 * g + i] = v;
    }
  p += H;
#pragma unroll
  for (int k = 1; k < NH; ++k) {
#pragma unroll
    for (int ob = 0; ob < S::HB; ++ob)
#pragma unroll
      for (int ib = 0; ib < S::HB; ++ib)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          p[(16 * ob + 4 * g + i) * H + 16 * ib + n] = gr.dwk[k - 1][ob][ib][i];
    p += H * H;
#pragma unroll
    for (int a = 0; a < S::HB; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = sum16(gr.db[k][a][i]);
        if (n == 0) p[16 * a + 4 * g + i] = v;
      }
    p += H;
  }
#pragma unroll
  for (int a = 0; a < S::HB; ++a)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float v = sum16(gr.dwout[a][i]);
      if (n == 0) p[16 * a + 4 * g + i] = v;
    }
  const float bo = sum16(gr.dbout);
  if (lane == 0) p[H] = bo;
}

}  // namespace fh
