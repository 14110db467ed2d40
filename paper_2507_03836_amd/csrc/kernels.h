// Host launchers of the HIP kernels (internal to libfhash).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace fh {

// index.hip
int64_t index_dir_words(const fhash_grid_desc* g, int l);
size_t index_workspace_bytes(const fhash_grid_desc* g, const int64_t* dims);
hipError_t launch_build_index(const fhash_grid_desc* g, const uint64_t* mask, const int64_t* dims,
                              ulonglong2* dir, const int64_t* dir_off, void* ws,
                              uint64_t* counts_host, hipStream_t st);

// encode.hip
hipError_t launch_encode_fwd(const GridDev& g, const float* pos, int64_t n, const void* table,
                             fhash_dtype dt, float* enc, hipStream_t st);
hipError_t launch_encode_bwd(const GridDev& g, const float* pos, int64_t n, const float* d_enc,
                             float* d_table, hipStream_t st);
hipError_t launch_corner_rows(const GridDev& g, const float* pos, int64_t n, int64_t* out_dir,
                              int64_t* out_slot, hipStream_t st);

// mlp.hip
bool mlp_supported(int in_w, int H, int NH);
size_t mlp_bwd_ws_bytes(int64_t n, int64_t P);
hipError_t launch_mlp_fwd(int in_w, int H, int NH, const float* params, const float* x, int64_t n,
                          float* y, hipStream_t st);
hipError_t launch_mlp_bwd(int in_w, int H, int NH, const float* params, const float* x,
                          const float* dy, int64_t n, float* d_params, float* dx, void* ws,
                          int64_t P, hipStream_t st);

// fused*.hip.  ddt: decoder arithmetic (FHASH_F32: FP32 MFMA; FHASH_F16 /
// FHASH_BF16: 16-bit MFMA with FP32 accumulation; 16-bit backward and BF16
// forward for two features per level only).
bool fused_supported(int F, int in_w, int H, int NH);
size_t fused_ws_bytes(int64_t n, int64_t P);
int64_t fused_partials(int64_t n);
hipError_t launch_fused_fwd(const GridDev& g, int H, int NH, const float* pos, int64_t n,
                            const void* table, fhash_dtype tdt, const float* params, float* y,
                            hipStream_t st);
hipError_t launch_fused_fwd16(const GridDev& g, int H, int NH, fhash_dtype ddt, const float* pos,
                              int64_t n, const void* table, fhash_dtype tdt, const float* params,
                              float* y, hipStream_t st);
hipError_t launch_fused_bwd(const GridDev& g, int H, int NH, fhash_dtype ddt, const float* pos,
                            int64_t n, const void* table, fhash_dtype tdt, const float* params,
                            const float* dy, float* d_table, float* d_params, void* ws, int64_t P,
                            hipStream_t st);
hipError_t launch_fused_bwd16(const GridDev& g, int H, int NH, fhash_dtype ddt, const float* pos,
                              int64_t n, const void* table, fhash_dtype tdt, const float* params,
                              const float* dy, float* d_table, float* d_params, void* ws,
                              int64_t P, hipStream_t st);
hipError_t launch_fused_train(const GridDev& g, int H, int NH, fhash_dtype ddt, const float* pos,
                              const float* target, int64_t n, const void* table, fhash_dtype tdt,
                              const float* params, float loss_scale, float* d_table,
                              float* d_params, double* loss_sum, void* ws, int64_t P,
                              hipStream_t st);
hipError_t launch_fused_train16(const GridDev& g, int H, int NH, fhash_dtype ddt,
                                const float* pos, const float* target, int64_t n,
                                const void* table, fhash_dtype tdt, const float* params,
                                float loss_scale, float* d_table, float* d_params,
                                double* loss_sum, void* ws, int64_t P, hipStream_t st);

// static_ws.hip: library-owned scratch for the entry points that allocate nothing
size_t static_scratch_bytes();
hipError_t static_scratch(void** ptr);

// optim.hip
// Adam over the parameters [first, first + n) of a vector: p, g, m, v and
// shadow point at the vector's start (o->moments layout).
hipError_t launch_adam(const fhash_adam_desc* o, float* p, float* g, float* m, float* v,
                       void* shadow, fhash_dtype sdt, int64_t n, int64_t first,
                       const int32_t* found_inf, const fhash_touch* touch, hipStream_t st);
// coarse.hip: the LDS scatter of levels 0 .. g.coarse - 1 from g.dxc
hipError_t launch_coarse_scatter(const GridDev& g, const float* pos, int64_t n, float* d_table,
                                 hipStream_t st);
hipError_t launch_reduce_partials(const float* part, int64_t nwav, int64_t P, float* d_params,
                                  hipStream_t st);
hipError_t launch_check_finite(const float* g, int64_t n, int32_t* found, hipStream_t st);
hipError_t launch_cast(const float* src, void* dst, fhash_dtype dt, int64_t n, hipStream_t st);
hipError_t launch_sq_err(const float* y, const float* v, int64_t n, double* sum, hipStream_t st);
hipError_t launch_mse_grad(const float* y, const float* v, int64_t n, float coef, float* dy,
                           double* sum, hipStream_t st);

// lazy.hip: deferred Adam over a table range
int64_t lazy_num_segments(int64_t range_floats);
size_t lazy_ws_bytes(int64_t range_floats, int64_t max_steps);
hipError_t launch_lazy_init(const fhash_lazy* lz, hipStream_t st);
hipError_t launch_lazy_prepare(const GridDev& g, int l0, int l1, const float* pos, int64_t n,
                               const fhash_lazy* lz, float* p, float* gr, float* m, float* v,
                               void* shadow, fhash_dtype sdt, uint32_t phases, hipStream_t st);
hipError_t lazy_read_stats(const fhash_lazy* lz, int64_t* out, hipStream_t st);
hipError_t launch_lazy_step(const fhash_adam_desc* o, const fhash_lazy* lz,
                            const int32_t* found_inf, hipStream_t st);
hipError_t launch_lazy_flush(const fhash_lazy* lz, float* p, float* gr, float* m, float* v,
                             void* shadow, fhash_dtype sdt, hipStream_t st);

// sampler.hip
hipError_t launch_sample(uint64_t seed, uint64_t step, int64_t n, const uint64_t* coreset,
                         uint64_t M, const int64_t* dims, const float* field,
                         const float* frame_t, const int32_t* box, float* pos, float* target,
                         hipStream_t st);

// sort.hip
size_t sort_ws_bytes(int64_t n);
hipError_t launch_sort_samples(float* pos, float* target, int64_t n, void* ws, hipStream_t st);

// render.hip
size_t render_ws_bytes(int64_t NR, const int64_t* dims);
// mask: the voxel mask rows (brick_grid false) or the occupancy grid of
// fhash_occupancy_grid (brick_grid true).
hipError_t launch_render_begin(const fhash_view* v, int W, int H, const uint64_t* mask,
                               bool brick_grid, const int64_t* dims, float t, void* ws,
                               int32_t* n_alive_host, float* rgba, hipStream_t st);
// One request of a batched march / composite (host view of its render state).
struct RenderBatch {
  void* ws;
  int32_t W, H, cur, n_alive, pace;
  float t01;
  const int64_t* dims;
  const float* tf;
  float* rgba;
};
hipError_t launch_render_march_batch(const RenderBatch* b, int32_t n, float ds, int32_t max_steps,
                                     float* pos, int64_t out_base, int32_t* counts_dev,
                                     int32_t* counts_host, hipStream_t st);
hipError_t launch_render_composite_batch(const RenderBatch* b, int32_t n, const float* y,
                                         float alpha_stop, int32_t* counts_dev,
                                         int32_t* counts_host, hipStream_t st);
hipError_t launch_render_march(void* ws, int W, int H, const int64_t* dims, float t01, float ds,
                               int32_t max_steps, int32_t pace, int cur, int32_t n_alive,
                               float* pos_out, int32_t* n_samples_host, hipStream_t st);
hipError_t launch_render_composite(void* ws, int W, int H, int cur, int32_t n_alive,
                                   const float* y, const float* tf, float alpha_stop, float* rgba,
                                   int32_t* n_alive_host, hipStream_t st);

// coreset.hip: feature extraction, dilation, boxes, occupancy, coreset list
int64_t mask_words(const int64_t* dims);
size_t feature_ws_bytes(const int64_t* dims, int kind);
hipError_t launch_feature_mask(const float* field, const int64_t* dims, int kind, float lo,
                               float hi, uint64_t* bits, void* ws, hipStream_t st);
hipError_t launch_dilate_mask(const uint64_t* in, const int64_t* dims, int r, uint64_t* out,
                              hipStream_t st);
hipError_t launch_feature_boxes(const uint64_t* bits, const int64_t* dims, int32_t* box,
                                hipStream_t st);
int64_t occupancy_words(const int64_t* dims);
hipError_t launch_occupancy_morton(const uint64_t* bits, const int64_t* dims, uint64_t* occ,
                                   hipStream_t st);
size_t coreset_ws_bytes(const int64_t* dims);
size_t coreset_frames_ws_bytes(const int64_t* dims);
hipError_t launch_coreset_frames(const uint64_t* bits, const int64_t* dims, const int32_t* frames,
                                 int32_t n_frames, void* ws, uint64_t* ids, int64_t capacity,
                                 int64_t* count, hipStream_t st);
hipError_t launch_coreset(const uint64_t* bits, const int64_t* dims, void* ws, uint64_t* ids,
                          int64_t capacity, int64_t* count, hipStream_t st);

}  // namespace fh
