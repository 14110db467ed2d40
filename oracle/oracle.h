/*
 * F-Hash FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct reference of what the F-Hash hot path
 * computes.  It is called only by the test-suite, by the smoke check and by
 * the CPU-baseline leg of the benchmark; the product path never links it.
 * It shares no source, header, table or helper with the HIP library.
 *
 * Conventions
 *   - A sample position is (x, y, z, t) in [0,1]^4 (FP32).  Level vertex v of
 *     a dimension with R vertices sits at v/(R-1); voxel i of a dimension with
 *     S samples sits at i/(S-1).
 *   - Levels are numbered 0 = coarsest.  res[l][0..3] = vertex counts (x,y,z,t).
 *   - Vertex linearisation of a level (Sec. 3.2.3, the F-Hash equation):
 *       lin = ((t*Rz + z)*Ry + y)*Rx + x
 *   - Embedding table rows are slots; row s holds F values.  Level l owns the
 *     slot range [slot_offset[l], slot_offset[l+1]).
 *   - slot maps: for level l, map[vtx_offset[l] + lin] = slot within the level
 *     (0-based, in linearisation order) or -1 for an inactive vertex.
 */
#ifndef FHASH_ORACLE_H
#define FHASH_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LEVELS 32

typedef struct {
  int32_t n_levels;
  int32_t n_features;
  int64_t res[OR_MAX_LEVELS][4];
  int64_t slot_offset[OR_MAX_LEVELS + 1];  /* global first slot of each level */
  int64_t vtx_offset[OR_MAX_LEVELS + 1];   /* first entry of each level in a slot map */
  const int64_t* slot_map;                 /* NULL: every vertex active (dense box) */
} or_grid;

/* ---- resolution policies ------------------------------------------------ */
int or_fold_num_levels(int64_t S, int64_t f);
int or_fold_resolutions(const int64_t S[4], int64_t f, int max_levels, int64_t* res_out);
int or_geometric_resolutions(int L, int64_t rmin_s, int64_t rmax_s, int64_t rmin_t,
                             int64_t rmax_t, const int64_t S[4], int64_t* res_out);

/* ---- active set and index ----------------------------------------------- */
void or_voxel_cells(int64_t i, int64_t S, int64_t R, int64_t* c_lo, int64_t* c_hi);
int64_t or_level_vertices(const int64_t res[4]);
int64_t or_level_cells(const int64_t res[4]);
void or_cell_activity(const int64_t res[4], const uint8_t* mask, const int64_t S[4],
                      uint8_t* cell_active);
int64_t or_build_level_slots(const int64_t res[4], const uint8_t* mask, const int64_t S[4],
                             int64_t* slot_map_level);
int64_t or_build_level_slots_bricks(const int64_t res[4], const uint8_t* mask,
                                    const int64_t S[4], int64_t* slot_map_level);

int or_cell_active_bits(const int64_t res[4], const uint64_t* bits, const int64_t S[4],
                        const int64_t c[4]);
int or_vertex_active_bits(const int64_t res[4], const uint64_t* bits, const int64_t S[4],
                          const int64_t v[4]);

/* ---- cell location and encoding ---------------------------------------- */
void or_locate(float p, int64_t R, int64_t* cell, double* frac);
int64_t or_vertex_slot(const or_grid* g, int l, const int64_t v[4]);
void or_corners(const or_grid* g, const float* pos, int64_t n, int64_t* slots, double* w);
void or_encode_fwd(const or_grid* g, const float* pos, int64_t n, const double* table,
                   double* enc, double* mag);
void or_encode_bwd(const or_grid* g, const float* pos, int64_t n, const double* d_enc,
                   double* d_table, double* mag);

/* ---- MLP decoder ---------------------------------------------------------- */
int64_t or_mlp_num_params(int n_layers, const int32_t* width);
void or_mlp_fwd(int n_layers, const int32_t* width, const double* params, const double* x,
                int64_t n, double* y, double* acts, const double* x_mag, double* y_mag);
void or_mlp_bwd(int n_layers, const int32_t* width, const double* params, const double* acts,
                const double* dy, const double* dy_mag, const double* x_mag, int64_t n,
                double* d_params, double* dx, double* dp_mag, double* dx_mag);

/* ---- loss, optimiser, reductions ---------------------------------------- */
double or_mse(const double* y, const double* v, int64_t n, double* dy);
void or_adam(double* p, const double* g, double* m, double* v, int64_t n, double lr,
             double beta1, double beta2, double eps, int64_t step);
double or_psnr(double mse);

/* ---- counter-based RNG and training sampler ----------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_sample_ids(uint64_t seed, uint64_t step, int64_t n, uint64_t M, uint64_t* ids);
void or_voxel_positions(const uint64_t* lin, int64_t n, const int64_t S[4], float* pos);
void or_sample_batch(uint64_t seed, uint64_t step, int64_t n, const uint64_t* coreset,
                     uint64_t M, const int64_t S[4], const float* field, float* pos,
                     float* target);

/* ---- rendering --------------------------------------------------------- */
int or_occupied(const uint8_t* mask, const int64_t S[4], const float p[3], float t);
int64_t or_render(const or_grid* g, const double* table, int n_layers, const int32_t* width,
                  const double* params, const uint8_t* mask, const int64_t S[4], const float* cam,
                  float t, float t01, const float* tf, int W, int H, float ds, float alpha_stop,
                  int max_steps, double* rgba, uint8_t* amb, double* pix);

#ifdef __cplusplus
}
#endif
#endif
