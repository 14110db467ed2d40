/*
 * F-Hash FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Every routine is the plain definition of one step of the method, written as
 * loops in the order the paper states it.  No blocking, fusion or reordering.
 * Floating-point work is FP64 except where FP32 decides an integer (cell
 * location, sample positions); there both sides use the same FP32 operation.
 * Build without -ffast-math (the FP32 operations must be IEEE single ops).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ========================================================================= */
/* Resolution policies                                                       */
/* ========================================================================= */

/* Number of fold levels of one dimension: L_d = ceil(log_f S_d)  (Sec. 3.2.1,
 * level-count equation).  Computed in integers: the smallest L with f^L >= S. */
int or_fold_num_levels(int64_t S, int64_t f) {
  int L = 0;
  int64_t p = 1;
  while (p < S) {
    p *= f;
    ++L;
  }
  return L;
}

/* Fold policy of Sec. 3.2.1 (spatial) and Sec. 3.2.2 (temporal).
 * Level 1 is the native FBB resolution; each further level divides the
 * previous one by f (rounded up) while it is above f, and is padded with the
 * minimal resolution 2 otherwise.  The level count is L_s, the maximum of the
 * three spatial level counts; the time axis follows the same recursion over
 * the same L_s levels.  res_out[(l-1)*4 + d] holds paper level l (l = 1 is the
 * finest).  Returns L_s, or -1 if it exceeds max_levels. */
int or_fold_resolutions(const int64_t S[4], int64_t f, int max_levels, int64_t* res_out) {
  int Ls = 0;
  for (int d = 0; d < 3; ++d) {
    int Ld = or_fold_num_levels(S[d], f);
    if (Ld > Ls) Ls = Ld;
  }
  if (Ls > max_levels) return -1;
  for (int d = 0; d < 4; ++d) {
    int64_t r = S[d];
    for (int l = 1; l <= Ls; ++l) {
      if (l > 1) r = (r > f) ? (r + f - 1) / f : 2;
      res_out[(l - 1) * 4 + d] = r;
    }
  }
  return Ls;
}

/* Geometric level policy: R_l = floor(Rmin * b^l + 0.5), b = (Rmax/Rmin)^(1/(L-1)),
 * clamped to [2, S_d] (the native resolution is the upper bound, Sec. 3.2.1).
 * res_out[l*4 + d], l = 0 is the coarsest level. */
int or_geometric_resolutions(int L, int64_t rmin_s, int64_t rmax_s, int64_t rmin_t,
                             int64_t rmax_t, const int64_t S[4], int64_t* res_out) {
  if (L < 1 || L > OR_MAX_LEVELS) return -1;
  for (int l = 0; l < L; ++l) {
    for (int d = 0; d < 4; ++d) {
      double rmin = (d < 3) ? (double)rmin_s : (double)rmin_t;
      double rmax = (d < 3) ? (double)rmax_s : (double)rmax_t;
      double r = rmin;
      if (L > 1) {
        double b = pow(rmax / rmin, 1.0 / (double)(L - 1));
        r = rmin * pow(b, (double)l);
      }
      int64_t R = (int64_t)floor(r + 0.5);
      if (R > S[d]) R = S[d];
      if (R < 2) R = 2;
      res_out[l * 4 + d] = R;
    }
  }
  return L;
}

/* ========================================================================= */
/* Active set and index                                                      */
/* ========================================================================= */

/* Cells of a level that contain voxel i of a dimension.  The voxel sits at
 * i/(S-1); cell c is the closed interval [c/(R-1), (c+1)/(R-1)].  With
 * q = i(R-1) and d = S-1 the voxel lies inside cell floor(q/d), and when q/d is
 * an integer k (the voxel sits on level vertex k) it lies on the shared face of
 * cells k-1 and k.  Integer arithmetic only. */
void or_voxel_cells(int64_t i, int64_t S, int64_t R, int64_t* c_lo, int64_t* c_hi) {
  int64_t q = i * (R - 1);
  int64_t d = S - 1;
  int64_t k = q / d;
  if (q % d == 0) {
    *c_lo = k - 1;
    *c_hi = k;
  } else {
    *c_lo = k;
    *c_hi = k;
  }
  if (*c_lo < 0) *c_lo = 0;
  if (*c_hi > R - 2) *c_hi = R - 2;
}

int64_t or_level_vertices(const int64_t res[4]) { return res[0] * res[1] * res[2] * res[3]; }

int64_t or_level_cells(const int64_t res[4]) {
  return (res[0] - 1) * (res[1] - 1) * (res[2] - 1) * (res[3] - 1);
}

/* A 4D cell of the level is active iff its closed box contains a masked voxel
 * (the feature region of Sec. 3.1 restricted to the level's cells).  mask is
 * one byte per voxel, [T][Sz][Sy][Sx], x fastest.  cell_active is one byte per
 * cell, [Rt-1][Rz-1][Ry-1][Rx-1], x fastest. */
void or_cell_activity(const int64_t res[4], const uint8_t* mask, const int64_t S[4],
                      uint8_t* cell_active) {
  const int64_t cx = res[0] - 1, cy = res[1] - 1, cz = res[2] - 1;
  memset(cell_active, 0, (size_t)or_level_cells(res));
  for (int64_t n = 0; n < S[3]; ++n)
    for (int64_t k = 0; k < S[2]; ++k)
      for (int64_t j = 0; j < S[1]; ++j)
        for (int64_t i = 0; i < S[0]; ++i) {
          if (!mask[((n * S[2] + k) * S[1] + j) * S[0] + i]) continue;
          int64_t lo[4], hi[4];
          or_voxel_cells(i, S[0], res[0], &lo[0], &hi[0]);
          or_voxel_cells(j, S[1], res[1], &lo[1], &hi[1]);
          or_voxel_cells(k, S[2], res[2], &lo[2], &hi[2]);
          or_voxel_cells(n, S[3], res[3], &lo[3], &hi[3]);
          for (int64_t ct = lo[3]; ct <= hi[3]; ++ct)
            for (int64_t cz2 = lo[2]; cz2 <= hi[2]; ++cz2)
              for (int64_t cy2 = lo[1]; cy2 <= hi[1]; ++cy2)
                for (int64_t cx2 = lo[0]; cx2 <= hi[0]; ++cx2)
                  cell_active[((ct * cz + cz2) * cy + cy2) * cx + cx2] = 1;
        }
}

/* Slot map of one level.  Embeddings live at cell corners (Sec. 3.2.4, step 3),
 * so a vertex is active iff it is one of the 16 corners of an active cell.  The
 * slot of an active vertex is its rank among the active vertices in the
 * linearisation order of the F-Hash equation (Sec. 3.2.3):
 *   lin = ((t*Rz + z)*Ry + y)*Rx + x.
 * The map is therefore a minimal perfect hash of the active set.  mask == NULL
 * makes every vertex active, which reduces the rank to the F-Hash equation
 * itself.  slot_map_level has one entry per vertex (-1 = inactive).
 * Returns the number of active vertices. */
int64_t or_build_level_slots(const int64_t res[4], const uint8_t* mask, const int64_t S[4],
                             int64_t* slot_map_level) {
  const int64_t Rx = res[0], Ry = res[1], Rz = res[2], Rt = res[3];
  const int64_t nv = or_level_vertices(res);
  if (mask == NULL) {
    for (int64_t v = 0; v < nv; ++v) slot_map_level[v] = v;
    return nv;
  }
  uint8_t* cell = (uint8_t*)malloc((size_t)or_level_cells(res));
  uint8_t* vert = (uint8_t*)calloc((size_t)nv, 1);
  or_cell_activity(res, mask, S, cell);
  for (int64_t ct = 0; ct < Rt - 1; ++ct)
    for (int64_t cz = 0; cz < Rz - 1; ++cz)
      for (int64_t cy = 0; cy < Ry - 1; ++cy)
        for (int64_t cx = 0; cx < Rx - 1; ++cx) {
          if (!cell[((ct * (Rz - 1) + cz) * (Ry - 1) + cy) * (Rx - 1) + cx]) continue;
          for (int c = 0; c < 16; ++c) {
            int64_t x = cx + (c & 1), y = cy + ((c >> 1) & 1);
            int64_t z = cz + ((c >> 2) & 1), t = ct + ((c >> 3) & 1);
            vert[((t * Rz + z) * Ry + y) * Rx + x] = 1;
          }
        }
  int64_t count = 0;
  for (int64_t v = 0; v < nv; ++v) slot_map_level[v] = vert[v] ? count++ : -1;
  free(cell);
  free(vert);
  return count;
}

/* The same active set ranked in another linearisation with preserved locality
 * (Sec. 3.2.3 allows linearisations other than the F-Hash equation's): the
 * level is cut into bricks of 2 x 2 x 2 x 2 vertices, brick (bx, by, bz, bt) =
 * (x/2, y/2, z/2, t/2); bricks are ordered like vertices in the F-Hash
 * equation (bx fastest, then by, bz, bt) and the vertices inside a brick by
 *   inner = (x mod 2) + 2 (y mod 2) + 4 (z mod 2) + 8 (t mod 2).
 * Bricks at an odd upper edge are partial (their missing vertices do not
 * exist and take no slot).  The slot of an active vertex is its rank among the
 * active vertices in this order; the map has the same form as above (indexed
 * by the F-Hash linear vertex id).  mask == NULL makes every vertex active.
 * Returns the number of active vertices. */
int64_t or_build_level_slots_bricks(const int64_t res[4], const uint8_t* mask,
                                    const int64_t S[4], int64_t* slot_map_level) {
  const int64_t R[4] = {res[0], res[1], res[2], res[3]};
  const int64_t nv = or_level_vertices(res);
  /* activity as in the F-Hash order (a map entry >= 0 marks an active vertex) */
  int64_t count = or_build_level_slots(res, mask, S, slot_map_level);
  int64_t B[4];
  for (int d = 0; d < 4; ++d) B[d] = (R[d] + 1) / 2;
  int64_t next = 0;
  for (int64_t bt = 0; bt < B[3]; ++bt)
    for (int64_t bz = 0; bz < B[2]; ++bz)
      for (int64_t by = 0; by < B[1]; ++by)
        for (int64_t bx = 0; bx < B[0]; ++bx)
          for (int inner = 0; inner < 16; ++inner) {
            const int64_t x = 2 * bx + (inner & 1), y = 2 * by + ((inner >> 1) & 1);
            const int64_t z = 2 * bz + ((inner >> 2) & 1), t = 2 * bt + ((inner >> 3) & 1);
            if (x >= R[0] || y >= R[1] || z >= R[2] || t >= R[3]) continue;
            const int64_t lin = ((t * R[2] + z) * R[1] + y) * R[0] + x;
            if (slot_map_level[lin] >= 0) slot_map_level[lin] = next++;
          }
  (void)nv;
  return next == count ? count : -1;
}

/* Activity of one vertex decided from a bit-packed mask, for volumes too large
 * for the whole-level enumeration above.  Same definitions: the vertex is
 * active iff one of the (up to 16) cells having it as a corner contains a
 * masked voxel in its closed box.  bits: rows of W = ceil(Sx/64) words,
 * [T][Sz][Sy][W], bit b of word w = voxel x = 64 w + b. */
static int voxel_in_cell(int64_t i, int64_t S, int64_t R, int64_t c) {
  int64_t lo, hi;
  or_voxel_cells(i, S, R, &lo, &hi);
  return lo <= c && c <= hi;
}

static int bit_set(const uint64_t* bits, const int64_t S[4], int64_t i, int64_t j, int64_t k,
                   int64_t n) {
  const int64_t W = (S[0] + 63) / 64;
  return (int)((bits[((n * S[2] + k) * S[1] + j) * W + i / 64] >> (i % 64)) & 1u);
}

int or_cell_active_bits(const int64_t res[4], const uint64_t* bits, const int64_t S[4],
                        const int64_t c[4]) {
  int64_t lo[4], hi[4];
  for (int d = 0; d < 4; ++d) {
    if (c[d] < 0 || c[d] > res[d] - 2) return 0;
    /* candidate voxels around the cell: i(R-1)/(S-1) within [c-1, c+2] */
    lo[d] = (c[d] - 1) * (S[d] - 1) / (res[d] - 1) - 1;
    hi[d] = (c[d] + 2) * (S[d] - 1) / (res[d] - 1) + 1;
    if (lo[d] < 0) lo[d] = 0;
    if (hi[d] > S[d] - 1) hi[d] = S[d] - 1;
  }
  for (int64_t n = lo[3]; n <= hi[3]; ++n) {
    if (!voxel_in_cell(n, S[3], res[3], c[3])) continue;
    for (int64_t k = lo[2]; k <= hi[2]; ++k) {
      if (!voxel_in_cell(k, S[2], res[2], c[2])) continue;
      for (int64_t j = lo[1]; j <= hi[1]; ++j) {
        if (!voxel_in_cell(j, S[1], res[1], c[1])) continue;
        for (int64_t i = lo[0]; i <= hi[0]; ++i) {
          if (!voxel_in_cell(i, S[0], res[0], c[0])) continue;
          if (bit_set(bits, S, i, j, k, n)) return 1;
        }
      }
    }
  }
  return 0;
}

int or_vertex_active_bits(const int64_t res[4], const uint64_t* bits, const int64_t S[4],
                          const int64_t v[4]) {
  for (int m = 0; m < 16; ++m) {
    int64_t c[4];
    for (int d = 0; d < 4; ++d) c[d] = v[d] - ((m >> d) & 1);
    if (or_cell_active_bits(res, bits, S, c)) return 1;
  }
  return 0;
}

/* ========================================================================= */
/* Cell location and the input encoding (Sec. 3.2.4)                        */
/* ========================================================================= */

/* Steps 1 and 2 of the encoding: the cell of a level that contains coordinate
 * p, and the fractional position inside it.  Positions outside [0,1] (and NaN)
 * are clamped.  The cell is decided in FP32 with a single multiply, exactly as
 * the GPU does, so both sides agree on the integer; the fraction u - i is exact
 * in FP32 and is promoted to FP64. */
void or_locate(float p, int64_t R, int64_t* cell, double* frac) {
  if (!(p >= 0.0f)) p = 0.0f;
  if (p > 1.0f) p = 1.0f;
  float u = p * (float)(R - 1);
  int64_t i = (int64_t)floorf(u);
  if (i > R - 2) i = R - 2;
  *cell = i;
  *frac = (double)(u - (float)i);
}

/* Global slot of vertex v = (x,y,z,t) of level l, or -1 if the vertex is not
 * active.  Dense box: the F-Hash equation plus the level's table offset. */
int64_t or_vertex_slot(const or_grid* g, int l, const int64_t v[4]) {
  const int64_t* r = g->res[l];
  int64_t lin = ((v[3] * r[2] + v[2]) * r[1] + v[1]) * r[0] + v[0];
  if (g->slot_map == NULL) return g->slot_offset[l] + lin;
  int64_t s = g->slot_map[g->vtx_offset[l] + lin];
  return s < 0 ? -1 : g->slot_offset[l] + s;
}

/* The 16 corner slots (8 spatial corners at t_prev and t_next, step 3) and
 * their quadrilinear weights (step 4) of every sample and level.
 * Corner c has offsets dx = c&1, dy = (c>>1)&1, dz = (c>>2)&1, dt = (c>>3)&1.
 * slots/w are [n][L][16]. */
void or_corners(const or_grid* g, const float* pos, int64_t n, int64_t* slots, double* w) {
  const int L = g->n_levels;
  for (int64_t s = 0; s < n; ++s)
    for (int l = 0; l < L; ++l) {
      int64_t cell[4];
      double f[4];
      for (int d = 0; d < 4; ++d) or_locate(pos[s * 4 + d], g->res[l][d], &cell[d], &f[d]);
      for (int c = 0; c < 16; ++c) {
        int64_t v[4];
        double wc = 1.0;
        for (int d = 0; d < 4; ++d) {
          int b = (c >> d) & 1;
          v[d] = cell[d] + b;
          wc *= b ? f[d] : (1.0 - f[d]);
        }
        slots[(s * L + l) * 16 + c] = or_vertex_slot(g, l, v);
        w[(s * L + l) * 16 + c] = wc;
      }
    }
}

/* Encoding forward.  For each level: trilinear interpolation of the 8 corner
 * embeddings at t_prev and at t_next (Eqs. 10 and 11), then linear
 * interpolation between the two in time (Eq. 12, read as a linear blend with
 * the in-cell time fraction).  Inactive corners contribute nothing.  The
 * levels are concatenated: enc is [n][L*F], level-major, feature-minor.
 * mag (optional) receives the sum of the magnitudes of the 16 terms, the
 * scale of the FP32 rounding error of any evaluation order. */
void or_encode_fwd(const or_grid* g, const float* pos, int64_t n, const double* table,
                   double* enc, double* mag) {
  const int L = g->n_levels, F = g->n_features;
  for (int64_t s = 0; s < n; ++s)
    for (int l = 0; l < L; ++l) {
      int64_t cell[4];
      double f[4];
      for (int d = 0; d < 4; ++d) or_locate(pos[s * 4 + d], g->res[l][d], &cell[d], &f[d]);
      for (int k = 0; k < F; ++k) {
        double V[2] = {0.0, 0.0}, M[2] = {0.0, 0.0};
        for (int dt = 0; dt < 2; ++dt)
          for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
              for (int dx = 0; dx < 2; ++dx) {
                int64_t v[4] = {cell[0] + dx, cell[1] + dy, cell[2] + dz, cell[3] + dt};
                int64_t slot = or_vertex_slot(g, l, v);
                if (slot < 0) continue;
                double wx = dx ? f[0] : 1.0 - f[0];
                double wy = dy ? f[1] : 1.0 - f[1];
                double wz = dz ? f[2] : 1.0 - f[2];
                double e = table[slot * F + k];
                V[dt] += e * wx * wy * wz;
                M[dt] += fabs(e * wx * wy * wz);
              }
        double tau = f[3];
        enc[s * L * F + l * F + k] = (1.0 - tau) * V[0] + tau * V[1];
        if (mag) mag[s * L * F + l * F + k] = (1.0 - tau) * M[0] + tau * M[1];
      }
    }
}

/* Adjoint of the encoding (linear in the tables):
 *   dL/dE[slot][k] += w_c * dL/denc[s][l*F + k]   for every corner c with that slot.
 * d_table (and mag, the magnitude sum of the terms) are accumulated into. */
void or_encode_bwd(const or_grid* g, const float* pos, int64_t n, const double* d_enc,
                   double* d_table, double* mag) {
  const int L = g->n_levels, F = g->n_features;
  for (int64_t s = 0; s < n; ++s)
    for (int l = 0; l < L; ++l) {
      int64_t cell[4];
      double f[4];
      for (int d = 0; d < 4; ++d) or_locate(pos[s * 4 + d], g->res[l][d], &cell[d], &f[d]);
      for (int c = 0; c < 16; ++c) {
        int64_t v[4];
        double wc = 1.0;
        for (int d = 0; d < 4; ++d) {
          int b = (c >> d) & 1;
          v[d] = cell[d] + b;
          wc *= b ? f[d] : (1.0 - f[d]);
        }
        int64_t slot = or_vertex_slot(g, l, v);
        if (slot < 0) continue;
        for (int k = 0; k < F; ++k) {
          double term = wc * d_enc[s * L * F + l * F + k];
          d_table[slot * F + k] += term;
          if (mag) mag[slot * F + k] += fabs(term);
        }
      }
    }
}

/* ========================================================================= */
/* MLP decoder: ReLU hidden layers, linear output, biases on                 */
/* ========================================================================= */

/* Parameters are packed per layer k: W_k [width[k+1]][width[k]] row-major,
 * then b_k [width[k+1]]. */
int64_t or_mlp_num_params(int n_layers, const int32_t* width) {
  int64_t p = 0;
  for (int k = 0; k < n_layers; ++k) p += (int64_t)width[k + 1] * width[k] + width[k + 1];
  return p;
}

static int64_t act_offset(int layer, const int32_t* width, int64_t n) {
  int64_t o = 0;
  for (int j = 0; j < layer; ++j) o += n * width[j];
  return o;
}

/* Forward: a_{k+1} = ReLU(W_k a_k + b_k) for hidden layers, y = W a + b last.
 * acts (optional) receives a_0..a_{n_layers} concatenated, each [n][width].
 * y_mag (optional) receives the running magnitude |W||a| + |b| through the
 * same ReLU pattern, started from x_mag (or |x| when x_mag is NULL). */
void or_mlp_fwd(int n_layers, const int32_t* width, const double* params, const double* x,
                int64_t n, double* y, double* acts, const double* x_mag, double* y_mag) {
  int wmax = 0;
  for (int k = 0; k <= n_layers; ++k)
    if (width[k] > wmax) wmax = width[k];
  double* a = (double*)malloc(sizeof(double) * wmax);
  double* b = (double*)malloc(sizeof(double) * wmax);
  double* am = (double*)malloc(sizeof(double) * wmax);
  double* bm = (double*)malloc(sizeof(double) * wmax);
  for (int64_t s = 0; s < n; ++s) {
    for (int i = 0; i < width[0]; ++i) {
      a[i] = x[s * width[0] + i];
      am[i] = x_mag ? x_mag[s * width[0] + i] : fabs(a[i]);
      if (acts) acts[s * width[0] + i] = a[i];
    }
    const double* P = params;
    for (int k = 0; k < n_layers; ++k) {
      const int in = width[k], out = width[k + 1];
      const double* W = P;
      const double* bias = P + (int64_t)out * in;
      for (int o = 0; o < out; ++o) {
        double acc = bias[o], accm = fabs(bias[o]);
        for (int i = 0; i < in; ++i) {
          acc += W[(int64_t)o * in + i] * a[i];
          accm += fabs(W[(int64_t)o * in + i]) * am[i];
        }
        if (k < n_layers - 1 && !(acc > 0.0)) {
          acc = 0.0;
          accm = 0.0;
        }
        b[o] = acc;
        bm[o] = accm;
      }
      for (int o = 0; o < out; ++o) {
        a[o] = b[o];
        am[o] = bm[o];
        if (acts) acts[act_offset(k + 1, width, n) + s * out + o] = a[o];
      }
      P += (int64_t)out * in + out;
    }
    for (int o = 0; o < width[n_layers]; ++o) {
      y[s * width[n_layers] + o] = a[o];
      if (y_mag) y_mag[s * width[n_layers] + o] = am[o];
    }
  }
  free(a);
  free(b);
  free(am);
  free(bm);
}

/* Backward (textbook reverse mode through the forward above), given the saved
 * activations of or_mlp_fwd:
 *   dW_k += delta_{k+1} a_k^T,  db_k += delta_{k+1},
 *   delta_k = (W_k^T delta_{k+1}) * [a_k > 0]  (hidden layers),  dx = W_0^T delta_1.
 * d_params is accumulated into; dx (optional) is written.
 * dp_mag / dx_mag (optional) receive the same recursion run on magnitudes
 * (|W|, |dy| or dy_mag, the running forward magnitude from x_mag or |x|): the
 * scale of the FP32 rounding error of the gradients. */
void or_mlp_bwd(int n_layers, const int32_t* width, const double* params, const double* acts,
                const double* dy, const double* dy_mag, const double* x_mag, int64_t n,
                double* d_params, double* dx, double* dp_mag, double* dx_mag) {
  int wmax = 0;
  for (int k = 0; k <= n_layers; ++k)
    if (width[k] > wmax) wmax = width[k];
  const double** Wk = (const double**)malloc(sizeof(double*) * n_layers);
  int64_t* poff = (int64_t*)malloc(sizeof(int64_t) * n_layers);
  {
    int64_t o = 0;
    for (int k = 0; k < n_layers; ++k) {
      poff[k] = o;
      Wk[k] = params + o;
      o += (int64_t)width[k + 1] * width[k] + width[k + 1];
    }
  }
  double* d = (double*)malloc(sizeof(double) * wmax);
  double* dn = (double*)malloc(sizeof(double) * wmax);
  double* dm = (double*)malloc(sizeof(double) * wmax);
  double* dnm = (double*)malloc(sizeof(double) * wmax);
  /* forward magnitudes per layer for this sample */
  double* fm = (double*)malloc(sizeof(double) * wmax * (n_layers + 1));
  for (int64_t s = 0; s < n; ++s) {
    /* running forward magnitude (needed only for the error scales) */
    for (int i = 0; i < width[0]; ++i) {
      double xv = acts[s * width[0] + i];
      fm[i] = x_mag ? x_mag[s * width[0] + i] : fabs(xv);
    }
    for (int k = 0; k < n_layers; ++k) {
      const int in = width[k], out = width[k + 1];
      const double* W = Wk[k];
      const double* bias = W + (int64_t)out * in;
      for (int o = 0; o < out; ++o) {
        double accm = fabs(bias[o]);
        for (int i = 0; i < in; ++i) accm += fabs(W[(int64_t)o * in + i]) * fm[k * wmax + i];
        if (k < n_layers - 1 && !(acts[act_offset(k + 1, width, n) + s * out + o] > 0.0))
          accm = 0.0;
        fm[(k + 1) * wmax + o] = accm;
      }
    }
    const int outw = width[n_layers];
    for (int o = 0; o < outw; ++o) {
      d[o] = dy[s * outw + o];
      dm[o] = dy_mag ? dy_mag[s * outw + o] : fabs(d[o]);
    }
    for (int k = n_layers - 1; k >= 0; --k) {
      const int in = width[k], out = width[k + 1];
      const double* W = Wk[k];
      const double* a = acts + act_offset(k, width, n) + s * in;
      double* dW = d_params + poff[k];
      double* db = dW + (int64_t)out * in;
      for (int o = 0; o < out; ++o) {
        for (int i = 0; i < in; ++i) {
          dW[(int64_t)o * in + i] += d[o] * a[i];
          if (dp_mag) dp_mag[poff[k] + (int64_t)o * in + i] += dm[o] * fm[k * wmax + i];
        }
        db[o] += d[o];
        if (dp_mag) dp_mag[poff[k] + (int64_t)out * in + o] += dm[o];
      }
      for (int i = 0; i < in; ++i) {
        double acc = 0.0, accm = 0.0;
        for (int o = 0; o < out; ++o) {
          acc += W[(int64_t)o * in + i] * d[o];
          accm += fabs(W[(int64_t)o * in + i]) * dm[o];
        }
        if (k > 0 && !(a[i] > 0.0)) {
          acc = 0.0;
          accm = 0.0;
        }
        dn[i] = acc;
        dnm[i] = accm;
      }
      for (int i = 0; i < in; ++i) {
        d[i] = dn[i];
        dm[i] = dnm[i];
      }
    }
    for (int i = 0; i < width[0]; ++i) {
      if (dx) dx[s * width[0] + i] = d[i];
      if (dx_mag) dx_mag[s * width[0] + i] = dm[i];
    }
  }
  free(Wk);
  free(poff);
  free(d);
  free(dn);
  free(dm);
  free(dnm);
  free(fm);
}

/* ========================================================================= */
/* Loss, optimiser, reductions                                               */
/* ========================================================================= */

/* Mean squared error over the batch and its gradient dL/dy = 2(y - v)/n. */
double or_mse(const double* y, const double* v, int64_t n, double* dy) {
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double r = y[i] - v[i];
    acc += r * r;
    if (dy) dy[i] = 2.0 * r / (double)n;
  }
  return n > 0 ? acc / (double)n : 0.0;
}

/* Adam (Kingma & Ba) with bias correction and no weight decay, applied to
 * every parameter, as the paper's PyTorch training does (Sec. 5.1.3):
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void or_adam(double* p, const double* g, double* m, double* v, int64_t n, double lr,
             double beta1, double beta2, double eps, int64_t step) {
  const double bc1 = 1.0 - pow(beta1, (double)step);
  const double bc2 = 1.0 - pow(beta2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    double mhat = m[i] / bc1;
    double vhat = v[i] / bc2;
    p[i] -= lr * mhat / (sqrt(vhat) + eps);
  }
}

/* PSNR for data normalised to [0,1] (Sec. 5.1.2): 10 log10(1 / MSE). */
double or_psnr(double mse) { return 10.0 * log10(1.0 / mse); }

/* ========================================================================= */
/* Counter-based RNG and the training sampler                                */
/* ========================================================================= */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
 * multiplies with the published multipliers and Weyl key increments. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Draw n indices uniformly from [0, M) with replacement.  Draw i of a step
 * uses counter (i_lo, i_hi, step_lo, step_hi) and key (seed_lo, seed_hi); the
 * 64-bit word r = out1:out0 is mapped to floor(r * M / 2^64). */
void or_sample_ids(uint64_t seed, uint64_t step, int64_t n, uint64_t M, uint64_t* ids) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)step,
                       (uint32_t)(step >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    uint64_t r = ((uint64_t)out[1] << 32) | out[0];
    ids[i] = (uint64_t)(((unsigned __int128)r * (unsigned __int128)M) >> 64);
  }
}

/* Sample positions of linear voxel ids: (i/(Sx-1), j/(Sy-1), k/(Sz-1), n/(T-1))
 * in FP32 (the position part of the training sampler). */
void or_voxel_positions(const uint64_t* lin, int64_t n, const int64_t S[4], float* pos) {
  for (int64_t s = 0; s < n; ++s) {
    uint64_t v = lin[s];
    int64_t i = (int64_t)(v % (uint64_t)S[0]);
    int64_t j = (int64_t)((v / (uint64_t)S[0]) % (uint64_t)S[1]);
    int64_t k = (int64_t)((v / ((uint64_t)S[0] * S[1])) % (uint64_t)S[2]);
    int64_t t = (int64_t)(v / ((uint64_t)S[0] * S[1] * S[2]));
    pos[s * 4 + 0] = (float)i / (float)(S[0] - 1);
    pos[s * 4 + 1] = (float)j / (float)(S[1] - 1);
    pos[s * 4 + 2] = (float)k / (float)(S[2] - 1);
    pos[s * 4 + 3] = (float)t / (float)(S[3] - 1);
  }
}

/* One training batch (Sec. 3.1, time-step concatenation): each draw picks a
 * voxel, either from the coreset list (linear voxel ids) or, when coreset is
 * NULL, from the whole grid; the sample is the voxel position
 * (i/(Sx-1), j/(Sy-1), k/(Sz-1), n/(T-1)) in FP32 and the label is the field
 * value there.  field is [T][Sz][Sy][Sx], x fastest. */
void or_sample_batch(uint64_t seed, uint64_t step, int64_t n, const uint64_t* coreset,
                     uint64_t M, const int64_t S[4], const float* field, float* pos,
                     float* target) {
  uint64_t* ids = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  or_sample_ids(seed, step, n, M, ids);
  for (int64_t s = 0; s < n; ++s) {
    uint64_t lin = coreset ? coreset[ids[s]] : ids[s];
    int64_t i = (int64_t)(lin % (uint64_t)S[0]);
    int64_t j = (int64_t)((lin / (uint64_t)S[0]) % (uint64_t)S[1]);
    int64_t k = (int64_t)((lin / ((uint64_t)S[0] * S[1])) % (uint64_t)S[2]);
    int64_t t = (int64_t)(lin / ((uint64_t)S[0] * S[1] * S[2]));
    pos[s * 4 + 0] = (float)i / (float)(S[0] - 1);
    pos[s * 4 + 1] = (float)j / (float)(S[1] - 1);
    pos[s * 4 + 2] = (float)k / (float)(S[2] - 1);
    pos[s * 4 + 3] = (float)t / (float)(S[3] - 1);
    target[s] = field[lin];
  }
  free(ids);
}

/* ========================================================================= */
/* Rendering (Sec. 3.3, Algorithm 1)                                         */
/* ========================================================================= */

/* Occupancy of lattice position p (voxel units) at fractional timestep t
 * (reading of the "linearly interpolated occupancy grid" for a bit grid): the
 * sample counts as occupied iff one of the 8 corner voxels of its voxel cell
 * is in the feature mask at floor(t) or at ceil(t).  mask: bytes [T][Sz][Sy][Sx]. */
int or_occupied(const uint8_t* mask, const int64_t S[4], const float p[3], float t) {
  int64_t c[3];
  for (int d = 0; d < 3; ++d) {
    int64_t i = (int64_t)floorf(p[d]);
    if (i < 0) i = 0;
    if (i > S[d] - 2) i = S[d] - 2;
    c[d] = i;
  }
  int64_t t0 = (int64_t)floorf(t), t1 = (int64_t)ceilf(t);
  if (t0 < 0) t0 = 0;
  if (t1 > S[3] - 1) t1 = S[3] - 1;
  if (t0 > S[3] - 1) t0 = S[3] - 1;
  for (int64_t n = t0; n <= t1; ++n)
    for (int m = 0; m < 8; ++m) {
      int64_t x = c[0] + (m & 1), y = c[1] + ((m >> 1) & 1), z = c[2] + ((m >> 2) & 1);
      if (mask[((n * S[2] + z) * S[1] + y) * S[0] + x]) return 1;
    }
  return 0;
}

/* Ray of pixel (px, py): pinhole camera with basis (fwd, right, up) already
 * normalised on the host, tan_half = tan(fovy/2), aspect = W/H.  All FP32
 * with the operation order below (no contraction). */
static void pixel_ray(const float* cam, int W, int H, int px, int py, float org[3], float dir[3]) {
  /* cam: eye[3], fwd[3], right[3], up[3], tan_half, aspect */
  const float* eye = cam;
  const float *fw = cam + 3, *rt = cam + 6, *up = cam + 9;
  const float th = cam[12], asp = cam[13];
  float u = (2.0f * ((float)px + 0.5f) / (float)W - 1.0f) * th * asp;
  float v = (1.0f - 2.0f * ((float)py + 0.5f) / (float)H) * th;
  float d[3];
  for (int k = 0; k < 3; ++k) d[k] = fw[k] + u * rt[k] + v * up[k];
  float nrm = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int k = 0; k < 3; ++k) {
    dir[k] = d[k] / nrm;
    org[k] = eye[k];
  }
}

/* Slab intersection with the box [0, S_d - 1]^3 (Kay & Kajiya 1986). */
static int ray_box(const float org[3], const float dir[3], const int64_t S[4], float* s0,
                   float* s1) {
  float lo = 0.0f, hi = 3.0e38f;
  for (int k = 0; k < 3; ++k) {
    float a = (0.0f - org[k]) / dir[k];
    float b = ((float)(S[k] - 1) - org[k]) / dir[k];
    float mn = a < b ? a : b, mx = a < b ? b : a;
    if (mn > lo) lo = mn;
    if (mx < hi) hi = mx;
  }
  *s0 = lo;
  *s1 = hi;
  return lo < hi;
}

/* Transfer function: 256 RGBA entries, value clamped to [0,1], linear blend. */
static void apply_tf(const float* tf, double v, double rgba[4]) {
  if (!(v >= 0.0)) v = 0.0;
  if (v > 1.0) v = 1.0;
  double x = v * 255.0;
  int i = (int)floor(x);
  if (i > 254) i = 254;
  double f = x - i;
  for (int k = 0; k < 4; ++k) rgba[k] = (1.0 - f) * tf[i * 4 + k] + f * tf[(i + 1) * 4 + k];
}

/* Render one image: every pixel's ray walks the lattice s_k = s_near + (k+1/2) ds
 * (p_k = fma(s_k, dir, org) per component, FP32); an occupied sample is
 * evaluated by the model at (p / (S - 1), t / (T - 1)) in FP64, mapped through
 * the transfer function and composited front to back
 *   C += (1 - A) a c,  A += (1 - A) a,
 * stopping after the first sample with A >= alpha_stop, or after max_steps
 * lattice steps.  The adaptive marching pace of Algorithm 1 only changes
 * which samples are evaluated together, never the image, so this walk is one
 * sample at a time.  rgba: [H][W][4]; amb[H][W] flags pixels whose opacity came
 * within 1e-5 of alpha_stop at some step (termination point rounding-sensitive).
 * pix (may be NULL): per pixel [H][W][3] the number of composited samples, the
 * sum of their decoder-output magnitudes (sum of |terms| of each output) and
 * the smallest |A - alpha_stop| over the composited steps (1 when none), the
 * quantities an error bound of another evaluation order needs.
 * Returns the number of evaluated samples. */
int64_t or_render(const or_grid* g, const double* table, int n_layers, const int32_t* width,
                  const double* params, const uint8_t* mask, const int64_t S[4], const float* cam,
                  float t, float t01, const float* tf, int W, int H, float ds, float alpha_stop,
                  int max_steps, double* rgba, uint8_t* amb, double* pix) {
  int64_t evals = 0;
  const int L = g->n_levels, F = g->n_features;
  double* enc = (double*)malloc(sizeof(double) * L * F * 2);
  const float tn = t01 >= 0.0f ? t01 : t / (float)(S[3] - 1);
  for (int py = 0; py < H; ++py)
    for (int px = 0; px < W; ++px) {
      double C[3] = {0, 0, 0}, A = 0.0;
      double n_comp = 0.0, ymag_sum = 0.0, margin = 1.0;
      int ambiguous = 0;
      float org[3], dir[3], s0, s1;
      pixel_ray(cam, W, H, px, py, org, dir);
      if (ray_box(org, dir, S, &s0, &s1)) {
        if (s0 < 0.0f) s0 = 0.0f;
        for (int k = 0; k < max_steps; ++k) {
          float sk = fmaf((float)k + 0.5f, ds, s0);
          if (!(sk < s1)) break;
          float p[3];
          for (int d = 0; d < 3; ++d) p[d] = fmaf(sk, dir[d], org[d]);
          if (!or_occupied(mask, S, p, t)) continue;
          float q[4] = {p[0] / (float)(S[0] - 1), p[1] / (float)(S[1] - 1),
                        p[2] / (float)(S[2] - 1), tn};
          double y, ym;
          double* encm = enc + L * F;
          or_encode_fwd(g, q, 1, table, enc, encm);
          or_mlp_fwd(n_layers, width, params, enc, 1, &y, NULL, encm, &ym);
          ++evals;
          n_comp += 1.0;
          ymag_sum += ym;
          double c[4];
          apply_tf(tf, y, c);
          double a = c[3];
          for (int d = 0; d < 3; ++d) C[d] += (1.0 - A) * a * c[d];
          A += (1.0 - A) * a;
          if (fabs(A - alpha_stop) < 1e-5) ambiguous = 1;
          if (fabs(A - alpha_stop) < margin) margin = fabs(A - alpha_stop);
          if (A >= alpha_stop) break;
        }
      }
      double* o = rgba + ((int64_t)py * W + px) * 4;
      o[0] = C[0];
      o[1] = C[1];
      o[2] = C[2];
      o[3] = A;
      if (amb) amb[(int64_t)py * W + px] = (uint8_t)ambiguous;
      if (pix) {
        double* q = pix + ((int64_t)py * W + px) * 3;
        q[0] = n_comp;
        q[1] = ymag_sum;
        q[2] = margin;
      }
    }
  free(enc);
  return evals;
}
