// C ABI of libfhash: host-side validation, workspace sizing and dispatch to the
// HIP kernels.  No exception crosses this boundary; every entry point returns a
// status code and records a message for fhash_last_error().
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "common.h"
#include "fhash.h"
#include "kernels.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return FHASH_OK;
  return fail(FHASH_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_grid(const fhash_grid_desc* g) {
  if (g == nullptr) return fail(FHASH_EINVAL, "grid descriptor is NULL");
  if (g->n_levels < 1 || g->n_levels > FHASH_MAX_LEVELS)
    return fail(FHASH_EINVAL, "n_levels %d outside [1, %d]", g->n_levels, FHASH_MAX_LEVELS);
  const int F = g->n_features;
  if (F != 1 && F != 2 && F != 4 && F != 8)
    return fail(FHASH_EINVAL, "n_features %d not in {1, 2, 4, 8}", F);
  for (int l = 0; l < g->n_levels; ++l) {
    double nv = 1.0;
    for (int d = 0; d < 4; ++d) {
      const int r = g->res[l][d];
      if (r < 2 || r > (1 << 24))
        return fail(FHASH_EINVAL, "res[%d][%d] = %d outside [2, 2^24]", l, d, r);
      nv *= r;
    }
    if (nv >= 4.0e18) return fail(FHASH_ERANGE, "level %d has too many vertices", l);
    // the kernels index a level's vertex rows and directory words in 32 bits
    const double words = (double)g->res[l][1] * g->res[l][2] * g->res[l][3] *
                         (double)((g->res[l][0] + 63) / 64);
    const double bwords = (double)((g->res[l][1] + 1) / 2) * ((g->res[l][2] + 1) / 2) *
                          ((g->res[l][3] + 1) / 2) * (double)(((g->res[l][0] + 1) / 2 + 3) / 4);
    if (words >= 2147483648.0 || (g->layout == FHASH_LAYOUT_BRICKS && bwords >= 2147483648.0))
      return fail(FHASH_ERANGE, "level %d has 2^31 directory words or more", l);
  }
  if (g->layout != FHASH_LAYOUT_ROWS && g->layout != FHASH_LAYOUT_BRICKS)
    return fail(FHASH_EINVAL, "layout %d is neither rows nor bricks", g->layout);
  return FHASH_OK;
}

int check_index(const fhash_index* idx) {
  if (idx == nullptr) return fail(FHASH_EINVAL, "index is NULL");
  int rc = check_grid(&idx->grid);
  if (rc) return rc;
  if (idx->active != 0 && idx->active != 1) return fail(FHASH_EINVAL, "index.active must be 0/1");
  if (idx->hash_bits != 0 && (idx->active || idx->hash_bits < 4 || idx->hash_bits > 31))
    return fail(FHASH_EINVAL, "index.hash_bits must be 0, or in [4, 31] with a dense index");
  if (idx->active && idx->dir == nullptr) return fail(FHASH_EINVAL, "active index without dir");
  for (int l = 0; l < idx->grid.n_levels; ++l)
    if (idx->slot_offset[l + 1] < idx->slot_offset[l] || idx->slot_offset[l] < 0)
      return fail(FHASH_EINVAL, "slot_offset not monotone at level %d", l);
  return FHASH_OK;
}

int64_t total_rows(const fhash_index* idx) { return idx->slot_offset[idx->grid.n_levels]; }

int check_table_dt(fhash_dtype dt) {
  if (dt != FHASH_F32 && dt != FHASH_F16 && dt != FHASH_F32_PAIRED)
    return fail(FHASH_ENOTSUP, "table dtype %d not supported (F32, F32_PAIRED or F16)", (int)dt);
  return FHASH_OK;
}

// The element type the kernels read for table dtype dt; a paired FP32 table
// is read through the run mask of g.
fhash_dtype table_view(fhash_dtype dt, fh::GridDev* g) {
  if (dt != FHASH_F32_PAIRED) return dt;
  g->tmask = ~(int64_t)15;
  return FHASH_F32;
}

// Flags of the backward calls; FHASH_GRAD_PAIRED sets the gradient's run mask
// (g may be NULL: check only).
int apply_bwd_flags(uint32_t flags, fh::GridDev* g) {
  if ((flags & ~(FHASH_SAMPLES_SORTED | FHASH_GRAD_PAIRED | FHASH_COARSE_LDS)) != 0)
    return fail(FHASH_EINVAL, "unknown flags 0x%x", (unsigned)flags);
  if (g != nullptr) g->gmask = (flags & FHASH_GRAD_PAIRED) ? ~(int64_t)15 : 0;
  return FHASH_OK;
}

// Decoder shape: width[0] input, hidden widths all equal H, output width 1.
// allow_f16: the FP16-MFMA decoder is built for the forward-only calls.
int check_mlp(const fhash_mlp_desc* m, int* H, int* NH, bool allow_f16 = false) {
  if (m == nullptr) return fail(FHASH_EINVAL, "mlp descriptor is NULL");
  if (m->n_layers < 2 || m->n_layers > FHASH_MAX_LAYERS)
    return fail(FHASH_EINVAL, "n_layers %d outside [2, %d]", m->n_layers, FHASH_MAX_LAYERS);
  for (int k = 0; k <= m->n_layers; ++k)
    if (m->width[k] < 1) return fail(FHASH_EINVAL, "width[%d] = %d", k, m->width[k]);
  if (m->width[m->n_layers] != 1) return fail(FHASH_ENOTSUP, "output width must be 1");
  const int h = m->width[1];
  for (int k = 1; k < m->n_layers; ++k)
    if (m->width[k] != h) return fail(FHASH_ENOTSUP, "hidden widths must be equal");
  if (m->compute_dt != FHASH_F32 &&
      !(allow_f16 && (m->compute_dt == FHASH_F16 || m->compute_dt == FHASH_BF16)))
    return fail(FHASH_ENOTSUP, "mlp compute dtype %d not built for this call",
                (int)m->compute_dt);
  if (!fh::mlp_supported(m->width[0], h, m->n_layers - 1))
    return fail(FHASH_ENOTSUP, "mlp shape in=%d hidden=%d x %d not built", m->width[0], h,
                m->n_layers - 1);
  *H = h;
  *NH = m->n_layers - 1;
  return FHASH_OK;
}

int64_t num_params(const fhash_mlp_desc* m) {
  int64_t p = 0;
  for (int k = 0; k < m->n_layers; ++k) p += (int64_t)m->width[k + 1] * m->width[k] + m->width[k + 1];
  return p;
}

int ws_check(void* ws, size_t* ws_bytes, size_t need, bool* query) {
  *query = false;
  if (ws_bytes == nullptr) return fail(FHASH_EINVAL, "ws_bytes is NULL");
  if (ws == nullptr) {
    *ws_bytes = need;
    *query = true;
    return FHASH_OK;
  }
  if (*ws_bytes < need)
    return fail(FHASH_ENOMEM, "workspace %zu bytes, need %zu", *ws_bytes, need);
  if (!aligned16(ws)) return fail(FHASH_EINVAL, "workspace not 16-byte aligned");
  return FHASH_OK;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// Validate a touched-segment descriptor against a gradient of `len` floats and
// install it in g (NULL: not tracked).
static int apply_touch(const fhash_touch* t, int64_t len, fh::GridDev* g) {
  if (t == nullptr) return FHASH_OK;
  if (t->flags == nullptr) return fail(FHASH_EINVAL, "touch flags are NULL");
  if (t->begin < 0 || t->begin % FHASH_TOUCH_FLOATS != 0 || t->end < t->begin || t->end > len)
    return fail(FHASH_EINVAL, "touch range [%lld, %lld) invalid for %lld floats",
                (long long)t->begin, (long long)t->end, (long long)len);
  if (g != nullptr) {
    g->touch = t->flags;
    g->touch_begin = t->begin;
  }
  return FHASH_OK;
}

extern "C" {

int fhash_version(void) { return FHASH_VERSION; }
const char* fhash_last_error(void) { return g_err; }

int fhash_index_dir_entries(const fhash_grid_desc* grid, int64_t* entries) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (entries == nullptr) return fail(FHASH_EINVAL, "entries is NULL");
  int64_t e = 0;
  for (int l = 0; l < grid->n_levels; ++l) e += fh::index_dir_words(grid, l);
  *entries = e;
  return FHASH_OK;
}

int fhash_dense_index(const fhash_grid_desc* grid, fhash_index* out, int64_t* slots_per_level) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (grid->layout != FHASH_LAYOUT_ROWS)
    return fail(FHASH_ENOTSUP, "the brick layout is built for the active-vertex index only");
  if (out == nullptr) return fail(FHASH_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->grid = *grid;
  out->active = 0;
  out->dir = nullptr;
  int64_t off = 0;
  for (int l = 0; l < grid->n_levels; ++l) {
    const int32_t* r = grid->res[l];
    const int64_t nv = (int64_t)r[0] * r[1] * r[2] * r[3];
    out->slot_offset[l] = off;
    if (slots_per_level) slots_per_level[l] = nv;
    off += nv;
  }
  for (int l = grid->n_levels; l <= FHASH_MAX_LEVELS; ++l) out->slot_offset[l] = off;
  return FHASH_OK;
}

int fhash_hash_index(const fhash_grid_desc* grid, int32_t hash_bits, fhash_index* out,
                     int64_t* slots_per_level) {
  if (hash_bits < 4 || hash_bits > 31) return fail(FHASH_EINVAL, "hash_bits %d outside [4, 31]", hash_bits);
  int rc = fhash_dense_index(grid, out, nullptr);
  if (rc) return rc;
  out->hash_bits = hash_bits;
  int64_t off = 0;
  for (int l = 0; l < grid->n_levels; ++l) {
    const int32_t* r = grid->res[l];
    const int64_t nv = (int64_t)r[0] * r[1] * r[2] * r[3];
    const int64_t rows = nv > (1ll << hash_bits) ? (1ll << hash_bits) : nv;
    out->slot_offset[l] = off;
    if (slots_per_level) slots_per_level[l] = rows;
    off += rows;
  }
  for (int l = grid->n_levels; l <= FHASH_MAX_LEVELS; ++l) out->slot_offset[l] = off;
  return FHASH_OK;
}

int fhash_build_index(const fhash_grid_desc* grid, const fhash_mask_desc* mask, void* dir,
                      void* ws, size_t* ws_bytes, fhash_index* out, int64_t* slots_per_level,
                      void* stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  if (mask == nullptr) return fail(FHASH_EINVAL, "mask descriptor is NULL");
  if (mask->bits == nullptr) {
    if (ws == nullptr && ws_bytes != nullptr) {
      *ws_bytes = 0;
      return FHASH_OK;
    }
    return fhash_dense_index(grid, out, slots_per_level);
  }
  for (int d = 0; d < 4; ++d)
    if (mask->dims[d] < 2 || mask->dims[d] > (int64_t)1 << 31)
      return fail(FHASH_EINVAL, "mask dims[%d] = %lld outside [2, 2^31]", d,
                  (long long)mask->dims[d]);
  const size_t need = fh::index_workspace_bytes(grid, mask->dims);
  bool query;
  rc = ws_check(ws, ws_bytes, need, &query);
  if (rc || query) return rc;
  if (dir == nullptr || out == nullptr || slots_per_level == nullptr)
    return fail(FHASH_EINVAL, "dir, out and slots_per_level must be non-NULL");
  if (!aligned16(dir)) return fail(FHASH_EINVAL, "dir not 16-byte aligned");
  std::memset(out, 0, sizeof(*out));
  out->grid = *grid;
  out->active = 1;
  out->dir = dir;
  int64_t e = 0;
  for (int l = 0; l < grid->n_levels; ++l) {
    out->dir_offset[l] = e;
    e += fh::index_dir_words(grid, l);
  }
  for (int l = grid->n_levels; l <= FHASH_MAX_LEVELS; ++l) out->dir_offset[l] = e;
  uint64_t counts[FHASH_MAX_LEVELS];
  hipError_t he = fh::launch_build_index(grid, mask->bits, mask->dims,
                                         reinterpret_cast<ulonglong2*>(dir), out->dir_offset, ws,
                                         counts, S(stream));
  if (he != hipSuccess) return hip_status(he, "fhash_build_index");
  int64_t off = 0;
  for (int l = 0; l < grid->n_levels; ++l) {
    out->slot_offset[l] = off;
    slots_per_level[l] = (int64_t)counts[l];
    off += (int64_t)counts[l];
  }
  for (int l = grid->n_levels; l <= FHASH_MAX_LEVELS; ++l) out->slot_offset[l] = off;
  return FHASH_OK;
}

int fhash_encode_fwd(const fhash_index* idx, const float* pos, int64_t n, const void* table,
                     fhash_dtype table_dt, float* enc, void* stream) {
  int rc = check_index(idx);
  if (rc) return rc;
  if ((rc = check_table_dt(table_dt))) return rc;
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  if (n == 0) return FHASH_OK;
  if (pos == nullptr || enc == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  if (!aligned16(pos)) return fail(FHASH_EINVAL, "pos not 16-byte aligned");
  const int64_t L = idx->grid.n_levels, F = idx->grid.n_features;
  if (total_rows(idx) == 0)
    return hip_status(hipMemsetAsync(enc, 0, sizeof(float) * n * L * F, S(stream)),
                      "fhash_encode_fwd");
  if (table == nullptr) return fail(FHASH_EINVAL, "table is NULL");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  const fhash_dtype tdt = table_view(table_dt, &g);
  return hip_status(fh::launch_encode_fwd(g, pos, n, table, tdt, enc, S(stream)),
                    "fhash_encode_fwd");
}

int fhash_corner_rows(const fhash_index* idx, const float* pos, int64_t n, int64_t* out_dir,
                      int64_t* out_slot, void* stream) {
  int rc = check_index(idx);
  if (rc) return rc;
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  if (n == 0) return FHASH_OK;
  if (pos == nullptr || out_dir == nullptr || out_slot == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (!aligned16(pos)) return fail(FHASH_EINVAL, "pos not 16-byte aligned");
  if (n > (int64_t)1 << 40) return fail(FHASH_ERANGE, "n too large");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  return hip_status(fh::launch_corner_rows(g, pos, n, out_dir, out_slot, S(stream)),
                    "fhash_corner_rows");
}

int fhash_encode_bwd(const fhash_index* idx, const float* pos, int64_t n, const float* d_enc,
                     float* d_table, const fhash_touch* touch, void* stream) {
  int rc = check_index(idx);
  if (rc) return rc;
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  if ((rc = apply_touch(touch, total_rows(idx) * idx->grid.n_features, &g))) return rc;
  if (n == 0 || total_rows(idx) == 0) return FHASH_OK;
  if (pos == nullptr || d_enc == nullptr || d_table == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (!aligned16(pos)) return fail(FHASH_EINVAL, "pos not 16-byte aligned");
  return hip_status(fh::launch_encode_bwd(g, pos, n, d_enc, d_table, S(stream)),
                    "fhash_encode_bwd");
}

int64_t fhash_mlp_num_params(const fhash_mlp_desc* mlp) {
  if (mlp == nullptr || mlp->n_layers < 1 || mlp->n_layers > FHASH_MAX_LAYERS) return -1;
  return num_params(mlp);
}

int fhash_mlp_fwd(const fhash_mlp_desc* mlp, const float* params, const void* shadow,
                  const float* x, int64_t n, float* y, void* stream) {
  (void)shadow;
  int H, NH;
  int rc = check_mlp(mlp, &H, &NH);
  if (rc) return rc;
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  if (n == 0) return FHASH_OK;
  if (params == nullptr || x == nullptr || y == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  return hip_status(fh::launch_mlp_fwd(mlp->width[0], H, NH, params, x, n, y, S(stream)),
                    "fhash_mlp_fwd");
}

int fhash_mlp_bwd(const fhash_mlp_desc* mlp, const float* params, const void* shadow,
                  const float* x, const float* dy, int64_t n, float* d_params, float* dx,
                  void* ws, size_t* ws_bytes, void* stream) {
  (void)shadow;
  int H, NH;
  int rc = check_mlp(mlp, &H, &NH);
  if (rc) return rc;
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  const int64_t P = num_params(mlp);
  bool query;
  rc = ws_check(ws, ws_bytes, fh::mlp_bwd_ws_bytes(n, P), &query);
  if (rc || query) return rc;
  if (n == 0) return FHASH_OK;
  if (params == nullptr || x == nullptr || dy == nullptr || d_params == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  return hip_status(
      fh::launch_mlp_bwd(mlp->width[0], H, NH, params, x, dy, n, d_params, dx, ws, P, S(stream)),
      "fhash_mlp_bwd");
}

// Levels whose cell count is at most 8 samples' worth: sorted neighbours share
// their vertices often enough for the merge of a scatter pass to pay.
static uint32_t dedup_mask(const fhash_index* idx, int64_t n, uint32_t flags) {
  if (!(flags & FHASH_SAMPLES_SORTED)) return 0u;
  uint32_t m = 0;
  for (int l = 0; l < idx->grid.n_levels; ++l) {
    const int32_t* r = idx->grid.res[l];
    const double cells = (double)(r[0] - 1) * (r[1] - 1) * (r[2] - 1) * (r[3] - 1);
    if (cells <= 8.0 * (double)n) m |= 1u << l;
  }
  return m;
}

// FHASH_COARSE_LDS: levels 0 .. lc - 1, the coarse levels with at most one
// cell per sample of the batch, go through the LDS scatter (row order only).
static int coarse_levels(const fhash_index* idx, int64_t n, uint32_t flags) {
  if (!(flags & FHASH_COARSE_LDS) || idx->grid.layout != FHASH_LAYOUT_ROWS) return 0;
  int lc = 0;
  for (int l = 0; l < idx->grid.n_levels; ++l) {
    const int32_t* r = idx->grid.res[l];
    const double cells = (double)(r[0] - 1) * (r[1] - 1) * (r[2] - 1) * (r[3] - 1);
    if (cells > (double)n) break;
    lc = l + 1;
  }
  return lc;
}

// Workspace of a fused backward: the decoder-gradient partials, then the
// coarse levels' encoding gradient (lc levels x n samples x F floats).
static size_t fused_bwd_ws(int64_t n, int64_t P, int lc, int F) {
  const size_t part = (fh::fused_ws_bytes(n, P) + 255) & ~(size_t)255;
  return part + (size_t)lc * (size_t)n * (size_t)F * sizeof(float);
}

static void set_coarse(fh::GridDev* g, int lc, int64_t n, int64_t P, void* ws) {
  g->coarse = lc;
  g->nsamp = n;
  g->dxc = lc > 0 ? reinterpret_cast<float*>(static_cast<char*>(ws) +
                                             ((fh::fused_ws_bytes(n, P) + 255) & ~(size_t)255))
                  : nullptr;
}

static int check_fused(const fhash_index* idx, const fhash_mlp_desc* mlp, const float* pos,
                       int64_t n, const void* table, fhash_dtype tdt, const float* params,
                       int* H, int* NH, bool backward) {
  int rc = check_index(idx);
  if (rc) return rc;
  if ((rc = check_mlp(mlp, H, NH, true))) return rc;
  // 16-bit decoders: FP16 forward for every feature count; BF16, and every
  // 16-bit backward, for two features per level
  if (mlp->compute_dt != FHASH_F32 && idx->grid.n_features != 2 &&
      (backward || mlp->compute_dt == FHASH_BF16))
    return fail(FHASH_ENOTSUP, "16-bit decoder dtype %d not built for F=%d%s",
                (int)mlp->compute_dt, idx->grid.n_features, backward ? " (backward)" : "");
  if ((rc = check_table_dt(tdt))) return rc;
  const int in_w = idx->grid.n_levels * idx->grid.n_features;
  if (mlp->width[0] != in_w)
    return fail(FHASH_EINVAL, "mlp input width %d != L*F = %d", mlp->width[0], in_w);
  if (!fh::fused_supported(idx->grid.n_features, in_w, *H, *NH))
    return fail(FHASH_ENOTSUP, "fused path not built for F=%d in=%d hidden=%dx%d",
                idx->grid.n_features, in_w, *H, *NH);
  if (idx->grid.layout == FHASH_LAYOUT_BRICKS) {
    const int F = idx->grid.n_features, inp = (in_w + 15) / 16 * 16;
    if (!((F == 2 || F == 4) && inp == 32 && *H == 64 && (*NH == 2 || *NH == 3)))
      return fail(FHASH_ENOTSUP, "fused kernels on a brick-ordered index are built for 17-32 "
                  "decoder inputs, F = 2 or 4, 2 or 3 hidden layers of 64 only");
  }
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  if (n > 0 && (pos == nullptr || params == nullptr)) return fail(FHASH_EINVAL, "NULL pointer");
  if (n > 0 && !aligned16(pos)) return fail(FHASH_EINVAL, "pos not 16-byte aligned");
  if (n > 0 && total_rows(idx) == 0)
    return fail(FHASH_EINVAL, "index has no active vertex (empty table)");
  if (n > 0 && table == nullptr) return fail(FHASH_EINVAL, "table is NULL");
  return FHASH_OK;
}

int fhash_fused_fwd(const fhash_index* idx, const fhash_mlp_desc* mlp, const float* pos, int64_t n,
                    const void* table, fhash_dtype table_dt, const float* params,
                    const void* shadow, float* y, void* stream) {
  (void)shadow;
  int H, NH;
  int rc = check_fused(idx, mlp, pos, n, table, table_dt, params, &H, &NH, false);
  if (rc) return rc;
  if (n == 0) return FHASH_OK;
  if (y == nullptr) return fail(FHASH_EINVAL, "y is NULL");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  const fhash_dtype tdt = table_view(table_dt, &g);
  const hipError_t e =
      mlp->compute_dt != FHASH_F32
          ? fh::launch_fused_fwd16(g, H, NH, mlp->compute_dt, pos, n, table, tdt, params, y,
                                   S(stream))
          : fh::launch_fused_fwd(g, H, NH, pos, n, table, tdt, params, y, S(stream));
  return hip_status(e, "fhash_fused_fwd");
}

int fhash_fused_bwd(const fhash_index* idx, const fhash_mlp_desc* mlp, const float* pos, int64_t n,
                    const void* table, fhash_dtype table_dt, const float* params,
                    const void* shadow, const float* dy, float* d_table, float* d_params,
                    uint32_t flags, const fhash_touch* touch, void* ws, size_t* ws_bytes,
                    void* stream) {
  (void)shadow;
  int H, NH;
  int rc = check_fused(idx, mlp, pos, n, table, table_dt, params, &H, &NH, true);
  if (rc) return rc;
  if ((rc = apply_bwd_flags(flags, nullptr))) return rc;
  const int64_t P = num_params(mlp);
  const int lc = coarse_levels(idx, n, flags);
  bool query;
  rc = ws_check(ws, ws_bytes, fused_bwd_ws(n, P, lc, idx->grid.n_features), &query);
  if (rc || query) return rc;
  if (n == 0) return FHASH_OK;
  if (dy == nullptr || d_table == nullptr || d_params == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  if ((rc = apply_bwd_flags(flags, &g))) return rc;
  g.dedup = dedup_mask(idx, n, flags);
  set_coarse(&g, lc, n, P, ws);
  if ((rc = apply_touch(touch, total_rows(idx) * idx->grid.n_features, &g))) return rc;
  const fhash_dtype tdt = table_view(table_dt, &g);
  return hip_status(fh::launch_fused_bwd(g, H, NH, mlp->compute_dt, pos, n, table, tdt,
                                         params, dy, d_table, d_params, ws, P, S(stream)),
                    "fhash_fused_bwd");
}

int fhash_fused_train(const fhash_index* idx, const fhash_mlp_desc* mlp, const float* pos,
                      const float* target, int64_t n, const void* table, fhash_dtype table_dt,
                      const float* params, const void* shadow, float loss_scale, float* d_table,
                      float* d_params, double* loss_sum, uint32_t flags,
                      const fhash_touch* touch, void* ws, size_t* ws_bytes, void* stream) {
  (void)shadow;
  int H, NH;
  int rc = check_fused(idx, mlp, pos, n, table, table_dt, params, &H, &NH, true);
  if (rc) return rc;
  if ((rc = apply_bwd_flags(flags, nullptr))) return rc;
  const int64_t P = num_params(mlp);
  const int lc = coarse_levels(idx, n, flags);
  bool query;
  rc = ws_check(ws, ws_bytes, fused_bwd_ws(n, P, lc, idx->grid.n_features), &query);
  if (rc || query) return rc;
  if (n == 0) return FHASH_OK;
  if (target == nullptr || d_table == nullptr || d_params == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  if ((rc = apply_bwd_flags(flags, &g))) return rc;
  g.dedup = dedup_mask(idx, n, flags);
  set_coarse(&g, lc, n, P, ws);
  if ((rc = apply_touch(touch, total_rows(idx) * idx->grid.n_features, &g))) return rc;
  const fhash_dtype tdt = table_view(table_dt, &g);
  return hip_status(fh::launch_fused_train(g, H, NH, mlp->compute_dt, pos, target, n, table,
                                           tdt, params, loss_scale, d_table, d_params, loss_sum,
                                           ws, P, S(stream)),
                    "fhash_fused_train");
}

int fhash_fused_train_static(const fhash_index* idx, const fhash_mlp_desc* mlp,
                             const float* pos, const float* target, int64_t n, const void* table,
                             fhash_dtype table_dt, const float* params, const void* shadow,
                             float loss_scale, float* d_table, float* d_params, double* loss_sum,
                             uint32_t flags, const fhash_touch* touch, void* stream) {
  (void)shadow;
  int H, NH;
  int rc = check_fused(idx, mlp, pos, n, table, table_dt, params, &H, &NH, true);
  if (rc) return rc;
  if ((rc = apply_bwd_flags(flags, nullptr))) return rc;
  if (flags & FHASH_COARSE_LDS)
    return fail(FHASH_EINVAL, "FHASH_COARSE_LDS needs the workspace of fhash_fused_train");
  if (n == 0) return FHASH_OK;
  if (target == nullptr || d_table == nullptr || d_params == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  const int64_t P = num_params(mlp);
  const size_t need = fh::fused_ws_bytes(n, P);
  if (need > fh::static_scratch_bytes())
    return fail(FHASH_ENOMEM, "decoder-gradient partials need %zu bytes, the static scratch "
                "holds %zu", need, fh::static_scratch_bytes());
  void* ws = nullptr;
  hipError_t e = fh::static_scratch(&ws);
  if (e != hipSuccess) return hip_status(e, "fhash_fused_train_static scratch");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  if ((rc = apply_bwd_flags(flags, &g))) return rc;
  g.dedup = dedup_mask(idx, n, flags);
  if ((rc = apply_touch(touch, total_rows(idx) * idx->grid.n_features, &g))) return rc;
  const fhash_dtype tdt = table_view(table_dt, &g);
  return hip_status(fh::launch_fused_train(g, H, NH, mlp->compute_dt, pos, target, n, table,
                                           tdt, params, loss_scale, d_table, d_params,
                                           loss_sum, ws, P, S(stream)),
                    "fhash_fused_train_static");
}

// Where the optimiser layout ties the arrays together (fhash_adam_desc).
static int check_state_pointers(int64_t layout, const float* param, const float* grad,
                                const float* m, const float* v) {
  if (layout == FHASH_MOMENTS_PAIRED && v != m + 16)
    return fail(FHASH_EINVAL, "paired moments: v must start 16 floats after m");
  if (layout == FHASH_MOMENTS_WITH_PARAMS && (m != param + 16 || v != grad + 16))
    return fail(FHASH_EINVAL, "moments with parameters: m must start 16 floats after param "
                "and v 16 floats after grad");
  return FHASH_OK;
}

static int check_step(const fhash_adam_desc* opt, const float* param, const float* grad,
                      const float* m, const float* v, const void* shadow, fhash_dtype shadow_dt,
                      int64_t n) {
  if (opt == nullptr) return fail(FHASH_EINVAL, "optimiser descriptor is NULL");
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  if (opt->step < 1) return fail(FHASH_EINVAL, "step must be >= 1");
  if (!(opt->lr >= 0.0) || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) ||
      !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) || !(opt->eps > 0.0))
    return fail(FHASH_EINVAL, "bad Adam hyper-parameters");
  if (opt->moments != FHASH_MOMENTS_SEPARATE && opt->moments != FHASH_MOMENTS_PAIRED &&
      opt->moments != FHASH_MOMENTS_WITH_PARAMS)
    return fail(FHASH_EINVAL, "moments layout %lld unknown", (long long)opt->moments);
  if (n == 0) return FHASH_OK;
  if (param == nullptr || grad == nullptr || m == nullptr || v == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (!aligned16(param) || !aligned16(grad) || !aligned16(m) || !aligned16(v))
    return fail(FHASH_EINVAL, "optimiser arrays must be 16-byte aligned");
  if (int rc = check_state_pointers(opt->moments, param, grad, m, v)) return rc;
  if (shadow != nullptr) {
    if (shadow_dt != FHASH_F16 && shadow_dt != FHASH_BF16)
      return fail(FHASH_EINVAL, "shadow dtype must be F16 or BF16");
    if ((reinterpret_cast<uintptr_t>(shadow) & 7u) != 0)
      return fail(FHASH_EINVAL, "shadow must be 8-byte aligned");
  }
  return FHASH_OK;
}

int fhash_step(const fhash_adam_desc* opt, float* param, float* grad, float* m, float* v,
               void* shadow, fhash_dtype shadow_dt, int64_t n, const int32_t* found_inf,
               const fhash_touch* touch, void* stream) {
  int rc = check_step(opt, param, grad, m, v, shadow, shadow_dt, n);
  if (rc) return rc;
  if (n == 0) return FHASH_OK;
  if ((rc = apply_touch(touch, n, nullptr))) return rc;
  return hip_status(
      fh::launch_adam(opt, param, grad, m, v, shadow, shadow_dt, n, 0, found_inf, touch,
                      S(stream)),
      "fhash_step");
}

size_t fhash_lazy_workspace_bytes(int64_t range_floats, int64_t max_steps) {
  if (range_floats < 0 || max_steps < 0) return 0;
  return fh::lazy_ws_bytes(range_floats, max_steps);
}

static int check_lazy(const fhash_lazy* lz) {
  if (lz == nullptr) return fail(FHASH_EINVAL, "lazy descriptor is NULL");
  if (lz->ws == nullptr || !aligned16(lz->ws))
    return fail(FHASH_EINVAL, "lazy workspace is NULL or not 16-byte aligned");
  if (lz->begin < 0 || lz->begin % FHASH_LAZY_FLOATS != 0 || lz->end < lz->begin ||
      lz->end % 4 != 0)
    return fail(FHASH_EINVAL, "lazy range [%lld, %lld): begin must be a multiple of %d, end of 4",
                (long long)lz->begin, (long long)lz->end, FHASH_LAZY_FLOATS);
  if (fh::lazy_num_segments(lz->end - lz->begin) >= (int64_t)UINT32_MAX)
    return fail(FHASH_ERANGE, "lazy range has 2^32 segments or more");
  if (lz->max_steps < 0 || lz->max_steps >= (int64_t)UINT32_MAX)
    return fail(FHASH_ERANGE, "max_steps outside [0, 2^32 - 1)");
  if (lz->steps < 0 || lz->steps > lz->max_steps)
    return fail(FHASH_EINVAL, "steps %lld outside [0, max_steps]", (long long)lz->steps);
  if (lz->moments != FHASH_MOMENTS_SEPARATE && lz->moments != FHASH_MOMENTS_PAIRED &&
      lz->moments != FHASH_MOMENTS_WITH_PARAMS)
    return fail(FHASH_EINVAL, "moments layout %lld unknown", (long long)lz->moments);
  return FHASH_OK;
}

int fhash_lazy_init(fhash_lazy* lz, void* stream) {
  if (lz == nullptr) return fail(FHASH_EINVAL, "lazy descriptor is NULL");
  lz->steps = 0;
  int rc = check_lazy(lz);
  if (rc) return rc;
  lz->beta1 = lz->beta2 = lz->eps = -1.0;  // recorded by the first step
  lz->flags = 0;
  return hip_status(fh::launch_lazy_init(lz, S(stream)), "fhash_lazy_init");
}

// The levels whose table floats intersect [begin, end).
static void lazy_levels(const fhash_index* idx, const fhash_lazy* lz, int* l0, int* l1) {
  const int L = idx->grid.n_levels, F = idx->grid.n_features;
  *l0 = L;
  *l1 = 0;
  for (int l = 0; l < L; ++l) {
    const int64_t a = idx->slot_offset[l] * F, b = idx->slot_offset[l + 1] * F;
    if (b > lz->begin && a < lz->end && a < b) {
      if (l < *l0) *l0 = l;
      *l1 = l + 1;
    }
  }
  if (*l0 > *l1) *l0 = *l1;
}

int fhash_lazy_prepare(const fhash_index* idx, const float* pos, int64_t n, fhash_lazy* lz,
                       float* param, float* grad, float* m, float* v, void* shadow,
                       fhash_dtype shadow_dt, uint32_t phases, void* stream) {
  int rc = check_index(idx);
  if (rc) return rc;
  if ((rc = check_lazy(lz))) return rc;
  if (n < 0) return fail(FHASH_EINVAL, "n < 0");
  if (phases == 0 || (phases & ~(uint32_t)(FHASH_LAZY_MARK | FHASH_LAZY_CATCH_UP)) != 0)
    return fail(FHASH_EINVAL, "phases must be a nonempty set of FHASH_LAZY_MARK, FHASH_LAZY_CATCH_UP");
  if (lz->end > total_rows(idx) * idx->grid.n_features + 3)
    return fail(FHASH_EINVAL, "lazy range ends past the table");
  if (n > 0 && (pos == nullptr || !aligned16(pos)))
    return fail(FHASH_EINVAL, "pos is NULL or not 16-byte aligned");
  if (param == nullptr || grad == nullptr || m == nullptr || v == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (!aligned16(param) || !aligned16(grad) || !aligned16(m) || !aligned16(v))
    return fail(FHASH_EINVAL, "optimiser arrays must be 16-byte aligned");
  if ((rc = check_state_pointers(lz->moments, param, grad, m, v))) return rc;
  if (shadow != nullptr && shadow_dt != FHASH_F16 && shadow_dt != FHASH_BF16)
    return fail(FHASH_EINVAL, "shadow dtype must be F16 or BF16");
  if (shadow != nullptr && (reinterpret_cast<uintptr_t>(shadow) & 7u) != 0)
    return fail(FHASH_EINVAL, "shadow must be 8-byte aligned");
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  int l0, l1;
  lazy_levels(idx, lz, &l0, &l1);
  return hip_status(fh::launch_lazy_prepare(g, l0, l1, pos, n, lz, param, grad, m, v, shadow,
                                            shadow_dt, phases, S(stream)),
                    "fhash_lazy_prepare");
}

int fhash_step_lazy(const fhash_adam_desc* opt, float* param, float* grad, float* m, float* v,
                    void* shadow, fhash_dtype shadow_dt, int64_t n, const int32_t* found_inf,
                    fhash_lazy* lz, void* stream) {
  int rc = check_step(opt, param, grad, m, v, shadow, shadow_dt, n);
  if (rc) return rc;
  if ((rc = check_lazy(lz))) return rc;
  if (lz->end > n) return fail(FHASH_EINVAL, "lazy range ends past the parameters");
  if (lz->steps + 1 > lz->max_steps)
    return fail(FHASH_ERANGE, "lazy record full (%lld steps)", (long long)lz->max_steps);
  if (opt->moments != lz->moments)
    return fail(FHASH_EINVAL, "the step's moments layout differs from the deferred state's");
  if (lz->beta1 < 0.0) {
    lz->beta1 = opt->beta1;
    lz->beta2 = opt->beta2;
    lz->eps = opt->eps;
  } else if (lz->beta1 != opt->beta1 || lz->beta2 != opt->beta2 || lz->eps != opt->eps) {
    return fail(FHASH_EINVAL, "beta1, beta2 and eps must not change under lazy updates");
  }
  hipStream_t st = S(stream);
  // dense part: [0, begin) and [end, n)
  hipError_t e = fh::launch_adam(opt, param, grad, m, v, shadow, shadow_dt, lz->begin, 0,
                                 found_inf, nullptr, st);
  if (e == hipSuccess)
    e = fh::launch_adam(opt, param, grad, m, v, shadow, shadow_dt, n - lz->end, lz->end,
                        found_inf, nullptr, st);
  if (e == hipSuccess)
    e = fh::launch_lazy_step(opt, lz, found_inf, st);
  if (e != hipSuccess) return hip_status(e, "fhash_step_lazy");
  if (!std::isfinite((float)opt->grad_scale)) lz->flags |= 1;
  lz->steps += 1;
  return FHASH_OK;
}

int fhash_lazy_stats(const fhash_lazy* lz, int64_t stats[4], void* stream) {
  int rc = check_lazy(lz);
  if (rc) return rc;
  if (stats == nullptr) return fail(FHASH_EINVAL, "stats is NULL");
  return hip_status(fh::lazy_read_stats(lz, stats, S(stream)), "fhash_lazy_stats");
}

int fhash_lazy_flush(fhash_lazy* lz, float* param, float* grad, float* m, float* v, void* shadow,
                     fhash_dtype shadow_dt, void* stream) {
  int rc = check_lazy(lz);
  if (rc) return rc;
  if (param == nullptr || grad == nullptr || m == nullptr || v == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (!aligned16(param) || !aligned16(grad) || !aligned16(m) || !aligned16(v))
    return fail(FHASH_EINVAL, "optimiser arrays must be 16-byte aligned");
  if ((rc = check_state_pointers(lz->moments, param, grad, m, v))) return rc;
  if (shadow != nullptr && shadow_dt != FHASH_F16 && shadow_dt != FHASH_BF16)
    return fail(FHASH_EINVAL, "shadow dtype must be F16 or BF16");
  if (shadow != nullptr && (reinterpret_cast<uintptr_t>(shadow) & 7u) != 0)
    return fail(FHASH_EINVAL, "shadow must be 8-byte aligned");
  return hip_status(fh::launch_lazy_flush(lz, param, grad, m, v, shadow, shadow_dt, S(stream)),
                    "fhash_lazy_flush");
}

int fhash_check_finite(const float* grad, int64_t n, int32_t* found_inf, void* stream) {
  if (n < 0 || found_inf == nullptr || (n > 0 && grad == nullptr))
    return fail(FHASH_EINVAL, "bad arguments");
  return hip_status(fh::launch_check_finite(grad, n, found_inf, S(stream)), "fhash_check_finite");
}

int fhash_cast(const float* src, void* dst, fhash_dtype dst_dt, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (src == nullptr || dst == nullptr)))
    return fail(FHASH_EINVAL, "bad arguments");
  if (dst_dt != FHASH_F16 && dst_dt != FHASH_BF16)
    return fail(FHASH_EINVAL, "cast target must be F16 or BF16");
  return hip_status(fh::launch_cast(src, dst, dst_dt, n, S(stream)), "fhash_cast");
}

int fhash_sample(uint64_t seed, uint64_t step, int64_t n, const uint64_t* coreset, uint64_t M,
                 const int64_t dims[4], const float* field, const float* frame_t,
                 const int32_t* box, float* pos, float* target, void* stream) {
  if (n < 0 || dims == nullptr) return fail(FHASH_EINVAL, "bad arguments");
  for (int d = 0; d < 4; ++d)
    if (dims[d] < 2 || dims[d] > (1 << 24))
      return fail(FHASH_EINVAL, "dims[%d] outside [2, 2^24]", d);
  const uint64_t nvox = (uint64_t)dims[0] * dims[1] * dims[2] * dims[3];
  if (coreset == nullptr && M != nvox)
    return fail(FHASH_EINVAL, "without a coreset M must be the voxel count");
  if (n == 0) return FHASH_OK;
  if (M == 0) return fail(FHASH_EINVAL, "M == 0");
  if (field == nullptr || pos == nullptr || target == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (!aligned16(pos)) return fail(FHASH_EINVAL, "pos not 16-byte aligned");
  if (box != nullptr)
    for (int d = 0; d < 3; ++d)
      if (box[d] < 0 || box[d + 3] <= box[d] || box[d + 3] >= dims[d])
        return fail(FHASH_EINVAL, "box axis %d [%d, %d] not inside [0, %lld) with two voxels",
                    d, box[d], box[d + 3], (long long)dims[d]);
  return hip_status(fh::launch_sample(seed, step, n, coreset, M, dims, field, frame_t, box, pos,
                                      target, S(stream)),
                    "fhash_sample");
}

int fhash_sort_samples(float* pos, float* target, int64_t n, void* ws, size_t* ws_bytes,
                       void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(FHASH_EINVAL, "n outside [0, 2^31)");
  bool query;
  int rc = ws_check(ws, ws_bytes, fh::sort_ws_bytes(n), &query);
  if (rc || query) return rc;
  if (n == 0) return FHASH_OK;
  if (pos == nullptr || !aligned16(pos)) return fail(FHASH_EINVAL, "pos NULL or not 16-byte aligned");
  return hip_status(fh::launch_sort_samples(pos, target, n, ws, S(stream)), "fhash_sort_samples");
}

int fhash_sq_err_sum(const float* y, const float* v, int64_t n, double* sum, void* stream) {
  if (n < 0 || sum == nullptr || (n > 0 && (y == nullptr || v == nullptr)))
    return fail(FHASH_EINVAL, "bad arguments");
  return hip_status(fh::launch_sq_err(y, v, n, sum, S(stream)), "fhash_sq_err_sum");
}

int fhash_mse_grad(const float* y, const float* v, int64_t n, float loss_scale, float* dy,
                   double* loss_sum, void* stream) {
  if (n < 0 || (n > 0 && (y == nullptr || v == nullptr || dy == nullptr)))
    return fail(FHASH_EINVAL, "bad arguments");
  const float coef = n > 0 ? (float)(2.0 * (double)loss_scale / (double)n) : 0.0f;
  return hip_status(fh::launch_mse_grad(y, v, n, coef, dy, loss_sum, S(stream)), "fhash_mse_grad");
}

static int check_dims(const int64_t* dims) {
  if (dims == nullptr) return fail(FHASH_EINVAL, "dims is NULL");
  for (int d = 0; d < 4; ++d)
    if (dims[d] < 2 || dims[d] > (1 << 24)) return fail(FHASH_EINVAL, "dims[%d] outside [2, 2^24]", d);
  return FHASH_OK;
}

static int check_opts(const fhash_render_opts* o) {
  if (o == nullptr) return fail(FHASH_EINVAL, "render options are NULL");
  if (!(o->ds > 0.0f) || !(o->alpha_stop > 0.0f && o->alpha_stop <= 1.0f) || o->arm_max < 1 ||
      o->max_steps < 1)
    return fail(FHASH_EINVAL, "bad render options");
  return FHASH_OK;
}

int fhash_render_state_bytes(int32_t W, int32_t H, const int64_t dims[4], size_t* bytes) {
  int rc = check_dims(dims);
  if (rc) return rc;
  if (W < 1 || H < 1 || (int64_t)W * H > (int64_t)1 << 30 || bytes == nullptr)
    return fail(FHASH_EINVAL, "bad image size");
  *bytes = fh::render_ws_bytes((int64_t)W * H, dims);
  return FHASH_OK;
}

static int render_begin(const fhash_view* view, float t, int32_t W, int32_t H,
                        const uint64_t* mask_bits, bool brick_grid, const int64_t dims[4],
                        void* ws, size_t ws_bytes, float* rgba, fhash_render_state* state,
                        void* stream) {
  size_t need;
  int rc = fhash_render_state_bytes(W, H, dims, &need);
  if (rc) return rc;
  if (view == nullptr || mask_bits == nullptr || ws == nullptr || rgba == nullptr ||
      state == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (ws_bytes < need) return fail(FHASH_ENOMEM, "render workspace %zu < %zu", ws_bytes, need);
  if (!aligned16(ws) || !aligned16(rgba)) return fail(FHASH_EINVAL, "ws/rgba not 16-byte aligned");
  if (!(t >= 0.0f) || t > (float)(dims[3] - 1)) return fail(FHASH_EINVAL, "t outside [0, T-1]");
  std::memset(state, 0, sizeof(*state));
  state->W = W;
  state->H = H;
  state->t = t;
  state->t01 = t / (float)(dims[3] - 1);
  state->ws = ws;
  for (int d = 0; d < 4; ++d) state->dims[d] = dims[d];
  int32_t na = 0;
  hipError_t e =
      fh::launch_render_begin(view, W, H, mask_bits, brick_grid, dims, t, ws, &na, rgba, S(stream));
  if (e != hipSuccess) return hip_status(e, "fhash_render_begin");
  state->n_alive = na;
  state->cur = 0;
  return FHASH_OK;
}

int fhash_render_begin(const fhash_view* view, float t, int32_t W, int32_t H,
                       const uint64_t* mask_bits, const int64_t dims[4], void* ws,
                       size_t ws_bytes, float* rgba, fhash_render_state* state, void* stream) {
  return render_begin(view, t, W, H, mask_bits, false, dims, ws, ws_bytes, rgba, state, stream);
}

int fhash_render_begin_grid(const fhash_view* view, float t, int32_t W, int32_t H,
                            const uint64_t* occ, const int64_t dims[4], void* ws,
                            size_t ws_bytes, float* rgba, fhash_render_state* state,
                            void* stream) {
  if (dims != nullptr && fhash_occupancy_words(dims) < 0)
    return fail(FHASH_EINVAL, "dims outside the occupancy grid's range");
  return render_begin(view, t, W, H, occ, true, dims, ws, ws_bytes, rgba, state, stream);
}

int32_t fhash_render_pace(int64_t budget, int64_t alive, int32_t arm_max) {
  if (alive <= 0) return 1;
  int64_t p = budget / alive;
  if (p > arm_max) p = arm_max;
  if (p < 1) p = 1;
  return (int32_t)p;
}

int fhash_render_march(fhash_render_state* state, const fhash_render_opts* opts, int32_t pace,
                       float* pos_out, int64_t cap, int64_t* n_samples, void* stream) {
  int rc = check_opts(opts);
  if (rc) return rc;
  if (state == nullptr || state->ws == nullptr || n_samples == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (pace < 1 || pace > opts->arm_max) return fail(FHASH_EINVAL, "pace outside [1, arm_max]");
  if (state->pending) return fail(FHASH_EINVAL, "previous samples not composited");
  if ((int64_t)pace * state->n_alive > cap)
    return fail(FHASH_EINVAL, "sample buffer %lld < pace * alive", (long long)cap);
  if ((int64_t)pace * state->n_alive > (int64_t)INT32_MAX)
    return fail(FHASH_EINVAL, "pace * alive exceeds 2^31 - 1 samples per march");
  if (state->n_alive > 0 && (pos_out == nullptr || !aligned16(pos_out)))
    return fail(FHASH_EINVAL, "pos_out NULL or not 16-byte aligned");
  int32_t ns = 0;
  hipError_t e = fh::launch_render_march(state->ws, state->W, state->H, state->dims, state->t01,
                                         opts->ds, opts->max_steps, pace, state->cur,
                                         state->n_alive, pos_out, &ns, S(stream));
  if (e != hipSuccess) return hip_status(e, "fhash_render_march");
  *n_samples = ns;
  state->pending = 1;
  state->samples += ns;
  return FHASH_OK;
}

int fhash_render_composite(fhash_render_state* state, const float* y, const float* tf,
                           const fhash_render_opts* opts, float* rgba, void* stream) {
  int rc = check_opts(opts);
  if (rc) return rc;
  if (state == nullptr || state->ws == nullptr || tf == nullptr || rgba == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (!state->pending) return fail(FHASH_EINVAL, "composite without a march");
  int32_t na = 0;
  hipError_t e = fh::launch_render_composite(state->ws, state->W, state->H, state->cur,
                                             state->n_alive, y, tf, opts->alpha_stop, rgba, &na,
                                             S(stream));
  if (e != hipSuccess) return hip_status(e, "fhash_render_composite");
  state->cur = 1 - state->cur;
  state->n_alive = na;
  state->pending = 0;
  state->iterations += 1;
  return FHASH_OK;
}

// n distinct states with distinct workspaces (the batched kernels update
// each request's rays through its own workspace).
static int check_batch(fhash_render_state* const* states, int32_t n, bool pending) {
  if (states == nullptr) return fail(FHASH_EINVAL, "states is NULL");
  if (n < 1 || n > FHASH_RENDER_BATCH_MAX)
    return fail(FHASH_EINVAL, "batch of %d requests outside [1, %d]", n, FHASH_RENDER_BATCH_MAX);
  for (int32_t r = 0; r < n; ++r) {
    const fhash_render_state* s = states[r];
    if (s == nullptr || s->ws == nullptr) return fail(FHASH_EINVAL, "state %d is NULL", r);
    if ((s->pending != 0) != pending)
      return fail(FHASH_EINVAL, pending ? "state %d: composite without a march"
                                        : "state %d: previous samples not composited", r);
    for (int32_t q = 0; q < r; ++q)
      if (states[q] == s || states[q]->ws == s->ws)
        return fail(FHASH_EINVAL, "states %d and %d share a state or workspace", q, r);
  }
  return FHASH_OK;
}

int fhash_render_march_batch(fhash_render_state* const* states, const int32_t* paces, int32_t n,
                             const fhash_render_opts* opts, float* pos, int64_t out_base,
                             int64_t cap, int32_t* counts, int64_t* n_samples, void* stream) {
  int rc = check_opts(opts);
  if (rc) return rc;
  if ((rc = check_batch(states, n, false))) return rc;
  if (paces == nullptr || counts == nullptr || n_samples == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (out_base < 0) return fail(FHASH_EINVAL, "out_base < 0");
  int64_t need = out_base;
  for (int32_t r = 0; r < n; ++r) {
    if (paces[r] < 1 || paces[r] > opts->arm_max)
      return fail(FHASH_EINVAL, "pace of request %d outside [1, arm_max]", r);
    need += (int64_t)paces[r] * states[r]->n_alive;
  }
  if (need > cap) return fail(FHASH_EINVAL, "sample buffer %lld < out_base + sum pace * alive",
                              (long long)cap);
  // (the launch pads each request's rays to whole waves: 63 more per request)
  if (need + 64 * (int64_t)n > (int64_t)INT32_MAX)
    return fail(FHASH_EINVAL, "out_base + sum pace * alive exceeds 2^31 - 1 - 64 n");
  if (need > out_base && (pos == nullptr || !aligned16(pos)))
    return fail(FHASH_EINVAL, "pos NULL or not 16-byte aligned");
  fh::RenderBatch b[FHASH_RENDER_BATCH_MAX];
  for (int32_t r = 0; r < n; ++r) {
    const fhash_render_state* s = states[r];
    b[r] = fh::RenderBatch{s->ws, s->W, s->H, s->cur, s->n_alive, paces[r], s->t01, s->dims,
                           nullptr, nullptr};
  }
  int32_t host[1 + FHASH_RENDER_BATCH_MAX];
  hipError_t e = fh::launch_render_march_batch(b, n, opts->ds, opts->max_steps, pos, out_base,
                                               counts, host, S(stream));
  if (e != hipSuccess) return hip_status(e, "fhash_render_march_batch");
  for (int32_t r = 0; r < n; ++r) {
    n_samples[r] = host[1 + r];
    states[r]->pending = 1;
    states[r]->samples += host[1 + r];
  }
  return FHASH_OK;
}

int fhash_render_composite_batch(fhash_render_state* const* states, int32_t n, const float* y,
                                 const float* const* tf, float* const* rgba,
                                 const fhash_render_opts* opts, int32_t* counts, void* stream) {
  int rc = check_opts(opts);
  if (rc) return rc;
  if ((rc = check_batch(states, n, true))) return rc;
  if (tf == nullptr || rgba == nullptr || counts == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  int64_t rays = 0;
  for (int32_t r = 0; r < n; ++r) rays += ((int64_t)states[r]->n_alive + 63) & ~(int64_t)63;
  if (rays > (int64_t)INT32_MAX)
    return fail(FHASH_EINVAL, "the batch's alive rays, padded to whole waves, exceed 2^31 - 1");
  fh::RenderBatch b[FHASH_RENDER_BATCH_MAX];
  for (int32_t r = 0; r < n; ++r) {
    const fhash_render_state* s = states[r];
    if (tf[r] == nullptr || rgba[r] == nullptr)
      return fail(FHASH_EINVAL, "request %d: NULL transfer function or image", r);
    b[r] = fh::RenderBatch{s->ws, s->W, s->H, s->cur, s->n_alive, 0, s->t01, s->dims, tf[r],
                           rgba[r]};
  }
  int32_t host[1 + FHASH_RENDER_BATCH_MAX];
  hipError_t e = fh::launch_render_composite_batch(b, n, y, opts->alpha_stop, counts, host,
                                                   S(stream));
  if (e != hipSuccess) return hip_status(e, "fhash_render_composite_batch");
  for (int32_t r = 0; r < n; ++r) {
    fhash_render_state* s = states[r];
    s->cur = 1 - s->cur;
    s->n_alive = host[1 + r];
    s->pending = 0;
    s->iterations += 1;
  }
  return FHASH_OK;
}

int fhash_render(const fhash_index* idx, const fhash_mlp_desc* mlp, const void* table,
                 fhash_dtype table_dt, const float* params, const uint64_t* mask_bits,
                 const int64_t dims[4], const fhash_view* view, float t, const float* tf,
                 int32_t W, int32_t H, const fhash_render_opts* opts, float* rgba, void* ws,
                 size_t* ws_bytes, fhash_render_stats* stats, void* stream) {
  size_t sbytes;
  int rc = fhash_render_state_bytes(W, H, dims, &sbytes);
  if (rc) return rc;
  if ((rc = check_opts(opts))) return rc;
  const int64_t NR = (int64_t)W * H;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t need = al(sbytes) + al(NR * 16) + al(NR * 4);
  bool query;
  rc = ws_check(ws, ws_bytes, need, &query);
  if (rc || query) return rc;
  int H_, NH;
  if ((rc = check_fused(idx, mlp, nullptr, 0, table, table_dt, params, &H_, &NH, false)))
    return rc;
  if (total_rows(idx) == 0) return fail(FHASH_EINVAL, "index has no active vertex");
  char* p = static_cast<char*>(ws);
  float* pos = reinterpret_cast<float*>(p + al(sbytes));
  float* y = reinterpret_cast<float*>(p + al(sbytes) + al(NR * 16));
  fhash_render_state st;
  rc = fhash_render_begin(view, t, W, H, mask_bits, dims, ws, sbytes, rgba, &st, stream);
  if (rc) return rc;
  fh::GridDev g;
  fh::make_grid_dev(idx, &g);
  const fhash_dtype tdt = table_view(table_dt, &g);
  while (st.n_alive > 0) {
    const int32_t pace = fhash_render_pace(NR, st.n_alive, opts->arm_max);
    int64_t ns = 0;
    rc = fhash_render_march(&st, opts, pace, pos, NR, &ns, stream);
    if (rc) return rc;
    if (ns > 0) {
      hipError_t e =
          mlp->compute_dt != FHASH_F32
              ? fh::launch_fused_fwd16(g, H_, NH, mlp->compute_dt, pos, ns, table, tdt,
                                       params, y, S(stream))
              : fh::launch_fused_fwd(g, H_, NH, pos, ns, table, tdt, params, y, S(stream));
      if (e != hipSuccess) return hip_status(e, "fhash_render decode");
    }
    rc = fhash_render_composite(&st, y, tf, opts, rgba, stream);
    if (rc) return rc;
  }
  if (stats) {
    stats->iterations = st.iterations;
    stats->samples = st.samples;
  }
  return FHASH_OK;
}

// ------------------------------------------------------------------ coreset

static int check_mask_dims(const int64_t dims[4]) {
  if (dims == nullptr) return fail(FHASH_EINVAL, "dims is NULL");
  for (int d = 0; d < 4; ++d)
    if (dims[d] < 2 || dims[d] > 0x7fffffffLL)
      return fail(FHASH_EINVAL, "dims[%d] = %lld outside [2, 2^31 - 1]", d, (long long)dims[d]);
  if (dims[3] > 65535) return fail(FHASH_EINVAL, "T = %lld above 65535", (long long)dims[3]);
  const double words = (double)dims[3] * dims[2] * dims[1] * ((dims[0] + 63) / 64);
  if (words >= 70368744177664.0) return fail(FHASH_ERANGE, "2^46 mask words or more");
  // one workgroup per (t, z) slice, 32-bit word index inside a slice
  if ((double)dims[3] * dims[2] >= 2147483648.0 ||
      (double)dims[1] * ((dims[0] + 63) / 64) >= 2147483648.0 ||
      (double)((dims[1] + 3) / 4) * ((dims[0] + 3) / 4) >= 2147483648.0)
    return fail(FHASH_ERANGE, "T Sz, or the words or bricks of one slice, reach 2^31");
  return FHASH_OK;
}

// Byte ranges [a, a + na) and [b, b + nb) share a byte.
static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return na > 0 && nb > 0 && pa < pb + nb && pb < pa + na;
}

int fhash_feature_mask(const float* field, const int64_t dims[4], int32_t kind, float lo,
                       float hi, uint64_t* bits, void* ws, size_t* ws_bytes, void* stream) {
  if (int rc = check_mask_dims(dims)) return rc;
  if (kind != FHASH_FEATURE_INTERVAL && kind != FHASH_FEATURE_ISOSURFACE)
    return fail(FHASH_EINVAL, "unknown feature kind %d", kind);
  const size_t need = fh::feature_ws_bytes(dims, kind);
  if (ws == nullptr && ws_bytes != nullptr) {
    *ws_bytes = need;
    return FHASH_OK;
  }
  if (need > 0) {
    bool query;
    if (int rc = ws_check(ws, ws_bytes, need, &query)) return rc;
  }
  if (field == nullptr || bits == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  const size_t mask_bytes = (size_t)fh::mask_words(dims) * 8;
  const size_t field_bytes = (size_t)dims[0] * dims[1] * dims[2] * dims[3] * sizeof(float);
  if (ranges_overlap(bits, mask_bytes, field, field_bytes))
    return fail(FHASH_EINVAL, "bits overlap the field");
  if (kind == FHASH_FEATURE_ISOSURFACE &&
      (ranges_overlap(ws, need, bits, mask_bytes) || ranges_overlap(ws, need, field, field_bytes)))
    return fail(FHASH_EINVAL, "workspace overlaps an argument");
  return hip_status(fh::launch_feature_mask(field, dims, kind, lo, hi, bits, ws, S(stream)),
                    "fhash_feature_mask");
}

int fhash_dilate_mask(const uint64_t* in, const int64_t dims[4], int32_t r, uint64_t* out,
                      void* stream) {
  if (int rc = check_mask_dims(dims)) return rc;
  if (r < 0 || r > 63) return fail(FHASH_EINVAL, "radius %d outside [0, 63]", r);
  if (in == nullptr || out == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  const uint64_t* oend = out + fh::mask_words(dims);
  const uint64_t* iend = in + fh::mask_words(dims);
  if (in < oend && out < iend) return fail(FHASH_EINVAL, "in and out overlap");
  return hip_status(fh::launch_dilate_mask(in, dims, r, out, S(stream)), "fhash_dilate_mask");
}

int fhash_feature_boxes(const uint64_t* bits, const int64_t dims[4], int32_t* box, void* stream) {
  if (int rc = check_mask_dims(dims)) return rc;
  if (bits == nullptr || box == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  return hip_status(fh::launch_feature_boxes(bits, dims, box, S(stream)), "fhash_feature_boxes");
}

int64_t fhash_occupancy_words(const int64_t dims[4]) {
  if (check_mask_dims(dims)) return -1;
  return fh::occupancy_words(dims);
}

int fhash_occupancy_grid(const uint64_t* bits, const int64_t dims[4], uint64_t* occ,
                         void* stream) {
  if (int rc = check_mask_dims(dims)) return rc;
  if (bits == nullptr || occ == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  return hip_status(fh::launch_occupancy_morton(bits, dims, occ, S(stream)),
                    "fhash_occupancy_grid");
}

int fhash_coreset(const uint64_t* bits, const int64_t dims[4], uint64_t* ids, int64_t capacity,
                  void* ws, size_t* ws_bytes, int64_t* count, void* stream) {
  if (int rc = check_mask_dims(dims)) return rc;
  bool query;
  if (int rc = ws_check(ws, ws_bytes, fh::coreset_ws_bytes(dims), &query)) return rc;
  if (query) return FHASH_OK;
  if (bits == nullptr || count == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  if (ids != nullptr && capacity < 0) return fail(FHASH_EINVAL, "negative capacity");
  const size_t mask_bytes = (size_t)fh::mask_words(dims) * 8;
  if (ranges_overlap(ws, fh::coreset_ws_bytes(dims), bits, mask_bytes))
    return fail(FHASH_EINVAL, "workspace overlaps the mask");
  if (ids != nullptr && (ranges_overlap(ids, (size_t)capacity * 8, bits, mask_bytes) ||
                         ranges_overlap(ids, (size_t)capacity * 8, ws,
                                        fh::coreset_ws_bytes(dims))))
    return fail(FHASH_EINVAL, "ids overlap the mask or the workspace");
  return hip_status(fh::launch_coreset(bits, dims, ws, ids, capacity, count, S(stream)),
                    "fhash_coreset");
}

int fhash_coreset_frames(const uint64_t* bits, const int64_t dims[4], const int32_t* frames,
                         int32_t n_frames, uint64_t* ids, int64_t capacity, void* ws,
                         size_t* ws_bytes, int64_t* count, void* stream) {
  if (int rc = check_mask_dims(dims)) return rc;
  bool query;
  if (int rc = ws_check(ws, ws_bytes, fh::coreset_frames_ws_bytes(dims), &query)) return rc;
  if (query) return FHASH_OK;
  if (bits == nullptr || count == nullptr) return fail(FHASH_EINVAL, "NULL pointer");
  if (n_frames < 0 || (n_frames > 0 && frames == nullptr))
    return fail(FHASH_EINVAL, "bad frame list");
  for (int32_t k = 0; k < n_frames; ++k) {
    if (frames[k] < 0 || frames[k] >= dims[3])
      return fail(FHASH_EINVAL, "frame %d outside [0, %lld)", frames[k], (long long)dims[3]);
    if (k > 0 && frames[k] <= frames[k - 1])
      return fail(FHASH_EINVAL, "frames must be strictly increasing");
  }
  if (ids != nullptr && capacity < 0) return fail(FHASH_EINVAL, "negative capacity");
  const size_t mask_bytes = (size_t)fh::mask_words(dims) * 8;
  const size_t ws_need = fh::coreset_frames_ws_bytes(dims);
  if (ranges_overlap(ws, ws_need, bits, mask_bytes))
    return fail(FHASH_EINVAL, "workspace overlaps the mask");
  if (ids != nullptr && (ranges_overlap(ids, (size_t)capacity * 8, bits, mask_bytes) ||
                         ranges_overlap(ids, (size_t)capacity * 8, ws, ws_need)))
    return fail(FHASH_EINVAL, "ids overlap the mask or the workspace");
  return hip_status(fh::launch_coreset_frames(bits, dims, frames, n_frames, ws, ids, capacity,
                                              count, S(stream)),
                    "fhash_coreset_frames");
}

int fhash_fold_resolutions(const int64_t size[4], int32_t fold, int32_t* res,
                           int32_t* n_levels) {
  if (size == nullptr || res == nullptr || n_levels == nullptr)
    return fail(FHASH_EINVAL, "NULL pointer");
  if (fold < 2) return fail(FHASH_EINVAL, "fold %d < 2", fold);
  // levels of each dimension: the smallest L with fold^L >= S (exact integers)
  int32_t L = 0;
  for (int d = 0; d < 4; ++d) {
    if (size[d] < 2 || size[d] > (1 << 24))
      return fail(FHASH_EINVAL, "size[%d] = %lld outside [2, 2^24]", d, (long long)size[d]);
    int32_t Ld = 0;
    for (int64_t p = 1; p < size[d]; p *= fold) ++Ld;
    if (Ld > L) L = Ld;
  }
  if (L > FHASH_MAX_LEVELS)
    return fail(FHASH_ERANGE, "%d levels exceed FHASH_MAX_LEVELS", L);
  // paper level 1 (finest) = the native size; each coarser level divides by the
  // fold (rounding up) while above it, else the tail resolution 2.  Stored
  // coarsest first: row L - 1 is the native size.
  for (int d = 0; d < 4; ++d) {
    int64_t r = size[d];
    for (int32_t l = 0; l < L; ++l) {
      res[(L - 1 - l) * 4 + d] = (int32_t)r;
      r = (r > fold) ? (r + fold - 1) / fold : 2;
    }
  }
  *n_levels = L;
  return FHASH_OK;
}

int fhash_key_frame_times(int64_t T, const int32_t* frames, int32_t n_frames, float* frame_t) {
  if (T < 2 || frames == nullptr || frame_t == nullptr || n_frames < 2)
    return fail(FHASH_EINVAL, "need T >= 2 and at least two key frames");
  for (int32_t k = 0; k < n_frames; ++k) {
    if (frames[k] < 0 || frames[k] >= T)
      return fail(FHASH_EINVAL, "key frame %d outside [0, %lld)", frames[k], (long long)T);
    if (k > 0 && frames[k] <= frames[k - 1])
      return fail(FHASH_EINVAL, "key frames must be strictly increasing");
  }
  const double last = (double)(n_frames - 1);
  int32_t k = 0;
  for (int64_t n = 0; n < T; ++n) {
    double tau;
    if (n <= frames[0]) {
      tau = 0.0;
    } else if (n >= frames[n_frames - 1]) {
      tau = 1.0;
    } else {
      while (frames[k + 1] <= n) ++k;
      tau = ((double)k + (double)(n - frames[k]) / (double)(frames[k + 1] - frames[k])) / last;
    }
    frame_t[n] = (float)tau;
  }
  return FHASH_OK;
}

}  // extern "C"
