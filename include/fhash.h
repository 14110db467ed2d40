/*
 * fhash.h -- C ABI of the MI355X (gfx950) F-Hash hot path.
 *
 * F-Hash (feature-based hash for time-varying volumes, arXiv 2507.03836)
 * encodes a 4D sample (x, y, z, t) with a stack of multi-resolution
 * "tesseract" embedding grids (Sec. 3.2), each addressed by a collision-free
 * per-level hash (Sec. 3.2.3), interpolates the 16 corner embeddings of the
 * containing 4D cell (Sec. 3.2.4), concatenates the levels and decodes them
 * with a small MLP.  Training is Adam (Sec. 5.1.3); rendering is ray marching
 * with an adaptive marching pace (Sec. 3.3, Algorithm 1).
 *
 * Conventions shared by every call
 *  - Every call returns an int status (FHASH_OK = 0, negative on error) and
 *    never throws.  A message for the last failure on the calling thread is
 *    available from fhash_last_error().
 *  - All arguments are validated on the host before any launch; invalid ones
 *    return FHASH_EINVAL and launch nothing.
 *  - "device" pointers are HIP device memory owned by the caller.  The library
 *    allocates nothing; calls that need scratch memory take a workspace
 *    (void* ws, size_t* ws_bytes): with ws == NULL the call only writes the
 *    required size to *ws_bytes and returns FHASH_OK.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = default
 *    stream) unless stated otherwise.  Launch failures surface as FHASH_EHIP.
 *  - Positions are FP32 (x, y, z, t) in [0,1]^4, 16-byte aligned, one float4
 *    per sample.  Values outside [0,1] are clamped (NaN -> 0).
 *  - Level vertex i of a dimension with R vertices sits at i/(R-1); level 0 is
 *    the coarsest level and the MLP input is levels 0..L-1 concatenated,
 *    F features per level.
 */
#ifndef FHASH_H
#define FHASH_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FHASH_VERSION 1
#define FHASH_MAX_LEVELS 24
#define FHASH_MAX_LAYERS 8

enum {
  FHASH_OK = 0,
  FHASH_EINVAL = -1,  /* bad argument (NULL, size, shape, alignment)        */
  FHASH_ENOMEM = -2,  /* workspace too small                                 */
  FHASH_EHIP = -3,    /* HIP launch / runtime error                          */
  FHASH_ERANGE = -4,  /* a count or index exceeds its representable range    */
  FHASH_ENOTSUP = -5  /* valid but not built (dtype, feature count, width)   */
};

/* FHASH_F32_PAIRED (a table dtype only): FP32 values stored in runs of 16
 * floats, each run followed by 16 floats of another array (in the optimiser
 * layout FHASH_MOMENTS_WITH_PARAMS below, those are the same parameters'
 * first moments): value i at float i + 16 floor(i / 16). */
typedef enum { FHASH_F32 = 0, FHASH_F16 = 1, FHASH_BF16 = 2, FHASH_F32_PAIRED = 3 } fhash_dtype;

/* Level structure of the multi-resolution tesseract grid (Sec. 3.2.1-3.2.2).
 * res[l] = vertex counts (x, y, z, t) of level l, each in [2, 2^24], with
 * y * z * t * ceil(x / 64) < 2^31 per level (FHASH_ERANGE otherwise: the
 * kernels index a level's vertex rows and directory words in 32 bits).
 * n_features = F, the embedding size of a vertex (Sec. 4.1): 1, 2, 4 or 8. */
/* Slot order of an active-vertex index (layout below). */
enum { FHASH_LAYOUT_ROWS = 0, FHASH_LAYOUT_BRICKS = 1 };

typedef struct {
  int32_t n_levels;
  int32_t n_features;
  int32_t res[FHASH_MAX_LEVELS][4];
  int32_t layout;  /* FHASH_LAYOUT_ROWS or FHASH_LAYOUT_BRICKS (see the index section) */
} fhash_grid_desc;

/* Voxel feature mask (the dilated feature region d_k of Sec. 3.1, one bit per
 * voxel and timestep).  dims = (Sx, Sy, Sz, T), each >= 2; voxel i of a
 * dimension with S samples sits at i/(S-1).  Layout: rows of ceil(Sx/64)
 * uint64 words, [T][Sz][Sy][ceil(Sx/64)]; bit b of word w of a row is voxel
 * x = 64 w + b; padding bits must be zero.  bits == NULL: the dense box. */
typedef struct {
  const uint64_t* bits; /* device */
  int64_t dims[4];
} fhash_mask_desc;

/* Built index (a plain view; valid while `dir` lives).  Filled by
 * fhash_build_index; callers treat it as read-only and may share it. */
typedef struct {
  fhash_grid_desc grid;
  int32_t active;   /* 0: dense box, every vertex has a slot; 1: active vertices only */
  int32_t hash_bits; /* 0, or b (dense box only): levels of more than 2^b vertices hash
                        into 2^b rows (fhash_hash_index) */
  const void* dir;  /* device rank directory (16-byte entries), NULL when dense */
  int64_t dir_offset[FHASH_MAX_LEVELS + 1];  /* first directory entry of each level */
  int64_t slot_offset[FHASH_MAX_LEVELS + 1]; /* first table row of each level; [L] = rows */
} fhash_index;

int fhash_version(void);
const char* fhash_last_error(void);

/* ---------------------------------------------------------------- index ----
 * The per-level collision-free hash (Sec. 3.2.3, the F-Hash equation, and the
 * "irregular feature region" variant of Sec. 3.1 that it makes fast).
 *
 * A 4D cell of level l is active iff its closed box contains a masked voxel;
 * a vertex is active iff it is a corner of an active cell (embeddings live at
 * cell corners, Sec. 3.2.4 step 3).  The slot of an active vertex is its rank
 * among the level's active vertices in the F-Hash linearisation
 *   lin = ((t*Rz + z)*Ry + y)*Rx + x,
 * so the table has exactly one row per active vertex: no collision and no
 * unused bucket.  With mask->bits == NULL every vertex is active and the slot
 * is the F-Hash equation itself.  Level l owns rows
 * [slot_offset[l], slot_offset[l+1]) of every table.
 *
 * Directory of an active index (per level, from dir_offset[l]): one 16-byte
 * entry {uint64 bits, uint64 rank} per 64-vertex word w of every vertex row
 * (t, z, y): bit b of `bits` is vertex x = 64 w + b, `rank` the number of
 * active vertices before that word in F-Hash order; the entry sits at
 * ((t*Rz + z)*ceil(Rx/64) + w)*Ry + y, so rows y and y+1 are neighbours.
 *
 * Brick layout (grid->layout = FHASH_LAYOUT_BRICKS; active index only, Sec.
 * 3.2.3 allows linearisations other than the F-Hash equation's): the same
 * active set ranked in bricks of 2 x 2 x 2 x 2 vertices, brick (bx, by, bz, bt)
 * = (x/2, y/2, z/2, t/2), bricks in the F-Hash equation's order (bx fastest),
 * vertices inside a brick by inner = x%2 + 2 (y%2) + 4 (z%2) + 8 (t%2); missing
 * vertices of edge bricks take no slot.  A cell then touches about 5 table
 * lines instead of 8.  Directory: one entry per 64 bits = 4 bricks of a brick
 * row (bt, bz, by): bit 16 (bx % 4) + inner of word bx / 4, `rank` the active
 * vertices before the word in brick order; the entry sits at
 * ((bt*Bz + bz)*Wb + w)*By + by, Bz = ceil(Rz/2), By = ceil(Ry/2),
 * Wb = ceil(ceil(Rx/2)/4).  fhash_dense_index and fhash_hash_index return
 * FHASH_ENOTSUP for this layout; the fused calls support it for 17-32 decoder
 * inputs with F = 2 or 4 and 2 or 3 hidden layers of 64 (FHASH_ENOTSUP
 * otherwise).
 *
 * fhash_index_dir_entries: number of 16-byte directory entries the grid needs
 * (0 for a dense index is not implied: the size is for the active form).
 * fhash_build_index: fills dir (device, dir_entries*16 bytes, caller-owned)
 * and *out, and writes the per-level active-vertex counts to the HOST array
 * slots_per_level[L].  This call synchronises `stream` (it returns counts).
 * ws: device workspace (query with ws == NULL).  Returns FHASH_ERANGE if a
 * level has 2^62 vertices or more. */
int fhash_index_dir_entries(const fhash_grid_desc* grid, int64_t* entries);
int fhash_build_index(const fhash_grid_desc* grid, const fhash_mask_desc* mask, void* dir,
                      void* ws, size_t* ws_bytes, fhash_index* out, int64_t* slots_per_level,
                      void* stream);
/* Dense index (every vertex active): no device memory, no launch. */
int fhash_dense_index(const fhash_grid_desc* grid, fhash_index* out, int64_t* slots_per_level);

/* Comparison index, not the method: a 4D spatial hash in the manner of
 * multiresolution hash encodings (the alternative discussed around Fig. 5 of
 * Sec. 3.2.3), on the same kernels.  Levels of at most 2^hash_bits vertices
 * keep the F-Hash equation (collision-free); a larger level has 2^hash_bits
 * rows and vertex (x, y, z, t) lives in row
 *   (x ^ y*2654435761 ^ z*805459861 ^ t*3674653429) mod 2^32 mod 2^hash_bits
 * (32-bit unsigned products), so distinct vertices may share a row and every
 * row may be used.  hash_bits in [4, 31].  Host only, no device memory. */
int fhash_hash_index(const fhash_grid_desc* grid, int32_t hash_bits, fhash_index* out,
                     int64_t* slots_per_level);

/* Level resolutions by the fold policy (Sec. 3.2.1 spatial, Sec. 3.2.2
 * temporal), host only.  size = (Sx, Sy, Sz, n_kf): the vertex counts of the
 * finest level, i.e. the FBB size in voxels and the number of key frames, each
 * in [2, 2^24]; fold >= 2.  Per dimension the finest level has `size`
 * vertices and each coarser level ceil(R / fold) while R > fold, else 2 (the
 * tail); the level count is the largest over the four dimensions of the
 * smallest L with fold^L >= size.  res (HOST int32 [FHASH_MAX_LEVELS][4]) row l
 * = level l, coarsest first (the fhash_grid_desc order); *n_levels = L.
 * FHASH_ERANGE when L > FHASH_MAX_LEVELS. */
int fhash_fold_resolutions(const int64_t size[4], int32_t fold, int32_t* res, int32_t* n_levels);

/* Time coordinate of every frame under key-frame training (Sec. 3.2.2), host
 * only: key frame k (frames: HOST int32[n_frames], strictly increasing, in
 * [0, T), n_frames >= 2) sits on vertex k of a temporal level of n_frames
 * vertices, tau = k / (n_frames - 1); a frame n between key frames k and k+1
 * gets tau = (k + (n - frames[k]) / (frames[k+1] - frames[k])) / (n_frames - 1)
 * (linear in the frame index between neighbouring key frames), frames before
 * the first key frame 0, after the last 1.  Evaluated in FP64, rounded to
 * FP32 into frame_t (HOST float[T]); the sampler and the renderer take these
 * as the model's time coordinate. */
int fhash_key_frame_times(int64_t T, const int32_t* frames, int32_t n_frames, float* frame_t);

/* -------------------------------------------------------------- encoding ----
 * Input encoding (Sec. 3.2.4): per level, locate the 4D cell containing the
 * sample (u = p*(R-1) as one FP32 multiply, cell = min(floor(u), R-2),
 * fraction = u - cell), look up the 16 corner slots, and blend the corner
 * embeddings with quadrilinear weights prod_d (f_d or 1 - f_d).  Inactive
 * corners contribute zero (no renormalisation).
 * pos: device float4[n]; table: device [rows][F] of table_dt (FHASH_F32 master,
 * FHASH_F32_PAIRED master in the paired layout, or FHASH_F16 shadow); enc:
 * device float [n][L*F], level-major.
 * FP32 accumulation. */
int fhash_encode_fwd(const fhash_index* idx, const float* pos, int64_t n, const void* table,
                     fhash_dtype table_dt, float* enc, void* stream);

/* Instrumentation, not part of the method: the memory one encoding (or its
 * adjoint) touches.  For sample s, level l and corner row r of the cell (the
 * vertex pair (x, x+1) at (y + (r & 1), z + (r >> 1 & 1), t + (r >> 2))):
 * out_dir[((s L + l) 8 + r) 2 + j] = the global index of the 16-byte directory
 * entry read (j = 0; j = 1 holds the next word's entry when x sits on bit 63
 * of its word, else -1; both -1 for a dense or hashed level), out_slot[... + e]
 * = the table row of vertex x + e (global, i.e. including slot_offset), -1
 * when the vertex is inactive.  Both device int64 [n][L][8][2].  Positions are
 * located exactly as fhash_encode_fwd does. */
int fhash_corner_rows(const fhash_index* idx, const float* pos, int64_t n, int64_t* out_dir,
                      int64_t* out_slot, void* stream);

/* Touched-segment tracking of a table gradient (an optimisation of the dense
 * Adam sweep, not part of the method): the gradient is viewed as segments of
 * FHASH_TOUCH_FLOATS floats; flags (device uint8, one per segment of the
 * whole table, i.e. ceil(rows * F / FHASH_TOUCH_FLOATS) bytes, caller-owned,
 * all zero before the first tracked write) gets a nonzero byte for every
 * segment at or after float index `begin` that a scatter-add wrote.  fhash_step then reads the gradient in [begin, end) only
 * where the segment is flagged (elsewhere it is zero by construction) and
 * clears the flags it read.  begin: a multiple of FHASH_TOUCH_FLOATS;
 * 0 <= begin <= end <= the gradient length.  Every writer of the gradient in
 * [begin, end) between two steps must be given the same descriptor. */
#define FHASH_TOUCH_FLOATS 16
typedef struct {
  uint8_t* flags;
  int64_t begin, end;
} fhash_touch;

/* Adjoint of the encoding: d_table[slot][k] += w_c * d_enc[s][l*F + k] for every
 * active corner c of every sample and level (FP32 atomics; summation order is
 * not deterministic).  The corner weights are recomputed from pos, not stored.
 * d_enc: device float [n][L*F]; d_table: device float [rows][F], accumulated
 * (dense; the fused calls below also write a gradient in the paired layout).
 * touch: NULL, or segment flags to set (see fhash_touch). */
int fhash_encode_bwd(const fhash_index* idx, const float* pos, int64_t n, const float* d_enc,
                     float* d_table, const fhash_touch* touch, void* stream);

/* ------------------------------------------------------------------- MLP ----
 * Shallow decoder (Sec. 3.2.4 end; 2 hidden layers of 64 in Sec. 4.2):
 * width[0] = input (<= 64), n_layers-1 hidden layers of equal width H
 * (16, 32 or 64) with ReLU, and a linear output of width 1; biases on.
 * params: device float, packed per layer k as W_k[width[k+1]][width[k]]
 * row-major then b_k[width[k+1]].  compute_dt: FHASH_F32 (FP32 MFMA) for
 * every call; FHASH_F16 (weights and hidden-layer inputs rounded to FP16 (RNE),
 * FP16 MFMA with FP32 accumulation, FP32 biases and output layer) for the
 * forward-only calls fhash_fused_fwd and fhash_render; other combinations
 * return FHASH_ENOTSUP.  `shadow` is reserved (pass NULL).
 */
typedef struct {
  int32_t n_layers;
  int32_t width[FHASH_MAX_LAYERS + 1];
  fhash_dtype compute_dt;
} fhash_mlp_desc;

int64_t fhash_mlp_num_params(const fhash_mlp_desc* mlp);

/* y[n] = MLP(x[n][width[0]]).  x, y: device float. */
int fhash_mlp_fwd(const fhash_mlp_desc* mlp, const float* params, const void* shadow,
                  const float* x, int64_t n, float* y, void* stream);

/* Reverse mode of fhash_mlp_fwd (activations are recomputed from x):
 * d_params (device float [P]) += dL/dparams, dx (device float [n][width[0]],
 * may be NULL) = dL/dx, for dy = dL/dy (device float [n]).  The parameter
 * gradient is reduced deterministically through the workspace. */
int fhash_mlp_bwd(const fhash_mlp_desc* mlp, const float* params, const void* shadow,
                  const float* x, const float* dy, int64_t n, float* d_params, float* dx,
                  void* ws, size_t* ws_bytes, void* stream);

/* ------------------------------------------------------------ fused path ----
 * Encoding fused with the decoder.  fhash_fused_fwd: y = MLP(encode(pos)).
 * fhash_fused_bwd: given dy, recompute the encoding and activations and
 * accumulate d_table (atomics) and d_params (each workgroup's waves add into
 * one LDS image in arrival order, the workgroups' images are then summed in a
 * fixed order: reproducible up to FP32 rounding, not bit for bit).
 * fhash_fused_train: forward, MSE loss against target, backward in one pass:
 *   dL/dy_s = loss_scale * 2 (y_s - target_s) / n,
 * loss_sum (device double, accumulated) += sum_s (y_s - target_s)^2. */
int fhash_fused_fwd(const fhash_index* idx, const fhash_mlp_desc* mlp, const float* pos, int64_t n,
                    const void* table, fhash_dtype table_dt, const float* params,
                    const void* shadow, float* y, void* stream);
/* flags: FHASH_SAMPLES_SORTED declares that the batch is ordered by
 * fhash_sort_samples; on the levels coarse enough for neighbouring samples to
 * share vertices, the scatter-add then sums a corner across the samples that
 * one of its instructions covers (16 at F = 1 and 2, 8 at F = 4) when they all
 * hit the same slot, and adds the sum with one atomic (atomics of different
 * lanes into one float cannot share a memory request).  Results are the same
 * up to FP32 summation order.  FHASH_GRAD_PAIRED: d_table is stored in runs
 * of 16 floats separated by 16-float gaps (gradient value i at
 * d_table[i + 16 floor(i / 16)]; the gradient array of the optimiser layout
 * FHASH_MOMENTS_WITH_PARAMS below); the table read is independent of it
 * (table_dt).  FHASH_COARSE_LDS: the levels with at most one cell per
 * sample of the batch (0 .. lc - 1, coarsest first; row-ordered indexes only,
 * ignored on brick-ordered ones) are not added by the fused kernel: their
 * encoding gradient goes to the workspace, and a second kernel on the same
 * stream sums it per chunk of 2048 consecutive samples into an LDS image of
 * the vertex box the chunk touches and adds that box with one atomic per
 * touched vertex and feature (a chunk whose box exceeds 16000 floats is taken
 * in 4 parts, and a part that still exceeds it adds its samples directly).
 * Sorted batches give compact boxes; the results are the same up to FP32
 * summation order.  The workspace then grows by lc x n x F floats (the size
 * query includes it).  Other bits: FHASH_EINVAL.  touch: NULL, or segment
 * flags of d_table to set, by logical float index (see fhash_touch). */
#define FHASH_SAMPLES_SORTED 1u
#define FHASH_GRAD_PAIRED 2u
#define FHASH_COARSE_LDS 4u
int fhash_fused_bwd(const fhash_index* idx, const fhash_mlp_desc* mlp, const float* pos, int64_t n,
                    const void* table, fhash_dtype table_dt, const float* params,
                    const void* shadow, const float* dy, float* d_table, float* d_params,
                    uint32_t flags, const fhash_touch* touch, void* ws, size_t* ws_bytes,
                    void* stream);
int fhash_fused_train(const fhash_index* idx, const fhash_mlp_desc* mlp, const float* pos,
                      const float* target, int64_t n, const void* table, fhash_dtype table_dt,
                      const float* params, const void* shadow, float loss_scale, float* d_table,
                      float* d_params, double* loss_sum, uint32_t flags, const fhash_touch* touch,
                      void* ws, size_t* ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving and training loops, harnesses that forbid
 * hipMalloc): fhash_fused_train with no workspace argument.  The decoder-
 * gradient partials go to a scratch array owned by the library, one copy per
 * GPU (FHASH_STATIC_SCRATCH_BYTES = 10,813,440 bytes, held until the process
 * ends); its device address is resolved on the first call on each device, and
 * the call allocates nothing.  Every partial the reduction reads is written by
 * the same call, so nothing has to start at zero.  All calls on one GPU share
 * the array: calls that overlap on one GPU (different streams, or threads
 * without ordering) race and give wrong d_params.  Otherwise the arguments,
 * results and errors are those of fhash_fused_train; FHASH_ENOMEM if the
 * partials of a launch would exceed the array (never for the decoders the
 * fused path is built for); FHASH_EINVAL for FHASH_COARSE_LDS, whose encoding
 * gradient needs a workspace. */
#define FHASH_STATIC_SCRATCH_BYTES 10813440
int fhash_fused_train_static(const fhash_index* idx, const fhash_mlp_desc* mlp,
                             const float* pos, const float* target, int64_t n, const void* table,
                             fhash_dtype table_dt, const float* params, const void* shadow,
                             float loss_scale, float* d_table, float* d_params, double* loss_sum,
                             uint32_t flags, const fhash_touch* touch, void* stream);

/* ------------------------------------------------------------ optimiser ----
 * Adam (Sec. 5.1.3: Adam, lr 0.01; PyTorch semantics, bias-corrected, no
 * weight decay), applied densely to every parameter:
 *   g = grad * grad_scale;  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= (lr / (1 - b1^step)) * m / (sqrt(v) / sqrt(1 - b2^step) + eps)
 * in FP32, the square root and the reciprocal of the denominator from the
 * hardware (within 1 ulp each).
 * grad is zeroed.  If found_inf (device int32, may be NULL) is non-zero the
 * whole update is skipped (grad is still zeroed).  shadow (device, may be
 * NULL) receives p rounded to shadow_dt (FHASH_F16 or FHASH_BF16, RNE).
 * touch (may be NULL): the gradient in [touch->begin, touch->end) is read only
 * in flagged segments and taken as zero elsewhere; the flags of that range are
 * cleared.  Results are bit for bit those of the untracked call whenever the
 * gradient is zero in every unflagged segment.
 * All arrays device float[n], 16-byte aligned.
 * Moments layout (opt->moments): FHASH_MOMENTS_SEPARATE, m and v each float[n];
 * FHASH_MOMENTS_PAIRED, one array in blocks of 32 floats, the m of parameters
 * 16b .. 16b+15 followed by their v (float[2 * ceil(n / 16) * 16]): pass its
 * start as m and its start + 16 floats as v (FHASH_EINVAL otherwise).  The
 * paired layout keeps a segment's two moments in one 128-byte line, which the
 * deferred update below reads and writes per segment.
 * FHASH_MOMENTS_WITH_PARAMS: two arrays in blocks of 32 floats (each
 * float[2 * ceil(n / 16) * 16]), one holding parameters 16b .. 16b+15 followed
 * by their m, the other their gradients followed by their v: pass param and
 * grad at the arrays' starts, m = param + 16 floats, v = grad + 16 floats
 * (FHASH_EINVAL otherwise).  A segment's whole optimiser state is then two
 * lines, the same number as with paired moments while parameters and
 * gradients stay dense, and the fused calls read such a table as
 * FHASH_F32_PAIRED and write its gradient with FHASH_GRAD_PAIRED; the lines
 * the forward gathers parameters from are never the lines the backward's
 * atomics add into.  shadow stays dense in every layout: shadow[i] is
 * parameter i. */
enum { FHASH_MOMENTS_SEPARATE = 0, FHASH_MOMENTS_PAIRED = 1, FHASH_MOMENTS_WITH_PARAMS = 2 };
typedef struct {
  double lr, beta1, beta2, eps; /* the kernel uses FP32 roundings of b1, 1-b1, b2, 1-b2 */
  int64_t step;                 /* 1-based */
  double grad_scale;
  int64_t moments;              /* FHASH_MOMENTS_SEPARATE, _PAIRED or _WITH_PARAMS */
} fhash_adam_desc;

int fhash_step(const fhash_adam_desc* opt, float* param, float* grad, float* m, float* v,
               void* shadow, fhash_dtype shadow_dt, int64_t n, const int32_t* found_inf,
               const fhash_touch* touch, void* stream);

/* ------------------------------------------------ deferred (lazy) Adam ----
 * An optimisation of the memory traffic of the dense update above, not part
 * of the method.  On a float range [begin, end) of the parameter vector (the
 * large table levels; the table starts at float 0 of the vector) no step is
 * applied when it happens.  Every segment of FHASH_LAZY_FLOATS floats records
 * the last step it has received and the step it was last enrolled in, the
 * constants of every step are kept, and the steps a segment missed are
 * replayed with the dense update's own per-parameter arithmetic the next time
 * the segment is prepared, or by fhash_lazy_flush: the step it was enrolled in
 * with its gradient (which is then zeroed), all others with a zero gradient
 * (there its gradient was zero).  A value read after its segment was
 * prepared, or after a flush, equals bit for bit what fhash_step applied to
 * every parameter at every step would hold there.  (A parameter with m and v
 * both +0 and no pending gradient is a fixed point of such a replay.)
 *
 * Per step: fhash_lazy_prepare with the positions of every sample whose
 * encoding or encoding gradient the step computes (any number of calls), then
 * those calls, then fhash_step_lazy.  Before the whole table is read (render,
 * checkpoint, export) or the table gradient is inspected, fhash_lazy_flush.
 * Reading a segment of the range that was not prepared gives a stale value;
 * between a step and the segment's next prepare or flush, the gradient of an
 * enrolled segment still holds that step's (unapplied) gradient.
 *
 * ws: device memory of fhash_lazy_workspace_bytes(end - begin, max_steps)
 * bytes, 16-byte aligned, caller-owned (8 bytes of state and a 1-byte claim
 * flag per segment, 16 bytes of constants per step).  begin: a multiple of
 * FHASH_LAZY_FLOATS; end: a multiple of 4; fewer than 2^32 segments.  steps:
 * the number of fhash_step_lazy calls so far (0 after fhash_lazy_init, one
 * more after each; at most max_steps < 2^32 - 1).  beta1, beta2, eps: recorded
 * by the first step, which every later step must repeat (FHASH_EINVAL
 * otherwise); lr and grad_scale may change from step to step.  The library
 * writes steps and the recorded constants; the caller sets the rest before
 * fhash_lazy_init.  Calls that share one descriptor must be ordered on one
 * stream. */
#define FHASH_LAZY_FLOATS 16
typedef struct {
  void* ws;
  int64_t begin, end;
  int64_t max_steps;
  int64_t steps;
  double beta1, beta2, eps;
  int64_t flags; /* library-owned: bit 0, a step with a non-finite grad_scale was recorded */
  int64_t moments; /* optimiser state layout (see fhash_adam_desc), set by the caller;
                      every fhash_step_lazy must pass the same */
} fhash_lazy;

size_t fhash_lazy_workspace_bytes(int64_t range_floats, int64_t max_steps);

/* Zero the workspace (a fill kernel on `stream`), steps = 0.  The deferred
 * update starts a fresh optimiser: m and v of the range must be zero (as Adam
 * starts), since segments never enrolled are not read or replayed. */
int fhash_lazy_init(fhash_lazy* lz, void* stream);

/* Enrol for step steps+1 every segment of [begin, end) that the samples pos
 * (device float4 [n], 16-byte aligned) read through the corner rows of their
 * cells (Sec. 3.2.4) at idx (phase FHASH_LAZY_MARK), and bring the segments
 * enrolled since the last catch-up up to step `steps` (phase
 * FHASH_LAZY_CATCH_UP): param, m, v (and shadow, when not NULL, rounded to
 * shadow_dt as by fhash_step) are updated in place, applied gradients in grad
 * are zeroed.  phases: FHASH_LAZY_PREPARE for both; a mark must be followed by
 * a catch-up before the enrolled segments are read and before the step. */
#define FHASH_LAZY_MARK 1u
#define FHASH_LAZY_CATCH_UP 2u
#define FHASH_LAZY_PREPARE 3u
int fhash_lazy_prepare(const fhash_index* idx, const float* pos, int64_t n, fhash_lazy* lz,
                       float* param, float* grad, float* m, float* v, void* shadow,
                       fhash_dtype shadow_dt, uint32_t phases, void* stream);

/* Workload counters accumulated by the catch-ups since fhash_lazy_init
 * (copied to host; synchronises `stream`): stats[0] segments caught up,
 * stats[1] of them with data to load (stepped before), stats[2] with a pending
 * gradient, stats[3] segment-steps replayed. */
int fhash_lazy_stats(const fhash_lazy* lz, int64_t stats[4], void* stream);

/* fhash_step with the range [begin, end) deferred: the dense update on
 * [0, begin) and [end, n); the step's constants (and whether found_inf skipped
 * it) are recorded for the range; steps += 1.  FHASH_ERANGE when
 * steps == max_steps. */
int fhash_step_lazy(const fhash_adam_desc* opt, float* param, float* grad, float* m, float* v,
                    void* shadow, fhash_dtype shadow_dt, int64_t n, const int32_t* found_inf,
                    fhash_lazy* lz, void* stream);

/* Bring every segment of the range up to step `steps` (a pass over the whole
 * range: replays what each segment missed, applies and zeroes pending
 * gradients). */
int fhash_lazy_flush(fhash_lazy* lz, float* param, float* grad, float* m, float* v,
                     void* shadow, fhash_dtype shadow_dt, void* stream);

/* *found_inf |= any(!isfinite(grad[i])) over device float grad[n]. */
int fhash_check_finite(const float* grad, int64_t n, int32_t* found_inf, void* stream);

/* Round a device float array to a device f16/bf16 copy (RNE). */
int fhash_cast(const float* src, void* dst, fhash_dtype dst_dt, int64_t n, void* stream);

/* -------------------------------------------------------------- coreset ----
 * Feature-based coreset selection (Sec. 3.1: feature extraction, feature
 * dilation with the occupancy grid, bounding boxes and temporal fusion into
 * the FBB, and the coreset union of Eq. (3)).  Every call works on a voxel
 * mask in the layout of fhash_mask_desc ([T][Sz][Sy][ceil(Sx/64)] uint64
 * words, bit b of word w = voxel x = 64 w + b, padding bits zero) over a field
 * of dims = (Sx, Sy, Sz, T), each in [2, 2^31 - 1] with T <= 65535, fewer
 * than 2^46 mask words, and T Sz, Sy ceil(Sx/64) and ceil(Sy/4) ceil(Sx/4)
 * each below 2^31 (FHASH_ERANGE otherwise).  Outputs are device buffers owned
 * by the caller.
 *
 * fhash_feature_mask: feature extraction per timestep from the device field
 * float [T][Sz][Sy][Sx] into bits (mask words, every word written).
 *   FHASH_FEATURE_INTERVAL: voxel set iff lo < v <= hi (a value-range feature).
 *   FHASH_FEATURE_ISOSURFACE: the vertices needed to interpolate the level
 *   set v = lo inside each frame: a spatial cell (8 voxels, within one
 *   timestep) is crossed iff some corner has v >= lo and some corner v < lo;
 *   a voxel is set iff it is a corner of a crossed cell.  hi is unused.
 *   ws: device workspace of *ws_bytes (one mask for the isosurface, 0 for the
 *   interval); with ws == NULL and ws_bytes != NULL only *ws_bytes is written
 *   (a size query); the interval kind runs with ws == NULL and ws_bytes == NULL.
 * fhash_dilate_mask: feature dilation inside each timestep by a cube of
 * radius r in [0, 63]: out voxel set iff an in voxel of the same timestep lies
 * within r voxels along each of x, y and z.  in and out must not overlap.
 * fhash_feature_boxes: box (int32 [T + 1][6], device) row k = bounding box
 * b_k of timestep k as (xmin, ymin, zmin, xmax, ymax, zmax), inclusive voxel
 * indices; row T = the FBB, the smallest box containing every b_k (temporal
 * fusion).  An empty timestep (or an empty mask, row T) reads
 * (Sx, Sy, Sz, -1, -1, -1).
 * fhash_occupancy_words: words of the occupancy grid of dims (-1 if dims are
 * invalid).
 * fhash_occupancy_grid: occupancy bits for rendering, Morton order inside
 * 4x4x4 bricks: occ (uint64, fhash_occupancy_words(dims) words, device) holds
 * one word per brick, bricks in [T][ceil(Sz/4)][ceil(Sy/4)][ceil(Sx/4)] order;
 * voxel (4bx + lx, 4by + ly, 4bz + lz) is bit
 *   (lx&1) | (ly&1)<<1 | (lz&1)<<2 | (lx>>1)<<3 | (ly>>1)<<4 | (lz>>1)<<5.
 * Voxels outside the volume read 0.
 * fhash_coreset: the coreset of Eq. (3) as linear voxel ids
 * ((t Sz + z) Sy + y) Sx + x of the set voxels, in increasing order, the form
 * fhash_sample draws from.  Writes the count to the HOST *count and, when ids
 * != NULL and count <= capacity, the ids (device uint64[count]); synchronises
 * `stream`.  ws: device workspace (query with ws == NULL). */
enum { FHASH_FEATURE_INTERVAL = 0, FHASH_FEATURE_ISOSURFACE = 1 };
int fhash_feature_mask(const float* field, const int64_t dims[4], int32_t kind, float lo,
                       float hi, uint64_t* bits, void* ws, size_t* ws_bytes, void* stream);
int fhash_dilate_mask(const uint64_t* in, const int64_t dims[4], int32_t r, uint64_t* out,
                      void* stream);
int fhash_feature_boxes(const uint64_t* bits, const int64_t dims[4], int32_t* box, void* stream);
int64_t fhash_occupancy_words(const int64_t dims[4]);
int fhash_occupancy_grid(const uint64_t* bits, const int64_t dims[4], uint64_t* occ,
                         void* stream);
int fhash_coreset(const uint64_t* bits, const int64_t dims[4], uint64_t* ids, int64_t capacity,
                  void* ws, size_t* ws_bytes, int64_t* count, void* stream);

/* fhash_coreset_frames: the coreset of the listed frames only (key-frame
 * training, Sec. 3.1 and 3.2.2): frames (HOST int32[n_frames], strictly
 * increasing, each in [0, T)); ids as fhash_coreset (linear voxel ids of the
 * whole volume, increasing).  *count (host) = their number; when ids != NULL
 * and the count exceeds capacity, ids holds those of the leading frames that
 * fit.  Synchronises `stream` once per frame.  ws: device workspace (query
 * with ws == NULL). */
int fhash_coreset_frames(const uint64_t* bits, const int64_t dims[4], const int32_t* frames,
                         int32_t n_frames, uint64_t* ids, int64_t capacity, void* ws,
                         size_t* ws_bytes, int64_t* count, void* stream);

/* -------------------------------------------------------------- sampler ----
 * Training batch from the coreset (Sec. 3.1, time-step concatenation): draw i
 * of step `step` is voxel id floor(r * M / 2^64), r the 64-bit word out1:out0
 * of Philox4x32-10 with counter (i, step) and key seed; the voxel is
 * coreset[id] (device uint64 linear voxel ids) or id itself when coreset is
 * NULL.  pos = (i/(Sx-1), j/(Sy-1), k/(Sz-1), tau(n)) in FP32 (IEEE
 * division), target = field[voxel] (device float [T][Sz][Sy][Sx]); tau(n) =
 * n/(T-1), or frame_t[n] when frame_t (device float [T]) is given: the time
 * coordinate of each frame under key-frame training (Sec. 3.2.2), see
 * fhash_key_frame_times.  box (HOST int32[6] = xmin, ymin, zmin, xmax, ymax,
 * zmax, inclusive voxel bounds with min < max < S, e.g. the FBB row of
 * fhash_feature_boxes; or NULL): the spatial coordinates become those of the
 * box, ((i - xmin)/(xmax - xmin), ...) (Sec. 3.1, position translation and
 * scaling to the FBB, on [0,1]); every drawn voxel must lie in the box.
 * dims = (Sx, Sy, Sz, T). */
int fhash_sample(uint64_t seed, uint64_t step, int64_t n, const uint64_t* coreset, uint64_t M,
                 const int64_t dims[4], const float* field, const float* frame_t,
                 const int32_t* box, float* pos, float* target, void* stream);

/* Reorder a batch of samples (pos float4[n], target float[n] or NULL, both
 * device, in place) by a 4D Morton key of the positions quantised to 256
 * cells per axis (stable LSD radix sort).  Samples of the same cells become
 * neighbours, which the gathers and the merge of equal slots before the
 * scatter-add's atomics (FHASH_SAMPLES_SORTED) exploit; the MSE loss and its gradient do not depend on the
 * order.  ws: device workspace (query with ws == NULL); n < 2^31. */
int fhash_sort_samples(float* pos, float* target, int64_t n, void* ws, size_t* ws_bytes,
                       void* stream);

/* ----------------------------------------------------------- reductions ----
 * *sum (device double, accumulated) += sum_i (y[i] - v[i])^2 in FP64
 * (the loss / PSNR reduction, PSNR = 10 log10(1/MSE), Sec. 5.1.2). */
int fhash_sq_err_sum(const float* y, const float* v, int64_t n, double* sum, void* stream);

/* MSE loss gradient of the unfused path (L = mean over the batch of (y_s - v_s)^2):
 * dy[s] = loss_scale * 2 (y[s] - v[s]) / n; *loss_sum (device double, may be
 * NULL, accumulated) += sum_s (y[s] - v[s])^2 in FP64. */
int fhash_mse_grad(const float* y, const float* v, int64_t n, float loss_scale, float* dy,
                   double* loss_sum, void* stream);

/* ------------------------------------------------------------- rendering ----
 * Volume rendering of the trained representation by ray marching with the
 * adaptive marching pace (ARM) of Sec. 3.3, Algorithm 1.
 *
 * Geometry: the volume occupies the box [0, Sx-1] x [0, Sy-1] x [0, Sz-1] in
 * voxel units.  Pixel (px, py) of a W x H image casts the ray from `eye` along
 * normalize(fwd + u right + v up), u = (2 (px + 1/2)/W - 1) tan_half_fovy aspect,
 * v = (1 - 2 (py + 1/2)/H) tan_half_fovy; the slab test gives [s_near, s_far].
 * Samples sit on the lattice s_k = s_near + (k + 1/2) ds, p_k = fma(s_k, dir, eye)
 * (FP32, IEEE operations, k < max_steps).  A sample is taken iff its voxel cell
 * is occupied at time t (reading of the interpolated occupancy grid for a bit
 * grid: one of the cell's 8 corner voxels is in the feature mask at floor(t)
 * or ceil(t)); its value is the decoder output at (p / (S - 1), t / (T - 1)).
 * The value is mapped through a 256-entry RGBA transfer function (value
 * clamped to [0,1], linear interpolation) and composited front to back,
 * C += (1 - A) a c, A += (1 - A) a, until A >= alpha_stop.
 * ARM: while rays are alive, each alive ray emits up to
 * pace = clamp(floor(budget / alive), 1, arm_max) occupied samples per
 * iteration (budget = number of rays for a single request), all emitted samples
 * are decoded in one batch, then composited.  The pace changes only the
 * schedule: the image equals the pace-1 image.
 * The view basis (fwd, right, up orthonormal, tan of half the vertical field of
 * view, aspect = W / H) is an input; rgba: device float [H][W][4]. */
typedef struct {
  float eye[3], fwd[3], right[3], up[3];
  float tan_half_fovy, aspect;
} fhash_view;

typedef struct {
  float ds;          /* lattice step in voxel units (> 0) */
  float alpha_stop;  /* early-termination opacity, e.g. 0.99 */
  int32_t arm_max;   /* maximum pace, 64 in Algorithm 1; 1 disables ARM */
  int32_t max_steps; /* lattice steps per ray */
} fhash_render_opts;

/* Per-request render state (host POD, owned by the caller). */
typedef struct {
  int32_t W, H;
  float t;
  int32_t cur;       /* current alive list */
  int32_t n_alive;   /* alive rays */
  int32_t pending;   /* samples emitted by the last march, not yet composited */
  int64_t iterations, samples;
  void* ws;
  int64_t dims[4];
  float t01;         /* the model's time coordinate of the samples; begin sets
                        t / (T - 1); a model trained on key frames takes its
                        frame time (fhash_key_frame_times, interpolated at t),
                        set by the caller before the first march */
} fhash_render_state;

/* Device workspace of one request's ray state (W*H rays + occupancy bits).
 * W, H >= 1 and W * H <= 2^30, else FHASH_EINVAL. */
int fhash_render_state_bytes(int32_t W, int32_t H, const int64_t dims[4], size_t* bytes);

/* Set up rays and the occupancy at time t (fractional timestep in [0, T-1]),
 * clear rgba.  Synchronises `stream` (returns the alive-ray count in *state). */
int fhash_render_begin(const fhash_view* view, float t, int32_t W, int32_t H,
                       const uint64_t* mask_bits, const int64_t dims[4], void* ws,
                       size_t ws_bytes, float* rgba, fhash_render_state* state, void* stream);

/* fhash_render_begin with the occupancy grid of the coreset selection
 * (Sec. 3.1, used by the renderer to skip empty space, Sec. 3.3): occ is the
 * Morton-brick grid of fhash_occupancy_grid (device) over the same dims,
 * in place of the mask rows; everything else as fhash_render_begin.  A grid
 * made from mask_bits gives the state (and so the image) of
 * fhash_render_begin(mask_bits) bit for bit. */
int fhash_render_begin_grid(const fhash_view* view, float t, int32_t W, int32_t H,
                            const uint64_t* occ, const int64_t dims[4], void* ws,
                            size_t ws_bytes, float* rgba, fhash_render_state* state,
                            void* stream);

/* pace = clamp(floor(budget / alive), 1, arm_max) (Algorithm 1). */
int32_t fhash_render_pace(int64_t budget, int64_t alive, int32_t arm_max);

/* Emit up to `pace` occupied samples per alive ray into pos_out (device
 * float4[cap], model inputs); cap must be >= pace * alive and pace * alive
 * <= 2^31 - 1 (FHASH_EINVAL otherwise).  Writes the number of samples to
 * *n_samples.  Synchronises `stream`. */
int fhash_render_march(fhash_render_state* state, const fhash_render_opts* opts, int32_t pace,
                       float* pos_out, int64_t cap, int64_t* n_samples, void* stream);

/* Composite the decoded values y (device float[n_samples], in the order of the
 * last march) into the rays; finished rays write their pixel.  Synchronises
 * `stream` (updates state->n_alive). */
int fhash_render_composite(fhash_render_state* state, const float* y, const float* tf,
                           const fhash_render_opts* opts, float* rgba, void* stream);

/* Batched steps: n render requests (1 <= n <= FHASH_RENDER_BATCH_MAX) advanced
 * by one march launch and one composite launch between them, the continuous
 * batching of requests that share the decode (Sec. 3.3, ARM over a shared
 * sample budget).  Each request behaves exactly as under the single-request
 * calls with its own pace: the images are bit for bit those of
 * fhash_render_march / fhash_render_composite.
 *
 * fhash_render_march_batch: states (HOST array of n distinct states, none
 * pending), paces (HOST int32[n], each in [1, opts->arm_max]); the samples of
 * all n requests go to pos[out_base, out_base + total) (device float4[cap]),
 * total = sum of n_samples, with the requests' samples interleaved; the
 * caller decodes that range (one model per call) into y with the same
 * indexing, y[j] = decode(pos[j]).  Requires out_base + sum_r pace_r alive_r
 * <= cap and <= 2^31 - 1 - 64 n.  counts: device int32[1 + n] (scratch, written by
 * the call).  n_samples: HOST int64[n], per request.  Synchronises `stream`.
 * fhash_render_composite_batch: composites the values y (the frame of the
 * march's pos) into the rays of the n states (all pending, from one march
 * batch or from single marches into the same frame); tf and rgba are HOST
 * arrays of n device pointers (transfer function float[256][4] and image of
 * each request).  Updates each state's n_alive.  Synchronises `stream`. */
#define FHASH_RENDER_BATCH_MAX 32
int fhash_render_march_batch(fhash_render_state* const* states, const int32_t* paces, int32_t n,
                             const fhash_render_opts* opts, float* pos, int64_t out_base,
                             int64_t cap, int32_t* counts, int64_t* n_samples, void* stream);
int fhash_render_composite_batch(fhash_render_state* const* states, int32_t n, const float* y,
                                 const float* const* tf, float* const* rgba,
                                 const fhash_render_opts* opts, int32_t* counts, void* stream);

typedef struct {
  int64_t iterations, samples;
} fhash_render_stats;

/* Whole image for one request: begin, then march / fused decode / composite
 * until no ray is alive.  ws: device workspace (query with ws == NULL).
 * Synchronises `stream`. */
int fhash_render(const fhash_index* idx, const fhash_mlp_desc* mlp, const void* table,
                 fhash_dtype table_dt, const float* params, const uint64_t* mask_bits,
                 const int64_t dims[4], const fhash_view* view, float t, const float* tf,
                 int32_t W, int32_t H, const fhash_render_opts* opts, float* rgba, void* ws,
                 size_t* ws_bytes, fhash_render_stats* stats, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FHASH_H */
