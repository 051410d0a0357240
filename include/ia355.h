/*
 * ia355.h -- C ABI of libia355.so, the MI355X (gfx950) deform-and-query path
 * of InstantAvatar (arXiv 2212.10550): march posed rays through an occupancy
 * grid, map each posed sample to canonical space by root finding on linear
 * blend skinning, encode it with a multiresolution hash grid, decode it with
 * a small MLP and alpha-composite per ray -- forward and backward.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array pointers are DEVICE pointers owned by the caller unless marked
 *    "host".  The library never allocates or frees device memory and keeps
 *    no global state; scratch space is a caller buffer sized by the matching
 *    *_workspace_size() call.
 *  - Every call only enqueues work on `stream` (a hipStream_t; NULL = the
 *    default stream) and returns without synchronising.  The return value
 *    reports argument validation and launch errors only.
 *  - Point sets are structure-of-arrays: [3][ld] floats (x row, y row,
 *    z row, each of leading dimension ld >= S).  Rays are [R][3] floats.
 *    Bone transforms B are [nb][3][4] row-major rigid transforms
 *    (canonical -> posed).  The skinning grid W is [Dz][Dy][Dx][nb].  The hash
 *    table is [L][T][F] with T = 2^log2T.  Features are level-major
 *    [L][ld][F].  Boxes (aabb) are host float[6] = (lo x, lo y, lo z,
 *    hi x, hi y, hi z).
 *  - A sample whose `bone` is negative has no canonical correspondence: it
 *    gets density 0, zero features and zero gradients (Sec. 3.3 gives
 *    skipped points zero density).
 *  - grad_* outputs documented as "accumulated" are added to (+=), so the
 *    caller zeroes them (ia355_zero) or sums over several calls.
 *  - Device sample counts: every entry point that takes a sample count S
 *    also takes `S_dev` (device int64, nullable).  With S_dev NULL the count
 *    is S.  With S_dev given, the count is min(S, *S_dev) read on the device
 *    when the kernels run, and S is the capacity the buffers, workspaces and
 *    launches are sized for.  A whole step (march, whose sample count lands
 *    in device memory, then every later stage) can so be enqueued without a
 *    host round trip, and captured in a HIP graph.
 *  - Features are level-major [L][ld][F]: level l of sample n is at
 *    (l * ld + n) * F, with ld the leading dimension of the point set.
 */
#ifndef IA355_H
#define IA355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IA355_OK 0
#define IA355_ERR_INVALID_ARG 1 /* null required pointer, bad size, dtype or shape */
#define IA355_ERR_WORKSPACE 2   /* workspace smaller than *_workspace_size() */
#define IA355_ERR_UNSUPPORTED 3 /* valid but unimplemented combination */
#define IA355_ERR_HIP 4         /* a HIP launch failed; see ia355_error_string */
#define IA355_ERR_SCRATCH 5     /* the problem exceeds the fixed scratch of an allocation-free entry point */
#define IA355_ERR_CAPACITY 6    /* the sample buffer is too small; *n_required holds the count needed */

/* flags of the backward entry points */
#define IA355_OVERWRITE 1u /* write the gradient instead of adding to it */
/* Hash-table gradient level groups (ia355_hashgrid_encode_bwd): the coarse
 * dense levels (resolution <= 32, summed by run aggregation) or the rest;
 * neither flag, or both, means every level.  The groups write disjoint
 * slices of grad_table, so they may run concurrently on two streams. */
#define IA355_TABLE_COARSE 2u
#define IA355_TABLE_FINE 4u
/* Two-phase use of ia355_hashgrid_table_grad: IA355_TABLE_PLAN runs only
 * the passes that depend on the positions (binning the corner updates by
 * table tile); a later call with IA355_TABLE_REUSE_PLAN, the same workspace
 * and the same positions, bones, count, sizes and level-group flags runs the
 * rest.  The plan can so run as soon as the positions are known (during the
 * forward), off the backward's critical path. */
#define IA355_TABLE_PLAN 8u
#define IA355_TABLE_REUSE_PLAN 16u

#define IA355_F32 0
#define IA355_F16 1
#define IA355_BF16 2

typedef void *ia355_stream_t; /* hipStream_t */

/* Library version (major*10000 + minor*100 + patch). */
int32_t ia355_version(void);
/* Human-readable text for a status code (static storage, never NULL). */
const char *ia355_error_string(int32_t status);

/* Fill `bytes` bytes at device pointer p with zeros (a kernel, not a
 * memset node, so the call may be captured in a HIP graph). */
int32_t ia355_zero(void *p, size_t bytes, ia355_stream_t stream);

/* ------------------------------------------------------------------ */
/* Occupancy grid (Sec. 3.3, "Empty Space Skipping").                  */
/* ------------------------------------------------------------------ */
/* Number of 32-bit words of a packed G^3 grid (0 unless 0 < G <= 2048). */
size_t ia355_occ_words(int32_t G);
/* Pack a binary occupancy grid occ [G][G][G] (uint8, z-major, x fastest,
 * non-zero = occupied) into bits [ia355_occ_words(G)].  Layout: bricks of
 * 8 x 8 x 16 cells (x, y, z), 32 words (one 128-byte line) each, in
 * x-fastest brick order over ceil(G/8) x ceil(G/8) x ceil(G/16) bricks;
 * cell (x, y, z) is bit lx + 8 ly + 64 lz of its brick (l = offset in the
 * brick), i.e. bit (lx + 8 ly) mod 32 of word 32 brick + ly/4 + 2 lz.
 * Cells past G in a brick are 0.  The march reads this layout. */
int32_t ia355_occ_pack(const uint8_t *occ, int32_t G, uint32_t *bits, ia355_stream_t stream);

/* Ray marching with empty-space skipping (Sec. 3.2 ray r = o + t d with N
 * samples between the near and far bound; Sec. 3.3 samples in
 * non-occupied cells are skipped).
 * Each ray is clipped to `aabb` (t >= 0); samples sit at the midpoints
 * t_k = t_near + (k + 1/2) dt, k < max_steps, t_k < t_far; with n_per_ray > 0
 * the step is dt = (t_far - t_near) / n_per_ray, otherwise `dt`.  A sample is
 * kept iff its cell in the G^3 grid over `aabb` is occupied (occ_bits NULL:
 * all cells occupied).  Positions and decisions use IEEE single precision
 * with no fused operations.
 * occ_bits: the packed grid of ia355_occ_pack.
 * Outputs (compacted, rays in order, samples in t order):
 *   xs [3][cap] positions, ts [cap] ray parameter, ray_id [cap],
 *   ray_off [R+1] first-sample offsets (int64), ray_cnt [R], ray_dt [R]
 *   (the ray's uniform step: every kept sample's delta, Eq. 8),
 *   n_samples [1] device int64 total kept count.
 * With cap == 0 the call only counts: ray_cnt, ray_dt and n_samples are
 * written, ray_off is not final.
 * If *n_samples > cap, samples at offsets >= cap are not written.
 * n_required (host, nullable): NULL leaves the call asynchronous (it may then
 * be captured in a graph) and the caller compares *n_samples with cap once
 * the stream completes; otherwise the call waits for the stream, writes the
 * kept count to *n_required and returns IA355_ERR_CAPACITY when it exceeds
 * cap (the outputs then hold the first cap samples), IA355_OK otherwise.
 * ws: ia355_march_workspace_size(R, max_steps) bytes (per-block totals,
 * and each ray's keep masks, 8 bytes per 64 steps, and entry distance). */
size_t ia355_march_workspace_size(int64_t R, int32_t max_steps);
int32_t ia355_occgrid_march(const float *rays_o, const float *rays_d, int64_t R,
                            const uint32_t *occ_bits, int32_t G, const float *aabb,
                            float dt, int32_t n_per_ray, int32_t max_steps,
                            float *xs, float *ts, int32_t *ray_id, int64_t cap,
                            int64_t *ray_off, int32_t *ray_cnt, float *ray_dt, int64_t *n_samples,
                            int64_t *n_required, void *ws, size_t ws_bytes, ia355_stream_t stream);

/* Occupancy from densities: cell c of the G^3 grid (c = x + G (y + G z) in
 * sigma [G^3]) is occupied when some cell within `dilate` cells of it
 * (Chebyshev distance, clipped at the grid) has sigma > sigma_thresh
 * (Sec. 3.3: thresholded densities, occupied region dilated).  Writes the
 * packed bits [ia355_occ_words(G)] in the layout of ia355_occ_pack.
 * 0 <= dilate <= 4. */
int32_t ia355_occ_from_density(const float *sigma, int32_t G, float sigma_thresh, int32_t dilate,
                               uint32_t *occ_bits, ia355_stream_t stream);

/* Per-pose occupancy grid for rendering (Sec. 3.3, inference stage).  The
 * cell centres of a G^3 lattice over the posed box `aabb` (point
 * n = x + G (y + G z) at lo + ((i + 1/2) / G) (hi - lo), IEEE single, no
 * fused operations) are mapped to canonical space exactly as by
 * ia355_snarf_deform (same arguments), their density is taken from the
 * canonical field as by ia355_hashgrid_encode + ia355_mlp_fwd (table_dtype
 * IA355_F32 / IA355_F16; mlp_dtype IA355_F32 with FP32 features or
 * IA355_BF16 with BF16 features), a point without a valid root has density
 * 0, and occ_bits are made by ia355_occ_from_density.
 *   sigma [G^3]  lattice densities (nullable)
 *   ws: ia355_occgrid_build_workspace_size(G, L, F, mlp_dtype, Dx, Dy, Dz)
 *   bytes (0 unless 0 < G <= 256). */
size_t ia355_occgrid_build_workspace_size(int32_t G, int32_t L, int32_t F, int32_t mlp_dtype,
                                          int32_t Dx, int32_t Dy, int32_t Dz);
int32_t ia355_occgrid_build(int32_t G, const float *aabb, const float *B, int32_t nb, const float *W,
                            int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                            const float *hash_aabb, int32_t max_iter, float tol_stop, float tol_valid,
                            const void *table, int32_t table_dtype, int32_t L, int32_t F, int32_t log2T,
                            double base_res, double growth, const float *params, int32_t mlp_dtype,
                            float sigma_thresh, int32_t dilate, uint32_t *occ_bits, float *sigma,
                            void *ws, size_t ws_bytes, ia355_stream_t stream);

/* Training-stage occupancy grid (Sec. 3.3): one update of the grid shared
 * by all frames.  For the frame given by B, one point in each cell listed
 * in cells [M] (distinct indices c = x + G (y + G z); NULL: every cell, M
 * ignored), at lo + ((i + u) / G) (hi - lo) with u = jitter [3][M] (or
 * [3][G^3]) in [0, 1) (the caller draws both; IEEE single, no fused
 * operations), gets its density as in ia355_occgrid_build (no root: 0); the
 * listed cells' values [G^3] (FP32, in/out) become beta * values +
 * (1 - beta) * sigma (an index outside the grid is skipped), and occ_bits
 * are made from all values by ia355_occ_from_density.  0 <= beta <= 1.
 * ws: ia355_occgrid_build_workspace_size(G, L, F, mlp_dtype, Dx, Dy, Dz). */
int32_t ia355_occgrid_update(int32_t G, const float *aabb, const float *jitter, const int32_t *cells, int64_t M,
                             const float *B, int32_t nb,
                             const float *W, int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                             const float *hash_aabb, int32_t max_iter, float tol_stop, float tol_valid,
                             const void *table, int32_t table_dtype, int32_t L, int32_t F, int32_t log2T,
                             double base_res, double growth, const float *params, int32_t mlp_dtype,
                             float beta, float sigma_thresh, int32_t dilate, float *values,
                             uint32_t *occ_bits, void *ws, size_t ws_bytes, ia355_stream_t stream);

/* Occupancy-based density regulariser (Sec. 3.4, L_density): with n the
 * point count, loss[0] = (lam / n) sum |sigma_i| over the points x [3][ld]
 * whose cell of the grid (occ_bits, layout of ia355_occ_pack, over aabb;
 * cell as in ia355_occgrid_march) is empty; grad_sigma [S] = dloss/dsigma
 * (overwritten; 0 for points in occupied cells).  A fixed summation order
 * for a given S.  ws: ia355_density_reg_workspace_size(S) bytes. */
size_t ia355_density_reg_workspace_size(int64_t S);
int32_t ia355_density_reg(const float *x, const float *sigma, int64_t S, const int64_t *S_dev, int64_t ld,
                          const uint32_t *occ_bits, int32_t G, const float *aabb, float lam,
                          float *loss, float *grad_sigma, void *ws, size_t ws_bytes, ia355_stream_t stream);

/* ------------------------------------------------------------------ */
/* Articulation (Sec. 3.1, Eq. 5-7): canonical correspondences x* of    */
/* posed points x' as roots of x' = sum_i w_i(x) B_i x, by multi-init   */
/* Broyden root finding (the paper's Fast-SNARF root finding).         */
/* ------------------------------------------------------------------ */
/* w(x) is the trilinear interpolant of W over skin_aabb (vertices on the
 * box corners, coordinates clamped to the box).  For each bone i the solver
 * starts at x0 = B_i^{-1} x' with the inverse Jacobian H0 = J(x0)^{-1},
 * takes up to max_iter Broyden steps (good update, Sherman-Morrison form)
 * and stops once ||g|| < tol_stop.  An init is valid when its final
 * ||g|| < tol_valid and its point lies in hash_aabb; the valid init with the
 * lowest residual is kept (ties: lowest bone).  All arithmetic is FP32.
 *   xp [3][ld]   posed points
 *   xc [3][ld]   canonical roots (the start point of bone 0 when invalid)
 *   bone [S]     chosen init, -1 when no init is valid
 *   resid [S]    residual of the chosen init (nullable)
 *   steps [S]    Broyden steps summed over all inits (nullable)
 * ws: ia355_deform_workspace_size(Dx, Dy, Dz) bytes (the per-pose blended
 * transform grid sum_i W[v][i] B_i). */
size_t ia355_deform_workspace_size(int32_t Dx, int32_t Dy, int32_t Dz);
int32_t ia355_snarf_deform(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld,
                           const float *B, int32_t nb, const float *W,
                           int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb, const float *hash_aabb,
                           int32_t max_iter, float tol_stop, float tol_valid,
                           float *xc, int16_t *bone, float *resid, int16_t *steps,
                           void *ws, size_t ws_bytes, ia355_stream_t stream);

/* Allocation-free form of ia355_snarf_deform, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments minus the workspace and
 * the same results, bit for bit: the blended transform grid lives in a
 * library-owned device array of IA355_DEFORM_NOALLOC_MAX_VERTS vertices x 12
 * floats (6 MiB), which each GPU the library runs on holds until the process
 * ends.  The call allocates and frees nothing.  Dx * Dy * Dz above the limit
 * returns IA355_ERR_SCRATCH.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams, or from several host
 * threads) race and must be serialised by the caller. */
#define IA355_DEFORM_NOALLOC_MAX_VERTS (1 << 17) /* e.g. a 64 x 64 x 32 skinning grid */
int32_t ia355_snarf_deform_noalloc(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld,
                                   const float *B, int32_t nb, const float *W, int32_t Dx, int32_t Dy, int32_t Dz,
                                   const float *skin_aabb, const float *hash_aabb, int32_t max_iter, float tol_stop,
                                   float tol_valid, float *xc, int16_t *bone, float *resid, int16_t *steps,
                                   ia355_stream_t stream);

/* Backward through the root finder by the implicit function theorem (no
 * unrolling of Broyden): with J = dg/dx at x* and v = J^{-T} grad_xc,
 *   grad_xp [3][ld] = v                                  (overwritten, nullable)
 *   grad_B  [nb][3][4]       += -sum_s w_b(x*) v x*_h^T  (nullable)
 *   grad_W  [Dz][Dy][Dx][nb] += -tri_c(x*) v^T (B_b x*_h) (nullable)
 * With IA355_OVERWRITE in flags grad_B / grad_W are written instead (every
 * entry).  Samples with bone < 0 contribute nothing (grad_xp = 0).
 * The parameter gradients go through the per-vertex moment
 * Q_v = sum_s tri_v(x*_s) v_s x*_h,s^T (FP32 atomics; the summation order
 * inside an entry is not fixed).
 * ws: ia355_deform_bwd_workspace_size(S, Dx, Dy, Dz, nb) bytes (12 B per
 * sample, 48 B per grid vertex and the dL/dB block partials). */
size_t ia355_deform_bwd_workspace_size(int64_t S, int32_t Dx, int32_t Dy, int32_t Dz, int32_t nb);
int32_t ia355_snarf_deform_bwd(const float *grad_xc, const float *xc, const int16_t *bone, int64_t S,
                               const int64_t *S_dev, int64_t ld,
                               const float *B, int32_t nb, const float *W,
                               int32_t Dx, int32_t Dy, int32_t Dz, const float *skin_aabb,
                               float *grad_xp, float *grad_B, float *grad_W, uint32_t flags,
                               void *ws, size_t ws_bytes, ia355_stream_t stream);

/* Learned root initialiser (an addition to the paper's root finding of
 * Sec. 3.1): an MLP (3 + 6 nb) -> 64 -> 64 -> (nb + 3) with ReLU hidden
 * layers maps (x', pose) to nb bone logits and a canonical offset; the start
 * point is x0 = B_k^{-1} x' + offset with k = argmax of the logits (ties:
 * lowest bone).
 *   xp [3][ld]; pose [nb][6] (axis-angle, translation per bone, device);
 *   params FP32 flat (per layer W [out][in] row-major, then b [out]);
 *   hidden must be 64 and nb + 3 <= 32; dtype IA355_F32 or IA355_BF16
 *   (BF16 MFMA for the two hidden-to-hidden/output layers, FP32 accumulate)
 *   init_bone [S] int16, x0 [3][ld] outputs. */
int32_t ia355_rootinit_fwd(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld, const float *pose,
                           const float *params,
                           int32_t hidden, const float *B, int32_t nb, int32_t dtype, int16_t *init_bone,
                           float *x0, ia355_stream_t stream);

/* Multi-root aggregation (an alternative to keeping the lowest-residual root
 * of Sec. 3.1).  ia355_snarf_deform_roots runs the same multi-init solve and
 * writes, per sample, up to K distinct valid roots in order of increasing
 * residual (ties: lower init), a candidate within dup_tol of a root already
 * taken counting as the same root:
 *   roots [3][K][S]  (slot k of sample n at (a K + k) S + n; past the
 *                    sample's count, init 0's final iterate)
 *   root_bone [K][S] the init of each root, -1 past the count
 *   n_roots [S]      the number of roots kept (0..K)
 * With K = 1 the root is ia355_snarf_deform's.  The K S slots can be fed to
 * ia355_hashgrid_encode / ia355_mlp_fwd as one batch of K S points (ld =
 * K S); ia355_select_max_density then keeps, per sample, the root with the
 * largest density (ties: the lower slot) and writes its point, bone,
 * density and colour (xc [3][ld], bone [S], sigma [S], rgb [3][ld]); a
 * sample without a root gets bone -1, density and colour 0.
 * ws: ia355_deform_workspace_size(Dx, Dy, Dz) bytes.  1 <= K <= nb. */
int32_t ia355_snarf_deform_roots(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld,
                                 const float *B, int32_t nb, const float *W, int32_t Dx, int32_t Dy,
                                 int32_t Dz, const float *skin_aabb, const float *hash_aabb,
                                 int32_t max_iter, float tol_stop, float tol_valid, int32_t K,
                                 float dup_tol, float *roots, int16_t *root_bone, int32_t *n_roots,
                                 void *ws, size_t ws_bytes, ia355_stream_t stream);
int32_t ia355_select_max_density(int32_t K, int64_t S, const float *sigma_k, const float *rgb_k,
                                 const float *roots, const int16_t *root_bone, const int32_t *n_roots,
                                 int64_t ld, float *xc, int16_t *bone, float *sigma, float *rgb,
                                 ia355_stream_t stream);

/* Guided root finding: one Broyden solve per sample from x0 (H0 = J(x0)^{-1},
 * the same iteration as ia355_snarf_deform).  A root with residual below
 * tol_valid inside hash_aabb is accepted with bone = init_bone; every other
 * sample falls back to the multi-init solve of ia355_snarf_deform.
 *   steps [S] (nullable) counts the guided steps plus, on fallback, every
 *   init's steps; n_fallback [1] (device int32, nullable) receives the
 *   number of fallback samples.
 * ws: ia355_deform_guided_workspace_size(S, Dx, Dy, Dz) bytes. */
size_t ia355_deform_guided_workspace_size(int64_t S, int32_t Dx, int32_t Dy, int32_t Dz);
int32_t ia355_snarf_deform_guided(const float *xp, int64_t S, const int64_t *S_dev, int64_t ld, const float *x0,
                                  const int16_t *init_bone,
                                  const float *B, int32_t nb, const float *W, int32_t Dx, int32_t Dy, int32_t Dz,
                                  const float *skin_aabb, const float *hash_aabb, int32_t max_iter, float tol_stop,
                                  float tol_valid, float *xc, int16_t *bone, float *resid, int16_t *steps,
                                  int32_t *n_fallback, void *ws, size_t ws_bytes, ia355_stream_t stream);

/* ------------------------------------------------------------------ */
/* Canonical field, Sec. 3.1 Eq. 1-2 (Instant-NGP encoding + MLP).      */
/* ------------------------------------------------------------------ */
/* Multiresolution hash encoding: level l has resolution
 * N_l = floor(base_res * growth^l); a canonical point (clamped to `aabb`)
 * is scaled to u = x_n N_l, the eight surrounding vertices are looked up --
 * densely (index x + (N+1)(y + (N+1) z)) when (N_l+1)^3 <= T, else by the
 * spatial hash (x*1 ^ y*2654435761 ^ z*805459861) mod 2^32 mod T -- and
 * trilinearly interpolated; the levels are concatenated.
 *   xc [3][ld], bone [S] (nullable: all valid)
 *   table [L][T][F] of table_dtype (IA355_F32 or IA355_F16)
 *   feat  [L][ld][F] of feat_dtype (IA355_F32 or IA355_BF16); zero for
 *         invalid samples.  F must be 2.  Interpolation is FP32. */
int32_t ia355_hashgrid_encode(const float *xc, const int16_t *bone, int64_t S, const int64_t *S_dev, int64_t ld,
                              const void *table, int32_t table_dtype, int32_t L, int32_t F, int32_t log2T,
                              double base_res, double growth, const float *aabb,
                              void *feat, int32_t feat_dtype, ia355_stream_t stream);

/* Backward of the encoding.  grad_feat [L][ld][F] FP32.
 *   grad_table [L][T][F] FP32 += sum over samples of w_c * grad_feat_l at each
 *   corner (nullable); with IA355_OVERWRITE in flags it is written instead
 *   (every entry, untouched ones set to 0).  IA355_TABLE_COARSE or
 *   IA355_TABLE_FINE limits the update (and the overwrite) to that level
 *   group's slice; the rest of grad_table is not touched.  Summation order inside a table
 *   entry is not fixed (atomic adds), so the last bits may vary run to run.
 *   grad_xc [3][ld] overwritten with sum_l sum_c (grad w_c)(theta_c . grad_feat_l)
 *   (nullable; needs the table and ws).  The levels are summed in order
 *   l = 0, 1, ..., so the result does not depend on the schedule.
 *   ws: ia355_hashgrid_encode_bwd_workspace_size(S, L) bytes (per-level
 *   partial position gradients); nullable when grad_xc is NULL.
 * The table gradient is added with FP32 global atomics laid out so that each
 * wave instruction touches few cache lines (run aggregation by a segmented
 * wave scan on the coarse dense levels, 16 lanes per sample and level
 * elsewhere). */
size_t ia355_hashgrid_encode_bwd_workspace_size(int64_t S, int32_t L);
int32_t ia355_hashgrid_encode_bwd(const float *grad_feat, const float *xc, const int16_t *bone,
                                  int64_t S, const int64_t *S_dev, int64_t ld, const void *table, int32_t table_dtype,
                                  int32_t L, int32_t F, int32_t log2T, double base_res, double growth,
                                  const float *aabb, float *grad_table, float *grad_xc, uint32_t flags,
                                  void *ws, size_t ws_bytes, ia355_stream_t stream);

/* Table gradient of the encoding (the grad_table output of
 * ia355_hashgrid_encode_bwd, same arguments, flags and result) computed
 * without global atomics on almost every entry: the corner updates are
 * binned by (level, table tile of 4096 entries), written once as 12-byte
 * records (the two FP32 values, the entry in the tile) and summed per tile
 * in LDS as exact 64-bit fixed point (a power-of-two scale per group of at
 * most 4096 records, chosen from its largest |value| m), then converted back
 * and written with plain stores.  Accuracy is absolute, relative to m: each
 * record is rounded to a quantum below m 2^-46, so an entry's error is at
 * most its record count times m 2^-47 plus one FP32 rounding of the entry
 * (values below m 2^-48 contribute zero).  A tile whose bin holds more than 4096
 * records is summed by several workgroups that add their nonzero entries
 * with FP32 atomics.  Every tile of the selected levels is written, so
 * IA355_OVERWRITE needs no separate clear.  A tile summed by one workgroup
 * does not depend on the order of its records; split tiles may vary in the
 * last bit from run to run.  NaN and infinite values are kept out of the
 * fixed-point sums and added to their entries as FP32 values, so they
 * propagate as with ia355_hashgrid_encode_bwd.
 *   grad_table: [L][T][F] FP32, 16-byte aligned, T = 2^log2T.
 *   ws: ia355_hashgrid_table_grad_workspace_size(S, L, log2T) bytes
 *       (S is the capacity when S_dev is given); about 96 bytes per sample
 *       and level.  Calls that may run at the same time need separate
 *       workspaces.
 * flags: IA355_OVERWRITE, a level group (IA355_TABLE_COARSE or _FINE) and
 * IA355_TABLE_PLAN (grad_feat and grad_table may then be NULL; nothing is
 * written but the workspace) or IA355_TABLE_REUSE_PLAN (xc, bone, S, S_dev
 * must be those of the plan; their contents must not have changed).  A
 * reuse without a matching plan gives wrong values; device-side checks keep
 * every access inside the workspace and the selected slice of grad_table.
 * Limits: L <= 16, L * 2^log2T <= 2^26 entries (at most 16384 tiles),
 * 8 L S < 2^32; otherwise IA355_ERR_INVALID_ARG (the workspace size is then
 * 0).  A workspace below the size returns IA355_ERR_WORKSPACE. */
size_t ia355_hashgrid_table_grad_workspace_size(int64_t S, int32_t L, int32_t log2T);
int32_t ia355_hashgrid_table_grad(const float *grad_feat, const float *xc, const int16_t *bone, int64_t S,
                                  const int64_t *S_dev, int64_t ld, int32_t L, int32_t F, int32_t log2T,
                                  double base_res, double growth, const float *aabb, float *grad_table,
                                  uint32_t flags, void *ws, size_t ws_bytes, ia355_stream_t stream);

/* The decoder of Sec. 3.1, Eq. 1-2: an MLP with ReLU hidden layers mapping
 * the concatenated features to sigma = exp(o_0) (clamped at exp(80)) and
 * c = sigmoid(o_1..3).
 *   widths (host) [n_layers + 1], n_layers: the layer widths; this library
 *   implements {32, 64, 64, 4} (n_layers 3), other shapes return
 *   IA355_ERR_UNSUPPORTED (a NULL widths, IA355_ERR_INVALID_ARG)
 *   feat [L][ld][F] (L*F = 32) of feat_dtype; params FP32 flat
 *   (per layer W [out][in] row-major, then b [out]; 6532 floats)
 *   dtype: IA355_F32 (FP32 MFMA) or IA355_BF16 (requires feat_dtype BF16):
 *   BF16 MFMA with FP32 accumulate; the weight matrices, the hidden
 *   activations (after the ReLU, decided on the FP32 pre-activation) and,
 *   in the backward, the deltas that multiply are bfloat16, the biases and
 *   their gradients FP32
 *   sigma [S], rgb [3][ld] FP32; invalid samples (bone < 0) get 0. */
int32_t ia355_mlp_fwd(const void *feat, int32_t feat_dtype, const int16_t *bone, int64_t S, const int64_t *S_dev,
                      int64_t ld, const float *params, const int32_t *widths, int32_t n_layers, int32_t dtype,
                      float *sigma, float *rgb, ia355_stream_t stream);

/* Backward of the MLP (the forward is recomputed from feat; nothing is
 * saved).  grad_sigma [S], grad_rgb [3][ld] FP32; widths as in the forward.
 *   grad_params [6532] FP32 accumulated (written with IA355_OVERWRITE)
 *   grad_feat [L][ld][F] FP32 overwritten (nullable)
 * ws: ia355_mlp_bwd_workspace_size(S) bytes (per-block weight-gradient
 * partials, reduced in a fixed order: the result is deterministic). */
size_t ia355_mlp_bwd_workspace_size(int64_t S);
int32_t ia355_mlp_bwd(const float *grad_sigma, const float *grad_rgb, const void *feat, int32_t feat_dtype,
                      const int16_t *bone, int64_t S, const int64_t *S_dev, int64_t ld, const float *params,
                      const int32_t *widths, int32_t n_layers, int32_t dtype, float *grad_params, float *grad_feat,
                      uint32_t flags, void *ws, size_t ws_bytes, ia355_stream_t stream);

/* ------------------------------------------------------------------ */
/* Volume rendering, Sec. 3.2 Eq. 8 (alpha_i = 1 - exp(-sigma_i delta_i)) */
/* with early termination (Sec. 3.4: stop once opacity reaches one).   */
/* ------------------------------------------------------------------ */
/* Per ray r, over its samples ray_off[r] .. ray_off[r+1]-1 in order, with
 * delta = ray_dt[r]: T_0 = 1, sample i is used iff T_i >= T_thresh (every
 * later one is then skipped), C = sum T_i alpha_i c_i, A = sum T_i alpha_i,
 * T_{i+1} = T_i (1 - alpha_i).  sigma [S], rgb [3][ld].
 * Outputs: color [R][3], opacity [R], n_used [R], T_final [R]. */
int32_t ia355_volrender_fwd(const float *sigma, const float *rgb, int64_t ld, const int64_t *ray_off,
                            const float *ray_dt, int64_t R, float T_thresh,
                            float *color, float *opacity, int32_t *n_used, float *T_final, ia355_stream_t stream);

/* Backward: grad_rgb_i = T_i alpha_i g_C,
 * grad_sigma_i = delta [T_{i+1} (g_C . c_i) - g_C . (C - C_<=i)] + g_A delta T_final;
 * unused samples get 0.  grad_color [R][3], grad_opacity [R] (nullable);
 * color, T_final are the forward outputs.  grad_sigma [S], grad_rgb [3][ld]
 * overwritten for every sample of every ray. */
int32_t ia355_volrender_bwd(const float *grad_color, const float *grad_opacity,
                            const float *sigma, const float *rgb, int64_t ld, const int64_t *ray_off,
                            const float *ray_dt, const int32_t *n_used, const float *color, const float *T_final,
                            int64_t R, float *grad_sigma, float *grad_rgb, ia355_stream_t stream);

/* Training loss of Sec. 3.4 over R rays: loss[4] = {total, L_rgb, L_alpha,
 * L_hard}, each the mean over the rays of, respectively, the sum of the
 * three, rho(|C - C_gt|) (Huber with threshold delta, whose value the paper
 * does not give), lam_alpha |A - A_gt| and lam_hard (-log(exp(-|A|) +
 * exp(-|A - 1|)) + log(1 + exp(-1))).  color, target [R][3], opacity,
 * alpha_gt [R] (alpha_gt nullable: no L_alpha).  grad_color [R][3] and
 * grad_opacity [R] (for ia355_volrender_bwd) are overwritten; at a kink the
 * gradient uses sign(0) = 0.  One workgroup, a fixed summation order. */
int32_t ia355_loss_full(const float *color, const float *opacity, const float *target, const float *alpha_gt,
                        int64_t R, float delta, float lam_alpha, float lam_hard, float *loss,
                        float *grad_color, float *grad_opacity, ia355_stream_t stream);

/* Adam (Kingma and Ba, bias-corrected) on a flat FP32 array of n
 * parameters: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * param -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), with t = step,
 * or t = *step_dev when step_dev is given (device memory, so a captured
 * step needs no host value).  param_f16 (nullable) receives the updated
 * parameters rounded to FP16 (the mixed-precision copy of the hash table).
 * ia355_count_step adds one to *step_dev: call it once per training step
 * before the updates. */
int32_t ia355_adam(float *param, const float *grad, float *m, float *v, int64_t n, float lr, float beta1,
                   float beta2, float eps, int32_t step, const int32_t *step_dev, void *param_f16,
                   ia355_stream_t stream);
int32_t ia355_count_step(int32_t *step_dev, ia355_stream_t stream);

/* Photometric L2 loss (the benchmark's stand-in for the Huber loss of
 * Eq. 9, whose threshold the paper does not give): loss[0] = mean over R*3
 * of (color - target)^2 (device float, overwritten); grad_color [R][3] =
 * dloss/dcolor (overwritten).  color, target [R][3]. */
int32_t ia355_l2_loss(const float *color, const float *target, int64_t R, float *loss, float *grad_color,
                      ia355_stream_t stream);

/* ------------------------------------------------------------------ */
/* Batched inference render: many poses of one avatar in one          */
/* persistent launch (the forward of Sec. 3.1-3.3 and Eq. 8 per ray). */
/* ------------------------------------------------------------------ */
#define IA355_BATCH_MAX_POSES 64

/* One pose.  Device pointers, owned by the caller; they must stay valid
 * (and the outputs unread) until the render calls that use them have run.
 *   rays_o, rays_d [R][3]; occ_bits (ia355_occ_pack layout, G^3 cells over
 *   occ_aabb; NULL keeps every step); dt / n_per_ray / max_steps as for
 *   ia355_occgrid_march, max_steps <= 128;
 *   B [nb][3][4] bone transforms; pose [nb][6] the initialiser's pose input;
 *   outputs as ia355_volrender_fwd: color [R][3], opacity [R], n_used [R],
 *   T_final [R]; n_fallback [1] (nullable) receives the number of evaluated
 *   samples whose guided solve was rejected, n_evaluated [1] (nullable) the
 *   number of samples evaluated (see below). */
typedef struct ia355_batch_pose {
  const float *rays_o, *rays_d;
  int64_t R;
  const uint32_t *occ_bits;
  int32_t G;
  float occ_aabb[6];
  float dt;
  int32_t n_per_ray, max_steps;
  const float *B, *pose;
  float *color, *opacity;
  int32_t *n_used;
  float *T_final;
  int32_t *n_fallback, *n_evaluated;
} ia355_batch_pose;

/* What the poses share (device pointers, owned by the caller):
 *   skinning grid W [Dz][Dy][Dx][nb] over skin_aabb; canonical box hash_aabb;
 *   Broyden max_iter, tol_stop, tol_valid (ia355_snarf_deform);
 *   FP16 hash table [L][2^log2T][2] (16-byte aligned), L = 16, per-level
 *   resolutions floor(base_res growth^l); decoder parameters (32-64-64-4,
 *   FP32 flat, 16-byte aligned, used as BF16 MFMA operands exactly as
 *   ia355_mlp_fwd with IA355_BF16); initialiser parameters (FP32 flat,
 *   hidden width init_hidden = 64, used as ia355_rootinit_fwd with
 *   IA355_BF16); compositing threshold T_thresh. */
typedef struct ia355_batch_model {
  const float *W;
  int32_t Dx, Dy, Dz, nb;
  float skin_aabb[6], hash_aabb[6];
  int32_t max_iter;
  float tol_stop, tol_valid;
  const void *table;
  int32_t L, log2T;
  double base_res, growth;
  const float *mlp_params, *init_params;
  int32_t init_hidden;
  float T_thresh;
} ia355_batch_model;

/* Every pose rendered as the staged path renders it (ia355_occgrid_march ->
 * ia355_rootinit_fwd -> ia355_snarf_deform_guided -> ia355_hashgrid_encode
 * (FP16 table, BF16 features) -> ia355_mlp_fwd (BF16) ->
 * ia355_volrender_fwd): the same operations on the same values, so the
 * same output bits, with no per-sample buffer in global memory.  Samples are
 * evaluated in the compositor's groups of 16 per ray, front to back, and a
 * ray's groups after the one where it terminates (Eq. 8 with T_thresh) are
 * not evaluated: they cannot change its outputs.
 * ia355_batch_plan validates the poses and the model and writes the plan
 * into ws (ia355_batch_workspace_size bytes: the plan, a work counter and
 * per pose the blended transform grid, the folded initialiser constant and
 * the bone inverses); it copies from host memory and synchronises the
 * stream, so it is not for graph capture.  ia355_batch_render enqueues two
 * kernels (per-pose preparation, then the persistent render) and is
 * capturable.  Its schedule: 256 * blocks_per_cu workgroups of
 * waves_per_group waves (4 or 8; blocks_per_cu 1-4 with 4 waves, 1-2 with 8,
 * else IA355_ERR_UNSUPPORTED); every wave takes tiles of rays_per_tile rays
 * (1..64) of one pose from a work counter and works through them in
 * segments of at most samples_per_segment samples (256..8192).  It reads
 * the plan from ws, which must be the ws the plan was written to (a ws
 * without a valid plan renders nothing).  ia355_batch_lds_bytes gives a
 * schedule's LDS per workgroup (0: invalid shape); a schedule needing more
 * than the device allows per workgroup returns IA355_ERR_UNSUPPORTED. */
size_t ia355_batch_workspace_size(int32_t n_poses, int32_t Dx, int32_t Dy, int32_t Dz, int32_t nb);
int32_t ia355_batch_plan(const ia355_batch_pose *poses, int32_t n_poses, const ia355_batch_model *model,
                         void *ws, size_t ws_bytes, ia355_stream_t stream);
size_t ia355_batch_lds_bytes(int32_t rays_per_tile, int32_t samples_per_segment, int32_t waves_per_group);
int32_t ia355_batch_render(const void *ws, size_t ws_bytes, int32_t rays_per_tile, int32_t samples_per_segment,
                           int32_t waves_per_group, int32_t blocks_per_cu, ia355_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* IA355_H */
