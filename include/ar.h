/*
 * ar.h -- C ABI of the MI355X (gfx950) abstract renderer for Gaussian-splat scenes.
 *
 * Abstract rendering (Li, Ji, Zhong, Zhang, Mitra, "Abstract Rendering: Computing All
 * that is Seen in Gaussian Splat Scenes", arXiv 2503.00308): given a scene of 3-D
 * Gaussians and a SET of camera poses, compute for every pixel a lower and an upper
 * RGB bound that contain the colour the splat renderer produces at every pose of the
 * set (Sec. 2.2, "Abstract rendering problem"; Theorem "all" of Sec. 3.3).
 *
 * The set of poses is a box in pose parameters (Sec. 4.2: position radius eps_t and
 * orientation radius eps_R around a nominal camera), or a cell of an orbit about a
 * vertical axis.  Every quantity of Alg. GaussianSplat is propagated as a pair of
 * linear forms over the normalised box, the 2x2 covariance inverse by MatrixInv
 * (Sec. 3.1) and the blend by BlendInd (Sec. 3.2), as in AbstractSplat (Sec. 3.3).
 *
 * Conventions
 *   camera axes x right, y down, z forward; a world point uw maps to
 *   uc = R (uw - t) with R world->camera and t the camera centre (Alg. GaussianSplat,
 *   Step 1); pixel (col, row) has centre (col + 1/2, row + 1/2); fx, fy, cx, cy the
 *   pinhole intrinsics (Sec. 2.2, matrix K).
 *
 * Memory
 *   Unless stated otherwise, pointers are host pointers.  Output images are DEVICE
 *   pointers (HBM) of H*W*3 floats in row-major [row][col][channel] order.  The caller
 *   owns every buffer it passes; a scene handle owns its device copy of the scene.
 *   Work is issued on the given HIP stream (NULL = the default stream).  The render
 *   calls synchronise that stream once mid-way (to size the tile lists) and again at
 *   the end, so outputs and statistics are complete when they return.
 *
 * Errors
 *   Every function returns AR_OK (0) or a negative AR_E_* code; nothing aborts.
 *   ar_last_error() returns a thread-local message for the last failure.
 */
#ifndef AR_H
#define AR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AR_OK = 0,
  AR_E_INVALID = -1,     /* an argument is out of range, non-finite or inconsistent */
  AR_E_OOM = -2,         /* device memory could not be allocated */
  AR_E_DEVICE = -3,      /* a HIP runtime call failed */
  AR_E_UNSUPPORTED = -4, /* a valid request the library does not handle */
  AR_E_BUDGET = -5,      /* a server request does not fit the memory budget */
  AR_PENDING = 1         /* ar_server_wait without blocking: the query has not finished */
};

enum { AR_POSE_CAMERA6 = 0, AR_POSE_ORBIT = 1 };

/* Opaque scene handle: a device-resident copy of the Gaussians. */
typedef struct ar_scene ar_scene;

/*
 * Scene of n Gaussians <uw, Mw, o, c> (Sec. 2.2): mean uw, covariance factor Mw with
 * Cov = Mw Mw^T (footnote of Sec. 2.2), opacity o in (0, 1], colour c in [0, 1]^3.
 * Structure-of-arrays, float32, host or device memory (see on_device):
 *   mean       [3][n]  (x of all Gaussians, then y, then z)
 *   cov_factor [9][n]  entry (r, c) of Mw at plane 3 r + c
 *   opacity    [n]
 *   rgb        [3][n]
 * or, in place of cov_factor (NULL), the rotation and scales a trained splat stores:
 *   quat       [4][n]  quaternion (w, x, y, z), any non-zero length (normalised here)
 *   scale      [3][n]  scales (standard deviations along the rotated axes), >= 0
 * from which Mw = R(q) diag(scale) (a factor of Cov = R diag(scale)^2 R^T), formed in
 * FP64 on the host and rounded to float32.  quat and scale are ignored when cov_factor
 * is given.
 * Rejected (AR_E_INVALID): n < 1, a NULL array (quat and scale only when cov_factor is
 * NULL), a non-finite value, a zero quaternion, a negative scale, o outside (0, 1], a
 * colour outside [0, 1].
 */
typedef struct {
  int32_t n;
  int32_t on_device; /* 0: the arrays are host memory, 1: device memory */
  const float *mean;
  const float *cov_factor;
  const float *opacity;
  const float *rgb;
  const float *quat;
  const float *scale;
} ar_scene_desc;

/* Pinhole intrinsics and image size (Sec. 2.2, K).  width, height in [1, 16384]. */
typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
} ar_intrinsics;

/*
 * A set of camera poses.
 *   AR_POSE_CAMERA6: p = (tx, ty, tz, yaw, pitch, roll) in the box lo <= p <= hi;
 *     R(p) = Ry(yaw) Rx(pitch) Rz(roll) R0 and t(p) = t0 + (tx, ty, tz), angles in
 *     radians, elementary rotations right-handed.  lo = hi on an axis fixes it.
 *   AR_POSE_ORBIT: the camera rig (R0, t0) turned by phi in [lo[0], hi[0]] about the
 *     vertical (y) axis through pivot: t(phi) = pivot + Ry(phi)(t0 - pivot),
 *     R(phi) = R0 Ry(phi)^T.  Entries 1..5 of lo / hi are ignored.
 * R0 is row-major world->camera.  Rejected: lo > hi, non-finite entries, angle
 * half-widths above 0.5 rad.
 */
typedef struct {
  int32_t model;
  double R0[9];
  double t0[3];
  double pivot[3];
  double lo[6];
  double hi[6];
} ar_pose_box;

/*
 * Options; a zero field takes the default.
 *   tile        pixel side of the binning tiles: 8 (default; one 64-lane wave per tile)
 *               or 16 (translation boxes only: a tile's list serves its four 8x8 blocks,
 *               one wave each; fewer list entries to sort, every entry walked four
 *               times).  The bounds enclose the same set with either (rounding aside,
 *               they agree to a few units of the last place); rotation boxes with 16 are
 *               rejected (AR_E_UNSUPPORTED), other values too
 *   ind_window  rotation boxes: which pairs of a tile list get the pairwise Ind test;
 *               0 = those inside the smaller of the two depth windows (default),
 *               1 = inside the window from the box of the list's means only,
 *               2 = every pair (slow; the result is the same, for checking)
 *   chunk       list positions per segment of the pixel loop (one wave each),
 *               8..4096 (default: translation boxes chosen from the number of pairs,
 *               rotation boxes 64)
 *   taylor_k    MatrixInv order k (Sec. 3.1; default 8, the paper's default), 1..16
 *   cull_budget bound E on the colour change from pruning faint Gaussians (default 1e-7);
 *               Gaussian i is dropped from pixel u when its alpha is provably below
 *               cull_budget / n at every pose; lower / upper bounds are widened by E
 *   z_near      near plane (default 0.01): depth <= z_near gives alpha 0
 *   prefix_entries  rotation boxes: tile-list entries whose per-pixel prefix sums one
 *               pixel-loop launch holds (64 x 16 bytes each; default 2^21; a longer
 *               single list gets its own launch)
 *   cells_per_launch  ar_render_batch: pose cells per launch (default: as many as fit a
 *               workspace of about 4 GiB, at most 256)
 *   t_min       translation boxes: stop a tile once every pixel's transmittance upper
 *               bound is below it, widening the upper bound by that transmittance;
 *               rotation boxes: take an entry's lower transmittance as 0 where its bound
 *               through the list positions surely in front of it, times the list's
 *               length, is below t_min (the lower bound moves by less than t_min);
 *               default 1e-7, negative disables both
 *   abs_sums, ind_copy, ind_masks   rotation boxes: switches of three layouts the
 *               library otherwise picks from the size of the call (0 = automatic,
 *               1 = on, 2 = off; any other value is rejected).  They change the speed,
 *               never the result (bit for bit):
 *                 abs_sums   the per-pixel running sums of the transmittance logs made
 *                            absolute in a pass of their own (automatic: on with at
 *                            least 8 Ind runs per list entry);
 *                 ind_copy   the Ind tests read a copy of the means and depth forms laid
 *                            out by list position (automatic: on when the Ind windows
 *                            average 32 positions or more);
 *                 ind_masks  the Ind masks of windows longer than 64 positions kept
 *                            between the counting and emitting passes (automatic and 1:
 *                            kept when they fit 8 GiB; 2: tested again instead)
 *   group_entries  rotation boxes: the Ind passes (windows, tests, runs) and the pixel
 *               loop run over groups of consecutive whole tile lists holding at most
 *               this many entries each (a longer single list is a group of its own;
 *               default 2^27).  Bounds the 32-bit counts of a group; the result does not
 *               depend on it (bit for bit).
 *   group_runs  rotation boxes: the most Ind runs one list group may hold (default and
 *               at most 2^32 - 1, the range of the runs' offsets).  A group whose runs
 *               exceed it is cut into smaller groups of whole lists and done again; only a
 *               single list with more runs is rejected (AR_E_UNSUPPORTED).  The result does
 *               not depend on it (bit for bit).
 *   ind_quick   rotation boxes: each Ind test first tries the identity bound's constant
 *               against a per-axis bound of all its other terms (3 + 3 multiply-adds),
 *               which decides most pairs of a window; where it decides, the full bound
 *               decides the same way (0 = automatic and 1: on; 2: off, every test takes
 *               the full bound).  Speed only, never the result (bit for bit)
 *   inverse     the covariance inverse of Step 3 (Conic): 0 = MatrixInv (Sec. 3.1) with
 *               its linear bounds propagated forward (default); 1 = MatrixInv with its
 *               bounds propagated backward (CROWN-style, as the paper's bound engine;
 *               usually tighter, about k^2 more work in the per-Gaussian stage);
 *               2 = the adjugate inverse adj(X) Div(det X) (Example 'matinv-vs-direct',
 *               a precision baseline, looser).  Where an inverse cannot be bounded (the
 *               assertion of MatrixInv fails, or det X is not provably positive) the
 *               Gaussian is a fallback (alpha in [0, footprint bound]), as always.
 */
typedef struct {
  int32_t tile;
  int32_t ind_window;
  int32_t chunk;
  int32_t taylor_k;
  double cull_budget;
  double z_near;
  double t_min;
  int32_t cells_per_launch;
  int32_t prefix_entries;
  int32_t abs_sums;
  int32_t ind_copy;
  int32_t ind_masks;
  int32_t group_entries;
  int32_t inverse;
  int32_t group_runs;
  int32_t ind_quick;
} ar_options;

/* Statistics of one call (filled when the call returns). */
typedef struct {
  int64_t pairs;         /* (pixel, Gaussian) pairs whose alpha bounds were evaluated */
  int64_t tile_pairs;    /* (tile, Gaussian) pairs produced by binning */
  int32_t n_fallback;    /* Gaussians whose MatrixInv assertion failed (alpha in [0, bound]) */
  int32_t n_wild;        /* Gaussians straddling the near plane (alpha in [0, o] everywhere) */
  int32_t n_dropped;     /* Gaussians behind the near plane at every pose */
  int32_t P;             /* number of pose variables of the box */
  int32_t max_window;    /* largest Ind window of uncertain depth order (rotations), after
                            its ends decided chunk by chunk are trimmed */
  int32_t segment_length; /* list positions per segment of the pixel loop (largest of the call) */
  double raster_ms;      /* device time of the main per-pixel kernel (HIP events on the call's stream) */
  double total_ms;       /* device time of the whole call from its first to its last kernel */
  int64_t runs;          /* rotation boxes: runs of list positions holding the Ind sets */
  int64_t cycles_a, cycles_b; /* rotation boxes: summed wave clock cycles of the pixel loop's two phases */
  int64_t ind_tests;     /* rotation boxes: pairwise Ind tests (summed window lengths;
                            depends on the options, never the result) */
  int64_t ind_borderline; /* rotation boxes: Ind tests decided by a bound within rounding of its
                             threshold (1e-12 (1 + |uw_i - uw_j|_1)), which another order of
                             the same operations might decide otherwise */
} ar_stats;

/* Copies the scene to the device on `stream` (synchronises it).  *out receives a
 * handle to release with ar_scene_destroy. */
int ar_scene_create(const ar_scene_desc *desc, void *hip_stream, ar_scene **out);

/*
 * A set of scenes around the Gaussians of an ar_scene_desc (Sec. 4.6, "abstract rendering
 * sets of scene": colour, mean position and opacity perturbations).  Every array may be
 * NULL (that attribute is exact); arrays are host or device memory (on_device):
 *   rgb_hi      [3][n]  colour upper bounds; the desc's rgb is the lower bound
 *                       (rgb <= rgb_hi <= 1)
 *   opacity_lo  [n]     opacity lower bounds; the desc's opacity is the upper bound
 *                       (0 <= opacity_lo <= opacity)
 *   mean_var    [n]     the scene variable (0..nvar-1) that moves Gaussian i's mean, or -1
 *   mean_dir    [3][n]  its direction: the mean is uw_i + mean_dir_i s_{mean_var[i]}
 *   nvar, lo, hi        scene variables s_v in [lo[v], hi[v]], v < nvar <= 6
 * Colours and opacities enter the blend as intervals (the lower colour in the lower, the
 * upper colour in the upper image; the lower opacity in the lower, the upper in the upper
 * alpha bound); a moved mean is a linear form in its variable, an extra variable after the
 * pose variables, and a render rejects (AR_E_UNSUPPORTED) a box whose pose variables plus
 * the scene's exceed 6.  Scenes with variables render on the general (depth-order)
 * path: a moved mean can change the depth order even under a translation box, so every
 * pair of a tile list is tested.  Rejected (AR_E_INVALID): bounds out of the ranges above,
 * non-finite values, nvar > 0 without mean_var and mean_dir, mean_var out of range.
 */
typedef struct {
  int32_t nvar;
  int32_t on_device; /* 0: the arrays are host memory, 1: device memory */
  double lo[6];
  double hi[6];
  const float *rgb_hi;
  const float *opacity_lo;
  const int32_t *mean_var;
  const float *mean_dir;
} ar_scene_set;

/* As ar_scene_create, for the set of scenes *set around *desc (set must not be NULL).
 * Every render call on the handle bounds every scene of the set at every pose of its box. */
int ar_scene_create_set(const ar_scene_desc *desc, const ar_scene_set *set, void *hip_stream, ar_scene **out);

/* Releases a scene handle and its device memory (NULL is ignored). */
void ar_scene_destroy(ar_scene *scene);

/* Number of Gaussians of a scene handle (0 for NULL). */
int32_t ar_scene_size(const ar_scene *scene);

/*
 * Lower / upper images over the pose box (AbstractSplat, Sec. 3.3).
 *   lo_rgb, hi_rgb: height*width*3 floats, [row][col][channel], both device memory or
 *   both host memory (pinned or pageable: the images are rendered into the scene
 *   handle's workspace and copied back before the call returns; with device memory the
 *   call returns once its work is complete on the stream as well);
 *   for every pose p of the box and every pixel, lo <= GaussianSplat(scene, p) <= hi.
 *   opts, stats may be NULL.  The scene handle's workspace is reused, so calls on the
 *   same scene handle must not overlap in time (serialise them on one stream).  One
 *   output in device memory and the other not is rejected (AR_E_INVALID).
 */
int ar_render_bounds(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                     const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream,
                     ar_stats *stats);

/*
 * For callers that cannot allocate memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ar_render_bounds without any allocation.
 * Arguments, result (bit for bit) and errors are those of ar_render_bounds, with these
 * limits:
 *   - translation boxes only (no yaw / pitch / roll, ORBIT width 0); a rotation box is
 *     rejected with AR_E_UNSUPPORTED;
 *   - the outputs are device memory (host outputs are rejected with AR_E_INVALID);
 *   - every device buffer of the render comes from one static device array of 256 MiB
 *     per GPU, which each GPU the library runs on holds until the process ends; a render
 *     that needs more (e.g. above about 10k Gaussians at 128x128 with a wide box) fails
 *     with AR_E_UNSUPPORTED and a message, nothing else is touched;
 *   - stats->raster_ms and stats->total_ms are 0 (no events are created).
 * All calls on one GPU share that array, which keeps the last call's contents; calls on
 * one GPU are serialised by a lock held until the call's work is complete, and work of
 * other code that reads the array's contents after a call races with the next call.
 * The call makes no hipMalloc, hipFree, hipHostMalloc or hipEventCreate; on its first
 * call on a device it looks up the array's address there (hipGetSymbolAddress).
 */
int ar_render_bounds_noalloc(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                             const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream,
                             ar_stats *stats);

/*
 * Bounds for ncells pose boxes of one scene (the partition of a larger set of poses,
 * Sec. 4.2 "#part"); lo_rgb / hi_rgb hold ncells images back to back, device or host
 * memory as for ar_render_bounds.  The result is
 * that of ncells calls of ar_render_bounds (bit for bit when opts->chunk is set);
 * consecutive cells with the same pose variables share one launch per stage, up to
 * opts->cells_per_launch cells (default: what fits a quarter of the free device
 * memory).  stats (may be NULL) accumulates over the cells.
 */
int ar_render_batch(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells,
                    int32_t ncells, const ar_options *opts, float *lo_rgb, float *hi_rgb,
                    void *hip_stream, ar_stats *stats);

/*
 * As ar_render_batch, with a scene per cell: cell c renders scenes[c] (scenes of any
 * sizes, repeated or not, all on the current device).  Consecutive cells with the same
 * pose variables share one launch per stage whatever their scenes: cell c's Gaussians
 * are its own range of the launch's items, and its images are those of
 * ar_render_batch(scenes[c], ...) for that cell (bit for bit for rotation boxes, and for
 * translation boxes when opts->chunk is set; the cull threshold is each scene's own).
 * Launches are sized for the largest scene of their cells.  The call uses the
 * workspace of scenes[0] (no call on scenes[0] may overlap it).  Sets of scenes (scene
 * variables) render only in calls of their own: a cell of one among other scenes is
 * rejected (AR_E_UNSUPPORTED); a NULL scene or one on another device is AR_E_INVALID.
 */
int ar_render_batch_scenes(const ar_scene *const *scenes, const ar_intrinsics *intr, const ar_pose_box *cells,
                           int32_t ncells, const ar_options *opts, float *lo_rgb, float *hi_rgb,
                           void *hip_stream, ar_stats *stats);

/*
 * Planned batched renders (the batched workload as one HIP graph).  A plan holds the
 * whole launch sequence of a batch of ncells pose boxes (all with the same pose
 * variables, as in ar_render_batch) captured in a HIP graph: every count stays on the
 * device, so a replay has no host synchronisation inside and no allocation.
 *   ar_plan_create   renders the cells once on the ordinary batched path to size every
 *                    launch of cells (the scene handle's workspace; calls on the scene
 *                    must not overlap), takes capacities with a quarter of headroom,
 *                    allocates the plan's own workspace, runs the launch sequence once and
 *                    captures it (on a stream of the plan's own).  lo_rgb / hi_rgb: device
 *                    images [ncells][H][W][3], fixed for the plan's life; they hold the
 *                    cells' bounds when the call returns.  Translation boxes give the
 *                    result of ar_render_batch bit for bit when opts->chunk is set,
 *                    rotation boxes always.  AR_E_UNSUPPORTED when a launch of cells needs
 *                    more than one list group (use fewer cells_per_launch).
 *   ar_plan_set_cells  new pose boxes for the next launch (ncells of them, with the pose
 *                    variables of the plan's cells; host memory, copied); they are copied
 *                    to the device by the graph itself.
 *   ar_plan_launch   replays the graph on the stream and waits for it; stats (may be NULL)
 *                    as ar_render_batch's, total_ms the graph's device time (raster_ms 0).
 *                    When the cells outgrew the capacities, the launch is rendered again on
 *                    the ordinary path, the plan is captured again with the new sizes and
 *                    *replanned (may be NULL) is set to 1 (else 0); the images are right in
 *                    both cases.
 *   ar_plan_destroy  releases the plan (NULL is ignored).
 */
typedef struct ar_plan ar_plan;

int ar_plan_create(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, int32_t ncells,
                   const ar_options *opts, float *lo_rgb, float *hi_rgb, void *hip_stream, ar_plan **out);
int ar_plan_set_cells(ar_plan *plan, const ar_pose_box *cells);
int ar_plan_launch(ar_plan *plan, void *hip_stream, ar_stats *stats, int32_t *replanned);
void ar_plan_destroy(ar_plan *plan);

/*
 * Bounds over one pose box partitioned into a grid of cells (Sec. 4.2: the set of
 * cameras split into subsets, bounds computed per subset and united).  Axis a of the box
 * is cut into splits[a] equal parts (splits: 6 entries, each >= 1; ORBIT boxes use
 * splits[0] only; a zero-width axis is not cut); the cells are rendered as by
 * ar_render_batch (in launches of up to 64 cells, or options.cells_per_launch) and the
 * output is their union, the elementwise minimum of the lower and maximum of the upper
 * images, which encloses every pose of the box and is usually tighter than the bounds of
 * the whole box.  lo_rgb / hi_rgb: [H][W][3] float32, device memory.  At most 65536
 * cells.  stats (may be NULL) accumulates over the cells.  Returns AR_OK or an error code.
 */
int ar_render_partitioned(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                          const int32_t *splits, const ar_options *opts, float *lo_rgb, float *hi_rgb,
                          void *hip_stream, ar_stats *stats);

/*
 * Per pose cell, the counts that drive the adaptive refinement (ar_render_refined):
 * counts[2c] = Gaussians whose MatrixInv convergence assertion fails over cell c
 * (Sec. 3.1, Alg. MatrixInv) and that the pruning test keeps at some pixel of the
 * image (the binning's float32 test on the rectangle of all pixel centres);
 * counts[2c + 1] = Gaussians straddling the near plane over cell c (alpha in [0, o]).
 * counts: host memory, 2 * ncells int64.  Synchronises the stream.  Returns AR_OK or an
 * error code (invalid cell, options or intrinsics; device failure).
 */
int ar_classify_cells(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, int32_t ncells,
                      const ar_options *opts, int64_t *counts, void *hip_stream);

/*
 * Per pose cell, the number of undecided depth-order tests (Sec. 3.2: Ind(d_i - d_j) is
 * piecewise constant, tight on every part of the pose domain where d_i - d_j keeps its
 * sign, so a cell whose tests stay undecided is one to cut): counts[c] = the ordered pairs
 * (i, j), i != j, of Gaussians in one tile list of cell c (summed over the tile lists)
 * whose three-valued Ind is 2 (unknown), with the bounds of ar_render_bounds (the
 * identity A_z (uw_i - uw_j) and the literal difference of the depth forms).  A box
 * whose depth order cannot change (translations only, scene without moved means) has 0.
 * counts: host memory, ncells int64.  Runs the rotation path up to its Ind tests (no
 * images); synchronises the stream.  Returns AR_OK or an error code as
 * ar_classify_cells.
 */
int ar_count_ind_uncertain(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells,
                           int32_t ncells, const ar_options *opts, int64_t *counts, void *hip_stream);

/* Criteria of ar_render_refined (bit mask; 0 means AR_REFINE_MATINV). */
enum {
  AR_REFINE_MATINV = 1,   /* cut cells holding a MatrixInv failure kept in the image */
  AR_REFINE_NEAR = 2,     /* cut cells holding a near-plane straddler */
  AR_REFINE_IND = 4       /* cut cells with undecided depth-order tests (ar_count_ind_uncertain) */
};

/*
 * Bounds over a pose box refined where MatrixInv fails (Sec. 3.1: the input range is
 * divided until the convergence assertion holds), where Gaussians straddle the near
 * plane, or where depth-order tests stay undecided (Sec. 3.2: Ind is tight on parts of
 * the domain where its argument keeps its sign); Sec. 4.2: bounds of subsets of the
 * cameras, united.  Cells are taken level by level, in order, starting from the whole
 * box; a cell flagged by the criteria (counts of ar_classify_cells, and with
 * AR_REFINE_IND of ar_count_ind_uncertain) at depth k (k
 * bisections from the box) is cut at the midpoint 0.5 (lo + hi) of its active axis
 * number k mod (number of active axes) (ORBIT: the angle), lower half first, while the
 * number of cells stays within max_cells (1..65536) and k < 24; every other cell is a
 * leaf.  The leaves are rendered as ar_render_batch and united (elementwise minimum of
 * the lower, maximum of the upper images) into lo_rgb / hi_rgb ([H][W][3] float32,
 * device memory), which enclose every pose of the box.  cells_out (may be NULL; room for
 * max_cells boxes) receives the leaves in the order they were settled and *ncells_out
 * (may be NULL) their number; stats (may be NULL) accumulates over the leaves' renders.
 * Returns AR_OK or an error code (AR_E_INVALID for max_cells or criteria out of range).
 */
int ar_render_refined(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *box,
                      const ar_options *opts, int32_t max_cells, int32_t criteria, float *lo_rgb, float *hi_rgb,
                      void *hip_stream, ar_pose_box *cells_out, int32_t *ncells_out, ar_stats *stats);

/*
 * Autotuning of the binning tile (options.tile), the pixel loop's segment length
 * (options.chunk) and, for a batch, the cells per launch (options.cells_per_launch) for
 * a workload: one pose box (ncells = 1) or a batch of cells, rendered as
 * ar_render_batch.  Per tile (translation boxes: 8 and 16 unless *opts fixes one;
 * rotation boxes: 8) the workload is rendered with the automatic length, then with
 * candidates (translation boxes: the automatic length times 1/2, 3/4, 5/4 and 3/2,
 * multiples of 8 in [8, 4096]; rotation boxes: 32, 48, 64, 96 and 128), reps times each
 * (1..16); tile and chunk are the pair with the least device time (stats.total_ms).
 * With ncells > 1 and no cells_per_launch in *opts, the counts
 * automatic (what fits the memory budget), half and a quarter of it, 16 and 8 (those
 * below the automatic count) are then timed by wall clock with that chunk.  *tuned
 * receives a copy of *opts (or of the defaults when opts is NULL) with the chosen tile,
 * chunk and cells per launch (0: the automatic count).  The workload is rendered once more with *tuned,
 * so lo_rgb / hi_rgb ([ncells][H][W][3], device memory) hold its bounds, and stats (may
 * be NULL) that render's statistics.  Results with any tile and chunk enclose the same
 * set; with the tuned ones they are those of ar_render_batch(..., tuned, ...) bit for bit.
 * Returns AR_OK or an error code as ar_render_batch (ar_last_error).
 */
int ar_autotune(const ar_scene *scene, const ar_intrinsics *intr, const ar_pose_box *cells, int32_t ncells,
                const ar_options *opts, int32_t reps, float *lo_rgb, float *hi_rgb, void *hip_stream,
                ar_options *tuned, ar_stats *stats);

/* Message of the last failure on the calling thread ("" if none). */
const char *ar_last_error(void);

/* Library version string. */
const char *ar_version(void);

/*
 * Query server: abstract-render queries over resident scenes with continuous batching.
 * A server owns `slots` HIP streams (default priority), each with its own workspace and
 * host worker thread.  Queries are taken in submission order; the next query starts as
 * soon as a slot is free and its estimated workspace fits the device-memory budget next
 * to the workspaces of the queries in flight, so queries of different scenes, image
 * sizes and boxes run on the device at the same time once a backlog builds up: a query
 * starts beside running ones only while at least overlap_queue queries wait (kernels of
 * concurrent queries interleave without preemption, so a query beside a long one takes
 * longer; overlap pays when it drains a backlog).  With batch_max > 1, under the same
 * backlog a slot also takes, with the query at the head, later queued queries that can
 * share its launches (same image size and intrinsics, options and pose variables;
 * rotation boxes, or translation boxes with options.chunk set; plain scenes, or all on
 * one scene), up to batch_max queries whose estimates fit the budget together: they
 * render as one batch of cells over their scenes (ar_render_batch_scenes) and complete
 * together.  Sharing pays for many small queries; queries that fill the device alone
 * gain nothing from it and wait for each other, so it is off by default.  A query's
 * result is the same as ar_render_bounds on the same arguments, bit for bit, alone or in
 * a shared launch.
 *
 * hbm_budget  device bytes all slot workspaces may hold (0: half of the free memory at
 *             creation); scenes are not counted.  A query whose estimate exceeds the
 *             budget on its own runs when no other query is in flight.  A slot keeps its
 *             workspace between queries unless the workspaces held exceed the budget,
 *             then it frees it (counted in ar_server_stats.releases).
 * slots       queries in flight at once, 1..16 (0: 4).
 * overlap_queue  queries waiting from which the next starts beside running ones, and
 *             from which queries share launches (0: the number of slots; 1: whenever a
 *             slot is free).
 * batch_max   most queries in one shared launch, 1..256 (0 and 1: never shared).
 */
typedef struct ar_server ar_server;

typedef struct {
  uint64_t hbm_budget;
  int32_t slots;
  int32_t overlap_queue;
  int32_t batch_max;
  int32_t reserved;     /* must be 0 */
} ar_server_config;

typedef struct {
  int32_t status;        /* AR_OK, AR_PENDING, or the AR_E_* code of a failed query */
  int32_t slot;          /* slot (stream) the query ran on */
  double queue_ms;       /* submission -> start on a slot (host clock) */
  double latency_ms;     /* submission -> outputs complete (host clock) */
  ar_stats stats;
  uint64_t est_bytes;    /* workspace bytes estimated for the query at admission */
  uint64_t ws_bytes;     /* workspace bytes the slot held when the query finished */
  int32_t batched;       /* queries in the launch that rendered it (1: alone); stats are
                            those of the whole launch */
  char error[256];       /* message of a failed query */
} ar_query_result;

typedef struct {
  int64_t submitted, completed, failed;
  int32_t slots, peak_inflight;
  double p50_ms, p99_ms, mean_ms;   /* latency of the completed queries */
  double busy_s;                    /* host time with at least one query in flight */
  uint64_t hbm_budget, peak_bytes;  /* budget and peak workspace bytes held */
  int64_t pairs;                    /* evaluated (pixel, Gaussian) pairs, all queries */
  int64_t releases;                 /* slot workspaces freed to stay within the budget */
  int64_t shared_launches;          /* launches that rendered more than one query */
  int64_t shared_queries;           /* queries rendered in them */
} ar_server_stats;

/* cfg may be NULL (defaults).  *out receives the handle. */
int ar_server_create(const ar_server_config *cfg, ar_server **out);

/* Waits for every submitted query, then frees the streams and workspaces. */
void ar_server_destroy(ar_server *srv);

/* Registers a scene (not copied; it must outlive the server and not be destroyed while
 * queries on it run).  *scene_id receives its index. */
int ar_server_add_scene(ar_server *srv, const ar_scene *scene, int32_t *scene_id);

/* Queues one query (arguments as ar_render_bounds; the structs are copied, the output
 * device buffers must stay valid until the query completes).  *ticket receives its id.
 * Invalid arguments are rejected here; errors while running are reported by wait. */
int ar_server_submit(ar_server *srv, int32_t scene_id, const ar_intrinsics *intr, const ar_pose_box *box,
                     const ar_options *opts, float *lo_rgb, float *hi_rgb, int64_t *ticket);

/* Result of a query.  block != 0 waits for it; block == 0 returns AR_PENDING in
 * out->status (and as the return value) while it is queued or running.  A finished
 * query's record is released by the first wait that returns it. */
int ar_server_wait(ar_server *srv, int64_t ticket, int32_t block, ar_query_result *out);

/* Latency percentiles and counters over the server's life so far. */
int ar_server_report(ar_server *srv, ar_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* AR_H */
