/*
 * ctis.h -- C ABI of the MI355X CTIS EM reconstruction library (libctis.so).
 *
 * The library reconstructs a hyperspectral datacube f from one computed-
 * tomographic-imaging-spectrometer frame g by the expectation-maximisation
 * iteration of White, Bell & Haygood (Sec. 2 eq. (em)):
 *
 *     f <- (f / h) . H^T (g / (H f)),      h_j = sum_i H_ij,
 *
 * where the n x m system matrix H is never stored.  Under the paper's spatial
 * shift-invariance (Sec. 2, calibration paragraph) every column of wavelength
 * block s is the calibration image c_s shifted by the voxel's field-stop
 * position; Sec. 3 writes this as H_s = C_s E (eq. (decomposition)), C_s the
 * n x n circulant with first column c_s and E the zero-padding embedding of
 * the a x alpha field stop into the gamma x xi focal plane array (FPA).
 * The library evaluates H f and H^T r directly as sparse gathers over the
 * nonzeros of each c_s (the paper evaluates them with FFTs; both give the
 * same operator).
 *
 * Conventions shared by every call
 * --------------------------------
 *  Sizes:   n = gamma * xi FPA pixels, ell = a * alpha field-stop pixels,
 *           m = ell * w voxels; n and m below 2^29.
 *  Layout:  the paper's column-major vectorisation (Sec. 2; Sec. 3 index map).
 *           Voxel (x, y, s), x < a, y < alpha, s < w, is f[x + a*y + ell*s]
 *           (a row-major (w, alpha, a) array).  FPA pixel (r, c), r < gamma,
 *           c < xi, is g[r + gamma*c] (a row-major (xi, gamma) array).
 *  Shift:   the shift of Sec. 3 is cyclic over the whole vectorised FPA of
 *           length n (an n x n circulant), so a shifted image that runs past
 *           the last FPA row continues at row 0 of the next FPA column, and
 *           past the last pixel at pixel 0.  The library reproduces this
 *           exactly; calibration layouts that never reach an FPA edge are the
 *           same computation.
 *  Numbers: float32 storage, float32 arithmetic and accumulation.
 *  Memory:  f, g, r, z and the workspace are DEVICE pointers on the plan's
 *           HIP device, contiguous, 4-byte aligned, owned by the caller, and
 *           must stay valid until the work queued on `stream` completes.
 *           Inputs and outputs must not overlap (except f in ctis_em_iterate,
 *           which is updated in place).  Inputs must be finite.
 *  Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *           Calls queue work and return; HIP faults surface at the caller's
 *           next synchronisation.  A plan is immutable after creation: calls
 *           on different streams may share it when their outputs and
 *           workspaces differ.
 *  Errors:  every call returns a ctis_status; none aborts or prints.
 *           ctis_last_error() gives a description of the last failure on the
 *           calling thread.
 */
#ifndef CTIS_H
#define CTIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CTIS_OK = 0,
    CTIS_E_ARG = 1,         /* null pointer, bad size or flag, wrong device   */
    CTIS_E_INDEX = 2,       /* calibration index outside [0, n)               */
    CTIS_E_VALUE = 3,       /* non-finite calibration value                   */
    CTIS_E_TOO_LARGE = 4,   /* n, ell, m or a table size beyond the limits    */
    CTIS_E_NOMEM = 5,       /* host or device allocation failed               */
    CTIS_E_HIP = 6,         /* a HIP runtime call or kernel launch failed     */
    CTIS_E_NEGATIVE = 7,    /* EM needs nonnegative calibration values        */
    CTIS_E_WORKSPACE = 8    /* workspace pointer null or too small            */
} ctis_status;

typedef struct ctis_plan ctis_plan;
typedef struct ctis_batch ctis_batch;

/* ctis_plan_create flags */
#define CTIS_PLAN_HOST_ONLY 0x1u        /* build the tables on the host only (no
                                           device memory); for inspection --
                                           compute calls on it return CTIS_E_ARG */
#define CTIS_PLAN_BOX(b) (((uint32_t)(b) & 0xFu) << 8)
                                        /* force the calibration box side B in
                                           1..8 (0 = chosen by the plan)         */
#define CTIS_PLAN_TILE_PATH 0x4u        /* EM on the tile path even where the
                                           region path applies (comparisons) */
#define CTIS_PLAN_REGION(k) (((uint32_t)(k) & 0x7u) << 12)
                                        /* region shape of the region path
                                           (pixels along gamma x xi): 1 = 8 x
                                           32, 2 = 16 x 16, 3 = 32 x 8, 4 =
                                           16 x 8, 5 = 8 x 16, 6 = 8 x 8, 0 =
                                           chosen by the plan (16 x 16); 7 is
                                           refused with CTIS_E_ARG            */
#define CTIS_PLAN_KEEP_ZEROS 0x2u       /* the structure is the set of given
                                           positions, whatever their values:
                                           entries that merge to an exact zero
                                           are kept (as zero-valued box slots)
                                           instead of dropped.  Needed for the
                                           value derivatives of ctis_em_vjp and
                                           for ctis_plan_set_values when some
                                           value may be zero                    */

typedef struct {
    int32_t a, alpha, w, gamma, xi;
    int64_t n, ell, m;
    int64_t nnz;             /* calibration nonzeros after merging duplicates
                                and dropping exact zeros                        */
    int64_t n_support;       /* FPA pixels whose row of H is not empty          */
    int32_t box;             /* side B of the dense boxes the nonzeros are
                                grouped into                                    */
    int32_t n_boxes;
    int32_t tile_fast, tile_slow;   /* FPA / field-stop tile (pixels)           */
    int32_t n_tiles;         /* FPA tiles                                       */
    int32_t n_active_tiles;  /* FPA tiles that meet the image of some box       */
    int64_t n_items;         /* (FPA tile, box) pairs of the forward work list  */
    size_t workspace_bytes;  /* device workspace ctis_em_iterate needs          */
    int32_t nonnegative;     /* 1 if every calibration value is >= 0            */
    int32_t device;          /* HIP device of the plan, -1 if host-only         */
    int32_t waves_forward;   /* wavefronts per forward workgroup                */
    int32_t waves_adjoint;   /* wavefronts per adjoint workgroup                */
    int64_t n_entries;       /* calibration entries as given (lambda_ptr[w])    */
    size_t vjp_workspace_bytes;  /* device workspace ctis_em_vjp needs (also
                                    enough for ctis_em_iterate)                 */
    int32_t dropped;         /* 1 if some entry merged to an exact zero and was
                                dropped (never with CTIS_PLAN_KEEP_ZEROS)       */
    /* The EM path's forward projection.  Region path: FPA regions of 64,
     * 128 or 256 pixels (region_fast x region_slow; CTIS_PLAN_REGION), 16,
     * 8 or 4 boxes per wavefront at a time (a lane group per box),
     * windows read from a zero-bordered copy of f; taken when the FPA leaves
     * region_fast + B - 2 pixels beside the field stop along gamma and
     * region_slow + B - 2 along xi (and CTIS_PLAN_TILE_PATH is not set).
     * Otherwise, and for ctis_forward, the tile path (tile_fast x tile_slow
     * FPA tiles).                                                           */
    int32_t region_fast, region_slow;   /* FPA region (pixels)                  */
    int32_t n_regions, n_active_regions;
    int64_t n_region_items;  /* (FPA region, box) pairs                         */
    int32_t em_region_path;  /* 1 if ctis_em_iterate takes the region path      */
    int32_t waves_region;    /* wavefronts per region-forward workgroup         */
    /* Multiply-adds of one projection: the method's own (every calibration
     * nonzero against every voxel of its wavelength, ell * nnz), and the ones
     * the kernels execute (every slot of a B x B box against every output of a
     * work item, overhang of the item past the box's image included).      */
    int64_t method_madds;
    int64_t tile_forward_madds;
    int64_t region_forward_madds;
    int64_t adjoint_madds;
    size_t solve_workspace_bytes;  /* workspace of ctis_solve_iterate with SART
                                      (EM and SMART need workspace_bytes)      */
} ctis_plan_info;

/*
 * Create a plan: the calibration images and geometry, validated, grouped and
 * uploaded to the current HIP device.
 *
 *   a, alpha      field stop (Sec. 2: a x alpha), 1 <= a <= gamma, 1 <= alpha <= xi
 *   w             number of wavelengths (calibration images), >= 1
 *   gamma, xi     FPA size (Sec. 2: gamma x xi)
 *   lambda_ptr    HOST int64[w+1]: entries of wavelength s are
 *                 [lambda_ptr[s], lambda_ptr[s+1]); lambda_ptr[0] = 0,
 *                 non-decreasing
 *   fpa_index     HOST int32[lambda_ptr[w]]: FPA index r + gamma*c of the
 *                 entry in the calibration image of field-stop pixel (0, 0)
 *                 (the first column c_s of H_s, Sec. 3)
 *   value         HOST float[lambda_ptr[w]]: its value; duplicates add up,
 *                 exact zeros are dropped; any sign is accepted, but
 *                 ctis_em_iterate needs all values >= 0
 *   flags         CTIS_PLAN_* bits
 *
 * The caller may free its arrays when the call returns.  Errors:
 * CTIS_E_ARG (sizes, pointers, lambda_ptr, flags), CTIS_E_INDEX, CTIS_E_VALUE,
 * CTIS_E_TOO_LARGE, CTIS_E_NOMEM, CTIS_E_HIP.  *out is NULL on failure.
 */
ctis_status ctis_plan_create(ctis_plan **out, int32_t a, int32_t alpha, int32_t w,
                             int32_t gamma, int32_t xi, const int64_t *lambda_ptr,
                             const int32_t *fpa_index, const float *value,
                             uint32_t flags);

/* Free a plan and its device tables (after the work using it has completed).
 * NULL is accepted. */
void ctis_plan_destroy(ctis_plan *plan);

/* Sizes and layout decisions of a plan (see ctis_plan_info). */
ctis_status ctis_plan_get_info(const ctis_plan *plan, ctis_plan_info *info);

/* HOST float[w]: the column sums h_j = sum_i H_ij (Sec. 2, below eq. (em)),
 * which are equal within a wavelength block (column sums of a circulant):
 * h for every voxel of wavelength s is the sum of the values of c_s. */
ctis_status ctis_plan_lambda_sums(const ctis_plan *plan, float *h_out);

/*
 * Inspection of the plan's grouping (host copies).  Boxes: box k belongs to
 * wavelength box_lambda[k]; its B x B values sit at FPA positions
 * (box_rc[2k] + dr, box_rc[2k+1] + dc), value box_values[k*B*B + dc*B + dr].
 * Work list: FPA tile t (fast index t % ceil(gamma/tile_fast)) lists the boxes
 * item_box[tile_ptr[t] .. tile_ptr[t+1]) whose shifted field-stop image meets
 * it.  Array sizes come from ctis_plan_info (n_boxes, n_tiles, n_items).
 * Any output pointer may be NULL to skip it.
 */
ctis_status ctis_plan_export_boxes(const ctis_plan *plan, int32_t *box_lambda,
                                   int32_t *box_rc, float *box_values);
ctis_status ctis_plan_export_worklist(const ctis_plan *plan, int32_t *tile_ptr,
                                      int32_t *item_box);
/* The same for the region path's grid (region_fast x region_slow regions,
 * fast index t % ceil(gamma/region_fast); sizes n_regions, n_region_items). */
ctis_status ctis_plan_export_regions(const ctis_plan *plan, int32_t *region_ptr,
                                     int32_t *item_box);

/*
 * Forward projection g_out = H f (Sec. 2 eq. (linear); Sec. 3 eq. (vs_linear):
 * g = sum_s C_s E f_s).
 *   f      DEVICE float[m], read
 *   g_out  DEVICE float[n], written everywhere (0 where no voxel projects)
 */
ctis_status ctis_forward(const ctis_plan *plan, const float *f, float *g_out, void *stream);

/*
 * Back projection z_out = H^T r (Sec. 3 eq. (Htu): the transposed circulants
 * followed by the transposed index map).
 *   r      DEVICE float[n], read (every pixel any voxel projects to, and the
 *          zero-valued padding around the calibration nonzeros, must be finite)
 *   z_out  DEVICE float[m], written
 */
ctis_status ctis_adjoint(const ctis_plan *plan, const float *r, float *z_out, void *stream);

/*
 * iters EM iterations in place (Sec. 2 eq. (em); the per-iteration steps of
 * the paper's Sec. 3 algorithm: g_k = H f, u = g / g_k, zeta = H^T u,
 * f = (f . zeta) / h), fused into two kernels per iteration:
 *   forward + ratio:  u_i = g_i / (H f)_i, or 0 where (H f)_i <= 0;
 *   adjoint + update: f_j = f_j * (H^T u)_j / h_j, or 0 where h_j == 0.
 *
 *   g          DEVICE float[n], the measured frame, >= 0 (not checked)
 *   f          DEVICE float[m], in: start (the paper starts from all ones),
 *              out: f after `iters` updates; iters = 0 leaves f unchanged
 *   workspace  DEVICE, >= info.workspace_bytes, 256-byte aligned; its
 *              contents are scratch (u; the partial sums of FPA tiles or
 *              regions whose boxes are split over several workgroups; on
 *              the region path (info.em_region_path) a zero-bordered copy of
 *              f, written at the start and kept current by the update)
 * Errors: CTIS_E_NEGATIVE if a calibration value is negative, CTIS_E_WORKSPACE,
 * CTIS_E_ARG, CTIS_E_HIP.
 */
ctis_status ctis_em_iterate(const ctis_plan *plan, const float *g, float *f, int32_t iters,
                            void *workspace, size_t workspace_bytes, void *stream);

/*
 * Other solvers on the same projections (Sec. 2 names MART and ART beside
 * EM and cites them to Gordon, Bender and Herman; Sec. 3 notes that the
 * decomposition does not depend on the solver).  The cited methods correct
 * one ray (one row of H) at a time; these are their simultaneous forms, in
 * which every voxel takes the H-weighted mean of the corrections of the rays
 * through it, one forward and one back projection per iteration:
 *   CTIS_SOLVER_SMART: f'_j = f_j exp((H^T l)_j / h_j),
 *       l_i = log(g_i / (H f)_i), 0 where g_i <= 0 or (H f)_i <= 0;
 *   CTIS_SOLVER_SART:  f'_j = max(0, f_j + relax (H^T r)_j / h_j),
 *       r_i = (g_i - (H f)_i) / R_i, R = H 1 (0 where R_i == 0),
 *       relax in (0, 2);
 *   CTIS_SOLVER_EM:    ctis_em_iterate (relax unused);
 * f'_j = 0 where h_j == 0.  iters iterations in place on f (DEVICE, the
 * start vector in, the result out); g DEVICE; workspace DEVICE, 256-byte
 * aligned, at least info.solve_workspace_bytes for SART and
 * info.workspace_bytes otherwise; f, g and the workspace must not overlap.
 * Errors: CTIS_E_ARG (unknown solver, relax outside (0, 2) for SART, NULL,
 * misaligned or overlapping buffers, iters < 0), CTIS_E_NEGATIVE (EM or
 * SMART with a negative calibration value; SART accepts any sign),
 * CTIS_E_WORKSPACE, CTIS_E_HIP.
 */
typedef enum { CTIS_SOLVER_EM = 0, CTIS_SOLVER_SMART = 1, CTIS_SOLVER_SART = 2 } ctis_solver;
ctis_status ctis_solve_iterate(const ctis_plan *plan, int32_t solver, const float *g, float *f, int32_t iters,
                               float relax, void *workspace, size_t workspace_bytes, void *stream);

/*
 * ctis_em_iterate without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The library keeps one file-scope device
 * array of 16 MiB per device (held until the process ends) and uses it as
 * the workspace; the call allocates nothing.  Same arguments, results and
 * kernels as ctis_em_iterate.  Every call on a device shares that device's
 * array: calls that overlap on one device (different streams, or several
 * host threads) race and must be serialised by the caller.
 * Errors: CTIS_E_TOO_LARGE if info.workspace_bytes exceeds 16 MiB, and those
 * of ctis_em_iterate (no CTIS_E_WORKSPACE).
 */
ctis_status ctis_em_iterate_static(const ctis_plan *plan, const float *g, float *f, int32_t iters,
                                   void *stream);

/*
 * Diagnostics of an EM iterate (Sec. 2: the column sums h below eq. (em); the
 * Poisson likelihood the EM iteration increases, after Shepp and Vardi), in
 * double precision:
 *   out[0] = sum_j h_j f_j               (flux; equals the sum of g over the
 *                                         pixels with (H f_prev)_i > 0 after
 *                                         an EM update)
 *   out[1] = sum_i g_i
 *   out[2] = sum_i (g_i log (H f)_i - (H f)_i), a g_i = 0 term contributing
 *            -(H f)_i; -HUGE_VAL if some g_i > 0 has (H f)_i <= 0
 *   out[3] = the number of such pixels
 *   g          DEVICE float[n];  f  DEVICE float[m]
 *   out        DEVICE double[4], 8-byte aligned, written
 *   workspace  DEVICE, >= info.workspace_bytes, 256-byte aligned (scratch:
 *              H f and the per-workgroup partial sums)
 * Two reduction passes in a fixed order: the result does not depend on
 * timing.  Errors: CTIS_E_ARG, CTIS_E_WORKSPACE, CTIS_E_HIP.
 */
ctis_status ctis_em_diagnostics(const ctis_plan *plan, const float *g, const float *f, double *out,
                                void *workspace, size_t workspace_bytes, void *stream);

/*
 * The two halves of one EM iteration, for callers that schedule the
 * iteration themselves.  ctis_em_iterate is `iters` pairs of these two calls
 * on one workspace (>= info.workspace_bytes, 256-byte aligned), apart from
 * writing the padded copy of f once instead of in every forward half.
 *
 *   ctis_em_forward_ratio:  u_i = g_i / (H f)_i, or 0 where (H f)_i <= 0, into
 *       the first n floats of the workspace, for every pixel of an FPA tile
 *       or region that meets the image of some calibration nonzero (the back
 *       projection reads no other pixel).  f DEVICE float[m], g DEVICE
 *       float[n].  On the region path this is two kernels: the zero-bordered
 *       copy of f into the workspace, then the projection.
 *   ctis_em_adjoint_update: f_out_j = f_in_j * (H^T u)_j / h_j, or 0 where
 *       h_j == 0, with u as left in the workspace by ctis_em_forward_ratio;
 *       on the region path it also writes f_out into the workspace's padded
 *       copy.  f_out may equal f_in (in place) but must not overlap it
 *       otherwise.
 * Errors: CTIS_E_NEGATIVE if a calibration value is negative, CTIS_E_WORKSPACE,
 * CTIS_E_ARG, CTIS_E_HIP.  Calls sharing one workspace must be ordered on one
 * stream.
 */
ctis_status ctis_em_forward_ratio(const ctis_plan *plan, const float *f, const float *g, void *workspace,
                                  size_t workspace_bytes, void *stream);
ctis_status ctis_em_adjoint_update(const ctis_plan *plan, void *workspace, size_t workspace_bytes,
                                   const float *f_in, float *f_out, void *stream);


/*
 * Batches: many frames, each with its own plan (geometry and calibration,
 * uneven sizes allowed), reconstructed together -- each EM iteration is one
 * forward+ratio launch and one adjoint+update launch for all frames, whose
 * workgroups walk one work list that holds the units of every frame.  No
 * host synchronisation, memset or allocation happens inside the calls, so a
 * caller may capture them in a HIP graph.
 *
 * Layout: frame k's datacube occupies f_all[f_offset_k, f_offset_k + m_k) and
 * its FPA image g_all[g_offset_k, g_offset_k + n_k), frames back to back in
 * order: f_offset_k = sum_{j<k} m_j, g_offset_k = sum_{j<k} n_j (each block in
 * the layout of the single-frame calls).  plans[k] may repeat (frames sharing
 * one calibration).  All plans need the same box side B (ctis_plan_info.box;
 * CTIS_PLAN_BOX forces it) and the batch's device.  The batch keeps pointers
 * to the plans, which must outlive it.
 */
#define CTIS_BATCH_WAVES_FORWARD(n) (((uint32_t)(n) & 0x1Fu) << 0)   /* 0 = chosen */
#define CTIS_BATCH_WAVES_ADJOINT(n) (((uint32_t)(n) & 0x1Fu) << 5)   /* 0 = chosen */
#define CTIS_BATCH_PERSISTENT 0x400u   /* launch only as many workgroups as fit on the chip
                                          at once, each walking the work list; default:
                                          one workgroup per work unit                    */
#define CTIS_BATCH_WAVES_REGION(n) (((uint32_t)(n) & 0xFu) << 11)  /* region forward, 0 = chosen */
#define CTIS_BATCH_TILE_PATH 0x8000u   /* EM on the tile path even where the region path applies */
#define CTIS_BATCH_REGION_SOLO 0x10000u /* region forward with a lane group per region walking
                                           all of its boxes (4, 8 or 16 regions per wavefront
                                           by region size), for batches of many short regions;
                                           the region waves setting is then unused           */

typedef struct {
    int32_t n_frames;
    int32_t box;
    int64_t m_total, n_total;      /* sizes of f_all and g_all (floats)          */
    int64_t forward_units, adjoint_units;
    int32_t waves_forward, waves_adjoint;
    size_t workspace_bytes;        /* EM workspace of ctis_batch_em_iterate      */
    int32_t n_plans;               /* distinct plans (frames may share one)      */
    int64_t n_entries;             /* calibration entries of the distinct plans  */
    size_t vjp_workspace_bytes;    /* workspace of ctis_batch_em_vjp             */
    int32_t em_region_path;        /* 1 if EM takes the region path (every plan
                                      allows it, all with one region shape,
                                      CTIS_BATCH_TILE_PATH not set)             */
    int32_t waves_region;
    int64_t region_units;
    size_t solve_workspace_bytes;  /* workspace of ctis_batch_solve_iterate with
                                      SART                                     */
} ctis_batch_info;

/* Create a batch over n_frames >= 1 frames.  flags: CTIS_BATCH_WAVES_FORWARD /
 * _ADJOINT (waves per workgroup of the tile kernels, 4..16 for B <= 5 and
 * 4..8 above, 1 for a wave per unit that walks all the unit's boxes, or 0 for
 * the built-in choice), CTIS_BATCH_WAVES_REGION (region
 * forward, 1..8 or 0), CTIS_BATCH_PERSISTENT, CTIS_BATCH_TILE_PATH,
 * CTIS_BATCH_REGION_SOLO.  Errors:
 * CTIS_E_ARG (different B, host-only or other-device plan, bad flags),
 * CTIS_E_TOO_LARGE (f_all of 2^29 floats or more, g_all of 2^31 or more),
 * CTIS_E_NOMEM, CTIS_E_HIP. */
ctis_status ctis_batch_create(ctis_batch **out, const ctis_plan *const *plans, int32_t n_frames, uint32_t flags);
void ctis_batch_destroy(ctis_batch *batch);
ctis_status ctis_batch_get_info(const ctis_batch *batch, ctis_batch_info *info);

/* g_all = H f_all frame by frame (DEVICE, layouts above). */
ctis_status ctis_batch_forward(const ctis_batch *batch, const float *f_all, float *g_all, void *stream);
/* z_all = H^T r_all frame by frame. */
ctis_status ctis_batch_adjoint(const ctis_batch *batch, const float *r_all, float *z_all, void *stream);
/* iters EM iterations of every frame, in place on f_all, with one workspace
 * (>= info.workspace_bytes, 256-byte aligned).  Same semantics per frame as
 * ctis_em_iterate; CTIS_E_NEGATIVE if any plan has a negative value. */
ctis_status ctis_batch_em_iterate(const ctis_batch *batch, const float *g_all, float *f_all, int32_t iters,
                                  void *workspace, size_t workspace_bytes, void *stream);
/* The two halves of one EM iteration of every frame, as ctis_em_forward_ratio
 * and ctis_em_adjoint_update for one frame (same semantics per frame, same
 * argument checks, same workspace as ctis_batch_em_iterate): the forward half
 * leaves u = g / (H f) of every frame at the start of the workspace (frame
 * k's block at g_offset_k) and, on the region path, refreshes the padded copy
 * of f_all that it reads; the update half reads u and writes f_out (f_in ==
 * f_out allowed).  In sequence they give ctis_batch_em_iterate's result bit
 * for bit. */
ctis_status ctis_batch_em_forward_ratio(const ctis_batch *batch, const float *f_all, const float *g_all,
                                        void *workspace, size_t workspace_bytes, void *stream);
ctis_status ctis_batch_em_adjoint_update(const ctis_batch *batch, void *workspace, size_t workspace_bytes,
                                         const float *f_in, float *f_out, void *stream);
/* ctis_solve_iterate for every frame of the batch at once (workspace at
 * least info.solve_workspace_bytes for SART, info.workspace_bytes
 * otherwise; CTIS_E_NEGATIVE if a plan of the batch has a negative value and
 * the solver is EM or SMART). */
ctis_status ctis_batch_solve_iterate(const ctis_batch *batch, int32_t solver, const float *g_all, float *f_all,
                                     int32_t iters, float relax, void *workspace, size_t workspace_bytes,
                                     void *stream);

/*
 * Derivatives of EM (reverse mode), for losses of f after K unrolled
 * iterations: each call differentiates ONE iteration (Sec. 2 eq. (em)), so a
 * caller keeps the iterates f^(1..K) (one checkpoint per iteration) and calls
 * ctis_em_vjp for k = K..1, feeding each call's df_out back as the next y.
 *
 * With f' = (f . zeta) / h, zeta = H^T u, u = g / H f (the step of
 * ctis_em_iterate, with its two zero rules) and the upstream gradient
 * y = dL/df', one call computes (in four projections and two reductions):
 *   b = y f / h,  e = -(H b) u / (H f)   (0 where u = 0 or h = 0),
 *   df_out = dL/df = y zeta / h + H^T e,
 *   dL/dv_t = sum over the voxels j of entry t's wavelength s of
 *             [u_i b_j + e_i f_j]  at  i = (p_t + q_j) mod n
 *             - sum_{j in s} y_j f'_j / h_s,
 * where p_t is entry t's FPA position and q_j the Sec. 3 shift of voxel j
 * (H_ij = c_s[(i - q_j) mod n], h_s = sum of c_s).  Entries that share a
 * position get the same derivative.
 *
 *   g          DEVICE float[n], the measured frame (as for EM)
 *   f          DEVICE float[m], the iteration's input f^(k)
 *   y          DEVICE float[m], dL/df^(k+1)
 *   df_out     DEVICE float[m], dL/df^(k); may equal y (in place), must not
 *              overlap f, g or the workspace otherwise
 *   dvalues    DEVICE float[n_entries] or NULL: dL/dv per calibration entry in
 *              the plan's input order; added to the array's contents if
 *              `accumulate` is nonzero, else overwritten
 *   workspace  DEVICE, >= info.vjp_workspace_bytes, 256-byte aligned; scratch
 * Errors: CTIS_E_ARG (also for dvalues on a plan that dropped an entry: create
 * it with CTIS_PLAN_KEEP_ZEROS), CTIS_E_NEGATIVE, CTIS_E_WORKSPACE, CTIS_E_HIP.
 * The launches are stream-ordered; nothing is allocated or synchronised.
 */
ctis_status ctis_em_vjp(const ctis_plan *plan, const float *g, const float *f, const float *y, float *df_out,
                        float *dvalues, int32_t accumulate, void *workspace, size_t workspace_bytes,
                        void *stream);

/*
 * New calibration values on the plan's structure (Sec. 2 calibration images;
 * same positions, same box grouping): values DEVICE float[n_entries] in the
 * plan's input order, duplicates of a position summed (in double) as at
 * creation.  Rewrites the plan's box values and column sums h on `stream`;
 * later calls on the stream see them.  The host-side readers of the values
 * (ctis_plan_get_info, ctis_plan_lambda_sums, ctis_plan_export_boxes,
 * ctis_batch_create, ctis_fourier_create) synchronise the device once after a
 * set_values, re-read the values and the sign flag from the device, and then
 * see the new values.  Until such a read, the sign check of EM keeps the sign
 * of the values last read: negative values set here are the caller's
 * contract violation.  Errors: CTIS_E_ARG (also if the plan dropped an entry:
 * use CTIS_PLAN_KEEP_ZEROS), CTIS_E_HIP.  Batches hold their own copy of their
 * plans' values, taken at ctis_batch_create (see ctis_batch_set_values).
 */
ctis_status ctis_plan_set_values(ctis_plan *plan, const float *values, void *stream);

/*
 * Batch forms.  Frames that share a plan share its values: dvalues and the
 * values of ctis_batch_set_values hold the entries of the batch's distinct
 * plans back to back, in order of first appearance in the plans array (see
 * ctis_batch_plan_entries), and the derivative of a shared value sums over
 * the frames that use it.  Layouts of g_all, f_all, y_all and df_all as for
 * ctis_batch_em_iterate.
 */
ctis_status ctis_batch_em_vjp(const ctis_batch *batch, const float *g_all, const float *f_all,
                              const float *y_all, float *df_all, float *dvalues, int32_t accumulate,
                              void *workspace, size_t workspace_bytes, void *stream);
/* New values for the plan of frame `frame` (and every frame sharing it), in
 * the batch's copy: values DEVICE float[that plan's n_entries]. */
ctis_status ctis_batch_set_values(ctis_batch *batch, int32_t frame, const float *values, void *stream);
/* Where the entries of frame `frame`'s plan sit in the batch's value arrays:
 * [*offset, *offset + *count). */
ctis_status ctis_batch_plan_entries(const ctis_batch *batch, int32_t frame, int64_t *offset, int64_t *count);

/*
 * The Fourier (WBH) form of the projections, for calibrations dense enough
 * that the FFT beats the gather over nonzeros (Sec. 3: the circulant blocks
 * C_s are diagonalised by the length-n DFT over the vectorised FPA, eqs.
 * (forward) and (backwards); Sec. 3 algorithm for the stage order of EM).
 * Needs n = gamma*xi a power of two in 2^4..2^20.  Two wavelengths share one
 * complex length-n FFT; each EM iteration is w/2 + 1 forward and w/2 + 1
 * inverse complex FFTs (the work of 2w + 2 real FFTs).  Results equal those
 * of the gather path up to FFT rounding.
 *
 * ctis_fourier_create computes the spectra e_t = F(c_{2t} - i c_{2t+1}) of the
 * plan's calibration on the current device (it synchronises the device before
 * returning) and keeps a pointer to the plan, which must outlive it.  The
 * spectra and the sums h_s are those of the plan's values at creation
 * (including values set by ctis_plan_set_values before it): after a later
 * ctis_plan_set_values, create the Fourier plan again.  The
 * spectra take info.spectra_bytes of device memory; the calls take a
 * workspace of info.workspace_bytes (256-byte aligned).  Layouts of f, g, r, z
 * as for the gather path.  Errors: CTIS_E_ARG (n not a power of two in range,
 * host-only plan, other device), CTIS_E_NOMEM, CTIS_E_HIP, CTIS_E_WORKSPACE,
 * CTIS_E_NEGATIVE (EM with a negative value).
 */
typedef struct ctis_fourier ctis_fourier;

typedef struct {
    int64_t n;                 /* FFT length (gamma*xi)                          */
    int32_t n1, n2;            /* four-step factors, n = n1*n2                   */
    int32_t pairs;             /* wavelength pairs, ceil(w/2)                    */
    size_t spectra_bytes;      /* device memory held by the Fourier plan        */
    size_t workspace_bytes;    /* workspace of the projection and EM calls      */
} ctis_fourier_info;

ctis_status ctis_fourier_create(ctis_fourier **out, const ctis_plan *plan);
void ctis_fourier_destroy(ctis_fourier *fourier);
ctis_status ctis_fourier_get_info(const ctis_fourier *fourier, ctis_fourier_info *info);
/* g_out = H f (DEVICE, n floats). */
ctis_status ctis_fourier_forward(const ctis_fourier *fourier, const float *f, float *g_out, void *workspace,
                                 size_t workspace_bytes, void *stream);
/* z_out = H^T r (DEVICE, m floats). */
ctis_status ctis_fourier_adjoint(const ctis_fourier *fourier, const float *r, float *z_out, void *workspace,
                                 size_t workspace_bytes, void *stream);
/* iters EM iterations in place on f (same rules as ctis_em_iterate). */
ctis_status ctis_fourier_em_iterate(const ctis_fourier *fourier, const float *g, float *f, int32_t iters,
                                    void *workspace, size_t workspace_bytes, void *stream);

/* Static description of a status code. */
const char *ctis_status_str(ctis_status status);

/* Description of the last failure on the calling thread ("" if none). */
const char *ctis_last_error(void);

/* Library version, "major.minor.patch". */
const char *ctis_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CTIS_H */
