// Internal types shared by the host plan builder, the C ABI glue and the HIP
// kernels of libctis.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ctis.h"

#ifndef __HIP_PLATFORM_AMD__
#define __HIP_PLATFORM_AMD__
#endif
#include <hip/hip_runtime_api.h>

namespace ctis {

// Tile shape of the back projection and of the tile forward projection: a
// wavefront covers 64 x 16 outputs (fast x slow axis) with a 4 x 4 register
// micro-tile per lane (16 lanes x 4 lanes).
constexpr int kTileFast = 64;
constexpr int kTileSlow = 16;
// Regions of the region forward projection (the EM path): a group of gl
// lanes covers 16 gl FPA pixels, gx x (gl / gx) lanes with a 4 x 4
// micro-tile each, i.e. (4 gx) x (4 gl / gx) pixels along gamma x xi; 64 / gl
// groups per wavefront, each on another box.  Shapes by code (the
// CTIS_PLAN_REGION value): 1 = 8 x 32, 2 = 16 x 16, 3 = 32 x 8 (gl = 16),
// 4 = 16 x 8, 5 = 8 x 16 (gl = 8), 6 = 8 x 8 (gl = 4).  Smaller regions
// follow the edges of the box images more closely (fewer multiply-adds on
// the zero border) at more set-up per output.
constexpr int kRegionPixels = 256;   // the largest region: a partial region slot
constexpr int kRegionShapes = 6;
constexpr int kDefaultRegionShape = 2;
constexpr int kFwdMaxWaves = 8;
constexpr int kMaxBox = 8;
// Work records of windows that run inside the FPA without wrapping carry
// this flag (tile forward: in the f-offset field; back projection: the third
// field is 1): the kernels then take scalar row offsets.
constexpr int kDirectFlag = 1 << 30;
constexpr int region_gx(int shape) { return shape == 3 ? 8 : (shape == 2 || shape == 4) ? 4 : 2; }
constexpr int region_gl(int shape) { return shape <= 3 ? 16 : shape <= 5 ? 8 : 4; }
constexpr int region_fast(int shape) { return 4 * region_gx(shape); }
constexpr int region_slow(int shape) { return 4 * region_gl(shape) / region_gx(shape); }
// Zero border of the padded copy of f the region forward reads, per axis: a
// window of a region (region + B - 1 slots per side) that meets the field
// stop lies inside [-hx, a + hx) x [-hy, alpha + hy).
constexpr int halo_fast(int shape, int B) { return region_fast(shape) + B - 2; }
constexpr int halo_slow(int shape, int B) { return region_slow(shape) + B - 2; }
// 32-bit buffer offsets (in bytes) address the FPA, a wavelength block and
// the whole f buffer (and its padded copy) of a plan or batch
constexpr int64_t kMaxPixels = (int64_t(1) << 29) - 1;

// ---------------------------------------------------------------------------
// Work description of one launch set.  A plan is a batch of one frame; a
// batch (ctis_batch) merges several plans (frames) that share the box side B.
// Every work unit carries its frame's geometry and buffer offsets, so the
// kernels never look up a frame table.
//
// forward unit meta, 3 x int4:
//   (r0, c0, n_chunks, partial slot)   FPA tile origin; a tile whose boxes are
//                                      split over n_chunks > 1 units writes its
//                                      partial tile to that slot
//   (a, alpha, gamma, xi)              frame geometry
//   (g_off, out_off, 0, 0)             frame offsets (floats) into g and out
// forward record, int4: (Xs, Ys, f_off, box): window origin
//   (r0 - (B-1) - rA, c0 - (B-1) - cA), offset of f_s in the f buffer, global
//   box id; box = -1 ends a unit's list.  A window that runs inside the FPA
//   without a carry or wrap is recorded decoded instead: (xr, y0,
//   f_off | kDirectFlag, box) with Xs + gamma*Ys = xr + gamma*y0 mod n
// split meta, 2 x int4: (r0, c0, n_chunks, first slot), (gamma, xi, g_off, out_off)
// adjoint unit meta, 3 x int4:
//   (x0, y0, global wavelength, f_off)  field-stop tile, offset of f_s
//   (a, alpha, gamma, xi)
//   (u_off, 0, 0, 0)                    frame offset into u
// adjoint record, int4: (rA, cA, direct, box), adj_stride records per global
//   wavelength; direct = 1 if the box's windows stay inside the FPA for
//   every field-stop tile
//
// Frames that share a plan share its boxes, wavelengths and values: the
// "global" box and wavelength ids run over the distinct plans of the work, in
// order of first appearance.
//
// Value-gradient tables (the calibration values as variables):
//   entry_slot[t]      global slot (box * B*B + position in the box) of
//                      calibration entry t, entries of the distinct plans back
//                      to back in each plan's input order; -1 if the entry was
//                      dropped (merged to an exact zero)
//   box_lam[b]         global wavelength of global box b
//   lam_box0[l]        first global box of global wavelength l (n_lambda + 1)
//   lam_units[..]      adjoint units of global wavelength l (every frame that
//                      uses it): lam_units[lam_units_ptr[l] .. lam_units_ptr[l+1])
//   slot_entries[..]   entries feeding global slot k (duplicates of one
//                      position): slot_entries[slot_entries_ptr[k] .. [k+1])
struct DevList {
    const int4 *meta = nullptr;
    const int4 *items = nullptr;
    int32_t n_units = 0, stride = 1, waves = 4;
};

struct DevWork {
    int32_t B = 1;
    DevList fwd_full;            // plain projection: every FPA tile once
    DevList fwd_em;              // tile forward for EM: tiles with boxes, heavy tiles split
    const int4 *split_meta = nullptr;
    int32_t n_split = 0;
    // region forward of the EM path (when pad_ok): regions with boxes, heavy
    // regions split; reads the padded copy of f in the workspace
    bool pad_ok = false;
    int32_t region_shape = kDefaultRegionShape;   // region shape code (region_fast x region_slow)
    int32_t halo_x = 0, halo_y = 0;   // zero border of the padded copy
    DevList fwd_pad;
    const int4 *rsplit_meta = nullptr;
    int32_t n_rsplit = 0;
    const int4 *pad_blocks = nullptr;   // per (frame, wavelength): (f_off, fp_off, a, alpha)
    int32_t n_pad_blocks = 0, pad_rows = 0;   // max alpha + 2 halo_y over the blocks
    int32_t f_floats = 0, fp_floats = 0, n_wf = 0;   // extents of f, of its padded copy, of box_wf
    DevList adj;                 // adjoint units; items indexed by global wavelength
    float *box_w = nullptr, *box_wf = nullptr, *h = nullptr;
    size_t partials_off = 0;     // byte offset of the partial tiles in the EM workspace
    size_t rpartials_off = 0;    // byte offset of the partial regions
    size_t fp_off = 0;           // byte offset of the padded copy of f
    size_t diag_off = 0;         // byte offset of the diagnostics partials
    size_t workspace_bytes = 0;  // u region + partial tiles + partial regions + padded f + diagnostics
    bool persistent = false;     // grid-stride workgroups instead of one per unit
    bool region_solo = false;    // region forward with a lane group per unit
    bool adj_direct = false;     // every back-projection box takes the direct window
    // value gradients and value updates
    const int32_t *entry_slot = nullptr, *box_lam = nullptr, *lam_box0 = nullptr;
    const int32_t *lam_units_ptr = nullptr, *lam_units = nullptr;
    const int32_t *slot_entries_ptr = nullptr, *slot_entries = nullptr;
    int64_t n_entries = 0;
    int32_t n_lambda = 0, n_boxes = 0;
    // VJP workspace: the EM workspace (u, partial tiles) followed by
    // e, zeta, b, per-unit flux partials and per-(unit, box) value partials
    size_t e_off = 0, zeta_off = 0, b_off = 0, hpart_off = 0, vg_off = 0, vjp_workspace_bytes = 0;
    // SART workspace: the EM workspace, then R = H 1 (like g) and a vector of
    // ones (like f), over the derivative parts (never used together)
    size_t solve_r_off = 0, solve_ones_off = 0, solve_workspace_bytes = 0;
    void *mem = nullptr;         // device allocation holding the tables
};

struct HostList {
    std::vector<int32_t> meta, items;   // int4 records, flattened
    int32_t n_units = 0, stride = 1, waves = 4;
};

struct HostWork {
    int32_t B = 1;
    HostList fwd_full, fwd_em, fwd_pad, adj;
    std::vector<int32_t> split_meta, rsplit_meta, pad_blocks;
    int32_t n_split = 0, partial_slots = 0, n_rsplit = 0, rpartial_slots = 0;
    bool pad_ok = false;
    int32_t region_shape = kDefaultRegionShape, halo_x = 0, halo_y = 0;
    int64_t fp_floats = 0;       // padded copy of f (all frames)
    int32_t pad_rows = 0;
    std::vector<float> box_w, box_wf, h;
    int64_t u_floats = 0;        // u region of the EM workspace
    int64_t g_floats = 0;        // extent of the g buffer
    bool adj_direct = false;     // every back-projection record is direct
    int64_t f_floats = 0;        // extent of the f buffer
    // value tables (layout as in DevWork)
    std::vector<int32_t> entry_slot, box_lam, lam_box0, lam_units_ptr, lam_units, slot_entries_ptr, slot_entries;
    // distinct plans: per frame its distinct plan, per distinct plan the first
    // global box, wavelength and entry
    std::vector<int32_t> frame_plan, plan_box0, plan_lam0;
    std::vector<int64_t> plan_entry0;
    bool dropped = false;        // some entry of some plan was dropped
};

// Workspace layout of a work description (byte offsets, 256-byte aligned).
struct Layout {
    size_t partials_off, rpartials_off, fp_off, diag_off, em_bytes, e_off, zeta_off, b_off, hpart_off, vg_off,
        vjp_bytes, solve_r_off, solve_ones_off, solve_bytes;
};

// Forward work list over a grid of FPA cells (tf x ts pixels): for every
// cell the boxes whose shifted, dilated field-stop image meets it.
struct WorkGrid {
    int32_t tf = 0, ts = 0;      // cell size along gamma and xi
    int32_t ntr = 0, ntc = 0, n_cells = 0, n_active = 0, max_items = 0;
    int32_t chunk = 64;          // max boxes per forward unit in EM
    std::vector<int32_t> order;  // cells, heaviest first (stable)
    std::vector<int32_t> item_ptr, item_box;   // boxes of cell t: item_box[item_ptr[t] .. item_ptr[t+1])
};
Layout layout_for(const HostWork &hw);

// Per-plan analysis of the calibration (host).
struct HostTables {
    int32_t B = 1;
    std::vector<int32_t> box_rc, box_lambda, lambda_box_ptr;
    std::vector<float> box_w, box_wf, h;
    WorkGrid tiles;              // 64 x 16 FPA tiles (plain projection, tile EM path)
    WorkGrid regions;            // FPA regions of the region EM path
    int32_t region_shape = kDefaultRegionShape;   // their shape code: region_fast x region_slow
    // the region path reads f through a zero-bordered copy; exact when the
    // FPA leaves halo_fast / halo_slow pixels beside the field stop
    bool pad_ok = false;
    int32_t nbx = 0, nby = 0;
    int64_t nnz = 0, n_support = 0;
    int32_t max_boxes = 0;
    bool nonneg = true;
    // calibration entries as given: count, slot of each (global box of the
    // plan * B*B + position in the box; -1 if dropped), any dropped
    int64_t n_in = 0;
    std::vector<int32_t> entry_slot;
    bool dropped = false;
};

}  // namespace ctis

struct ctis_plan {
    int32_t a, alpha, w, gamma, xi;
    int64_t n, ell, m;
    ctis::HostTables ht;
    int32_t device = -1;
    ctis::DevWork work;          // the plan as a batch of one frame
    size_t workspace_bytes = 0, vjp_workspace_bytes = 0, solve_workspace_bytes = 0;
    // ctis_plan_set_values rewrites the device copies of the box values and
    // column sums; the host copies in `ht` are re-read from the device by
    // refresh_host_tables before the next host-side reader uses them
    mutable bool host_stale = false;
};

struct ctis_batch {
    std::vector<const ctis_plan *> plans;
    std::vector<int64_t> f_base, g_base, u_base;   // per frame, in floats
    int64_t f_floats = 0, g_floats = 0;
    int32_t device = -1;
    bool nonneg = true;
    bool dropped = false;
    std::vector<int32_t> frame_plan, plan_box0, plan_lam0;   // distinct plans
    std::vector<int64_t> plan_entry0;
    ctis::DevWork work;
};

namespace ctis {

void set_error(const std::string &msg);
ctis_status fail(ctis_status st, const std::string &msg);

// Bring the host copies of a plan's box values, column sums and sign flag up
// to date after ctis_plan_set_values (synchronises the device once; a no-op
// otherwise).  api.cpp.
ctis_status refresh_host_tables(const ctis_plan *p);

// host plan builder (plan.cpp)
ctis_status build_host_tables(ctis_plan *p, const int64_t *lambda_ptr, const int32_t *fpa_index,
                              const float *value, int forced_box, bool keep_zeros, int region_shape);

// One frame of a work description: its plan and buffer offsets (floats).
struct FrameRef {
    const ctis_plan *plan;
    int64_t f_base, g_base, u_base;
};
ctis_status build_work(const std::vector<FrameRef> &frames, bool with_full, HostWork &hw);
ctis_status upload_work(const HostWork &hw, DevWork &dw);
void free_work(DevWork &dw);

// Scratch-free EM (static_scratch.hip): a file-scope device array of this
// size per device stands in for the workspace.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
int static_scratch(void **ptr);

// stream-ordered EM drivers shared by plans and batches (api.cpp)
ctis_status em_forward_half(const DevWork &w, const float *f, const float *g, void *workspace, void *stream);
ctis_status em_loop(const DevWork &w, const float *g, float *f, int32_t iters, void *workspace, void *stream);
// iters iterations of a solver (CTIS_SOLVER_*) in place; SART needs the
// solve workspace
ctis_status solve_loop(const DevWork &w, int solver, const float *g, float *f, int32_t iters, float relax,
                       void *workspace, void *stream);

// kernel launchers (kernels.hip); return hipError_t as int
int max_waves(int box);         // tile kernels: waves per workgroup
int min_waves();

// Epilogues of the forward projection v = (H x)_i:
enum FwdMode : int {
    kFwdPlain = 0,     // out = v                                  (every FPA tile)
    kFwdRatio = 1,     // out = g / v, 0 where v <= 0              (EM: u)
    kFwdVjp = 2,       // out = -v u^2 / g, 0 where u == 0          (EM derivative: e; aux = u)
    kFwdLogRatio = 3,  // out = log(g / v), 0 where g <= 0 or v <= 0 (SMART)
    kFwdResidual = 4,  // out = (g - v) / R, 0 where R == 0         (SART; aux = R = H 1,
                       //                                            laid out like g)
};
// Epilogues of the back projection v = (H^T r)_j:
enum AdjMode : int {
    kAdjPlain = 0,     // out = v
    kAdjUpdate = 1,    // out = in1 v / h, 0 where h == 0          (EM update)
    kAdjVjpPre = 2,    // out = v (zeta), out2 = in1 in2 / h (b = y f / h),
                       // flux[unit] = sum over the unit's voxels of b v
    kAdjVjpGrad = 3,   // out = in1 in2 / h + v (y zeta / h + H^T e)
    kAdjMulExp = 4,    // out = in1 exp(v / h), 0 where h == 0     (SMART update)
    kAdjAddClamp = 5,  // out = max(0, in1 + relax v / h), 0 where h == 0 (SART update)
};
// the modes that replace f (and its padded copy) by an update
inline constexpr bool adj_updates(int mode) {
    return mode == kAdjUpdate || mode == kAdjMulExp || mode == kAdjAddClamp;
}
int launch_forward(const DevWork &w, const float *x, const float *g, const float *u, float *out, int mode,
                   void *workspace, void *stream);
// Region path (w.pad_ok): launch_pad writes the zero-bordered copy of x into
// the workspace; launch_forward_pad projects that copy (modes as above).
int launch_pad(const DevWork &w, const float *x, void *workspace, void *stream);
int launch_forward_pad(const DevWork &w, const float *g, const float *u, float *out, int mode, void *workspace,
                       void *stream);
// `fpad`: with an update mode, also write the updated f into the padded copy
// at that workspace (nullptr: not); `relax`: kAdjAddClamp's relaxation
int launch_adjoint(const DevWork &w, const float *r, const float *in1, const float *in2, float *out, float *out2,
                   float *flux, int mode, void *stream, void *fpad = nullptr, float relax = 1.0f);
// x[0, n) = v
int launch_fill(float *x, int64_t n, float v, void *stream);
// per-(adjoint unit, box) partial derivatives of the calibration values, then
// their sums per entry into dv (accumulated if `accumulate`)
int launch_value_grad(const DevWork &w, const float *u, const float *e, const float *b, const float *f,
                      float *partial, void *stream);
int launch_value_finish(const DevWork &w, const float *partial, const float *flux, float *dv, int64_t entry0,
                        int64_t n_entries, bool accumulate, void *stream);
// EM diagnostics of one frame into out[4] = (flux, sum g, log-likelihood,
// pixels with g > 0 and ghat <= 0); `part` holds kDiagParts * 4 doubles
constexpr int kDiagParts = 256;
int launch_diagnostics(const float *g, const float *ghat, const float *f, const float *hsum, int64_t n, int64_t m,
                       int64_t ell, double *part, double *out, void *stream);
// box values and column sums of the global wavelengths [lam0, lam1) from
// the entry values `values` (entry `entry0` first)
int launch_set_values(const DevWork &w, const float *values, int64_t entry0, int32_t lam0, int32_t lam1,
                      void *stream);

}  // namespace ctis
