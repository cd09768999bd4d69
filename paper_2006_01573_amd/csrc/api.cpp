// C ABI of libctis: argument checking, plan lifetime and the stream-ordered
// drivers.  The arithmetic is in kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctis_internal.h"

namespace ctis {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

ctis_status fail(ctis_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

namespace {

ctis_status check_device(const ctis_plan *p) {
    if (p->device < 0) return fail(CTIS_E_ARG, "plan was created host-only");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CTIS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev != p->device)
        return fail(CTIS_E_ARG, "current HIP device " + std::to_string(dev) + " differs from the plan's device " +
                                    std::to_string(p->device));
    return CTIS_OK;
}

bool aligned4(const void *ptr) { return ((uintptr_t)ptr & 3u) == 0; }

bool overlaps(const void *x, size_t xb, const void *y, size_t yb) {
    const char *a = (const char *)x, *b = (const char *)y;
    return a < b + yb && b < a + xb;
}

ctis_status launch_status(int err, const char *what) {
    if (err != 0)
        return fail(CTIS_E_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)err));
    return CTIS_OK;
}

}  // namespace

// The first half of an EM iteration, u = g / (H f) into the workspace: on the
// region path the zero-bordered copy of f is written first.
ctis_status em_forward_half(const DevWork &w, const float *f, const float *g, void *workspace, void *stream) {
    if (w.pad_ok) {
        ctis_status st = launch_status(launch_pad(w, f, workspace, stream), "pad launch");
        if (st != CTIS_OK) return st;
        return launch_status(launch_forward_pad(w, g, nullptr, (float *)workspace, kFwdRatio, workspace, stream),
                             "forward+ratio launch");
    }
    return launch_status(launch_forward(w, f, g, nullptr, (float *)workspace, kFwdRatio, workspace, stream),
                         "forward+ratio launch");
}

// iters EM iterations in place.  Region path: the padded copy of f is
// written once, then kept current by the update epilogue.
ctis_status em_loop(const DevWork &w, const float *g, float *f, int32_t iters, void *workspace, void *stream) {
    float *u = (float *)workspace;
    ctis_status st = CTIS_OK;
    if (w.pad_ok && iters > 0) {
        st = launch_status(launch_pad(w, f, workspace, stream), "pad launch");
        if (st != CTIS_OK) return st;
    }
    for (int32_t k = 0; k < iters; ++k) {
        if (w.pad_ok)
            st = launch_status(launch_forward_pad(w, g, nullptr, u, kFwdRatio, workspace, stream), "forward+ratio launch");
        else
            st = launch_status(launch_forward(w, f, g, nullptr, u, kFwdRatio, workspace, stream), "forward+ratio launch");
        if (st != CTIS_OK) return st;
        st = launch_status(launch_adjoint(w, u, f, nullptr, f, nullptr, nullptr, kAdjUpdate, stream, workspace),
                           "adjoint+update launch");
        if (st != CTIS_OK) return st;
    }
    return CTIS_OK;
}

// Iterations of SMART or SART in place (EM: em_loop), the operation order of
// EM's loop with other epilogues: forward with the log-ratio (SMART) or the
// residual over R = H 1 (SART, R formed first from a vector of ones), then
// the back projection with the multiplicative or the additive, clamped
// update, which also keeps the padded copy of f current on the region path.
ctis_status solve_loop(const DevWork &w, int solver, const float *g, float *f, int32_t iters, float relax,
                       void *workspace, void *stream) {
    if (solver == CTIS_SOLVER_EM) return em_loop(w, g, f, iters, workspace, stream);
    if (iters <= 0) return CTIS_OK;
    float *u = (float *)workspace;
    const float *R = nullptr;
    ctis_status st = CTIS_OK;
    if (solver == CTIS_SOLVER_SART) {
        float *Rw = (float *)((char *)workspace + w.solve_r_off);
        float *ones = (float *)((char *)workspace + w.solve_ones_off);
        st = launch_status(launch_fill(ones, w.f_floats, 1.0f, stream), "fill launch");
        if (st != CTIS_OK) return st;
        st = launch_status(launch_forward(w, ones, nullptr, nullptr, Rw, kFwdPlain, nullptr, stream),
                           "row-sum projection launch");
        if (st != CTIS_OK) return st;
        R = Rw;
    }
    const int fmode = solver == CTIS_SOLVER_SMART ? kFwdLogRatio : kFwdResidual;
    const int amode = solver == CTIS_SOLVER_SMART ? kAdjMulExp : kAdjAddClamp;
    if (w.pad_ok) {
        st = launch_status(launch_pad(w, f, workspace, stream), "pad launch");
        if (st != CTIS_OK) return st;
    }
    for (int32_t k = 0; k < iters; ++k) {
        if (w.pad_ok)
            st = launch_status(launch_forward_pad(w, g, R, u, fmode, workspace, stream), "forward launch");
        else
            st = launch_status(launch_forward(w, f, g, R, u, fmode, workspace, stream), "forward launch");
        if (st != CTIS_OK) return st;
        st = launch_status(launch_adjoint(w, u, f, nullptr, f, nullptr, nullptr, amode, stream, workspace, relax),
                           "adjoint+update launch");
        if (st != CTIS_OK) return st;
    }
    return CTIS_OK;
}

ctis_status refresh_host_tables(const ctis_plan *p) {
    if (!p->host_stale) return CTIS_OK;
    ctis_status st = check_device(p);
    if (st != CTIS_OK) return st;
    // set_values may have been queued on any stream: wait for all of them
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(CTIS_E_HIP, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
    HostTables &T = const_cast<ctis_plan *>(p)->ht;
    const struct {
        std::vector<float> *host;
        const float *dev;
    } parts[] = {{&T.box_w, p->work.box_w}, {&T.box_wf, p->work.box_wf}, {&T.h, p->work.h}};
    for (const auto &pt : parts) {
        if (pt.host->empty()) continue;
        e = hipMemcpy(pt.host->data(), pt.dev, pt.host->size() * sizeof(float), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(CTIS_E_HIP, std::string("hipMemcpy of plan values: ") + hipGetErrorString(e));
    }
    T.nonneg = std::all_of(T.box_w.begin(), T.box_w.end(), [](float v) { return v >= 0.0f; });
    p->host_stale = false;
    return CTIS_OK;
}

}  // namespace ctis

using namespace ctis;

extern "C" {

const char *ctis_version(void) { return "0.1.0"; }

const char *ctis_status_str(ctis_status st) {
    switch (st) {
        case CTIS_OK: return "ok";
        case CTIS_E_ARG: return "invalid argument";
        case CTIS_E_INDEX: return "calibration index out of range";
        case CTIS_E_VALUE: return "non-finite calibration value";
        case CTIS_E_TOO_LARGE: return "size exceeds the supported range";
        case CTIS_E_NOMEM: return "out of memory";
        case CTIS_E_HIP: return "HIP runtime error";
        case CTIS_E_NEGATIVE: return "EM needs nonnegative calibration values";
        case CTIS_E_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

const char *ctis_last_error(void) { return g_last_error.c_str(); }

ctis_status ctis_plan_create(ctis_plan **out, int32_t a, int32_t alpha, int32_t w, int32_t gamma, int32_t xi,
                             const int64_t *lambda_ptr, const int32_t *fpa_index, const float *value,
                             uint32_t flags) {
    g_last_error.clear();
    if (!out) return fail(CTIS_E_ARG, "out is NULL");
    *out = nullptr;
    const uint32_t known =
        CTIS_PLAN_HOST_ONLY | CTIS_PLAN_KEEP_ZEROS | CTIS_PLAN_TILE_PATH | CTIS_PLAN_BOX(0xF) | CTIS_PLAN_REGION(7);
    if (flags & ~known) return fail(CTIS_E_ARG, "unknown flag bits");
    const int shape = (int)((flags >> 12) & 0x7u);
    if (shape > kRegionShapes) return fail(CTIS_E_ARG, "region shape code must be in 0..6");
    const int forced_box = (int)((flags >> 8) & 0xFu);
    if (forced_box > kMaxBox) return fail(CTIS_E_ARG, "forced box side must be in 1..8");
    if (a < 1 || alpha < 1 || w < 1 || gamma < 1 || xi < 1)
        return fail(CTIS_E_ARG, "a, alpha, w, gamma, xi must all be >= 1");
    if (a > gamma || alpha > xi) return fail(CTIS_E_ARG, "the field stop must fit on the FPA (a <= gamma, alpha <= xi)");
    const int64_t n = (int64_t)gamma * xi, ell = (int64_t)a * alpha, m = ell * w;
    if (n > kMaxPixels || m > kMaxPixels)
        return fail(CTIS_E_TOO_LARGE, "n = gamma*xi and m = a*alpha*w must be below 2^29");
    if (!lambda_ptr) return fail(CTIS_E_ARG, "lambda_ptr is NULL");
    if (lambda_ptr[0] != 0) return fail(CTIS_E_ARG, "lambda_ptr[0] must be 0");
    for (int32_t s = 0; s < w; ++s)
        if (lambda_ptr[s + 1] < lambda_ptr[s]) return fail(CTIS_E_ARG, "lambda_ptr must be non-decreasing");
    const int64_t total = lambda_ptr[w];
    if (total > INT32_MAX) return fail(CTIS_E_TOO_LARGE, "too many calibration entries");
    if (total > 0 && (!fpa_index || !value)) return fail(CTIS_E_ARG, "fpa_index or value is NULL");
    for (int64_t t = 0; t < total; ++t) {
        if (fpa_index[t] < 0 || (int64_t)fpa_index[t] >= n)
            return fail(CTIS_E_INDEX, "fpa_index[" + std::to_string(t) + "] = " + std::to_string(fpa_index[t]) +
                                          " is outside [0, n)");
        if (!std::isfinite(value[t])) return fail(CTIS_E_VALUE, "value[" + std::to_string(t) + "] is not finite");
    }

    ctis_plan *p = new (std::nothrow) ctis_plan();
    if (!p) return fail(CTIS_E_NOMEM, "plan allocation");
    p->a = a;
    p->alpha = alpha;
    p->w = w;
    p->gamma = gamma;
    p->xi = xi;
    p->n = n;
    p->ell = ell;
    p->m = m;
    ctis_status st;
    try {
        st = build_host_tables(p, lambda_ptr, fpa_index, value, forced_box, (flags & CTIS_PLAN_KEEP_ZEROS) != 0,
                               shape);
    } catch (const std::bad_alloc &) {
        st = fail(CTIS_E_NOMEM, "host allocation while building the plan");
    }
    if (st != CTIS_OK) {
        delete p;
        return st;
    }
    if (flags & CTIS_PLAN_TILE_PATH) p->ht.pad_ok = false;
    if (!(flags & CTIS_PLAN_HOST_ONLY)) {
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) {
            delete p;
            return fail(CTIS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
        }
        p->device = dev;
        HostWork hw;
        try {
            st = build_work({FrameRef{p, 0, 0, 0}}, true, hw);
        } catch (const std::bad_alloc &) {
            st = fail(CTIS_E_NOMEM, "host allocation while building the work tables");
        }
        if (st == CTIS_OK) st = upload_work(hw, p->work);
        if (st != CTIS_OK) {
            delete p;
            return st;
        }
        p->workspace_bytes = p->work.workspace_bytes;
        p->vjp_workspace_bytes = p->work.vjp_workspace_bytes;
        p->solve_workspace_bytes = p->work.solve_workspace_bytes;
    } else {
        // host-only plans still report the workspace an EM call would need
        HostWork hw;
        try {
            st = build_work({FrameRef{p, 0, 0, 0}}, false, hw);
        } catch (const std::bad_alloc &) {
            st = fail(CTIS_E_NOMEM, "host allocation while building the work tables");
        }
        if (st != CTIS_OK) {
            delete p;
            return st;
        }
        const Layout L = layout_for(hw);
        p->workspace_bytes = L.em_bytes;
        p->vjp_workspace_bytes = L.vjp_bytes;
        p->solve_workspace_bytes = L.solve_bytes;
        p->work.fwd_em.waves = hw.fwd_em.waves;
        p->work.fwd_pad.waves = hw.fwd_pad.waves;
        p->work.adj.waves = hw.adj.waves;
    }
    *out = p;
    return CTIS_OK;
}

void ctis_plan_destroy(ctis_plan *p) {
    if (!p) return;
    free_work(p->work);
    delete p;
}

ctis_status ctis_plan_get_info(const ctis_plan *p, ctis_plan_info *info) {
    if (!p || !info) return fail(CTIS_E_ARG, "plan or info is NULL");
    ctis_status st = refresh_host_tables(p);
    if (st != CTIS_OK) return st;
    std::memset(info, 0, sizeof(*info));
    info->a = p->a;
    info->alpha = p->alpha;
    info->w = p->w;
    info->gamma = p->gamma;
    info->xi = p->xi;
    info->n = p->n;
    info->ell = p->ell;
    info->m = p->m;
    info->nnz = p->ht.nnz;
    info->n_support = p->ht.n_support;
    info->box = p->ht.B;
    info->n_boxes = (int32_t)p->ht.box_lambda.size();
    const HostTables &T = p->ht;
    info->tile_fast = kTileFast;
    info->tile_slow = kTileSlow;
    info->n_tiles = T.tiles.n_cells;
    info->n_active_tiles = T.tiles.n_active;
    info->n_items = (int64_t)T.tiles.item_box.size();
    info->region_fast = T.regions.tf;
    info->region_slow = T.regions.ts;
    info->n_regions = T.regions.n_cells;
    info->n_active_regions = T.regions.n_active;
    info->n_region_items = (int64_t)T.regions.item_box.size();
    info->em_region_path = (p->device >= 0 ? p->work.pad_ok : T.pad_ok) ? 1 : 0;
    info->waves_region = p->work.fwd_pad.waves;
    // multiply-adds: the method's (every calibration nonzero against every
    // voxel of its wavelength), and the ones the kernels execute (every slot
    // of a B x B box against every output of a work item)
    const int64_t BB = (int64_t)T.B * T.B;
    info->method_madds = p->ell * T.nnz;
    info->tile_forward_madds = (int64_t)T.tiles.item_box.size() * kTileFast * kTileSlow * BB;
    info->region_forward_madds = (int64_t)T.regions.item_box.size() * T.regions.tf * T.regions.ts * BB;
    info->adjoint_madds = (int64_t)T.nbx * T.nby * kTileFast * kTileSlow * (int64_t)T.box_lambda.size() * BB;
    info->workspace_bytes = p->workspace_bytes;
    info->nonnegative = p->ht.nonneg ? 1 : 0;
    info->device = p->device;
    info->waves_forward = p->work.fwd_em.waves;
    info->waves_adjoint = p->work.adj.waves;
    info->n_entries = p->ht.n_in;
    info->vjp_workspace_bytes = p->vjp_workspace_bytes;
    info->solve_workspace_bytes = p->solve_workspace_bytes;
    info->dropped = p->ht.dropped ? 1 : 0;
    return CTIS_OK;
}

ctis_status ctis_plan_lambda_sums(const ctis_plan *p, float *h_out) {
    if (!p || !h_out) return fail(CTIS_E_ARG, "plan or h_out is NULL");
    ctis_status st = refresh_host_tables(p);
    if (st != CTIS_OK) return st;
    std::memcpy(h_out, p->ht.h.data(), sizeof(float) * p->ht.h.size());
    return CTIS_OK;
}

ctis_status ctis_plan_export_boxes(const ctis_plan *p, int32_t *box_lambda, int32_t *box_rc, float *box_values) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    ctis_status st = refresh_host_tables(p);
    if (st != CTIS_OK) return st;
    const auto &T = p->ht;
    if (box_lambda) std::memcpy(box_lambda, T.box_lambda.data(), T.box_lambda.size() * 4);
    if (box_rc) std::memcpy(box_rc, T.box_rc.data(), T.box_rc.size() * 4);
    if (box_values) std::memcpy(box_values, T.box_w.data(), T.box_w.size() * 4);
    return CTIS_OK;
}

ctis_status ctis_plan_export_worklist(const ctis_plan *p, int32_t *tile_ptr, int32_t *item_box) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    const auto &G = p->ht.tiles;
    if (tile_ptr) std::memcpy(tile_ptr, G.item_ptr.data(), G.item_ptr.size() * 4);
    if (item_box) std::memcpy(item_box, G.item_box.data(), G.item_box.size() * 4);
    return CTIS_OK;
}

ctis_status ctis_plan_export_regions(const ctis_plan *p, int32_t *region_ptr, int32_t *item_box) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    const auto &G = p->ht.regions;
    if (region_ptr) std::memcpy(region_ptr, G.item_ptr.data(), G.item_ptr.size() * 4);
    if (item_box) std::memcpy(item_box, G.item_box.data(), G.item_box.size() * 4);
    return CTIS_OK;
}

ctis_status ctis_forward(const ctis_plan *p, const float *f, float *g_out, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (!f || !g_out) return fail(CTIS_E_ARG, "f or g_out is NULL");
    if (!aligned4(f) || !aligned4(g_out)) return fail(CTIS_E_ARG, "f and g_out must be 4-byte aligned");
    if (overlaps(f, (size_t)p->m * 4, g_out, (size_t)p->n * 4)) return fail(CTIS_E_ARG, "f and g_out overlap");
    ctis_status st = check_device(p);
    if (st != CTIS_OK) return st;
    return launch_status(launch_forward(p->work, f, nullptr, nullptr, g_out, kFwdPlain, nullptr, stream), "forward launch");
}

ctis_status ctis_adjoint(const ctis_plan *p, const float *r, float *z_out, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (!r || !z_out) return fail(CTIS_E_ARG, "r or z_out is NULL");
    if (!aligned4(r) || !aligned4(z_out)) return fail(CTIS_E_ARG, "r and z_out must be 4-byte aligned");
    if (overlaps(r, (size_t)p->n * 4, z_out, (size_t)p->m * 4)) return fail(CTIS_E_ARG, "r and z_out overlap");
    ctis_status st = check_device(p);
    if (st != CTIS_OK) return st;
    return launch_status(launch_adjoint(p->work, r, nullptr, nullptr, z_out, nullptr, nullptr, kAdjPlain, stream), "adjoint launch");
}

namespace {
ctis_status workspace_check(const ctis_plan *p, const void *workspace, size_t workspace_bytes) {
    if (!workspace || workspace_bytes < p->workspace_bytes)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(p->workspace_bytes) + " bytes");
    if (((uintptr_t)workspace & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    return CTIS_OK;
}

ctis_status em_check(const ctis_plan *p, const float *g, float *f, int32_t iters, void *workspace,
                     size_t workspace_bytes) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (!g || !f) return fail(CTIS_E_ARG, "g or f is NULL");
    if (iters < 0) return fail(CTIS_E_ARG, "iters must be >= 0");
    if (!aligned4(g) || !aligned4(f)) return fail(CTIS_E_ARG, "g and f must be 4-byte aligned");
    if (!p->ht.nonneg) return fail(CTIS_E_NEGATIVE, "the plan has a negative calibration value");
    ctis_status st = workspace_check(p, workspace, workspace_bytes);
    if (st != CTIS_OK) return st;
    if (overlaps(g, (size_t)p->n * 4, f, (size_t)p->m * 4) ||
        overlaps(workspace, p->workspace_bytes, f, (size_t)p->m * 4) ||
        overlaps(workspace, p->workspace_bytes, g, (size_t)p->n * 4))
        return fail(CTIS_E_ARG, "g, f and the workspace must not overlap");
    return check_device(p);
}
}  // namespace

ctis_status ctis_em_iterate(const ctis_plan *p, const float *g, float *f, int32_t iters, void *workspace,
                            size_t workspace_bytes, void *stream) {
    ctis_status st = em_check(p, g, f, iters, workspace, workspace_bytes);
    if (st != CTIS_OK || iters == 0) return st;
    return em_loop(p->work, g, f, iters, workspace, stream);
}

ctis_status ctis_solve_iterate(const ctis_plan *p, int32_t solver, const float *g, float *f, int32_t iters,
                               float relax, void *workspace, size_t workspace_bytes, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (solver != CTIS_SOLVER_EM && solver != CTIS_SOLVER_SMART && solver != CTIS_SOLVER_SART)
        return fail(CTIS_E_ARG, "unknown solver " + std::to_string(solver));
    if (solver == CTIS_SOLVER_SART && !(relax > 0.0f && relax < 2.0f))
        return fail(CTIS_E_ARG, "the SART relaxation must lie in (0, 2)");
    if (!g || !f) return fail(CTIS_E_ARG, "g or f is NULL");
    if (!aligned4(g) || !aligned4(f)) return fail(CTIS_E_ARG, "g and f must be 4-byte aligned");
    if (iters < 0) return fail(CTIS_E_ARG, "iters must be >= 0");
    if (solver != CTIS_SOLVER_SART && !p->ht.nonneg)
        return fail(CTIS_E_NEGATIVE, "the plan has a negative calibration value");
    const size_t need = solver == CTIS_SOLVER_SART ? p->solve_workspace_bytes : p->workspace_bytes;
    if (!workspace || workspace_bytes < need)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (overlaps(g, (size_t)p->n * 4, f, (size_t)p->m * 4) || overlaps(workspace, need, f, (size_t)p->m * 4) ||
        overlaps(workspace, need, g, (size_t)p->n * 4))
        return fail(CTIS_E_ARG, "g, f and the workspace must not overlap");
    ctis_status st = check_device(p);
    if (st != CTIS_OK || iters == 0) return st;
    return solve_loop(p->work, solver, g, f, iters, relax, workspace, stream);
}

ctis_status ctis_em_forward_ratio(const ctis_plan *p, const float *f, const float *g, void *workspace,
                                  size_t workspace_bytes, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (!f || !g) return fail(CTIS_E_ARG, "f or g is NULL");
    if (!aligned4(f) || !aligned4(g)) return fail(CTIS_E_ARG, "f and g must be 4-byte aligned");
    if (!p->ht.nonneg) return fail(CTIS_E_NEGATIVE, "the plan has a negative calibration value");
    ctis_status st = workspace_check(p, workspace, workspace_bytes);
    if (st != CTIS_OK) return st;
    if (overlaps(workspace, p->workspace_bytes, f, (size_t)p->m * 4) ||
        overlaps(workspace, p->workspace_bytes, g, (size_t)p->n * 4))
        return fail(CTIS_E_ARG, "the workspace must not overlap f or g");
    st = check_device(p);
    if (st != CTIS_OK) return st;
    return em_forward_half(p->work, f, g, workspace, stream);
}

ctis_status ctis_em_adjoint_update(const ctis_plan *p, void *workspace, size_t workspace_bytes,
                                   const float *f_in, float *f_out, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (!f_in || !f_out) return fail(CTIS_E_ARG, "f_in or f_out is NULL");
    if (!aligned4(f_in) || !aligned4(f_out)) return fail(CTIS_E_ARG, "f_in and f_out must be 4-byte aligned");
    if (!p->ht.nonneg) return fail(CTIS_E_NEGATIVE, "the plan has a negative calibration value");
    ctis_status st = workspace_check(p, workspace, workspace_bytes);
    if (st != CTIS_OK) return st;
    const size_t mb = (size_t)p->m * 4;
    if (f_in != f_out && overlaps(f_in, mb, f_out, mb)) return fail(CTIS_E_ARG, "f_in and f_out overlap");
    if (overlaps(workspace, p->workspace_bytes, f_out, mb))
        return fail(CTIS_E_ARG, "the workspace and f_out overlap");
    st = check_device(p);
    if (st != CTIS_OK) return st;
    return launch_status(launch_adjoint(p->work, (const float *)workspace, f_in, nullptr, f_out, nullptr, nullptr,
                                        kAdjUpdate, stream, workspace),
                         "adjoint+update launch");
}

ctis_status ctis_em_iterate_static(const ctis_plan *p, const float *g, float *f, int32_t iters, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (!g || !f) return fail(CTIS_E_ARG, "g or f is NULL");
    if (iters < 0) return fail(CTIS_E_ARG, "iters must be >= 0");
    if (!aligned4(g) || !aligned4(f)) return fail(CTIS_E_ARG, "g and f must be 4-byte aligned");
    if (!p->ht.nonneg) return fail(CTIS_E_NEGATIVE, "the plan has a negative calibration value");
    if (p->workspace_bytes > kStaticScratchBytes)
        return fail(CTIS_E_TOO_LARGE, "the plan's EM workspace (" + std::to_string(p->workspace_bytes) +
                                          " bytes) exceeds the static scratch of " +
                                          std::to_string(kStaticScratchBytes) + " bytes; use ctis_em_iterate");
    if (overlaps(g, (size_t)p->n * 4, f, (size_t)p->m * 4)) return fail(CTIS_E_ARG, "g and f overlap");
    ctis_status st = check_device(p);
    if (st != CTIS_OK || iters == 0) return st;
    void *scratch = nullptr;
    st = launch_status(static_scratch(&scratch), "static scratch address");
    if (st != CTIS_OK) return st;
    return em_loop(p->work, g, f, iters, scratch, stream);
}

ctis_status ctis_em_diagnostics(const ctis_plan *p, const float *g, const float *f, double *out, void *workspace,
                                size_t workspace_bytes, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (!g || !f || !out) return fail(CTIS_E_ARG, "g, f or out is NULL");
    if (!aligned4(g) || !aligned4(f) || ((uintptr_t)out & 7u) != 0)
        return fail(CTIS_E_ARG, "g and f must be 4-byte aligned, out 8-byte aligned");
    ctis_status st = workspace_check(p, workspace, workspace_bytes);
    if (st != CTIS_OK) return st;
    if (overlaps(workspace, p->workspace_bytes, f, (size_t)p->m * 4) ||
        overlaps(workspace, p->workspace_bytes, g, (size_t)p->n * 4) ||
        overlaps(workspace, p->workspace_bytes, out, 4 * sizeof(double)))
        return fail(CTIS_E_ARG, "the workspace must not overlap g, f or out");
    st = check_device(p);
    if (st != CTIS_OK) return st;
    float *ghat = (float *)workspace;
    st = launch_status(launch_forward(p->work, f, nullptr, nullptr, ghat, kFwdPlain, nullptr, stream),
                       "diagnostics forward launch");
    if (st != CTIS_OK) return st;
    return launch_status(launch_diagnostics(g, ghat, f, p->work.h, p->n, p->m, p->ell,
                                            (double *)((char *)workspace + p->work.diag_off), out, stream),
                         "diagnostics launch");
}

}  // extern "C"
