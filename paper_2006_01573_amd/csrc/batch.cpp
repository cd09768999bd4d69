// Batches of frames (C ABI): several plans merged into one work description,
// so that each EM iteration of all frames is one forward+ratio launch and one
// adjoint+update launch.
#include <cstring>
#include <new>
#include <string>

#include "ctis_internal.h"

using namespace ctis;

namespace {

ctis_status batch_device(const ctis_batch *b) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CTIS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev != b->device) return fail(CTIS_E_ARG, "current HIP device differs from the batch's device");
    return CTIS_OK;
}

bool aligned4(const void *ptr) { return ((uintptr_t)ptr & 3u) == 0; }

bool overlaps(const void *x, size_t xb, const void *y, size_t yb) {
    const char *a = (const char *)x, *b = (const char *)y;
    return a < b + yb && b < a + xb;
}

ctis_status launched(int err, const char *what) {
    if (err != 0) return fail(CTIS_E_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)err));
    return CTIS_OK;
}

}  // namespace

extern "C" {

ctis_status ctis_batch_create(ctis_batch **out, const ctis_plan *const *plans, int32_t n_frames, uint32_t flags) {
    if (!out) return fail(CTIS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!plans || n_frames < 1) return fail(CTIS_E_ARG, "need at least one plan");
    if (flags & ~(0x3FFu | CTIS_BATCH_PERSISTENT | CTIS_BATCH_WAVES_REGION(0xF) | CTIS_BATCH_TILE_PATH |
                  CTIS_BATCH_REGION_SOLO))
        return fail(CTIS_E_ARG, "unknown flag bits");
    const int wf = (int)(flags & 0x1Fu), wa = (int)((flags >> 5) & 0x1Fu);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CTIS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::vector<FrameRef> frames;
    int64_t fo = 0, go = 0;
    bool nonneg = true;
    for (int32_t k = 0; k < n_frames; ++k) {
        const ctis_plan *p = plans[k];
        if (!p) return fail(CTIS_E_ARG, "plan " + std::to_string(k) + " is NULL");
        if (p->device < 0) return fail(CTIS_E_ARG, "plan " + std::to_string(k) + " is host-only");
        if (p->device != dev) return fail(CTIS_E_ARG, "plan " + std::to_string(k) + " lives on another device");
        if (p->ht.B != plans[0]->ht.B) return fail(CTIS_E_ARG, "all plans of a batch need the same box side B");
        const ctis_status rs = refresh_host_tables(p);
        if (rs != CTIS_OK) return rs;
        frames.push_back(FrameRef{p, fo, go, go});
        fo += p->m;
        go += p->n;
        nonneg = nonneg && p->ht.nonneg;
        if (fo > kMaxPixels || go > INT32_MAX)
            return fail(CTIS_E_TOO_LARGE, "batch buffers of 2^29 (f_all) or 2^31 (g_all) floats or more");
    }
    const int B = plans[0]->ht.B;
    for (int nw : {wf, wa})
        if (nw != 0 && nw != 1 && (nw < min_waves() || nw > max_waves(B)))
            return fail(CTIS_E_ARG, "waves per workgroup must be 0, 1 (a wave per unit) or in " +
                                        std::to_string(min_waves()) + ".." + std::to_string(max_waves(B)));
    const int wr = (int)((flags >> 11) & 0xFu);
    if (wr > kFwdMaxWaves)
        return fail(CTIS_E_ARG, "region waves per workgroup must be 0 or in 1.." + std::to_string(kFwdMaxWaves));
    ctis_batch *b = new (std::nothrow) ctis_batch();
    if (!b) return fail(CTIS_E_NOMEM, "batch allocation");
    ctis_status st;
    HostWork hw;
    try {
        st = build_work(frames, true, hw);
    } catch (const std::bad_alloc &) {
        st = fail(CTIS_E_NOMEM, "host allocation while building the work tables");
    }
    if (st == CTIS_OK) {
        if (wf) hw.fwd_em.waves = hw.fwd_full.waves = wf;
        if (wa) hw.adj.waves = wa;
        if (wr) hw.fwd_pad.waves = wr;
        if (flags & CTIS_BATCH_TILE_PATH) hw.pad_ok = false;
        st = upload_work(hw, b->work);
        b->work.persistent = (flags & CTIS_BATCH_PERSISTENT) != 0;
        b->work.region_solo = (flags & CTIS_BATCH_REGION_SOLO) != 0;
    }
    if (st != CTIS_OK) {
        delete b;
        return st;
    }
    for (const FrameRef &fr : frames) {
        b->plans.push_back(fr.plan);
        b->f_base.push_back(fr.f_base);
        b->g_base.push_back(fr.g_base);
        b->u_base.push_back(fr.u_base);
    }
    b->f_floats = fo;
    b->g_floats = go;
    b->dropped = hw.dropped;
    b->frame_plan = hw.frame_plan;
    b->plan_box0 = hw.plan_box0;
    b->plan_lam0 = hw.plan_lam0;
    b->plan_entry0 = hw.plan_entry0;
    b->device = dev;
    b->nonneg = nonneg;
    *out = b;
    return CTIS_OK;
}

void ctis_batch_destroy(ctis_batch *b) {
    if (!b) return;
    free_work(b->work);
    delete b;
}

ctis_status ctis_batch_get_info(const ctis_batch *b, ctis_batch_info *info) {
    if (!b || !info) return fail(CTIS_E_ARG, "batch or info is NULL");
    std::memset(info, 0, sizeof(*info));
    info->n_frames = (int32_t)b->plans.size();
    info->box = b->work.B;
    info->m_total = b->f_floats;
    info->n_total = b->g_floats;
    info->forward_units = b->work.fwd_em.n_units;
    info->adjoint_units = b->work.adj.n_units;
    info->waves_forward = b->work.fwd_em.waves;
    info->waves_adjoint = b->work.adj.waves;
    info->em_region_path = b->work.pad_ok ? 1 : 0;
    info->waves_region = b->work.fwd_pad.waves;
    info->region_units = b->work.fwd_pad.n_units;
    info->workspace_bytes = b->work.workspace_bytes;
    info->solve_workspace_bytes = b->work.solve_workspace_bytes;
    info->n_plans = (int32_t)b->plan_entry0.size();
    info->n_entries = b->work.n_entries;
    info->vjp_workspace_bytes = b->work.vjp_workspace_bytes;
    return CTIS_OK;
}

ctis_status ctis_batch_forward(const ctis_batch *b, const float *f_all, float *g_all, void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    if (!f_all || !g_all || !aligned4(f_all) || !aligned4(g_all))
        return fail(CTIS_E_ARG, "f_all and g_all must be non-NULL and 4-byte aligned");
    if (overlaps(f_all, (size_t)b->f_floats * 4, g_all, (size_t)b->g_floats * 4))
        return fail(CTIS_E_ARG, "f_all and g_all overlap");
    ctis_status st = batch_device(b);
    if (st != CTIS_OK) return st;
    return launched(launch_forward(b->work, f_all, nullptr, nullptr, g_all, kFwdPlain, nullptr, stream), "batch forward launch");
}

ctis_status ctis_batch_adjoint(const ctis_batch *b, const float *r_all, float *z_all, void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    if (!r_all || !z_all || !aligned4(r_all) || !aligned4(z_all))
        return fail(CTIS_E_ARG, "r_all and z_all must be non-NULL and 4-byte aligned");
    if (overlaps(r_all, (size_t)b->g_floats * 4, z_all, (size_t)b->f_floats * 4))
        return fail(CTIS_E_ARG, "r_all and z_all overlap");
    ctis_status st = batch_device(b);
    if (st != CTIS_OK) return st;
    return launched(launch_adjoint(b->work, r_all, nullptr, nullptr, z_all, nullptr, nullptr, kAdjPlain, stream), "batch adjoint launch");
}

ctis_status ctis_batch_em_iterate(const ctis_batch *b, const float *g_all, float *f_all, int32_t iters,
                                  void *workspace, size_t workspace_bytes, void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    if (!g_all || !f_all || !aligned4(g_all) || !aligned4(f_all))
        return fail(CTIS_E_ARG, "g_all and f_all must be non-NULL and 4-byte aligned");
    if (iters < 0) return fail(CTIS_E_ARG, "iters must be >= 0");
    if (!b->nonneg) return fail(CTIS_E_NEGATIVE, "a plan of the batch has a negative calibration value");
    if (!workspace || workspace_bytes < b->work.workspace_bytes)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(b->work.workspace_bytes) + " bytes");
    if (((uintptr_t)workspace & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t fb = (size_t)b->f_floats * 4, gb = (size_t)b->g_floats * 4, wb = b->work.workspace_bytes;
    if (overlaps(g_all, gb, f_all, fb) || overlaps(workspace, wb, f_all, fb) || overlaps(workspace, wb, g_all, gb))
        return fail(CTIS_E_ARG, "g_all, f_all and the workspace must not overlap");
    ctis_status st = batch_device(b);
    if (st != CTIS_OK) return st;
    return em_loop(b->work, g_all, f_all, iters, workspace, stream);
}

ctis_status ctis_batch_solve_iterate(const ctis_batch *b, int32_t solver, const float *g_all, float *f_all,
                                     int32_t iters, float relax, void *workspace, size_t workspace_bytes,
                                     void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    if (solver != CTIS_SOLVER_EM && solver != CTIS_SOLVER_SMART && solver != CTIS_SOLVER_SART)
        return fail(CTIS_E_ARG, "unknown solver " + std::to_string(solver));
    if (solver == CTIS_SOLVER_SART && !(relax > 0.0f && relax < 2.0f))
        return fail(CTIS_E_ARG, "the SART relaxation must lie in (0, 2)");
    if (!g_all || !f_all || !aligned4(g_all) || !aligned4(f_all))
        return fail(CTIS_E_ARG, "g_all and f_all must be non-NULL and 4-byte aligned");
    if (iters < 0) return fail(CTIS_E_ARG, "iters must be >= 0");
    if (solver != CTIS_SOLVER_SART && !b->nonneg)
        return fail(CTIS_E_NEGATIVE, "a plan of the batch has a negative calibration value");
    const size_t need = solver == CTIS_SOLVER_SART ? b->work.solve_workspace_bytes : b->work.workspace_bytes;
    if (!workspace || workspace_bytes < need)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t fb = (size_t)b->f_floats * 4, gb = (size_t)b->g_floats * 4;
    if (overlaps(g_all, gb, f_all, fb) || overlaps(workspace, need, f_all, fb) || overlaps(workspace, need, g_all, gb))
        return fail(CTIS_E_ARG, "g_all, f_all and the workspace must not overlap");
    ctis_status st = batch_device(b);
    if (st != CTIS_OK || iters == 0) return st;
    return solve_loop(b->work, solver, g_all, f_all, iters, relax, workspace, stream);
}

ctis_status ctis_batch_em_forward_ratio(const ctis_batch *b, const float *f_all, const float *g_all, void *workspace,
                                        size_t workspace_bytes, void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    if (!g_all || !f_all || !aligned4(g_all) || !aligned4(f_all))
        return fail(CTIS_E_ARG, "g_all and f_all must be non-NULL and 4-byte aligned");
    if (!b->nonneg) return fail(CTIS_E_NEGATIVE, "a plan of the batch has a negative calibration value");
    if (!workspace || workspace_bytes < b->work.workspace_bytes)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(b->work.workspace_bytes) + " bytes");
    if (((uintptr_t)workspace & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t fb = (size_t)b->f_floats * 4, gb = (size_t)b->g_floats * 4, wb = b->work.workspace_bytes;
    if (overlaps(workspace, wb, f_all, fb) || overlaps(workspace, wb, g_all, gb))
        return fail(CTIS_E_ARG, "the workspace must not overlap f_all or g_all");
    ctis_status st = batch_device(b);
    if (st != CTIS_OK) return st;
    return em_forward_half(b->work, f_all, g_all, workspace, stream);
}

ctis_status ctis_batch_em_adjoint_update(const ctis_batch *b, void *workspace, size_t workspace_bytes,
                                         const float *f_in, float *f_out, void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    if (!f_in || !f_out || !aligned4(f_in) || !aligned4(f_out))
        return fail(CTIS_E_ARG, "f_in and f_out must be non-NULL and 4-byte aligned");
    if (!b->nonneg) return fail(CTIS_E_NEGATIVE, "a plan of the batch has a negative calibration value");
    if (!workspace || workspace_bytes < b->work.workspace_bytes)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(b->work.workspace_bytes) + " bytes");
    if (((uintptr_t)workspace & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t fb = (size_t)b->f_floats * 4, wb = b->work.workspace_bytes;
    if (f_in != f_out && overlaps(f_in, fb, f_out, fb)) return fail(CTIS_E_ARG, "f_in and f_out overlap");
    if (overlaps(workspace, wb, f_out, fb)) return fail(CTIS_E_ARG, "the workspace and f_out overlap");
    ctis_status st = batch_device(b);
    if (st != CTIS_OK) return st;
    return launched(launch_adjoint(b->work, (const float *)workspace, f_in, nullptr, f_out, nullptr, nullptr,
                                   kAdjUpdate, stream, workspace),
                    "batch adjoint+update launch");
}

}  // extern "C"
