// Reverse-mode derivative of one EM iteration (C ABI) and updates of the
// calibration values on a fixed structure.
//
// One EM step (Sec. 2 eq. (em); stage order of the Sec. 3 algorithm) is
//   ghat = H f,  u = g / ghat,  zeta = H^T u,  f' = f zeta / h.
// Differentiating the stages last to first for an upstream y = dL/df':
//   b = y f / h = dL/dzeta,      dL/df (direct) = y zeta / h,
//   dL/dh_j = -y_j f'_j / h_j,    dL/du = H b,
//   e = dL/dghat = -(H b) u / ghat,  dL/df += H^T e,
//   dL/dH_ij = u_i b_j + e_i f_j,
// and H_ij = c_s[(i - q_j) mod n] (Sec. 3, H_s = C_s E) with every column
// sum h_j of wavelength s equal to the sum of c_s.  The six launches below:
//   1. forward + ratio          u        (the EM kernel)
//   2. back projection of u     zeta, b = y f / h, per-unit sums of b zeta
//   3. forward of b             e = -(H b) u^2 / g   (u / ghat = u^2 / g)
//   4. back projection of e     df = y zeta / h + H^T e
//   5. value partials           per (unit, box, slot): sum of u b + e f
//   6. value sums               per entry: partials over the wavelength's
//                               units minus (sum of b zeta) / h_s
#include <cstring>
#include <string>

#include "ctis_internal.h"

using namespace ctis;

namespace {

bool aligned4(const void *ptr) { return ((uintptr_t)ptr & 3u) == 0; }

bool overlaps(const void *x, size_t xb, const void *y, size_t yb) {
    const char *a = (const char *)x, *b = (const char *)y;
    return a < b + yb && b < a + xb;
}

ctis_status launched(int err, const char *what) {
    if (err != 0) return fail(CTIS_E_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)err));
    return CTIS_OK;
}

ctis_status on_device(int32_t device) {
    if (device < 0) return fail(CTIS_E_ARG, "plan was created host-only");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CTIS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev != device) return fail(CTIS_E_ARG, "current HIP device differs from the plan's or batch's device");
    return CTIS_OK;
}

struct Sizes {
    int64_t m, n;   // floats of f and g (all frames)
    bool nonneg, dropped;
    int32_t device;
};

ctis_status vjp_run(const DevWork &w, const Sizes &z, const float *g, const float *f, const float *y, float *df,
                    float *dv, int32_t accumulate, void *workspace, size_t workspace_bytes, void *stream) {
    if (!g || !f || !y || !df) return fail(CTIS_E_ARG, "g, f, y and df_out must not be NULL");
    if (!aligned4(g) || !aligned4(f) || !aligned4(y) || !aligned4(df) || (dv && !aligned4(dv)))
        return fail(CTIS_E_ARG, "arrays must be 4-byte aligned");
    if (!z.nonneg) return fail(CTIS_E_NEGATIVE, "a calibration value is negative");
    if (dv && z.dropped)
        return fail(CTIS_E_ARG, "value derivatives need every entry in the structure: create the plan with "
                                "CTIS_PLAN_KEEP_ZEROS");
    if (!workspace || workspace_bytes < w.vjp_workspace_bytes)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(w.vjp_workspace_bytes) + " bytes");
    if (((uintptr_t)workspace & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    const size_t mb = (size_t)z.m * 4, nb = (size_t)z.n * 4, wb = w.vjp_workspace_bytes;
    const size_t vb = (size_t)w.n_entries * 4;
    if (df != y && overlaps(df, mb, y, mb)) return fail(CTIS_E_ARG, "df_out overlaps y without being equal");
    if (overlaps(df, mb, f, mb) || overlaps(df, mb, g, nb) || overlaps(df, mb, workspace, wb) ||
        overlaps(y, mb, workspace, wb) || overlaps(f, mb, workspace, wb) || overlaps(g, nb, workspace, wb))
        return fail(CTIS_E_ARG, "df_out, f, g, y and the workspace must not overlap (df_out may equal y)");
    if (dv && (overlaps(dv, vb, workspace, wb) || overlaps(dv, vb, df, mb) || overlaps(dv, vb, y, mb) ||
               overlaps(dv, vb, f, mb) || overlaps(dv, vb, g, nb)))
        return fail(CTIS_E_ARG, "dvalues overlaps another argument");
    ctis_status st = on_device(z.device);
    if (st != CTIS_OK) return st;

    char *base = (char *)workspace;
    float *u = (float *)base;
    float *e = (float *)(base + w.e_off);
    float *zeta = (float *)(base + w.zeta_off);
    float *b = (float *)(base + w.b_off);
    float *flux = (float *)(base + w.hpart_off);
    float *part = (float *)(base + w.vg_off);
    st = launched(launch_forward(w, f, g, nullptr, u, kFwdRatio, workspace, stream), "vjp forward+ratio launch");
    if (st != CTIS_OK) return st;
    st = launched(launch_adjoint(w, u, y, f, zeta, b, flux, kAdjVjpPre, stream), "vjp back projection of u");
    if (st != CTIS_OK) return st;
    st = launched(launch_forward(w, b, g, u, e, kFwdVjp, workspace, stream), "vjp forward of b");
    if (st != CTIS_OK) return st;
    st = launched(launch_adjoint(w, e, y, zeta, df, nullptr, nullptr, kAdjVjpGrad, stream), "vjp back projection of e");
    if (st != CTIS_OK) return st;
    if (dv && w.n_entries > 0) {
        st = launched(launch_value_grad(w, u, e, b, f, part, stream), "vjp value partials");
        if (st != CTIS_OK) return st;
        st = launched(launch_value_finish(w, part, flux, dv, 0, w.n_entries, accumulate != 0, stream), "vjp value sums");
    }
    return st;
}

}  // namespace

extern "C" {

ctis_status ctis_em_vjp(const ctis_plan *p, const float *g, const float *f, const float *y, float *df_out,
                        float *dvalues, int32_t accumulate, void *workspace, size_t workspace_bytes,
                        void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    const Sizes z{p->m, p->n, p->ht.nonneg, p->ht.dropped, p->device};
    return vjp_run(p->work, z, g, f, y, df_out, dvalues, accumulate, workspace, workspace_bytes, stream);
}

ctis_status ctis_batch_em_vjp(const ctis_batch *b, const float *g_all, const float *f_all, const float *y_all,
                              float *df_all, float *dvalues, int32_t accumulate, void *workspace,
                              size_t workspace_bytes, void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    const Sizes z{b->f_floats, b->g_floats, b->nonneg, b->dropped, b->device};
    return vjp_run(b->work, z, g_all, f_all, y_all, df_all, dvalues, accumulate, workspace, workspace_bytes, stream);
}

ctis_status ctis_plan_set_values(ctis_plan *p, const float *values, void *stream) {
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (p->ht.dropped)
        return fail(CTIS_E_ARG, "the plan dropped an entry that merged to zero: create it with CTIS_PLAN_KEEP_ZEROS");
    if (p->ht.n_in > 0 && (!values || !aligned4(values))) return fail(CTIS_E_ARG, "values must be non-NULL and aligned");
    ctis_status st = on_device(p->device);
    if (st != CTIS_OK || p->w == 0) return st;
    st = launched(launch_set_values(p->work, values, 0, 0, p->w, stream), "set values launch");
    if (st == CTIS_OK) p->host_stale = true;
    return st;
}

ctis_status ctis_batch_set_values(ctis_batch *b, int32_t frame, const float *values, void *stream) {
    if (!b) return fail(CTIS_E_ARG, "batch is NULL");
    if (frame < 0 || frame >= (int32_t)b->plans.size()) return fail(CTIS_E_ARG, "frame out of range");
    const ctis_plan *p = b->plans[(size_t)frame];
    if (p->ht.dropped)
        return fail(CTIS_E_ARG, "the plan dropped an entry that merged to zero: create it with CTIS_PLAN_KEEP_ZEROS");
    if (p->ht.n_in > 0 && (!values || !aligned4(values))) return fail(CTIS_E_ARG, "values must be non-NULL and aligned");
    ctis_status st = on_device(b->device);
    if (st != CTIS_OK) return st;
    const size_t d = (size_t)b->frame_plan[(size_t)frame];
    const int32_t lam0 = b->plan_lam0[d];
    return launched(launch_set_values(b->work, values, b->plan_entry0[d], lam0, lam0 + p->w, stream),
                    "batch set values launch");
}

ctis_status ctis_batch_plan_entries(const ctis_batch *b, int32_t frame, int64_t *offset, int64_t *count) {
    if (!b || !offset || !count) return fail(CTIS_E_ARG, "batch, offset or count is NULL");
    if (frame < 0 || frame >= (int32_t)b->plans.size()) return fail(CTIS_E_ARG, "frame out of range");
    const size_t d = (size_t)b->frame_plan[(size_t)frame];
    *offset = b->plan_entry0[d];
    *count = b->plans[(size_t)frame]->ht.n_in;
    return CTIS_OK;
}

}  // extern "C"
