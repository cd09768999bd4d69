// C ABI of the Fourier (WBH) path: the spectra of a plan's calibration, and
// projections and EM through length-n FFTs (Sec. 3 eqs. (forward) and
// (backwards); the stage order of the Sec. 3 algorithm).  The FFT kernel is
// in fourier.hip.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fourier_internal.h"

using namespace ctis;
using namespace ctis::fourier;

struct ctis_fourier {
    const ctis_plan *plan = nullptr;
    int64_t n = 0;
    int32_t N1 = 0, N2 = 0, log_n1 = 0, log_n2 = 0, pairs = 0, device = -1;
    Geo geo{};
    float2 *e = nullptr;          // pairs x n spectra e_t = F(c_{2t} - i c_{2t+1})
    float2 *tw1 = nullptr, *tw2 = nullptr, *tw_hi = nullptr, *tw_lo = nullptr;
    float *h = nullptr;           // w column sums
    void *mem = nullptr;
    size_t spectra_bytes = 0, workspace_bytes = 0;
    size_t off_b = 0, off_u = 0;  // workspace: A (pairs n complex), B (pairs n complex), u (n floats)
    bool nonneg = true;
};

namespace {

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

ctis_status launched(int err, const char *what) {
    if (err != 0) return fail(CTIS_E_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)err));
    return CTIS_OK;
}

int log2_exact(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return (int64_t(1) << l) == v ? l : -1;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// One complex FFT of length n over `batches` sequences: pass A then pass B.
ctis_status run_fft(const ctis_fourier *F, Pass a, Pass b, int batches_a, int batches_b, void *stream) {
    a.n = b.n = F->n;
    a.N1 = b.N1 = F->N1;
    a.N2 = b.N2 = F->N2;
    a.log_n2 = b.log_n2 = F->log_n2;
    a.geo = b.geo = F->geo;
    a.e = b.e = F->e;
    a.h = b.h = F->h;
    a.pass_a = 1;
    a.L = F->N1;
    a.log_l = F->log_n1;
    a.n_seq = F->N2;
    a.tw_stage = F->tw1;
    a.tw_hi = F->tw_hi;
    a.tw_lo = F->tw_lo;
    b.pass_a = 0;
    b.L = F->N2;
    b.log_l = F->log_n2;
    b.n_seq = F->N1;
    b.tw_stage = F->tw2;
    b.load = kLoadComplex;
    ctis_status st = launched(launch_pass(a, batches_a, stream), "fft pass A");
    if (st != CTIS_OK) return st;
    return launched(launch_pass(b, batches_b, stream), "fft pass B");
}

// ghat = H f (store kStoreReal into out) or u = g / H f (kStoreRatio)
ctis_status forward(const ctis_fourier *F, const float *f, const float *g, float *out, int store, char *ws,
                    void *stream) {
    float2 *A = (float2 *)ws, *B = (float2 *)(ws + F->off_b);
    Pass a{}, b{};
    a.fin = f;
    a.load = kLoadEmbedPair;
    a.out = A;
    b.in = A;
    b.out = B;
    b.store = kStoreComplex;
    ctis_status st = run_fft(F, a, b, F->pairs, F->pairs, stream);   // X_t = F(v_{2t} + i v_{2t+1})
    if (st != CTIS_OK) return st;
    st = launched(launch_combine(F->e, B, A, F->pairs, F->n, stream), "spectral products");   // sum_t e_t X_t
    if (st != CTIS_OK) return st;
    Pass c{}, d{};
    c.in = A;
    c.load = kLoadComplex;
    c.out = B;
    c.inverse = 1;
    d.in = B;
    d.inverse = 1;
    d.store = store;
    d.fout = out;
    d.g = g;
    return run_fft(F, c, d, 1, 1, stream);                           // F^-1 of the sum
}

// z = H^T r (kStoreCrop into out) or f = f . H^T u / h (kStoreUpdate on out)
ctis_status adjoint(const ctis_fourier *F, const float *r, float *out, int store, char *ws, void *stream) {
    float2 *A = (float2 *)ws, *B = (float2 *)(ws + F->off_b);
    Pass a{}, b{};
    a.fin = r;
    a.load = kLoadReal;
    a.out = A;
    b.in = A;
    b.out = B;
    b.store = kStoreComplex;
    ctis_status st = run_fft(F, a, b, 1, 1, stream);                 // U = F r
    if (st != CTIS_OK) return st;
    Pass c{}, d{};
    c.in = B;
    c.load = kLoadConjE;
    c.out = A;
    c.inverse = 1;
    d.in = A;
    d.inverse = 1;
    d.store = store;
    d.fout = out;
    return run_fft(F, c, d, F->pairs, F->pairs, stream);             // F^-1 conj(e_t) U
}

ctis_status on_device(const ctis_fourier *F) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CTIS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev != F->device) return fail(CTIS_E_ARG, "current HIP device differs from the Fourier plan's device");
    return CTIS_OK;
}

ctis_status check_ws(const ctis_fourier *F, const void *ws, size_t bytes) {
    if (!ws || bytes < F->workspace_bytes)
        return fail(CTIS_E_WORKSPACE, "workspace needs " + std::to_string(F->workspace_bytes) + " bytes");
    if (((uintptr_t)ws & 255u) != 0) return fail(CTIS_E_WORKSPACE, "workspace must be 256-byte aligned");
    return CTIS_OK;
}

bool overlaps(const void *x, size_t xb, const void *y, size_t yb) {
    const char *a = (const char *)x, *b = (const char *)y;
    return a < b + yb && b < a + xb;
}

}  // namespace

extern "C" {

ctis_status ctis_fourier_create(ctis_fourier **out, const ctis_plan *p) {
    if (!out) return fail(CTIS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(CTIS_E_ARG, "plan is NULL");
    if (p->device < 0) return fail(CTIS_E_ARG, "plan was created host-only");
    const int ln = log2_exact(p->n);
    if (ln < 4 || ln > 20) return fail(CTIS_E_ARG, "the Fourier path needs n = gamma*xi a power of two in 2^4..2^20");
    int dev = -1;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess || dev != p->device) return fail(CTIS_E_ARG, "current HIP device differs from the plan's");
    const ctis_status rs = refresh_host_tables(p);
    if (rs != CTIS_OK) return rs;
    ctis_fourier *F = new (std::nothrow) ctis_fourier();
    if (!F) return fail(CTIS_E_NOMEM, "Fourier plan allocation");
    F->plan = p;
    F->n = p->n;
    F->log_n1 = (ln + 1) / 2;
    F->log_n2 = ln / 2;
    F->N1 = 1 << F->log_n1;
    F->N2 = 1 << F->log_n2;
    F->pairs = (p->w + 1) / 2;
    F->geo = Geo{p->a, p->alpha, p->gamma, p->xi, p->w, (long long)p->ell, log2_exact(p->gamma)};
    F->device = dev;
    F->nonneg = p->ht.nonneg;
    const int64_t n = p->n;

    // dense calibration images c_s from the plan's boxes (merged values)
    std::vector<float> c;
    std::vector<float2> tw1((size_t)F->N1 / 2), tw2((size_t)std::max(1, F->N2 / 2)), hi((size_t)F->N1),
        lo((size_t)F->N2);
    try {
        c.assign((size_t)p->w * (size_t)n, 0.0f);
    } catch (const std::bad_alloc &) {
        delete F;
        return fail(CTIS_E_NOMEM, "host calibration images");
    }
    const auto &T = p->ht;
    const int B = T.B;
    for (size_t k = 0; k < T.box_lambda.size(); ++k) {
        const int s = T.box_lambda[k];
        const int64_t rA = T.box_rc[2 * k], cA = T.box_rc[2 * k + 1];
        for (int dc = 0; dc < B; ++dc)
            for (int dr = 0; dr < B; ++dr) {
                const float v = T.box_w[k * (size_t)(B * B) + (size_t)(dc * B + dr)];
                if (v == 0.0f) continue;
                const int64_t i = ((rA + dr) + (int64_t)p->gamma * (cA + dc)) % n;
                c[(size_t)s * (size_t)n + (size_t)i] += v;
            }
    }
    const double pi = 3.14159265358979323846;
    auto unit = [&](double frac) { return float2{(float)std::cos(-2.0 * pi * frac), (float)std::sin(-2.0 * pi * frac)}; };
    for (int j = 0; j < F->N1 / 2; ++j) tw1[(size_t)j] = unit((double)j / F->N1);
    for (int j = 0; j < F->N2 / 2; ++j) tw2[(size_t)j] = unit((double)j / F->N2);
    for (int j = 0; j < F->N1; ++j) hi[(size_t)j] = unit((double)j / F->N1);
    for (int j = 0; j < F->N2; ++j) lo[(size_t)j] = unit((double)j / (double)n);

    // one allocation: spectra, twiddles, h
    const size_t e_bytes = (size_t)F->pairs * (size_t)n * sizeof(float2);
    size_t off = 0;
    const size_t o_e = off;
    off += up256(e_bytes);
    const size_t o_t1 = off;
    off += up256(tw1.size() * sizeof(float2));
    const size_t o_t2 = off;
    off += up256(tw2.size() * sizeof(float2));
    const size_t o_hi = off;
    off += up256(hi.size() * sizeof(float2));
    const size_t o_lo = off;
    off += up256(lo.size() * sizeof(float2));
    const size_t o_h = off;
    off += up256((size_t)p->w * sizeof(float));
    he = hipMalloc(&F->mem, off);
    if (he != hipSuccess) {
        delete F;
        return fail(CTIS_E_NOMEM, std::string("hipMalloc of the spectra: ") + hipGetErrorString(he));
    }
    char *base = (char *)F->mem;
    F->e = (float2 *)(base + o_e);
    F->tw1 = (float2 *)(base + o_t1);
    F->tw2 = (float2 *)(base + o_t2);
    F->tw_hi = (float2 *)(base + o_hi);
    F->tw_lo = (float2 *)(base + o_lo);
    F->h = (float *)(base + o_h);
    F->spectra_bytes = off;
    F->off_b = up256((size_t)F->pairs * (size_t)n * sizeof(float2));
    F->off_u = F->off_b + up256((size_t)F->pairs * (size_t)n * sizeof(float2));
    F->workspace_bytes = F->off_u + up256((size_t)n * sizeof(float));

    // upload, and e_t = F(c_{2t} - i c_{2t+1}) through the FFT itself
    void *cdev = nullptr, *tmp = nullptr;
    ctis_status st = CTIS_OK;
    auto cleanup = [&]() {
        if (cdev) (void)hipFree(cdev);
        if (tmp) (void)hipFree(tmp);
    };
    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    };
    const Up ups[] = {{F->tw1, tw1.data(), tw1.size() * sizeof(float2)},
                      {F->tw2, tw2.data(), tw2.size() * sizeof(float2)},
                      {F->tw_hi, hi.data(), hi.size() * sizeof(float2)},
                      {F->tw_lo, lo.data(), lo.size() * sizeof(float2)},
                      {F->h, T.h.data(), (size_t)p->w * sizeof(float)}};
    for (const Up &u : ups) {
        he = hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice);
        if (he != hipSuccess) st = fail(CTIS_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(he));
        if (st != CTIS_OK) break;
    }
    if (st == CTIS_OK) {
        he = hipMalloc(&cdev, c.size() * sizeof(float));
        if (he == hipSuccess) he = hipMalloc(&tmp, e_bytes);
        if (he != hipSuccess) st = fail(CTIS_E_NOMEM, "device calibration images");
    }
    if (st == CTIS_OK) {
        he = hipMemcpy(cdev, c.data(), c.size() * sizeof(float), hipMemcpyHostToDevice);
        if (he != hipSuccess) st = fail(CTIS_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(he));
    }
    if (st == CTIS_OK) {
        Pass a{}, b{};
        a.fin = (const float *)cdev;
        a.load = kLoadCalPair;
        a.out = (float2 *)tmp;
        b.in = (const float2 *)tmp;
        b.out = F->e;
        b.store = kStoreComplex;
        st = run_fft(F, a, b, F->pairs, F->pairs, nullptr);
    }
    if (st == CTIS_OK) {
        he = hipDeviceSynchronize();
        if (he != hipSuccess) st = fail(CTIS_E_HIP, std::string("spectra: ") + hipGetErrorString(he));
    }
    cleanup();
    if (st != CTIS_OK) {
        (void)hipFree(F->mem);
        delete F;
        return st;
    }
    *out = F;
    return CTIS_OK;
}

void ctis_fourier_destroy(ctis_fourier *F) {
    if (!F) return;
    if (F->mem) (void)hipFree(F->mem);
    delete F;
}

ctis_status ctis_fourier_get_info(const ctis_fourier *F, ctis_fourier_info *info) {
    if (!F || !info) return fail(CTIS_E_ARG, "Fourier plan or info is NULL");
    std::memset(info, 0, sizeof(*info));
    info->n = F->n;
    info->n1 = F->N1;
    info->n2 = F->N2;
    info->pairs = F->pairs;
    info->spectra_bytes = F->spectra_bytes;
    info->workspace_bytes = F->workspace_bytes;
    return CTIS_OK;
}

ctis_status ctis_fourier_forward(const ctis_fourier *F, const float *f, float *g_out, void *workspace,
                                 size_t workspace_bytes, void *stream) {
    if (!F) return fail(CTIS_E_ARG, "Fourier plan is NULL");
    if (!f || !g_out || !aligned4(f) || !aligned4(g_out)) return fail(CTIS_E_ARG, "f and g_out must be non-NULL and aligned");
    ctis_status st = check_ws(F, workspace, workspace_bytes);
    if (st != CTIS_OK) return st;
    const size_t mb = (size_t)F->plan->m * 4, nb = (size_t)F->n * 4;
    if (overlaps(f, mb, g_out, nb) || overlaps(workspace, F->workspace_bytes, f, mb) ||
        overlaps(workspace, F->workspace_bytes, g_out, nb))
        return fail(CTIS_E_ARG, "f, g_out and the workspace must not overlap");
    st = on_device(F);
    if (st != CTIS_OK) return st;
    return forward(F, f, nullptr, g_out, kStoreReal, (char *)workspace, stream);
}

ctis_status ctis_fourier_adjoint(const ctis_fourier *F, const float *r, float *z_out, void *workspace,
                                 size_t workspace_bytes, void *stream) {
    if (!F) return fail(CTIS_E_ARG, "Fourier plan is NULL");
    if (!r || !z_out || !aligned4(r) || !aligned4(z_out)) return fail(CTIS_E_ARG, "r and z_out must be non-NULL and aligned");
    ctis_status st = check_ws(F, workspace, workspace_bytes);
    if (st != CTIS_OK) return st;
    const size_t mb = (size_t)F->plan->m * 4, nb = (size_t)F->n * 4;
    if (overlaps(r, nb, z_out, mb) || overlaps(workspace, F->workspace_bytes, r, nb) ||
        overlaps(workspace, F->workspace_bytes, z_out, mb))
        return fail(CTIS_E_ARG, "r, z_out and the workspace must not overlap");
    st = on_device(F);
    if (st != CTIS_OK) return st;
    return adjoint(F, r, z_out, kStoreCrop, (char *)workspace, stream);
}

ctis_status ctis_fourier_em_iterate(const ctis_fourier *F, const float *g, float *f, int32_t iters, void *workspace,
                                    size_t workspace_bytes, void *stream) {
    if (!F) return fail(CTIS_E_ARG, "Fourier plan is NULL");
    if (!g || !f || !aligned4(g) || !aligned4(f)) return fail(CTIS_E_ARG, "g and f must be non-NULL and aligned");
    if (iters < 0) return fail(CTIS_E_ARG, "iters must be >= 0");
    if (!F->nonneg) return fail(CTIS_E_NEGATIVE, "the plan has a negative calibration value");
    ctis_status st = check_ws(F, workspace, workspace_bytes);
    if (st != CTIS_OK) return st;
    const size_t mb = (size_t)F->plan->m * 4, nb = (size_t)F->n * 4;
    if (overlaps(g, nb, f, mb) || overlaps(workspace, F->workspace_bytes, f, mb) ||
        overlaps(workspace, F->workspace_bytes, g, nb))
        return fail(CTIS_E_ARG, "g, f and the workspace must not overlap");
    st = on_device(F);
    if (st != CTIS_OK) return st;
    char *ws = (char *)workspace;
    float *u = (float *)(ws + F->off_u);
    for (int32_t k = 0; k < iters && st == CTIS_OK; ++k) {
        st = forward(F, f, g, u, kStoreRatio, ws, stream);
        if (st == CTIS_OK) st = adjoint(F, u, f, kStoreUpdate, ws, stream);
    }
    return st;
}

}  // extern "C"
