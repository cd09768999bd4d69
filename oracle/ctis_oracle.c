/*
 * FP64 explicit-system-matrix oracle for CTIS EM reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the HIP implementation.
 *
 * What it computes (White, Bell & Haygood, "Accelerating computed tomographic
 * imaging spectrometer reconstruction using a parallel algorithm exploiting
 * spatial shift-invariance"):
 *
 *   Sec. 2, eq. (linear): g = H f with H of size n x m, n = gamma*xi,
 *     m = a*alpha*w.  Calibration: the image of a point source at one
 *     field-stop pixel, vectorised, is one column of H; shift-invariance gives
 *     the other columns of the same wavelength by shifting that image.
 *   Sec. 3, eq. (decomposition): H_s = C_s E, C_s the n x n circulant with
 *     first column c_s, E = [I_alpha (x) Q; 0], Q = [I_a; 0].  So column q of
 *     C_s is c_s cyclically shifted down by q (1-D, over the whole vectorised
 *     FPA), and column j' of E is the unit vector at the index the Sec. 3
 *     zero-based index map gives for j'.
 *   Sec. 2, eq. (em): f' = (f / h) . H^T (g / H f), h_j = sum_i H_ij, in the
 *     operation order of the paper's algorithm (WBH + EM): ghat = H f,
 *     u = g / ghat, zeta = H^T u, f' = (f . zeta) / h.
 *
 * Readings where the paper is silent (documented with the design notes):
 *   - u_i = 0 where ghat_i <= 0 (division by a zero projection);
 *   - f'_j = 0 where h_j == 0;
 *   - duplicate calibration entries of one wavelength add up;
 *   - "K iterations" means K multiplicative updates of the start vector.
 *
 * Arithmetic: double throughout.  OpenMP parallelises the two products over
 * rows (forward, CSR) and columns (adjoint, CSC): race-free, fixed order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int a, alpha, w, gamma, xi;
    int64_t n, ell, m;
    /* calibration vectors c_s, sparse: positions ascending, duplicates summed */
    int64_t *cptr;   /* w+1 */
    int64_t *cidx;   /* FPA index of each nonzero */
    double *cval;
    /* H column-compressed (CSC) */
    int64_t *colptr; /* m+1 */
    int32_t *rowidx;
    double *val;
    /* H row-compressed (CSR) */
    int64_t *rowptr; /* n+1 */
    int32_t *colidx;
    double *rval;
    /* column sums */
    double *h;
    int nthreads;
} oracle_t;

enum { OR_OK = 0, OR_E_ARG = 1, OR_E_INDEX = 2, OR_E_VALUE = 3, OR_E_NOMEM = 5,
       OR_E_NEGATIVE = 7 };

void oracle_free(oracle_t *o) {
    if (!o) return;
    free(o->cptr); free(o->cidx); free(o->cval);
    free(o->colptr); free(o->rowidx); free(o->val);
    free(o->rowptr); free(o->colidx); free(o->rval);
    free(o->h);
    free(o);
}

/* Sec. 3 zero-based index map, with the block offset s*n removed:
 *   i = j - s*ell + (gamma - a) * floor((j - s*ell) / a) + s*n,  s = floor(j / ell).
 * Returns i - s*n, the position of voxel j inside its length-n block of v. */
int64_t oracle_index_map(const oracle_t *o, int64_t j) {
    int64_t s = j / o->ell;
    int64_t jp = j - s * o->ell;
    return jp + (int64_t)(o->gamma - o->a) * (jp / o->a);
}

static int set_threads(const oracle_t *o) {
#ifdef _OPENMP
    return o->nthreads > 0 ? o->nthreads : omp_get_max_threads();
#else
    (void)o;
    return 1;
#endif
}

void oracle_set_threads(oracle_t *o, int nthreads) { o->nthreads = nthreads; }

int oracle_threads_used(const oracle_t *o) { return set_threads(o); }

/*
 * Build the calibration vectors and the explicit H, column by column.
 * lambda_ptr[w+1] (int64), fpa_index[] (int32, r + gamma*c), value[] (double).
 */
int oracle_create(oracle_t **out, int a, int alpha, int w, int gamma, int xi,
                  const int64_t *lambda_ptr, const int32_t *fpa_index,
                  const double *value, int build_csr) {
    *out = NULL;
    if (a < 1 || alpha < 1 || w < 1 || gamma < 1 || xi < 1) return OR_E_ARG;
    if (a > gamma || alpha > xi) return OR_E_ARG;
    int64_t n = (int64_t)gamma * xi, ell = (int64_t)a * alpha, m = ell * w;
    if (n > INT32_MAX || m > INT32_MAX) return OR_E_ARG;
    if (lambda_ptr[0] != 0) return OR_E_ARG;
    for (int s = 0; s < w; ++s)
        if (lambda_ptr[s + 1] < lambda_ptr[s]) return OR_E_ARG;
    int64_t nnz_in = lambda_ptr[w];
    for (int64_t t = 0; t < nnz_in; ++t) {
        if (fpa_index[t] < 0 || (int64_t)fpa_index[t] >= n) return OR_E_INDEX;
        if (!isfinite(value[t])) return OR_E_VALUE;
    }

    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    if (!o) return OR_E_NOMEM;
    o->a = a; o->alpha = alpha; o->w = w; o->gamma = gamma; o->xi = xi;
    o->n = n; o->ell = ell; o->m = m;

    /* O2: c_s[i_t] += v_t, accumulated densely, then kept sparse */
    double *dense = (double *)calloc((size_t)n, sizeof(double));
    o->cptr = (int64_t *)calloc((size_t)w + 1, sizeof(int64_t));
    o->cidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz_in > 0 ? nnz_in : 1));
    o->cval = (double *)malloc(sizeof(double) * (size_t)(nnz_in > 0 ? nnz_in : 1));
    if (!dense || !o->cptr || !o->cidx || !o->cval) { free(dense); oracle_free(o); return OR_E_NOMEM; }
    int64_t nc = 0;
    for (int s = 0; s < w; ++s) {
        for (int64_t t = lambda_ptr[s]; t < lambda_ptr[s + 1]; ++t)
            dense[fpa_index[t]] += value[t];
        for (int64_t i = 0; i < n; ++i) {
            if (dense[i] != 0.0) { o->cidx[nc] = i; o->cval[nc] = dense[i]; ++nc; }
            dense[i] = 0.0;
        }
        o->cptr[s + 1] = nc;
    }
    free(dense);

    /* O3: column j of H = c_s shifted by q_j (cyclic, length n) */
    o->colptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!o->colptr) { oracle_free(o); return OR_E_NOMEM; }
    o->colptr[0] = 0;
    for (int64_t j = 0; j < m; ++j) {
        int64_t s = j / ell;
        o->colptr[j + 1] = o->colptr[j] + (o->cptr[s + 1] - o->cptr[s]);
    }
    int64_t nnz = o->colptr[m];
    o->rowidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    o->val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    o->h = (double *)calloc((size_t)m, sizeof(double));
    if (!o->rowidx || !o->val || !o->h) { oracle_free(o); return OR_E_NOMEM; }
    for (int64_t j = 0; j < m; ++j) {
        int64_t s = j / ell;
        int64_t q = oracle_index_map(o, j);
        int64_t k = o->colptr[j];
        for (int64_t t = o->cptr[s]; t < o->cptr[s + 1]; ++t, ++k) {
            o->rowidx[k] = (int32_t)((o->cidx[t] + q) % n);
            o->val[k] = o->cval[t];
        }
    }
    /* O4: h_j = sum_i H_ij, from the assembled columns */
    for (int64_t j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int64_t k = o->colptr[j]; k < o->colptr[j + 1]; ++k) acc += o->val[k];
        o->h[j] = acc;
    }

    if (build_csr) {
        o->rowptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        o->colidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
        o->rval = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        if (!o->rowptr || !o->colidx || !o->rval) { oracle_free(o); return OR_E_NOMEM; }
        for (int64_t k = 0; k < nnz; ++k) o->rowptr[o->rowidx[k] + 1]++;
        for (int64_t i = 0; i < n; ++i) o->rowptr[i + 1] += o->rowptr[i];
        int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        if (!pos) { oracle_free(o); return OR_E_NOMEM; }
        memcpy(pos, o->rowptr, sizeof(int64_t) * (size_t)n);
        for (int64_t j = 0; j < m; ++j)
            for (int64_t k = o->colptr[j]; k < o->colptr[j + 1]; ++k) {
                int64_t p = pos[o->rowidx[k]]++;
                o->colidx[p] = (int32_t)j;
                o->rval[p] = o->val[k];
            }
        free(pos);
    }
    o->nthreads = 0;
    *out = o;
    return OR_OK;
}

int64_t oracle_nnz(const oracle_t *o) { return o->colptr[o->m]; }

/* copy out the CSC arrays (for comparison against dense constructions) */
void oracle_export_csc(const oracle_t *o, int64_t *colptr, int32_t *rowidx, double *val) {
    memcpy(colptr, o->colptr, sizeof(int64_t) * (size_t)(o->m + 1));
    int64_t nnz = o->colptr[o->m];
    memcpy(rowidx, o->rowidx, sizeof(int32_t) * (size_t)nnz);
    memcpy(val, o->val, sizeof(double) * (size_t)nnz);
}

void oracle_colsums(const oracle_t *o, double *h) {
    memcpy(h, o->h, sizeof(double) * (size_t)o->m);
}

/* O5: ghat = H f (rows of H, one output per row: race-free) */
int oracle_forward(const oracle_t *o, const double *f, double *g) {
    if (!o->rowptr) return OR_E_ARG;
    int nt = set_threads(o);
    int64_t n = o->n;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t k = o->rowptr[i]; k < o->rowptr[i + 1]; ++k)
            acc += o->rval[k] * f[o->colidx[k]];
        g[i] = acc;
    }
    return OR_OK;
}

/* O5: z = H^T r (columns of H) */
int oracle_adjoint(const oracle_t *o, const double *r, double *z) {
    int nt = set_threads(o);
    int64_t m = o->m;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int64_t k = o->colptr[j]; k < o->colptr[j + 1]; ++k)
            acc += o->val[k] * r[o->rowidx[k]];
        z[j] = acc;
    }
    return OR_OK;
}

/* O7: flux sum_j h_j f_j; Poisson log-likelihood sum_i (g_i log ghat_i - ghat_i)
 * (a term with g_i = 0 contributes -ghat_i; g_i > 0 with ghat_i <= 0 gives -inf). */
void oracle_diagnostics(const oracle_t *o, const double *g, const double *f,
                        const double *ghat, double *flux, double *loglik) {
    double fl = 0.0;
    for (int64_t j = 0; j < o->m; ++j) fl += o->h[j] * f[j];
    double L = 0.0;
    for (int64_t i = 0; i < o->n; ++i) {
        if (g[i] > 0.0) {
            if (ghat[i] <= 0.0) { L = -INFINITY; break; }
            L += g[i] * log(ghat[i]) - ghat[i];
        } else {
            L -= ghat[i];
        }
    }
    *flux = fl;
    *loglik = L;
}

/*
 * O6: K EM iterations in place on f (Sec. 3 algorithm, WBH + EM, with the
 * projections done by the explicit matrix).  If trace is non-null it receives
 * 2*K values: (flux of f^(k+1), loglik of f^(k)) per iteration.
 */
int oracle_em(const oracle_t *o, const double *g, double *f, int iters, double *trace) {
    if (iters < 0) return OR_E_ARG;
    for (int64_t t = 0; t < o->cptr[o->w]; ++t)
        if (o->cval[t] < 0.0) return OR_E_NEGATIVE;
    double *ghat = (double *)malloc(sizeof(double) * (size_t)o->n);
    double *u = (double *)malloc(sizeof(double) * (size_t)o->n);
    double *zeta = (double *)malloc(sizeof(double) * (size_t)o->m);
    if (!ghat || !u || !zeta) { free(ghat); free(u); free(zeta); return OR_E_NOMEM; }
    for (int k = 0; k < iters; ++k) {
        oracle_forward(o, f, ghat);                       /* g^(k) = H f^(k) */
        for (int64_t i = 0; i < o->n; ++i)                /* u = g / g^(k)   */
            u[i] = ghat[i] > 0.0 ? g[i] / ghat[i] : 0.0;
        double L = 0.0, fl = 0.0;
        if (trace) oracle_diagnostics(o, g, f, ghat, &fl, &L);
        oracle_adjoint(o, u, zeta);                       /* zeta = H^T u    */
        for (int64_t j = 0; j < o->m; ++j)                /* f = (f . zeta) / h */
            f[j] = o->h[j] != 0.0 ? (f[j] * zeta[j]) / o->h[j] : 0.0;
        if (trace) {
            double fl2 = 0.0;
            for (int64_t j = 0; j < o->m; ++j) fl2 += o->h[j] * f[j];
            trace[2 * k] = fl2;
            trace[2 * k + 1] = L;
        }
    }
    free(ghat); free(u); free(zeta);
    return OR_OK;
}

/*
 * The simultaneous forms of the other two solvers Sec. 2 names (MART and
 * ART, cited there to Gordon, Bender and Herman), built from the same two
 * products.  The cited methods correct one ray (one row of H) at a time;
 * here every ray's correction is applied at once, each voxel taking the
 * H-weighted mean of the corrections of the rays through it:
 *
 *   SMART (multiplicative):  ghat = H f,
 *     l_i = log(g_i / ghat_i)          (0 where g_i <= 0 or ghat_i <= 0),
 *     f'_j = f_j exp((H^T l)_j / h_j)  (0 where h_j == 0);
 *   SART (additive, kept nonnegative), relaxation lam:  ghat = H f,
 *     R = H 1 (row sums of H),
 *     r_i = (g_i - ghat_i) / R_i        (0 where R_i == 0),
 *     f'_j = max(0, f_j + lam (H^T r)_j / h_j)   (0 where h_j == 0).
 *
 * The zero rules follow those of EM (a ray with no data or no projection
 * carries no information).  g[n], f[m] in double, f updated in place.
 */
int oracle_smart(const oracle_t *o, const double *g, double *f, int iters) {
    if (!o->rowptr || iters < 0) return OR_E_ARG;
    for (int64_t t = 0; t < o->cptr[o->w]; ++t)
        if (o->cval[t] < 0.0) return OR_E_NEGATIVE;
    double *ghat = (double *)malloc(sizeof(double) * (size_t)o->n);
    double *l = (double *)malloc(sizeof(double) * (size_t)o->n);
    double *z = (double *)malloc(sizeof(double) * (size_t)o->m);
    if (!ghat || !l || !z) { free(ghat); free(l); free(z); return OR_E_NOMEM; }
    for (int k = 0; k < iters; ++k) {
        oracle_forward(o, f, ghat);
        for (int64_t i = 0; i < o->n; ++i)
            l[i] = (g[i] > 0.0 && ghat[i] > 0.0) ? log(g[i] / ghat[i]) : 0.0;
        oracle_adjoint(o, l, z);
        for (int64_t j = 0; j < o->m; ++j)
            f[j] = o->h[j] != 0.0 ? f[j] * exp(z[j] / o->h[j]) : 0.0;
    }
    free(ghat); free(l); free(z);
    return OR_OK;
}

int oracle_sart(const oracle_t *o, const double *g, double *f, int iters, double lam) {
    if (!o->rowptr || iters < 0) return OR_E_ARG;
    double *ghat = (double *)malloc(sizeof(double) * (size_t)o->n);
    double *R = (double *)malloc(sizeof(double) * (size_t)o->n);
    double *r = (double *)malloc(sizeof(double) * (size_t)o->n);
    double *z = (double *)malloc(sizeof(double) * (size_t)o->m);
    double *one = (double *)malloc(sizeof(double) * (size_t)o->m);
    if (!ghat || !R || !r || !z || !one) {
        free(ghat); free(R); free(r); free(z); free(one);
        return OR_E_NOMEM;
    }
    for (int64_t j = 0; j < o->m; ++j) one[j] = 1.0;
    oracle_forward(o, one, R);                            /* R = H 1 */
    for (int k = 0; k < iters; ++k) {
        oracle_forward(o, f, ghat);
        for (int64_t i = 0; i < o->n; ++i)
            r[i] = R[i] != 0.0 ? (g[i] - ghat[i]) / R[i] : 0.0;
        oracle_adjoint(o, r, z);
        for (int64_t j = 0; j < o->m; ++j) {
            const double v = o->h[j] != 0.0 ? f[j] + lam * z[j] / o->h[j] : 0.0;
            f[j] = v > 0.0 ? v : 0.0;
        }
    }
    free(ghat); free(R); free(r); free(z); free(one);
    return OR_OK;
}

/*
 * Single rows / columns of H straight from the definition, without the
 * assembled matrix (for sampled checks at sizes where assembly is too big):
 *   row i:    (H f)_i = sum_s sum_t c_s[t] * f_s(E^{-1}((i - t) mod n)),
 *             E^{-1}(p) = (p mod gamma, p div gamma) when inside the field stop;
 *   column j: (H^T r)_j = sum_t c_s[t] * r[(t + q_j) mod n].
 * These need only the calibration vectors (build with oracle_create(...,0)
 * still assembles H; oracle_create_kernels_only skips it).
 */
int oracle_create_kernels_only(oracle_t **out, int a, int alpha, int w, int gamma, int xi,
                               const int64_t *lambda_ptr, const int32_t *fpa_index,
                               const double *value) {
    *out = NULL;
    if (a < 1 || alpha < 1 || w < 1 || gamma < 1 || xi < 1) return OR_E_ARG;
    if (a > gamma || alpha > xi) return OR_E_ARG;
    int64_t n = (int64_t)gamma * xi, ell = (int64_t)a * alpha, m = ell * w;
    if (n > INT32_MAX || m > INT32_MAX) return OR_E_ARG;
    if (lambda_ptr[0] != 0) return OR_E_ARG;
    int64_t nnz_in = lambda_ptr[w];
    for (int64_t t = 0; t < nnz_in; ++t) {
        if (fpa_index[t] < 0 || (int64_t)fpa_index[t] >= n) return OR_E_INDEX;
        if (!isfinite(value[t])) return OR_E_VALUE;
    }
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    if (!o) return OR_E_NOMEM;
    o->a = a; o->alpha = alpha; o->w = w; o->gamma = gamma; o->xi = xi;
    o->n = n; o->ell = ell; o->m = m;
    double *dense = (double *)calloc((size_t)n, sizeof(double));
    o->cptr = (int64_t *)calloc((size_t)w + 1, sizeof(int64_t));
    o->cidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz_in > 0 ? nnz_in : 1));
    o->cval = (double *)malloc(sizeof(double) * (size_t)(nnz_in > 0 ? nnz_in : 1));
    if (!dense || !o->cptr || !o->cidx || !o->cval) { free(dense); oracle_free(o); return OR_E_NOMEM; }
    int64_t nc = 0;
    for (int s = 0; s < w; ++s) {
        for (int64_t t = lambda_ptr[s]; t < lambda_ptr[s + 1]; ++t)
            dense[fpa_index[t]] += value[t];
        for (int64_t t = lambda_ptr[s]; t < lambda_ptr[s + 1]; ++t) {
            int64_t i = fpa_index[t];
            if (dense[i] != 0.0) { o->cidx[nc] = i; o->cval[nc] = dense[i]; ++nc; dense[i] = 0.0; }
            else dense[i] = 0.0;
        }
        o->cptr[s + 1] = nc;
    }
    free(dense);
    *out = o;
    return OR_OK;
}

void oracle_forward_rows(const oracle_t *o, const double *f, const int64_t *rows,
                         int64_t nrows, double *out) {
    int nt = set_threads(o);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        double acc = 0.0;
        for (int s = 0; s < o->w; ++s)
            for (int64_t t = o->cptr[s]; t < o->cptr[s + 1]; ++t) {
                int64_t p = ((i - o->cidx[t]) % o->n + o->n) % o->n;
                int64_t x = p % o->gamma, y = p / o->gamma;
                if (x < o->a && y < o->alpha)
                    acc += o->cval[t] * f[(int64_t)s * o->ell + x + (int64_t)o->a * y];
            }
        out[k] = acc;
    }
}

void oracle_adjoint_cols(const oracle_t *o, const double *r, const int64_t *cols,
                         int64_t ncols, double *out) {
    int nt = set_threads(o);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t k = 0; k < ncols; ++k) {
        int64_t j = cols[k];
        int64_t s = j / o->ell;
        int64_t q = oracle_index_map(o, j);
        double acc = 0.0;
        for (int64_t t = o->cptr[s]; t < o->cptr[s + 1]; ++t)
            acc += o->cval[t] * r[(o->cidx[t] + q) % o->n];
        out[k] = acc;
    }
}

/* merged calibration vectors (positions and summed values), for tests */
int64_t oracle_cal_nnz(const oracle_t *o) { return o->cptr[o->w]; }
void oracle_export_cal(const oracle_t *o, int64_t *cptr, int64_t *cidx, double *cval) {
    memcpy(cptr, o->cptr, sizeof(int64_t) * (size_t)(o->w + 1));
    memcpy(cidx, o->cidx, sizeof(int64_t) * (size_t)o->cptr[o->w]);
    memcpy(cval, o->cval, sizeof(double) * (size_t)o->cptr[o->w]);
}

/*
 * Reverse-mode derivative of one EM step (Sec. 2 eq. (em), stage order of the
 * Sec. 3 algorithm), for a scalar loss L of the step's output f':
 *
 *   forward stages:  ghat = H f,  u_i = g_i / ghat_i (0 where ghat_i <= 0),
 *                    zeta = H^T u,  f'_j = f_j zeta_j / h_j (0 where h_j = 0),
 *                    with H_ij = c_s[(i - q_j) mod n] for voxel j of wavelength
 *                    s (Sec. 3, H_s = C_s E) and h_j = sum_i H_ij.
 *   given y = dL/df', the stages are differentiated last to first:
 *     f' stage:  b_j = dL/dzeta_j = y_j f_j / h_j,  dL/df_j = y_j zeta_j / h_j,
 *                hbar_j = dL/dh_j = -y_j f'_j / h_j   (all 0 where h_j = 0);
 *     zeta stage: dL/du = H b,  dL/dH_ij += u_i b_j;
 *     u stage:   e_i = dL/dghat_i = -(H b)_i g_i / ghat_i^2   (0 where ghat_i <= 0);
 *     ghat stage: dL/df += H^T e,  dL/dH_ij += e_i f_j;
 *     H from the calibration vectors: dL/dc_s[p] = sum over the voxels j of
 *                wavelength s of (dL/dH_{(p + q_j) mod n, j} + hbar_j),
 *                because H_ij is c_s[p] exactly at i = (p + q_j) mod n and
 *                every column sum h_j of wavelength s holds c_s[p] once.
 *
 * Inputs g[n], f[m] (the step's input), y[m].  Outputs df[m] = dL/df and, for
 * npos requested calibration positions (pos_lambda[k], pos_index[k]),
 * dv[k] = dL/dc_s[p].  dv may be NULL when npos = 0.
 */
int oracle_em_vjp(const oracle_t *o, const double *g, const double *f, const double *y,
                  double *df, int64_t npos, const int32_t *pos_lambda, const int64_t *pos_index,
                  double *dv) {
    if (!o->rowptr || npos < 0) return OR_E_ARG;
    for (int64_t k = 0; k < npos; ++k)
        if (pos_lambda[k] < 0 || pos_lambda[k] >= o->w || pos_index[k] < 0 || pos_index[k] >= o->n)
            return OR_E_INDEX;
    const int64_t n = o->n, m = o->m;
    double *ghat = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *Hb = (double *)malloc(sizeof(double) * (size_t)n);
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    double *zeta = (double *)malloc(sizeof(double) * (size_t)m);
    double *b = (double *)malloc(sizeof(double) * (size_t)m);
    double *hbar = (double *)malloc(sizeof(double) * (size_t)m);
    double *Hte = (double *)malloc(sizeof(double) * (size_t)m);
    if (!ghat || !u || !Hb || !e || !zeta || !b || !hbar || !Hte) {
        free(ghat); free(u); free(Hb); free(e); free(zeta); free(b); free(hbar); free(Hte);
        return OR_E_NOMEM;
    }
    /* forward stages, recomputed from the step's input */
    oracle_forward(o, f, ghat);
    for (int64_t i = 0; i < n; ++i) u[i] = ghat[i] > 0.0 ? g[i] / ghat[i] : 0.0;
    oracle_adjoint(o, u, zeta);
    /* f' stage */
    for (int64_t j = 0; j < m; ++j) {
        if (o->h[j] != 0.0) {
            const double fnew = f[j] * zeta[j] / o->h[j];
            b[j] = y[j] * f[j] / o->h[j];
            df[j] = y[j] * zeta[j] / o->h[j];
            hbar[j] = -y[j] * fnew / o->h[j];
        } else {
            b[j] = 0.0;
            df[j] = 0.0;
            hbar[j] = 0.0;
        }
    }
    /* zeta stage and u stage */
    oracle_forward(o, b, Hb);
    for (int64_t i = 0; i < n; ++i) e[i] = ghat[i] > 0.0 ? -Hb[i] * g[i] / (ghat[i] * ghat[i]) : 0.0;
    /* ghat stage */
    oracle_adjoint(o, e, Hte);
    for (int64_t j = 0; j < m; ++j) df[j] += Hte[j];
    /* calibration values, from the entries of H they appear in */
    int nt = set_threads(o);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t k = 0; k < npos; ++k) {
        const int64_t s = pos_lambda[k], p = pos_index[k];
        double acc = 0.0;
        for (int64_t j = s * o->ell; j < (s + 1) * o->ell; ++j) {
            const int64_t i = (p + oracle_index_map(o, j)) % n;
            acc += u[i] * b[j] + e[i] * f[j] + hbar[j];
        }
        dv[k] = acc;
    }
    free(ghat); free(u); free(Hb); free(e); free(zeta); free(b); free(hbar); free(Hte);
    return OR_OK;
}

/*
 * O8, the FP32 drift probe -- NOT the oracle.  The same EM iteration as
 * oracle_em (Sec. 2 eq. (em), in the order of the Sec. 3 algorithm) with
 * float storage and float accumulation: the assembled H's values rounded to
 * float, products summed in float along each row (forward) and each column
 * (adjoint) of H.  Its distance from oracle_em shows how much of a tolerance
 * float rounding alone uses after K iterations; a GPU sums the same terms in
 * another order, so it is an estimate of the floor, not a bound.
 * g[n] and f[m] are float; f is updated in place.
 */
int oracle_em_f32(const oracle_t *o, const float *g, float *f, int iters) {
    if (!o->rowptr || iters < 0) return OR_E_ARG;
    for (int64_t t = 0; t < o->cptr[o->w]; ++t)
        if (o->cval[t] < 0.0) return OR_E_NEGATIVE;
    const int64_t n = o->n, m = o->m, nnz = o->colptr[o->m];
    float *rv = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float *cv = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float *h = (float *)malloc(sizeof(float) * (size_t)m);
    float *ghat = (float *)malloc(sizeof(float) * (size_t)n);
    float *u = (float *)malloc(sizeof(float) * (size_t)n);
    float *zeta = (float *)malloc(sizeof(float) * (size_t)m);
    if (!rv || !cv || !h || !ghat || !u || !zeta) {
        free(rv); free(cv); free(h); free(ghat); free(u); free(zeta);
        return OR_E_NOMEM;
    }
    int nt = set_threads(o);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t k = 0; k < nnz; ++k) {
        rv[k] = (float)o->rval[k];
        cv[k] = (float)o->val[k];
    }
    for (int64_t j = 0; j < m; ++j) h[j] = (float)o->h[j];
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t i = 0; i < n; ++i) {
            float acc = 0.0f;
            for (int64_t k = o->rowptr[i]; k < o->rowptr[i + 1]; ++k) acc += rv[k] * f[o->colidx[k]];
            ghat[i] = acc;
            u[i] = acc > 0.0f ? g[i] / acc : 0.0f;
        }
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t j = 0; j < m; ++j) {
            float acc = 0.0f;
            for (int64_t k = o->colptr[j]; k < o->colptr[j + 1]; ++k) acc += cv[k] * u[o->rowidx[k]];
            zeta[j] = acc;
        }
        for (int64_t j = 0; j < m; ++j) f[j] = h[j] != 0.0f ? (f[j] * zeta[j]) / h[j] : 0.0f;
    }
    free(rv); free(cv); free(h); free(ghat); free(u); free(zeta);
    return OR_OK;
}
