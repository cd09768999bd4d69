// The Fourier (WBH) form of the projections for gfx950: the circulant
// blocks C_s are diagonalised by the length-n DFT over the vectorised FPA
// (White, Bell & Haygood, Sec. 3 eqs. (forward) and (backwards)).
//
// Two wavelengths share one complex sequence.  With e_t = F(c_{2t} - i c_{2t+1})
// (computed once per plan) and v_s = E f_s:
//   forward:  ghat = Re F^-1( sum_t e_t . F(v_{2t} + i v_{2t+1}) ) / n
//             (the imaginary cross terms c_{2t} * v_{2t+1} - c_{2t+1} * v_{2t}
//             fall into the imaginary part);
//   adjoint:  F^-1( conj(e_t) . F(u) ) / n = C_{2t}^T u + i C_{2t+1}^T u.
// Per EM iteration that is w/2 + 1 forward and w/2 + 1 inverse complex FFTs
// of length n -- the work of the paper's 2w + 2 real FFTs.
//
// FFT: n = N1 N2 (four-step).  Pass A: N2 transforms of length N1 over the
// strided sequences x[N2 n1 + n2], each output multiplied by w_N^(n2 k1),
// written to Y[n2 + N2 k1]; pass B: N1 transforms of length N2 over the rows
// of Y, written in natural order X[k1 + N1 k2].  A workgroup holds S
// sequences (S L = 8192 complex values when many transforms run together, 4
// sequences for a single transform) laid out [element][seq], loads them so
// that consecutive lanes touch consecutive addresses, applies the log2 L
// radix-2 stages in place after a bit-reversed load -- three at a time, in
// registers, with the stage twiddles staged in LDS -- and stores the same
// way.  Loads and stores carry the pipeline's own
// steps (embedding E f, the products conj(e_t) U, the ratio g / ghat, the
// crop E^T and the EM update); the sum over pairs of the forward's spectral
// products is one elementwise kernel.  Twiddles come from tables computed in
// double on the host.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fourier_internal.h"

namespace ctis {
namespace fourier {
namespace {

constexpr int kFftThreads = 512;   // threads per FFT-pass workgroup

struct C2 {
    float x, y;
};

__device__ __forceinline__ C2 cmul(C2 a, C2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ C2 cmulc(C2 a, C2 b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }  // conj(a) b

// (a, b) <- (a + w b, a - w b): one radix-2 butterfly of the decimation in time
__device__ __forceinline__ void bfly(C2 &a, C2 &b, C2 w) {
    const C2 t = cmul(b, w);
    b = {a.x - t.x, a.y - t.y};
    a = {a.x + t.x, a.y + t.y};
}

__device__ __forceinline__ C2 ld(const float2 *buf, int i, int S, int s) {
    const float2 v = buf[i * S + s];
    return {v.x, v.y};
}

__device__ __forceinline__ void st(float2 *buf, int i, int S, int s, C2 v) { buf[i * S + s] = make_float2(v.x, v.y); }

__device__ __forceinline__ C2 tw(const float2 *t, int j, int inverse) {
    const float2 v = t[j];
    return {v.x, inverse ? -v.y : v.y};
}

// Element i (natural index of the length-n sequence) of batch `bt` under the load mode.
__device__ __forceinline__ C2 load_elem(const Pass &P, int bt, long long i) {
    switch (P.load) {
        case kLoadEmbedPair:
        case kLoadCalPair: {
            const int s0 = 2 * bt, s1 = 2 * bt + 1;
            if (P.load == kLoadCalPair) {
                const float a = P.fin[(long long)s0 * P.n + i];
                const float b = s1 < P.geo.w ? P.fin[(long long)s1 * P.n + i] : 0.0f;
                return {a, -b};
            }
            const int r = (int)(i & (P.geo.gamma - 1)), c = (int)(i >> P.geo.log_gamma);
            if (r >= P.geo.a || c >= P.geo.alpha) return {0.0f, 0.0f};
            const long long j = r + (long long)P.geo.a * c;
            const float a = P.fin[(long long)s0 * P.geo.ell + j];
            const float b = s1 < P.geo.w ? P.fin[(long long)s1 * P.geo.ell + j] : 0.0f;
            return {a, b};
        }
        case kLoadReal:
            return {P.fin[i], 0.0f};
        case kLoadConjE: {
            const float2 ev = P.e[(long long)bt * P.n + i], uv = P.in[i];
            return cmulc({ev.x, ev.y}, {uv.x, uv.y});
        }
        default: {
            const float2 v = P.in[(long long)bt * P.n + i];
            return {v.x, v.y};
        }
    }
}

__device__ __forceinline__ void store_elem(const Pass &P, int bt, long long k, C2 v) {
    const float inv_n = 1.0f / (float)P.n;
    switch (P.store) {
        case kStoreReal:
            P.fout[k] = v.x * inv_n;
            return;
        case kStoreRatio: {
            const float gh = v.x * inv_n;
            P.fout[k] = gh > 0.0f ? P.g[k] / gh : 0.0f;
            return;
        }
        case kStoreCrop:
        case kStoreUpdate: {
            const int r = (int)(k & (P.geo.gamma - 1)), c = (int)(k >> P.geo.log_gamma);
            if (r >= P.geo.a || c >= P.geo.alpha) return;
            const long long j = r + (long long)P.geo.a * c;
            const int s0 = 2 * bt, s1 = 2 * bt + 1;
            const float z0 = v.x * inv_n, z1 = v.y * inv_n;
            float *f0 = P.fout + (long long)s0 * P.geo.ell + j;
            if (P.store == kStoreCrop) {
                *f0 = z0;
                if (s1 < P.geo.w) P.fout[(long long)s1 * P.geo.ell + j] = z1;
            } else {
                const float h0 = P.h[s0];
                *f0 = h0 != 0.0f ? (*f0 * z0) / h0 : 0.0f;
                if (s1 < P.geo.w) {
                    float *f1 = P.fout + (long long)s1 * P.geo.ell + j;
                    const float h1 = P.h[s1];
                    *f1 = h1 != 0.0f ? (*f1 * z1) / h1 : 0.0f;
                }
            }
            return;
        }
        default:
            P.out[(long long)bt * P.n + k] = make_float2(v.x, v.y);
    }
}

// One pass over S sequences of length L = 2^LOGL.  LDS: the S L values
// [element][sequence], then the L/2 stage twiddles.
template <int LOGL, int S>
__global__ void __launch_bounds__(kFftThreads) k_fft_pass(const Pass P) {
    constexpr int L = 1 << LOGL;
    constexpr int TOTAL = S * L;
    extern __shared__ float2 lds[];
    float2 *buf = lds;
    float2 *twl = lds + TOTAL;
    const int bt = blockIdx.y;
    const int seq0 = blockIdx.x * S;
    for (int j = threadIdx.x; j < L / 2; j += kFftThreads) {
        const float2 t = P.tw_stage[j];
        twl[j] = make_float2(t.x, P.inverse ? -t.y : t.y);
    }
    // pass A: sequence = column n2 (addresses N2 n1 + n2: consecutive seqs
    // are consecutive); pass B: sequence = row k1 (addresses N2 k1 + n2:
    // consecutive elements are consecutive)
#pragma unroll 4
    for (int idx = threadIdx.x; idx < TOTAL; idx += kFftThreads) {
        int s, j;
        if (P.pass_a) {
            s = idx % S;
            j = idx / S;
        } else {
            j = idx % L;
            s = idx / L;
        }
        const int sq = seq0 + s;
        C2 v = {0.0f, 0.0f};
        if (sq < P.n_seq) {
            if (P.pass_a) {
                v = load_elem(P, bt, (long long)P.N2 * j + sq);
            } else {
                const float2 t = P.in[(long long)bt * P.n + (long long)P.N2 * sq + j];
                v = {t.x, t.y};
            }
        }
        const int jr = (int)(__builtin_bitreverse32((unsigned)j) >> (32 - LOGL));
        buf[jr * S + s] = make_float2(v.x, v.y);
    }
    __syncthreads();
    // the log2 L radix-2 stages, three at a time (radix 8) after one radix-2
    // or radix-4 step for the remainder of log2 L mod 3: LOGL = 9 takes three
    // round trips through LDS, LOGL = 10 four
    constexpr int REM = LOGL % 3;
    if (REM == 1) {
#pragma unroll 4
        for (int b = threadIdx.x; b < (L / 2) * S; b += kFftThreads) {
            const int s = b % S, i0 = 2 * (b / S), i1 = i0 + 1;
            const float2 a = buf[i0 * S + s], c = buf[i1 * S + s];
            buf[i0 * S + s] = make_float2(a.x + c.x, a.y + c.y);
            buf[i1 * S + s] = make_float2(a.x - c.x, a.y - c.y);
        }
        __syncthreads();
    }
    if (REM == 2) {
        // stages of half 1 and 2: each thread takes a block of 4
#pragma unroll 2
        for (int b = threadIdx.x; b < (L / 4) * S; b += kFftThreads) {
            const int s = b % S, i0 = 4 * (b / S);
            const float2 w3 = twl[L / 4];   // w_4^1
            C2 a0 = ld(buf, i0, S, s), a1 = ld(buf, i0 + 1, S, s), a2 = ld(buf, i0 + 2, S, s),
               a3 = ld(buf, i0 + 3, S, s);
            bfly(a0, a1, {1.0f, 0.0f});
            bfly(a2, a3, {1.0f, 0.0f});
            bfly(a0, a2, {1.0f, 0.0f});
            bfly(a1, a3, {w3.x, w3.y});
            st(buf, i0, S, s, a0);
            st(buf, i0 + 1, S, s, a1);
            st(buf, i0 + 2, S, s, a2);
            st(buf, i0 + 3, S, s, a3);
        }
        __syncthreads();
    }
    // stages of half h, 2h and 4h in registers: each thread takes
    // i_k = 8h-block + m + k h (k < 8); twiddles w_2h^m, w_4h^(m + {0,h}),
    // w_8h^(m + {0,h,2h,3h}), all powers of w_L from the staged table
#pragma unroll
    for (int lh = REM; lh + 2 < LOGL; lh += 3) {
        const int h = 1 << lh;
#pragma unroll 2
        for (int b = threadIdx.x; b < (L / 8) * S; b += kFftThreads) {
            const int s = b % S, p = b / S;
            const int m = p & (h - 1);
            const int i0 = (p - m) * 8 + m;
            const int q1 = L / (2 * h), q2 = L / (4 * h), q3 = L / (8 * h);
            C2 x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = ld(buf, i0 + k * h, S, s);
            const float2 t1 = twl[m * q1];
            const C2 w1 = {t1.x, t1.y};
#pragma unroll
            for (int k = 0; k < 8; k += 2) bfly(x[k], x[k + 1], w1);
            const float2 t20 = twl[m * q2], t21 = twl[(m + h) * q2];
            const C2 w20 = {t20.x, t20.y}, w21 = {t21.x, t21.y};
            bfly(x[0], x[2], w20);
            bfly(x[1], x[3], w21);
            bfly(x[4], x[6], w20);
            bfly(x[5], x[7], w21);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float2 t3 = twl[(m + k * h) * q3];
                bfly(x[k], x[k + 4], {t3.x, t3.y});
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) st(buf, i0 + k * h, S, s, x[k]);
        }
        __syncthreads();
    }
    // pass A: Y[n2 + N2 k1] = X1[k1] w_N^(n2 k1) (consecutive seqs consecutive);
    // pass B: X[k1 + N1 k2] (consecutive seqs = rows k1 consecutive)
#pragma unroll 4
    for (int idx = threadIdx.x; idx < TOTAL; idx += kFftThreads) {
        const int s = idx % S, k = idx / S;
        const int sq = seq0 + s;
        if (sq >= P.n_seq) continue;
        const float2 t = buf[k * S + s];
        C2 v = {t.x, t.y};
        if (P.pass_a) {
            const long long e = ((long long)sq * k) & (P.n - 1);
            const C2 w = cmul(tw(P.tw_hi, (int)(e >> P.log_n2), P.inverse),
                              tw(P.tw_lo, (int)(e & (P.N2 - 1)), P.inverse));
            v = cmul(v, w);
            P.out[(long long)bt * P.n + sq + (long long)P.N2 * k] = make_float2(v.x, v.y);
        } else {
            store_elem(P, bt, sq + (long long)P.N1 * k, v);
        }
    }
}

// G[k] = sum_t e_t[k] X_t[k]: the spectral products of the forward
// projection, summed over the wavelength pairs (fixed order).
__global__ void __launch_bounds__(256) k_combine(const float2 *__restrict__ e, const float2 *__restrict__ X,
                                                 float2 *__restrict__ G, int pairs, long long n) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    C2 acc = {0.0f, 0.0f};
    for (int t = 0; t < pairs; ++t) {
        const float2 ev = e[(long long)t * n + k], xv = X[(long long)t * n + k];
        const C2 p = cmul({ev.x, ev.y}, {xv.x, xv.y});
        acc.x += p.x;
        acc.y += p.y;
    }
    G[k] = make_float2(acc.x, acc.y);
}

template <int LOGL, int S>
int launch_ls(const Pass &P, int batches, hipStream_t st) {
    constexpr int L = 1 << LOGL;
    const size_t lds = ((size_t)S * L + L / 2) * sizeof(float2);
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [lds]() {
        if (lds > 65536)
            attr = hipFuncSetAttribute((const void *)k_fft_pass<LOGL, S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    });
    if (attr != hipSuccess) return (int)attr;
    const int groups = (P.n_seq + S - 1) / S;
    hipLaunchKernelGGL((k_fft_pass<LOGL, S>), dim3(groups, batches), dim3(kFftThreads), lds, st, P);
    return (int)hipGetLastError();
}

// Sequences per workgroup: S L = 8192 values (64 KB, two workgroups per
// compute unit; S = 8 at L = 1024 makes the strided accesses of the column
// pass 64-byte segments) for batched passes; 4 for a single transform, so
// that it still spreads over the chip.  (Measured on c2/c3 frames against
// 4096 values with 256 threads: c3 forward 579 -> 455 us, adjoint
// 640 -> 491 us; 8192 values with 256 threads was slower than either.)
template <int LOGL>
int launch_l(const Pass &P, int batches, bool few, hipStream_t st) {
    constexpr int SB = (8192 >> LOGL) > 32 ? 32 : ((8192 >> LOGL) < 1 ? 1 : (8192 >> LOGL));
    constexpr int SS = SB < 4 ? SB : 4;
    return few ? launch_ls<LOGL, SS>(P, batches, st) : launch_ls<LOGL, SB>(P, batches, st);
}

}  // namespace

int launch_pass(const Pass &P, int batches, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const bool few = (long long)P.n_seq * batches < 4096;
    switch (P.log_l) {
        case 2: return launch_l<2>(P, batches, few, st);
        case 3: return launch_l<3>(P, batches, few, st);
        case 4: return launch_l<4>(P, batches, few, st);
        case 5: return launch_l<5>(P, batches, few, st);
        case 6: return launch_l<6>(P, batches, few, st);
        case 7: return launch_l<7>(P, batches, few, st);
        case 8: return launch_l<8>(P, batches, few, st);
        case 9: return launch_l<9>(P, batches, few, st);
        case 10: return launch_l<10>(P, batches, few, st);
    }
    return (int)hipErrorInvalidValue;
}

int launch_combine(const float2 *e, const float2 *X, float2 *G, int pairs, long long n, void *stream) {
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, e, X, G,
                       pairs, n);
    return (int)hipGetLastError();
}

}  // namespace fourier
}  // namespace ctis
