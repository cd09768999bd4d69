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
// sequences (S L <= 8192 complex values, 64 KB of LDS) laid out [element][seq],
// loads them so that consecutive lanes touch consecutive addresses, applies
// log2 L radix-2 stages in place after a bit-reversed load, and stores the
// same way.  Loads and stores carry the pipeline's own steps (embedding E f,
// the spectral products, the ratio g / ghat, the crop E^T and the EM update)
// so that no separate elementwise pass touches HBM.  Twiddles come from
// tables computed in double on the host.
#include <hip/hip_runtime.h>

#include "fourier_internal.h"

namespace ctis {
namespace fourier {
namespace {

struct C2 {
    float x, y;
};

__device__ __forceinline__ C2 cmul(C2 a, C2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ C2 cmulc(C2 a, C2 b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }  // conj(a) b

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
            const int r = (int)(i % P.geo.gamma), c = (int)(i / P.geo.gamma);
            if (r >= P.geo.a || c >= P.geo.alpha) return {0.0f, 0.0f};
            const long long j = r + (long long)P.geo.a * c;
            const float a = P.fin[(long long)s0 * P.geo.ell + j];
            const float b = s1 < P.geo.w ? P.fin[(long long)s1 * P.geo.ell + j] : 0.0f;
            return {a, b};
        }
        case kLoadReal:
            return {P.fin[i], 0.0f};
        case kLoadCombine: {
            C2 acc = {0.0f, 0.0f};
            for (int t = 0; t < P.pairs; ++t) {
                const float2 ev = P.e[(long long)t * P.n + i], xv = P.in[(long long)t * P.n + i];
                const C2 p = cmul({ev.x, ev.y}, {xv.x, xv.y});
                acc.x += p.x;
                acc.y += p.y;
            }
            return acc;
        }
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
            const int r = (int)(k % P.geo.gamma), c = (int)(k / P.geo.gamma);
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

__global__ void __launch_bounds__(256) k_fft_pass(const Pass P) {
    extern __shared__ float2 buf[];   // [element][sequence], S L values
    const int S = P.S, L = P.L;
    const int bt = blockIdx.y;
    const int seq0 = blockIdx.x * S;
    const int total = S * L;
    // pass A: sequence = column n2 (addresses N2 n1 + n2: consecutive seqs
    // are consecutive); pass B: sequence = row k1 (addresses N2 k1 + n2:
    // consecutive elements are consecutive)
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
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
        const int jr = (int)(__builtin_bitreverse32((unsigned)j) >> (32 - P.log_l));
        buf[jr * S + s] = make_float2(v.x, v.y);
    }
    __syncthreads();
    for (int half = 1; half < L; half <<= 1) {
        const int step = L / (2 * half);
        for (int b = threadIdx.x; b < (L / 2) * S; b += blockDim.x) {
            const int s = b % S, p = b / S;
            const int m = p & (half - 1);
            const int i0 = (p - m) * 2 + m, i1 = i0 + half;
            const C2 w = tw(P.tw_stage, m * step, P.inverse);
            const float2 a = buf[i0 * S + s], c = buf[i1 * S + s];
            const C2 cw = cmul({c.x, c.y}, w);
            buf[i0 * S + s] = make_float2(a.x + cw.x, a.y + cw.y);
            buf[i1 * S + s] = make_float2(a.x - cw.x, a.y - cw.y);
        }
        __syncthreads();
    }
    // pass A: Y[n2 + N2 k1] = X1[k1] w_N^(n2 k1) (consecutive seqs consecutive);
    // pass B: X[k1 + N1 k2] (consecutive seqs = rows k1 consecutive)
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
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

}  // namespace

int seqs_per_group(int L, int n_seq) {
    int S = 8192 / L;
    if (S > 16) S = 16;
    if (S > n_seq) S = n_seq;
    return S < 1 ? 1 : S;
}

int launch_pass(const Pass &P, int batches, void *stream) {
    const int groups = (P.n_seq + P.S - 1) / P.S;
    const size_t lds = (size_t)P.S * P.L * sizeof(float2);
    hipLaunchKernelGGL(k_fft_pass, dim3(groups, batches), dim3(256), lds, (hipStream_t)stream, P);
    return (int)hipGetLastError();
}

}  // namespace fourier
}  // namespace ctis
