// Internal types of the Fourier (WBH) path: the pass descriptor shared by the
// FFT kernel (fourier.hip) and the C ABI glue (fourier.cpp).
#pragma once

#include "ctis_internal.h"

namespace ctis {
namespace fourier {

// Load modes (pass A reads element i of the batch's sequence, i = N2 n1 + n2
// in natural order):
enum Load : int {
    kLoadComplex = 0,   // in[batch n + i]
    kLoadEmbedPair = 1, // (fE_{2t}(i), fE_{2t+1}(i)): E f of the pair's wavelengths
    kLoadCalPair = 2,   // (c_{2t}[i], -c_{2t+1}[i]) from a dense w x n calibration
    kLoadReal = 3,      // (u[i], 0)
    kLoadConjE = 4,     // conj(e_t[i]) U[i]
};
// Store modes (pass B writes element k of the batch's sequence in natural order):
enum Store : int {
    kStoreComplex = 0,  // out[batch n + k]
    kStoreReal = 1,     // ghat[k] = Re / n
    kStoreRatio = 2,    // u[k] = g[k] / ghat[k], 0 where ghat <= 0
    kStoreCrop = 3,     // z_s(x, y) = (Re, Im) / n for the pair's wavelengths
    kStoreUpdate = 4,   // f_s(x, y) = f_s zeta_s / h_s, 0 where h_s = 0
};

struct Geo {
    int a, alpha, gamma, xi, w;
    long long ell;
    int log_gamma;             // n = gamma xi is a power of two, so gamma is one
};

struct Pass {
    const float2 *in;          // complex input (mode complex; conj-e: U)
    float2 *out;               // complex output (pass A, complex store)
    const float *fin;          // real input (embed: f; real: u; cal: c)
    float *fout;               // real output (real, ratio: ghat / u; crop: z; update: f)
    const float *g;            // ratio: the measured frame
    const float2 *e;           // spectra e_t (conj-e)
    const float *h;            // column sums per wavelength (update)
    const float2 *tw_stage;    // exp(-2 pi i j / L), j < L / 2
    const float2 *tw_hi;       // exp(-2 pi i a / N1), a < N1   (pass A only)
    const float2 *tw_lo;       // exp(-2 pi i b / N),  b < N2   (pass A only)
    long long n;
    int L, log_l;              // transform length and its log2
    int n_seq;                 // sequences per batch (N2 for pass A, N1 for pass B)
    int pass_a;                // 1: pass A (strided columns, twiddle, Y layout); 0: pass B
    int N1, N2, log_n2;
    int inverse;
    int load, store;
    Geo geo;
};

// One FFT pass (pass A or B per P.pass_a) over `batches` sequences of P.n_seq
// transforms of length 2^P.log_l (2^2 .. 2^10).
int launch_pass(const Pass &P, int batches, void *stream);
// G = sum_t e_t . X_t over `pairs` spectra of length n.
int launch_combine(const float2 *e, const float2 *X, float2 *G, int pairs, long long n, void *stream);

}  // namespace fourier
}  // namespace ctis
