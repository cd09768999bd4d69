// HIP kernels for gfx950: the forward projection H f (fused with the EM ratio
// u = g / H f) and the back projection H^T u (fused with the EM update
// f = f . H^T u / h).  White, Bell & Haygood, Sec. 2 eq. (em); Sec. 3 eqs.
// (vs_linear) and (Htu).
//
// Both are atomic-free gathers over dense B x B boxes of calibration
// nonzeros.  A wavefront owns a 64 x 16 output tile (fast x slow axis) with a
// 4 x 4 register micro-tile per lane, stages the (64+B-1) x (16+B-1) input
// window a box needs into its own LDS region, and correlates it with the
// box's values, which are wave-uniform and come through scalar loads.  The
// waves of a workgroup split the boxes of one tile and meet in an LDS
// reduction in a fixed order, so results are deterministic.
//
//   forward  (one workgroup per FPA tile, the tile's boxes from the work list):
//     ghat(r, c) = sum_box sum_{dr,dc} v[dr,dc] * fE((r - rA - dr) + gamma*(c - cA - dc) mod n)
//     where fE(q) = f_s(q mod gamma, q div gamma) inside the a x alpha field
//     stop and 0 outside (the zero padding E of Sec. 3).
//   adjoint  (one workgroup per (wavelength, field-stop tile), all boxes of it):
//     zeta(x, y, s) = sum_box sum_{dr,dc} v[dr,dc] * u((rA + dr + x) + gamma*(cA + dc + y) mod n)
//
// The window loaders evaluate the 1-D address modulo n with a row/column
// decomposition, which is exact for the paper's cyclic shift over the whole
// vectorised FPA, including shifts that run past an FPA edge.
#include <hip/hip_runtime.h>

#include "ctis_internal.h"

namespace ctis {
namespace {

constexpr int TX = kTileFast;
constexpr int TY = kTileSlow;

template <int B>
struct Win {
    static constexpr int SX = TX + B - 1;          // window extent, fast axis
    static constexpr int SXP = (SX + 3) & ~3;      // LDS row pitch (16-byte rows)
    static constexpr int SY = TY + B - 1;          // window extent, slow axis
    static constexpr int REG = SXP * SY;           // floats per wavefront region
    static constexpr int NR = 4 + B - 1;           // row segment a lane reads
    static constexpr int NV = (NR + 3) / 4;        // float4 reads per segment
    static_assert(REG >= 1024, "the reduction reuses 1024 floats per wave");
    static_assert(4 * (TX / 4 - 1) + 4 * NV <= SXP, "segment reads stay inside the row");
};

// floor division / modulo for b > 0
__device__ __forceinline__ void floor_divmod(int x, int b, int &q, int &r) {
    q = x / b;
    r = x - q * b;
    if (r < 0) {
        r += b;
        q -= 1;
    }
}

__device__ __forceinline__ int step_mod(int y, int m) { return (y + 1 == m) ? 0 : y + 1; }

// Decode the fast-axis part of a 1-D FPA address for this lane's window
// column X = Xs + col: returns xm = X mod gamma and the slow-axis index
// y = (Ys + X div gamma) mod xi (both floor semantics).
__device__ __forceinline__ void decode_column(const KParams &p, int Xs, int Ys, int col, int &xm, int &y) {
    int q0, r0;
    floor_divmod(Xs, p.gamma, q0, r0);
    int yq, y0;
    floor_divmod(Ys + q0, p.xi, yq, y0);
    xm = r0 + col;
    y = y0;
    while (xm >= p.gamma) {
        xm -= p.gamma;
        y = step_mod(y, p.xi);
    }
}

// Forward window: slot (xx, yy) <- fE((Xs + xx) + gamma*(Ys + yy) mod n).
template <int B>
__device__ __forceinline__ void stage_forward(float *S, const float *__restrict__ fs, const KParams &p, int Xs,
                                              int Ys, int lane) {
    using Wn = Win<B>;
    {
        int xm, y;
        decode_column(p, Xs, Ys, lane, xm, y);
        const bool vx = xm < p.a;
        float v[Wn::SY];
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) {
            const bool ok = vx && (y < p.alpha);
            const float t = fs[ok ? xm + p.a * y : 0];
            v[yy] = ok ? t : 0.0f;
            y = step_mod(y, p.xi);
        }
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) S[yy * Wn::SXP + lane] = v[yy];
    }
    if constexpr (B > 1) {
        constexpr int E = B - 1;
        for (int k = lane; k < E * Wn::SY; k += 64) {
            const int e = k % E, yy = k / E;
            int xm, y;
            decode_column(p, Xs, Ys, TX + e, xm, y);
            y += yy;
            while (y >= p.xi) y -= p.xi;
            const bool ok = (xm < p.a) && (y < p.alpha);
            const float t = fs[ok ? xm + p.a * y : 0];
            S[yy * Wn::SXP + TX + e] = ok ? t : 0.0f;
        }
    }
}

// Adjoint window: slot (xx, yy) <- u((Xs + xx) + gamma*(Ys + yy) mod n) for
// xx < xlim, yy < ylim (the dilated field stop), else 0.
template <int B>
__device__ __forceinline__ void stage_adjoint(float *S, const float *__restrict__ u, const KParams &p, int Xs,
                                              int Ys, int xlim, int ylim, int lane) {
    using Wn = Win<B>;
    {
        int xm, y;
        decode_column(p, Xs, Ys, lane, xm, y);
        const bool vx = lane < xlim;
        float v[Wn::SY];
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) {
            const bool ok = vx && (yy < ylim);
            const float t = u[ok ? xm + p.gamma * y : 0];
            v[yy] = ok ? t : 0.0f;
            y = step_mod(y, p.xi);
        }
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) S[yy * Wn::SXP + lane] = v[yy];
    }
    if constexpr (B > 1) {
        constexpr int E = B - 1;
        for (int k = lane; k < E * Wn::SY; k += 64) {
            const int e = k % E, yy = k / E;
            int xm, y;
            decode_column(p, Xs, Ys, TX + e, xm, y);
            y += yy;
            while (y >= p.xi) y -= p.xi;
            const bool ok = (TX + e < xlim) && (yy < ylim);
            const float t = u[ok ? xm + p.gamma * y : 0];
            S[yy * Wn::SXP + TX + e] = ok ? t : 0.0f;
        }
    }
}

// acc[k][q] += sum_{i,j < B} W[j*B + i] * S[(4ly + k + j) * SXP + 4lx + q + i]
template <int B>
__device__ __forceinline__ void correlate(float (&acc)[4][4], const float *S, int lx, int ly,
                                          const float *__restrict__ W) {
    using Wn = Win<B>;
#pragma unroll
    for (int row = 0; row < Wn::NR; ++row) {
        float seg[4 * Wn::NV];
        const float4 *src = reinterpret_cast<const float4 *>(S + (4 * ly + row) * Wn::SXP + 4 * lx);
#pragma unroll
        for (int v = 0; v < Wn::NV; ++v) {
            const float4 t = src[v];
            seg[4 * v + 0] = t.x;
            seg[4 * v + 1] = t.y;
            seg[4 * v + 2] = t.z;
            seg[4 * v + 3] = t.w;
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int k = row - j;
            if (k < 0 || k >= 4) continue;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const float wij = W[j * B + i];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[k][q] = __builtin_fmaf(wij, seg[q + i], acc[k][q]);
            }
        }
    }
}

// Sum the other waves' accumulators into wave 0 (fixed order).  Returns false
// on waves other than 0, which then have nothing left to do.
__device__ __forceinline__ bool reduce_waves(float (&acc)[4][4], float *lds, int wv, int nw, int lane) {
    if (nw == 1) return true;
    __syncthreads();
    if (wv > 0) {
        float *R = lds + (wv - 1) * 1024;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) R[(k * 4 + q) * 64 + lane] = acc[k][q];
    }
    __syncthreads();
    if (wv != 0) return false;
    for (int w2 = 1; w2 < nw; ++w2) {
        const float *R = lds + (w2 - 1) * 1024;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[k][q] += R[(k * 4 + q) * 64 + lane];
    }
    return true;
}

template <int B>
__global__ void __launch_bounds__(256) k_forward(const KParams p, const int32_t *__restrict__ tile_order,
                                                 const int32_t *__restrict__ tile_item_ptr,
                                                 const int32_t *__restrict__ item_box,
                                                 const int32_t *__restrict__ box_rc,
                                                 const int32_t *__restrict__ box_lambda,
                                                 const float *__restrict__ box_wf, const float *__restrict__ f,
                                                 const float *__restrict__ g, float *__restrict__ out, int em,
                                                 int vec) {
    using Wn = Win<B>;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int tile = tile_order[blockIdx.x];
    const int r0 = (tile % p.ntr) * TX, c0 = (tile / p.ntr) * TY;
    const int it0 = tile_item_ptr[tile], it1 = tile_item_ptr[tile + 1];
    float *S = lds + wv * Wn::REG;
    const int lx = lane & 15, ly = lane >> 4;

    float acc[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[k][q] = 0.0f;

    for (int it = it0 + wv; it < it1; it += nw) {
        const int b = __builtin_amdgcn_readfirstlane(item_box[it]);
        const int rA = box_rc[2 * b], cA = box_rc[2 * b + 1];
        const int s = box_lambda[b];
        stage_forward<B>(S, f + (size_t)s * p.ell, p, r0 - (B - 1) - rA, c0 - (B - 1) - cA, lane);
        correlate<B>(acc, S, lx, ly, box_wf + (size_t)b * (B * B));
    }
    if (!reduce_waves(acc, lds, wv, nw, lane)) return;

    const int rb = r0 + 4 * lx;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = c0 + 4 * ly + k;
        if (c >= p.xi) continue;
        const size_t base = (size_t)rb + (size_t)p.gamma * c;
        if (vec && rb + 3 < p.gamma) {
            float4 v = make_float4(acc[k][0], acc[k][1], acc[k][2], acc[k][3]);
            if (em) {
                const float4 gv = *reinterpret_cast<const float4 *>(g + base);
                v.x = v.x > 0.0f ? gv.x / v.x : 0.0f;
                v.y = v.y > 0.0f ? gv.y / v.y : 0.0f;
                v.z = v.z > 0.0f ? gv.z / v.z : 0.0f;
                v.w = v.w > 0.0f ? gv.w / v.w : 0.0f;
            }
            *reinterpret_cast<float4 *>(out + base) = v;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (rb + q >= p.gamma) continue;
                float v = acc[k][q];
                if (em) v = v > 0.0f ? g[base + q] / v : 0.0f;
                out[base + q] = v;
            }
        }
    }
}

template <int B>
__global__ void __launch_bounds__(256) k_adjoint(const KParams p, const int32_t *__restrict__ lambda_box_ptr,
                                                 const int32_t *__restrict__ box_rc, const float *__restrict__ box_w,
                                                 const float *__restrict__ hsum, const float *__restrict__ u,
                                                 const float *fin, float *out, int em, int vec) {
    using Wn = Win<B>;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int per = p.nbx * p.nby;
    const int s = blockIdx.x / per, vt = blockIdx.x - s * per;
    const int x0 = (vt % p.nbx) * TX, y0 = (vt / p.nbx) * TY;
    const int b0 = lambda_box_ptr[s], b1 = lambda_box_ptr[s + 1];
    const int xlim = p.a + B - 1 - x0, ylim = p.alpha + B - 1 - y0;
    float *S = lds + wv * Wn::REG;
    const int lx = lane & 15, ly = lane >> 4;

    float acc[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[k][q] = 0.0f;

    for (int b = b0 + wv; b < b1; b += nw) {
        const int rA = box_rc[2 * b], cA = box_rc[2 * b + 1];
        stage_adjoint<B>(S, u, p, rA + x0, cA + y0, xlim, ylim, lane);
        correlate<B>(acc, S, lx, ly, box_w + (size_t)b * (B * B));
    }
    if (!reduce_waves(acc, lds, wv, nw, lane)) return;

    const float hs = hsum[s];
    const int xb = x0 + 4 * lx;
    const size_t sb = (size_t)s * p.ell;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int y = y0 + 4 * ly + k;
        if (y >= p.alpha) continue;
        const size_t base = sb + (size_t)xb + (size_t)p.a * y;
        if (vec && xb + 3 < p.a) {
            float4 v = make_float4(acc[k][0], acc[k][1], acc[k][2], acc[k][3]);
            if (em) {
                const float4 fv = *reinterpret_cast<const float4 *>(fin + base);
                v.x = hs != 0.0f ? (fv.x * v.x) / hs : 0.0f;
                v.y = hs != 0.0f ? (fv.y * v.y) / hs : 0.0f;
                v.z = hs != 0.0f ? (fv.z * v.z) / hs : 0.0f;
                v.w = hs != 0.0f ? (fv.w * v.w) / hs : 0.0f;
            }
            *reinterpret_cast<float4 *>(out + base) = v;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (xb + q >= p.a) continue;
                float v = acc[k][q];
                if (em) v = hs != 0.0f ? (fin[base + q] * v) / hs : 0.0f;
                out[base + q] = v;
            }
        }
    }
}

bool aligned16(const void *ptr) { return ptr == nullptr || ((uintptr_t)ptr & 15u) == 0; }

template <int B>
int forward_B(const ctis_plan *pl, const float *f, const float *g, float *out, bool em, hipStream_t st) {
    const int nwg = em ? pl->ht.n_active : pl->ht.n_tiles;
    if (nwg == 0) return 0;
    const int nw = pl->waves_fwd;
    const size_t lds = (size_t)nw * Win<B>::REG * sizeof(float);
    const int vec = (pl->gamma % 4 == 0) && aligned16(out) && aligned16(g);
    const DevTables &t = pl->dt;
    hipLaunchKernelGGL(k_forward<B>, dim3(nwg), dim3(64 * nw), lds, st, pl->kp, t.tile_order, t.tile_item_ptr,
                       t.item_box, t.box_rc, t.box_lambda, t.box_wf, f, g, out, em ? 1 : 0, vec);
    return (int)hipGetLastError();
}

template <int B>
int adjoint_B(const ctis_plan *pl, const float *u, const float *fin, float *out, bool em, hipStream_t st) {
    const int nwg = pl->kp.nbx * pl->kp.nby * pl->w;
    const int nw = pl->waves_adj;
    const size_t lds = (size_t)nw * Win<B>::REG * sizeof(float);
    const int vec = (pl->a % 4 == 0) && aligned16(out) && aligned16(fin);
    const DevTables &t = pl->dt;
    hipLaunchKernelGGL(k_adjoint<B>, dim3(nwg), dim3(64 * nw), lds, st, pl->kp, t.lambda_box_ptr, t.box_rc, t.box_w,
                       t.h, u, fin, out, em ? 1 : 0, vec);
    return (int)hipGetLastError();
}

}  // namespace

int launch_forward(const ctis_plan *p, const float *f, const float *g, float *out, bool em, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (p->ht.B) {
        case 1: return forward_B<1>(p, f, g, out, em, st);
        case 2: return forward_B<2>(p, f, g, out, em, st);
        case 3: return forward_B<3>(p, f, g, out, em, st);
        case 4: return forward_B<4>(p, f, g, out, em, st);
        case 5: return forward_B<5>(p, f, g, out, em, st);
        case 6: return forward_B<6>(p, f, g, out, em, st);
        case 7: return forward_B<7>(p, f, g, out, em, st);
        case 8: return forward_B<8>(p, f, g, out, em, st);
    }
    return (int)hipErrorInvalidValue;
}

int launch_adjoint(const ctis_plan *p, const float *u, const float *fin, float *out, bool em, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (p->ht.B) {
        case 1: return adjoint_B<1>(p, u, fin, out, em, st);
        case 2: return adjoint_B<2>(p, u, fin, out, em, st);
        case 3: return adjoint_B<3>(p, u, fin, out, em, st);
        case 4: return adjoint_B<4>(p, u, fin, out, em, st);
        case 5: return adjoint_B<5>(p, u, fin, out, em, st);
        case 6: return adjoint_B<6>(p, u, fin, out, em, st);
        case 7: return adjoint_B<7>(p, u, fin, out, em, st);
        case 8: return adjoint_B<8>(p, u, fin, out, em, st);
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace ctis
