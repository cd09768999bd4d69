// HIP kernels for gfx950: the forward projection H f (fused with the EM ratio
// u = g / H f) and the back projection H^T u (fused with the EM update
// f = f . H^T u / h).  White, Bell & Haygood, Sec. 2 eq. (em); Sec. 3 eqs.
// (vs_linear) and (Htu).  The same two kernels, with other epilogues, and a
// correlation-reduction kernel over the calibration boxes give the
// reverse-mode derivative of an EM step (forward of b = y f / h with
// e = -(H b) u / (H f); back projections with y zeta / h + H^T e; the value
// derivatives sum u b + e f over the voxels of each box slot).
//
// Both are atomic-free gathers over dense B x B boxes of calibration
// nonzeros.  A wavefront owns a 64 x 16 output tile (fast x slow axis) with a
// 4 x 4 register micro-tile per lane, stages the (64+B-1) x (16+B-1) input
// window of one box into its own LDS region, and correlates it with the box's
// values.  Each wave keeps the next box's window in flight in registers
// while it computes the current one.  The waves of a workgroup split the boxes of one tile and meet
// in an LDS reduction in a fixed order (deterministic results); the reduced
// tile leaves row by row, so every epilogue load and store is a contiguous
// 256-byte wavefront access.
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
// vectorised FPA, including shifts that run past an FPA edge.  Window slots
// outside the field stop (forward) or outside the dilated field stop
// (adjoint) are fetched with an out-of-range buffer offset, which the buffer
// unit returns as 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "ctis_internal.h"

namespace ctis {
namespace {

constexpr int TX = kTileFast;
constexpr int TY = kTileSlow;
constexpr int kMinWaves = 4;                     // so that a wave owns <= 4 epilogue rows
constexpr int kSoloWaves = 4;                    // solo kernels: units (waves) per workgroup
constexpr int kRowsPerWave = TY / kMinWaves;
constexpr unsigned kOutOfRange = 0x80000000u;   // buffer offset past num_records -> 0
constexpr int kRsrcWord3 = 0x00020000;           // raw 32-bit buffer, gfx9 family

template <int B>
struct Win {
    static constexpr int SX = TX + B - 1;          // window extent, fast axis
    static constexpr int SXP = (SX + 3) & ~3;      // LDS row pitch (16-byte rows)
    static constexpr int SY = TY + B - 1;          // window extent, slow axis
    static constexpr int REG = SXP * SY;           // floats per wavefront region
    static constexpr int NR = 4 + B - 1;           // row segment a lane reads
    static constexpr int NV = (NR + 3) / 4;        // float4 reads per segment
    static constexpr int E = B - 1;                // window columns beyond the 64 lanes
    static constexpr int ED = E > 0 ? E : 1;       // divisor for the extra slots (none when B = 1)
    static constexpr int NXT = (E * SY + 63) / 64; // extra slots per lane
    static constexpr int WREG = REG + 64;          // region incl. the box values (<= 64)
    static constexpr int MAXW = B <= 5 ? 16 : 8;   // waves per workgroup (VGPR budget)
    static_assert(REG >= TX * TY, "the reduction reuses 1024 floats per wave");
    static_assert(REG % 4 == 0 && B * B <= 64, "box values sit 16-byte aligned after the window");
    static_assert(4 * (TX / 4 - 1) + 4 * NV <= SXP, "segment reads stay inside the row");
};

// One window in flight, in registers: window column `lane`, this lane's
// slots of the extra columns, and (lanes < B*B) one of the box's values.
template <int B>
struct Pending {
    float v[Win<B>::SY];
    float x[Win<B>::NXT > 0 ? Win<B>::NXT : 1];
    float wt;
};

// Work records: int4 (X, Y, s, box); box < 0 ends a list.
__device__ __forceinline__ int4 record(const int4 *__restrict__ list, int k, int stride) {
    return k < stride ? list[k] : make_int4(0, 0, 0, -1);
}

// Unit lists are ordered for one unit per workgroup, position p running on
// XCD p mod 8 (workgroups are dealt to the 8 XCDs round-robin; batches put a
// frame's units on one XCD).  A solo workgroup takes `per_wg` units, so
// virtual workgroup v (blockIdx.x, then strided by the grid, a multiple of 8
// when persistent) takes the positions 8 (per_wg (v / 8) + i) + v mod 8,
// i < per_wg: all of them on v's own XCD.
__device__ __forceinline__ int solo_unit(int v, int i, int per_wg) {
    return 8 * (per_wg * (v >> 3) + i) + (v & 7);
}

// Virtual workgroups that cover n_units positions, per_wg at a time per XCD.
__host__ __device__ __forceinline__ int solo_groups(int n_units, int per_wg) {
    return 8 * ((((n_units + 7) >> 3) + per_wg - 1) / per_wg);
}

__device__ __forceinline__ void floor_divmod(int x, int b, int &q, int &r) {
    q = x / b;
    r = x - q * b;
    if (r < 0) {
        r += b;
        q -= 1;
    }
}

__device__ __forceinline__ int step_mod(int y, int m) { return (y + 1 == m) ? 0 : y + 1; }

// The lanes of a wavefront hand data to each other through LDS (a window and
// its box values written by some lanes, read by others).  The hardware runs a
// wavefront's LDS instructions in order; this fence pair keeps the compiler
// from moving LDS loads or stores across the hand-off (without it, a load of
// data another lane wrote may legally be hoisted out of the item loop).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the 64 lanes of a wavefront (every lane gets the total; a fixed
// butterfly order, so the result does not depend on timing).
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const float *base, int nfloats) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, nfloats * 4, kRsrcWord3);
}

// raw 32-bit buffer load at byte offset `off`, reinterpreted as float (the
// builtin returns the bits)
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// raw 128-bit buffer load at byte offset `off` (4-byte aligned)
__device__ __forceinline__ float4 bload4(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// raw 32-bit buffer load at byte offset voff + soff (soff wave-uniform: a
// scalar register)
__device__ __forceinline__ float bload2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// The SY rows of one window column, from a buffer with row pitch P floats:
// row yy sits at byte offset 4*(col + P*((y + yy) mod xi)), given
// o0 = 4*(col + P*y) and wrap = 4*P*xi.  For xi >= SY the row index wraps at
// most once over the window, so the offset is min(o, o - wrap) in unsigned
// arithmetic with o = o0 + 4*P*yy the unwrapped one (below wrap, o - wrap
// wraps round to more than o).  All offsets stay below 2^32: o0 < 4n, and
// 4*P*SY <= 4n for P <= gamma, with n < 2^29.  A column whose o0 lies past
// the buffer, with wrap = 0, reads 0 in every row.
template <int B>
__device__ __forceinline__ void column_rows(float (&v)[Win<B>::SY], __amdgpu_buffer_rsrc_t r, unsigned o0,
                                            unsigned step, unsigned wrap) {
#pragma unroll
    for (int yy = 0; yy < Win<B>::SY; ++yy) {
        const unsigned o = o0 + step * (unsigned)yy;
        v[yy] = bload(r, min(o, o - wrap));
    }
}

// Frame geometry of a work unit.
struct Geo {
    int a, alpha, gamma, xi;
};

template <int B>
__device__ __forceinline__ void load_values(Pending<B> &pd, const float *__restrict__ wtab, int box, int lane) {
    pd.wt = 0.0f;
    if (lane < B * B) pd.wt = wtab[(size_t)box * (B * B) + lane];
}

// Forward window of one (tile, box) item, rec = (Xs, Ys, f_off, box):
// slot (xx, yy) <- fE((Xs + xx) + gamma*(Ys + yy) mod n).  Each lane decodes
// its column once (the window origin needs two scalar divisions) and then
// steps row by row.  (Taking the row offset of windows that stay inside one
// FPA column as the buffer's scalar offset was measured slower.)
template <int B>
__device__ __forceinline__ void load_forward(Pending<B> &pd, const float *f, const float *__restrict__ wtab,
                                             const Geo &p, int4 rec, int lane) {
    using Wn = Win<B>;
    const __amdgpu_buffer_rsrc_t fr = rsrc(f + (size_t)(unsigned)rec.z, p.a * p.alpha);
    const int Xs = rec.x, Ys = rec.y;
    int q0, xr, yq, y0;
    floor_divmod(Xs, p.gamma, q0, xr);
    floor_divmod(Ys + q0, p.xi, yq, y0);
    int xm = xr + lane, y = y0;
    while (xm >= p.gamma) {
        xm -= p.gamma;
        y = step_mod(y, p.xi);
    }
    const bool vx = xm < p.a;
    if (p.xi >= Wn::SY) {
        // rows at or past alpha land at or past a*alpha floats and read 0;
        // columns outside the field stop start past the buffer and never wrap
        column_rows<B>(pd.v, fr, vx ? (unsigned)(xm + p.a * y) * 4u : kOutOfRange, 4u * (unsigned)p.a,
                       vx ? 4u * (unsigned)(p.a * p.xi) : 0u);
    } else {
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) {
            const bool ok = vx && (y < p.alpha);
            pd.v[yy] = bload(fr, ok ? (unsigned)(xm + p.a * y) * 4u : kOutOfRange);
            y = step_mod(y, p.xi);
        }
    }
#pragma unroll
    for (int t = 0; t < Wn::NXT; ++t) {
        const int k = lane + 64 * t;
        unsigned off = kOutOfRange;
        if (k < Wn::E * Wn::SY) {
            const int e = k % Wn::ED, yy = k / Wn::ED;
            int xe = xr + TX + e, ye = y0;
            while (xe >= p.gamma) {
                xe -= p.gamma;
                ye = step_mod(ye, p.xi);
            }
            ye += yy;
            while (ye >= p.xi) ye -= p.xi;
            if (xe < p.a && ye < p.alpha) off = (unsigned)(xe + p.a * ye) * 4u;
        }
        pd.x[t] = bload(fr, off);
    }
    load_values<B>(pd, wtab, rec.w, lane);
}

// Forward window of an item whose window reads the same values as a plain
// 2-D window over a zero-bordered f_s (decided on the host, rec = (x0, y0,
// f_off | kDirectFlag, box)): either the decoded origin runs inside the FPA
// without a carry into the next column or a wrap round its end, or the
// origin, possibly negative, keeps every position that the 1-D cyclic shift
// wraps on an FPA column or row outside the field stop.  Slot (xx, yy) is
// f_s(x0 + xx, y0 + yy) inside the field stop, 0 outside: a column outside
// [0, a) (compared unsigned) gets the out-of-range offset; a row at or past
// alpha lands at or past the block's a*alpha floats and a negative row wraps
// the unsigned offset past it, both reading 0.  One vector add per row.
template <int B>
__device__ __forceinline__ void load_forward_direct(Pending<B> &pd, const float *f, const float *__restrict__ wtab,
                                                    const Geo &p, int4 rec, int lane, const unsigned (&xo)[
                                                        Win<B>::NXT > 0 ? Win<B>::NXT : 1]) {
    using Wn = Win<B>;
    const __amdgpu_buffer_rsrc_t fr = rsrc(f + (size_t)(unsigned)(rec.z & (kDirectFlag - 1)), p.a * p.alpha);
    const int xm = rec.x + lane;
    const unsigned stp = 4u * (unsigned)p.a;
    const unsigned o0 = (unsigned)xm < (unsigned)p.a ? 4u * (unsigned)xm + stp * (unsigned)rec.y : kOutOfRange;
#pragma unroll
    for (int yy = 0; yy < Wn::SY; ++yy) pd.v[yy] = bload(fr, o0 + stp * (unsigned)yy);
    // extra slot t of this lane: column 64 + e, row yy, with xo[t] = (e, yy)
    // packed as e + 64*yy (or -1: no slot)
#pragma unroll
    for (int t = 0; t < Wn::NXT; ++t) {
        const int e = (int)(xo[t] & 63u), yy = (int)(xo[t] >> 6);
        const int xe = rec.x + TX + e;
        pd.x[t] = bload(fr, (xo[t] != ~0u && (unsigned)xe < (unsigned)p.a)
                                ? 4u * (unsigned)xe + stp * (unsigned)(rec.y + yy)
                                : kOutOfRange);
    }
    load_values<B>(pd, wtab, rec.w, lane);
}

// Adjoint window of one (field-stop tile, box) pair: slot (xx, yy) <-
// u((Xs + xx) + gamma*(Ys + yy) mod n).  Slots past the dilated field stop
// (xx >= a + B - 1 - x0 or yy >= alpha + B - 1 - y0) only ever meet output
// voxels outside the field stop, which are never written, so they need no
// masking; their addresses are still reduced mod n and stay in bounds.
template <int B>
__device__ __forceinline__ void load_adjoint(Pending<B> &pd, __amdgpu_buffer_rsrc_t ur,
                                             const float *__restrict__ wtab, const Geo &p, int Xs, int Ys,
                                             int box, int lane) {
    using Wn = Win<B>;
    int q0, xr, yq, y0;
    floor_divmod(Xs, p.gamma, q0, xr);
    floor_divmod(Ys + q0, p.xi, yq, y0);
    int xm = xr + lane, y = y0;
    while (xm >= p.gamma) {
        xm -= p.gamma;
        y = step_mod(y, p.xi);
    }
    if (p.xi >= Wn::SY) {
        column_rows<B>(pd.v, ur, (unsigned)(xm + p.gamma * y) * 4u, 4u * (unsigned)p.gamma,
                       4u * (unsigned)(p.gamma * p.xi));
    } else {
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) {
            pd.v[yy] = bload(ur, (unsigned)(xm + p.gamma * y) * 4u);
            y = step_mod(y, p.xi);
        }
    }
#pragma unroll
    for (int t = 0; t < Wn::NXT; ++t) {
        const int k = lane + 64 * t;
        unsigned off = kOutOfRange;
        if (k < Wn::E * Wn::SY) {
            const int e = k % Wn::ED, yy = k / Wn::ED;
            int xe = xr + TX + e, ye = y0;
            while (xe >= p.gamma) {
                xe -= p.gamma;
                ye = step_mod(ye, p.xi);
            }
            ye += yy;
            while (ye >= p.xi) ye -= p.xi;
            off = (unsigned)(xe + p.gamma * ye) * 4u;
        }
        pd.x[t] = bload(ur, off);
    }
    load_values<B>(pd, wtab, box, lane);
}

// Adjoint window of a box whose image of the dilated field stop runs inside
// the FPA without a carry or a wrap, and whose last tile's window ends inside
// u (flagged on the host): slot (xx, yy) at byte offset
// 4*xx + 4*(Xs + gamma*(Ys + yy)), the second term wave-uniform (a scalar
// offset), so the row loads take no vector arithmetic.  Slots of lanes past
// the field stop may hold other pixels of u; those lanes' outputs are never
// written.  xo[t]: byte offset of this lane's extra slot within the window
// (0 where it has none).
template <int B>
__device__ __forceinline__ void load_adjoint_direct(Pending<B> &pd, __amdgpu_buffer_rsrc_t ur,
                                                    const float *__restrict__ wtab, const Geo &p, int Xs, int Ys,
                                                    int box, int lane,
                                                    const unsigned (&xo)[Win<B>::NXT > 0 ? Win<B>::NXT : 1]) {
    using Wn = Win<B>;
    const unsigned s0 = 4u * (unsigned)(Xs + p.gamma * Ys), srow = 4u * (unsigned)p.gamma;
    const unsigned vo = 4u * (unsigned)lane;
#pragma unroll
    for (int yy = 0; yy < Wn::SY; ++yy) pd.v[yy] = bload2(ur, vo, s0 + srow * (unsigned)yy);
#pragma unroll
    for (int t = 0; t < Wn::NXT; ++t) pd.x[t] = bload2(ur, xo[t], s0);
    load_values<B>(pd, wtab, box, lane);
}

// Direct adjoint window in 16-byte pieces: piece k = lane + 64 t is row
// k / SX4, column quad k % SX4 of the window (SX4 = SXP / 4 pieces per row),
// at byte offset s0 + voff[t] of u with voff[t] = 4 gamma row + 16 quad
// precomputed per unit; the whole offset goes in the vector operand, so
// the range check covers the up to three floats a row's last piece reads
// past the window.  A lane holds NQ pieces instead of one float per window
// row: a quarter of the load instructions.
template <int B>
struct Pending4 {
    static constexpr int SX4 = Win<B>::SXP / 4, NP = SX4 * Win<B>::SY, NQ = (NP + 63) / 64;
    float4 q[NQ];
    float wt;
};

template <int B>
__device__ __forceinline__ void adjoint_piece_offsets(unsigned (&voff)[Pending4<B>::NQ], int lane, int gamma) {
    using P4 = Pending4<B>;
#pragma unroll
    for (int t = 0; t < P4::NQ; ++t) {
        const int k = lane + 64 * t;
        voff[t] = k < P4::NP ? 4u * (unsigned)gamma * (unsigned)(k / P4::SX4) + 16u * (unsigned)(k % P4::SX4) : 0u;
    }
}

template <int B>
__device__ __forceinline__ void load_adjoint_direct4(Pending4<B> &pd, __amdgpu_buffer_rsrc_t ur,
                                                     const float *__restrict__ wtab, const Geo &p, int Xs, int Ys,
                                                     int box, int lane,
                                                     const unsigned (&voff)[Pending4<B>::NQ]) {
    const unsigned s0 = 4u * (unsigned)(Xs + p.gamma * Ys);
#pragma unroll
    for (int t = 0; t < Pending4<B>::NQ; ++t) pd.q[t] = bload4(ur, s0 + voff[t]);
    pd.wt = lane < B * B ? wtab[(size_t)box * (B * B) + lane] : 0.0f;
}

// Pieces into S[0, REG) (piece k at float 4k: the row pitch is SX4 pieces),
// box values into S[REG, REG + B*B).
template <int B>
__device__ __forceinline__ void store_window4(float *S, const Pending4<B> &pd, int lane) {
    using P4 = Pending4<B>;
    static_assert(Win<B>::SXP == 4 * P4::SX4 && Win<B>::REG == 4 * P4::NP, "pieces are packed row after row");
#pragma unroll
    for (int t = 0; t < P4::NQ; ++t) {
        const int k = lane + 64 * t;
        if (t + 1 < P4::NQ || k < P4::NP) *reinterpret_cast<float4 *>(S + 4 * k) = pd.q[t];
    }
    if (lane < B * B) S[Win<B>::REG + lane] = pd.wt;
}

// Window into S[0, REG), box values into S[REG, REG + B*B) (kValues).
template <int B, bool kValues = true>
__device__ __forceinline__ void store_window(float *S, const Pending<B> &pd, int lane) {
    using Wn = Win<B>;
#pragma unroll
    for (int yy = 0; yy < Wn::SY; ++yy) S[yy * Wn::SXP + lane] = pd.v[yy];
#pragma unroll
    for (int t = 0; t < Wn::NXT; ++t) {
        const int k = lane + 64 * t;
        if (k < Wn::E * Wn::SY) S[(k / Wn::ED) * Wn::SXP + TX + k % Wn::ED] = pd.x[t];
    }
    if (kValues && lane < B * B) S[Wn::REG + lane] = pd.wt;
}

// acc[k][q] += sum_{i,j < B} W[j*B + i] * S[(4ly + k + j) * SXP + 4lx + q + i],
// W = S + WOFF: a window of row pitch SXP with the box values after it
template <int B, int SXP, int WOFF>
__device__ __forceinline__ void correlate(float (&acc)[4][4], const float *S, int lx, int ly) {
    constexpr int NR = 4 + B - 1, NV = (NR + 3) / 4;
    const float *W = S + WOFF;
#pragma unroll
    for (int row = 0; row < NR; ++row) {
        float seg[4 * NV];
        const float4 *src = reinterpret_cast<const float4 *>(S + (4 * ly + row) * SXP + 4 * lx);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
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

// Park every wave's 4x4 micro-tiles in LDS as a 16 x 64 row-major tile
// (region `wv`), so that rows can then be summed over the waves in a fixed order.
__device__ __forceinline__ void park_tile(const float (&acc)[4][4], float *lds, int wv, int lx, int ly) {
    __syncthreads();   // every wave is done with its window region
    float *P = lds + wv * (TX * TY);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        *reinterpret_cast<float4 *>(P + (4 * ly + k) * TX + 4 * lx) =
            make_float4(acc[k][0], acc[k][1], acc[k][2], acc[k][3]);
    __syncthreads();
}

__device__ __forceinline__ float row_sum(const float *lds, int nw, int row, int lane) {
    float v = 0.0f;
    for (int w2 = 0; w2 < nw; ++w2) v += lds[w2 * (TX * TY) + row * TX + lane];
    return v;
}

// Wave `wv` of `nw` owns output rows wv, wv + nw, ... of the tile (at most TY).
#define FOR_OWN_ROWS(j, row)                                  \
    _Pragma("unroll") for (int j = 0; j < kRowsPerWave; ++j)  \
        if (const int row = wv + j * nw; row < TY)

// Forward epilogue: v = (H x)_i, gv = g_i, uv = u_i.
//   ratio: u = g / v (0 where v <= 0);
//   vjp:   e = -v u / ghat = -v u (u / g), 0 where u == 0 (u != 0 implies g != 0)
//   logratio: log(g / v) (0 where g <= 0 or v <= 0);
//   residual: (g - v) / R, uv = R (0 where R == 0)
__device__ __forceinline__ float fwd_epilogue(int mode, float v, float gv, float uv) {
    if (mode == kFwdRatio) return v > 0.0f ? gv / v : 0.0f;
    if (mode == kFwdVjp) return uv != 0.0f ? -(v * uv) * (uv / gv) : 0.0f;
    if (mode == kFwdLogRatio) return (gv > 0.0f && v > 0.0f) ? logf(gv / v) : 0.0f;
    if (mode == kFwdResidual) return uv != 0.0f ? (gv - v) / uv : 0.0f;
    return v;
}

// Whether a forward epilogue reads the auxiliary vector, and at which frame
// offset: u (kFwdVjp) is laid out like the output, R (kFwdResidual) like g.
__device__ __forceinline__ bool fwd_aux(int mode) { return mode == kFwdVjp || mode == kFwdResidual; }
__device__ __forceinline__ size_t fwd_aux_off(int mode, int g_off, int out_off) {
    return (size_t)(unsigned)(mode == kFwdResidual ? g_off : out_off);
}

// Update epilogues of the back projection v = (H^T r)_j of voxel j with the
// column sum hs and the current value fj:
//   EM:    fj v / hs;   SMART: fj exp(v / hs);   SART: max(0, fj + relax v / hs);
// 0 where hs == 0 (a voxel that no pixel sees).
__device__ __forceinline__ float adj_update(int mode, float fj, float v, float hs, float relax) {
    if (hs == 0.0f) return 0.0f;
    if (mode == kAdjMulExp) return fj * expf(v / hs);
    if (mode == kAdjAddClamp) return fmaxf(0.0f, fj + relax * (v / hs));
    return (fj * v) / hs;
}

// Forward projection.  Workgroups walk the unit list (grid stride); a unit is
// a chunk of the boxes meeting one FPA tile of one frame.  A tile split into
// several units writes one partial tile per unit to `partials`;
// k_finish_split sums them (next launch on the stream).
template <int B>
__global__ void __launch_bounds__(64 * Win<B>::MAXW) k_forward(const int4 *__restrict__ meta,
                                                               const int4 *__restrict__ items, const int stride,
                                                               const int n_units, const float *__restrict__ box_wf,
                                                               const float *__restrict__ f,
                                                               const float *__restrict__ g,
                                                               const float *__restrict__ uaux, float *__restrict__ out,
                                                               float *__restrict__ partials, const int mode) {
    using Wn = Win<B>;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    float *S = lds + wv * Wn::WREG;
    const int lx = lane & 15, ly = lane >> 4;

    for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
        const int4 *list = items + (size_t)unit * stride;
        int k = wv;
        int4 rec0 = record(list, k, stride);
        int4 rec1 = record(list, k + nw, stride);
        const int4 m0 = meta[3 * unit], m1 = meta[3 * unit + 1], m2 = meta[3 * unit + 2];
        const Geo geo{m1.x, m1.y, m1.z, m1.w};
        const int r0 = m0.x, c0 = m0.y;
        const int r = r0 + lane;
        const bool whole = m0.z == 1;

        // operands of the epilogue, fetched up front
        float gpre[kRowsPerWave], upre[kRowsPerWave];
        FOR_OWN_ROWS(j, row) {
            const int c = c0 + row;
            const bool in = mode != kFwdPlain && whole && r < geo.gamma && c < geo.xi;
            const size_t i = (size_t)r + (size_t)geo.gamma * c;
            gpre[j] = in ? g[(size_t)m2.x + i] : 0.0f;
            upre[j] = (in && fwd_aux(mode)) ? uaux[fwd_aux_off(mode, m2.x, m2.y) + i] : 0.0f;
        }

        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = 0.0f;

        // this lane's extra window slots (column 64 + e, row yy) as e + 64 yy
        unsigned xs[Wn::NXT > 0 ? Wn::NXT : 1];
#pragma unroll
        for (int t = 0; t < Wn::NXT; ++t) {
            const int kk = lane + 64 * t;
            xs[t] = kk < Wn::E * Wn::SY ? (unsigned)(kk % Wn::ED) + 64u * (unsigned)(kk / Wn::ED) : ~0u;
        }

        // one window in flight: once item k's window is in LDS, the window of
        // the wave's next item (k + nw) is fetched into registers while item k
        // is correlated; the work records run one item further ahead
        Pending<B> pa;
        if (rec0.w >= 0) {
            if (rec0.z & kDirectFlag)
                load_forward_direct<B>(pa, f, box_wf, geo, rec0, lane, xs);
            else
                load_forward<B>(pa, f, box_wf, geo, rec0, lane);
        }
        while (rec0.w >= 0) {
            store_window<B>(S, pa, lane);
            wave_lds_sync();
            k += nw;
            const int4 rec3 = record(list, k + nw, stride);
            if (rec1.w >= 0) {
                if (rec1.z & kDirectFlag)
                    load_forward_direct<B>(pa, f, box_wf, geo, rec1, lane, xs);
                else
                    load_forward<B>(pa, f, box_wf, geo, rec1, lane);
            }
            correlate<B, Win<B>::SXP, Win<B>::REG>(acc, S, lx, ly);
            wave_lds_sync();
            rec0 = rec1;
            rec1 = rec3;
        }

        park_tile(acc, lds, wv, lx, ly);
        if (!whole) {
            float *mine = partials + (size_t)m0.w * (TX * TY);
            FOR_OWN_ROWS(j, row) mine[row * TX + lane] = row_sum(lds, nw, row, lane);
        } else {
            FOR_OWN_ROWS(j, row) {
                const int c = c0 + row;
                const float v = row_sum(lds, nw, row, lane);
                if (r < geo.gamma && c < geo.xi)
                    out[(size_t)m2.y + (size_t)r + (size_t)geo.gamma * c] = fwd_epilogue(mode, v, gpre[j], upre[j]);
            }
        }
        __syncthreads();   // the next unit reuses the LDS regions
    }
}

// Sum the partial tiles of every split FPA tile in chunk order and apply the
// forward epilogue.  One workgroup (4 waves, 4 rows each) per split tile.
__global__ void __launch_bounds__(256) k_finish_split(const int4 *__restrict__ split_meta,
                                                      const float *__restrict__ partials,
                                                      const float *__restrict__ g, const float *__restrict__ uaux,
                                                      float *__restrict__ out, int mode) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int4 s0 = split_meta[2 * blockIdx.x], s1 = split_meta[2 * blockIdx.x + 1];
    const int r = s0.x + lane;
#pragma unroll
    for (int j = 0; j < TY / 4; ++j) {
        const int row = wv + 4 * j, c = s0.y + row;
        if (r >= s1.x || c >= s1.y) continue;
        const size_t i = (size_t)r + (size_t)s1.x * c;
        const float gv = mode != kFwdPlain ? g[(size_t)s1.z + i] : 0.0f;
        const float uv = fwd_aux(mode) ? uaux[fwd_aux_off(mode, s1.z, s1.w) + i] : 0.0f;
        float v = 0.0f;
        for (int ch = 0; ch < s0.z; ++ch) v += partials[((size_t)s0.w + ch) * (TX * TY) + row * TX + lane];
        out[(size_t)s1.w + i] = fwd_epilogue(mode, v, gv, uv);
    }
}

// ---------------------------------------------------------------------------
// Region forward projection (the EM path).  A wavefront is G = 64 / GL
// groups of GL lanes (GL = 16, 8 or 4 by region shape SH).  A group owns an
// FPA region of 16 GL pixels, (4 GX) x (4 GY) with GX * GY = GL (GX x GY
// lanes with a 4 x 4 register micro-tile each), and takes one box of the
// region's work list at a time, so the G groups of a wave correlate G
// different boxes with the same region at once, and the waves of a
// workgroup split the region's boxes.  At the end the groups are summed with
// a fixed butterfly and the waves in LDS in a fixed order (deterministic
// results).  The small region keeps the outputs computed per box close to
// the box's shifted field-stop image: a larger output tile spends its
// multiply-adds on the overhang, where the window holds zeros.
//
// The windows come from a zero-bordered copy of f (per wavelength a block of
// (a + 2 Hx) x (alpha + 2 Hy) floats, Hx = 4 GX + B - 2, Hy = 4 GY + B - 2,
// written by k_pad and by the back projection's EM update): the host writes
// each window origin as a position of that block, so a window is a plain
// 2-D rectangle of it, read in 16-byte pieces with no field-stop test and no
// wrap arithmetic (exact when the FPA leaves Hx and Hy pixels beside the
// field stop; the tile kernel serves other plans).
template <int B, int SH>
struct RWin {
    static constexpr int GX = region_gx(SH), GL = region_gl(SH);
    static constexpr int GROUPS = 64 / GL;         // lane groups per wavefront
    static constexpr int GY = GL / GX;
    static constexpr int RX = 4 * GX, RY = 4 * GY;  // region (fast x slow)
    static constexpr int NPIX = RX * RY;           // outputs of a region
    static constexpr int SX = RX + B - 1;          // window extent, fast axis
    static constexpr int SX4 = (SX + 3) / 4;       // 16-byte pieces per window row
    static constexpr int SXP = 4 * SX4;            // LDS row pitch
    static constexpr int SY = RY + B - 1;          // window extent, slow axis
    static constexpr int REG = SXP * SY;           // window floats per group
    static constexpr int BB = B * B;
    static constexpr int GREG = REG + ((BB + 3) & ~3);   // window + box values
    static constexpr int WAVE = GROUPS * GREG;     // LDS floats per wavefront
    static constexpr int NSLOT = SX4 * SY;         // 16-byte pieces per window
    static constexpr int NT = (NSLOT + GL - 1) / GL;
    static constexpr int NWT = (BB + GL - 1) / GL;
    static constexpr int MAXW = kFwdMaxWaves;
    static_assert(SH >= 1 && SH <= kRegionShapes, "region shape code");
    static_assert(GL % GX == 0 && 64 % GL == 0 && GROUPS >= 4, "whole groups, at least four per wave");
    static_assert(NPIX == 16 * GL && NPIX <= kRegionPixels, "a group covers 16 GL pixels");
    static_assert(RX == region_fast(SH) && RY == region_slow(SH), "the host's region shape");
    static_assert(WAVE >= NPIX, "the reduction parks a region per wave");
    static_assert(REG % 4 == 0 && GREG % 4 == 0, "16-byte aligned group regions");
    static_assert(4 * (GX - 1) + 4 * ((4 + B - 1 + 3) / 4) <= SXP, "segment reads stay inside the row");
    static_assert(halo_fast(SH, B) >= SX - 1 && halo_slow(SH, B) >= SY - 1,
                  "a window meeting the field stop stays inside the padded block");
};

// One window in flight per group lane, in registers: its 16-byte pieces of
// the window and its share of the box's values.
template <int B, int SH>
struct RPend {
    float4 v[RWin<B, SH>::NT];
    float wt[RWin<B, SH>::NWT];
};


// Window of one (region, box) item, rec = (origin, 0, 0, box): piece t of
// this lane at byte offset 4*origin + poff[t] of the padded copy (poff: the
// piece's column and row within the window; 0 for a lane without a piece t,
// whose load is then not stored); box < 0 (an empty slot) reads zeros (the
// out-of-range offset).  A piece may run up to three floats past the
// window's last column (LDS pitch padding, never used).
template <int B, int SH>
__device__ __forceinline__ void load_region(RPend<B, SH> &pd, __amdgpu_buffer_rsrc_t fr, __amdgpu_buffer_rsrc_t wr,
                                            int4 rec, int gl, const unsigned (&poff)[RWin<B, SH>::NT]) {
    using Wn = RWin<B, SH>;
    const bool ok = rec.w >= 0;
    const unsigned base = ok ? 4u * (unsigned)rec.x : kOutOfRange;
#pragma unroll
    for (int t = 0; t < Wn::NT; ++t) pd.v[t] = bload4(fr, base + poff[t]);
#pragma unroll
    for (int t = 0; t < Wn::NWT; ++t) {
        const int k = gl + Wn::GL * t;
        pd.wt[t] = bload(wr, (ok && k < Wn::BB) ? 4u * (unsigned)(rec.w * Wn::BB + k) : kOutOfRange);
    }
}

// Window into S[0, REG), box values into S[REG, REG + B*B).  Piece k (row
// k / SX4, column quad k % SX4) lands at float 4k: the row pitch is 4 SX4.
template <int B, int SH>
__device__ __forceinline__ void store_region(float *S, const RPend<B, SH> &pd, int gl) {
    using Wn = RWin<B, SH>;
    static_assert(Wn::SXP == 4 * Wn::SX4, "pieces are packed row after row");
#pragma unroll
    for (int t = 0; t < Wn::NT; ++t) {
        const int k = gl + Wn::GL * t;
        if (t + 1 < Wn::NT || k < Wn::NSLOT) *reinterpret_cast<float4 *>(S + 4 * k) = pd.v[t];
    }
#pragma unroll
    for (int t = 0; t < Wn::NWT; ++t) {
        const int k = gl + Wn::GL * t;
        if (k < Wn::BB) S[Wn::REG + k] = pd.wt[t];
    }
}

// Byte offset, from the window origin in the padded copy (row pitch P
// floats), of piece t of group lane gl: piece k = gl + GL t sits at row
// k / SX4, column quad k % SX4, found from gl's own row and column by a
// compile-time step and one carry; 0 for a lane without a piece t.
template <int B, int SH>
__device__ __forceinline__ void region_piece_offsets(unsigned int (&poff)[RWin<B, SH>::NT], int gl, int P) {
    using Wn = RWin<B, SH>;
    const int row0 = gl / Wn::SX4, col0 = gl - row0 * Wn::SX4;
    const unsigned prow = 4u * (unsigned)P;
#pragma unroll
    for (int t = 0; t < Wn::NT; ++t) {
        const int dr = (Wn::GL * t) / Wn::SX4, dc = (Wn::GL * t) % Wn::SX4;
        const bool carry = col0 + dc >= Wn::SX4;
        const int row = row0 + dr + (carry ? 1 : 0), col = col0 + dc - (carry ? Wn::SX4 : 0);
        poff[t] = gl + Wn::GL * t < Wn::NSLOT ? 16u * (unsigned)col + prow * (unsigned)row : 0u;
    }
}

// Region forward.  Workgroups walk the unit list (grid stride); a unit is a
// chunk of the boxes meeting one FPA region of one frame (meta as the tile
// list's, with the padded block's row pitch P in the third record).  A region
// split into several units writes one partial region per unit to
// `partials` (slots of kRegionPixels floats); k_finish_regions sums them
// (next launch on the stream).
template <int B, int SH>
__global__ void __launch_bounds__(64 * kFwdMaxWaves) k_forward_region(
    const int4 *__restrict__ meta, const int4 *__restrict__ items, const int stride, const int n_units,
    const float *__restrict__ box_wf, const int n_wf, const float *__restrict__ fp, const int fp_floats,
    const float *__restrict__ g, const float *__restrict__ uaux, float *__restrict__ out,
    float *__restrict__ partials, const int mode) {
    using Wn = RWin<B, SH>;
    constexpr int RX = Wn::RX, GL = Wn::GL, NG = Wn::GROUPS, NPIX = Wn::NPIX;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int gi = lane / GL, gl = lane % GL, lx = gl % Wn::GX, ly = gl / Wn::GX;
    float *S = lds + wv * Wn::WAVE + gi * Wn::GREG;
    const __amdgpu_buffer_rsrc_t fr = rsrc(fp, fp_floats);
    const __amdgpu_buffer_rsrc_t wr = rsrc(box_wf, n_wf);
    const int tid = threadIdx.x, nt = blockDim.x;
    constexpr int kOut = NPIX / 64;   // outputs per thread at one wave per workgroup

    for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
        const int4 *list = items + (size_t)unit * stride;
        const int4 m0 = meta[3 * unit], m1 = meta[3 * unit + 1], m2 = meta[3 * unit + 2];
        const int gamma = m1.z, xi = m1.w;
        const int r0 = m0.x, c0 = m0.y;
        const bool whole = m0.z == 1;
        // byte offsets of this lane's window pieces from the window origin
        unsigned poff[Wn::NT];
        region_piece_offsets<B, SH>(poff, gl, m2.z);
        const int step = NG * nw;
        int k = NG * wv + gi;
        int4 rec0 = record(list, k, stride);
        int4 rec1 = record(list, k + step, stride);

        // operands of the epilogue (output o = tid + nt*j of the region): up
        // to B = 3 fetched here, off the critical path of short units (the
        // registers are there); for larger boxes after the item loop, which
        // keeps the loop at fewer VGPRs
        constexpr bool kEarly = B <= 3;
        float gpre[kOut], upre[kOut];
        auto fetch_operands = [&]() {
#pragma unroll
            for (int j = 0; j < kOut; ++j) {
                const int o = tid + nt * j;
                const int r = r0 + o % RX, c = c0 + o / RX;
                const bool in = o < NPIX && mode != kFwdPlain && whole && r < gamma && c < xi;
                const size_t i = (size_t)r + (size_t)gamma * c;
                gpre[j] = in ? g[(size_t)m2.x + i] : 0.0f;
                upre[j] = (in && fwd_aux(mode)) ? uaux[fwd_aux_off(mode, m2.x, m2.y) + i] : 0.0f;
            }
        };
        if (kEarly) fetch_operands();

        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = 0.0f;

        // one window in flight per group: while the groups correlate their
        // items, the windows of the wave's next NG items are fetched (an
        // empty record reads zeros); the work records run one pass further
        // ahead.  Lists are padded with empty records, so a wave is done once
        // its first group has none.
        RPend<B, SH> pa;
        load_region<B, SH>(pa, fr, wr, rec0, gl, poff);
        if (__builtin_amdgcn_readfirstlane(rec0.w) >= 0) {
            do {
                store_region<B, SH>(S, pa, gl);
                wave_lds_sync();
                k += step;
                const int4 rec3 = record(list, k + step, stride);
                load_region<B, SH>(pa, fr, wr, rec1, gl, poff);
                correlate<B, Wn::SXP, Wn::REG>(acc, S, lx, ly);
                wave_lds_sync();
                rec0 = rec1;
                rec1 = rec3;
            } while (__builtin_amdgcn_readfirstlane(rec0.w) >= 0);
        }

        if (!kEarly) fetch_operands();   // while the groups and waves are summed

        // sum of the groups (lanes l, l ^ GL, l ^ 2 GL, ... hold the same
        // outputs): a butterfly over the group index, every group ends with
        // the same sum (for four groups ((g0 + g1) + (g2 + g3)))
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float v = acc[a][q];
#pragma unroll
                for (int off = GL; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
                acc[a][q] = v;
            }
        // park the wave's region in LDS (group gi < 4 stores row gi of its
        // lanes' micro-tiles), then sum the waves in order
        __syncthreads();   // every wave is done with its windows
        if (gi < 4) {
            float4 row = make_float4(acc[0][0], acc[0][1], acc[0][2], acc[0][3]);
#pragma unroll
            for (int a = 1; a < 4; ++a)
                if (gi == a) row = make_float4(acc[a][0], acc[a][1], acc[a][2], acc[a][3]);
            *reinterpret_cast<float4 *>(lds + wv * Wn::WAVE + (4 * ly + gi) * RX + 4 * lx) = row;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kOut; ++j) {
            const int o = tid + nt * j;
            if (o >= NPIX) continue;
            float v = 0.0f;
            for (int w2 = 0; w2 < nw; ++w2) v += lds[w2 * Wn::WAVE + o];
            if (!whole) {
                partials[(size_t)m0.w * kRegionPixels + o] = v;
            } else {
                const int r = r0 + o % RX, c = c0 + o / RX;
                if (r < gamma && c < xi)
                    out[(size_t)m2.y + (size_t)r + (size_t)gamma * c] = fwd_epilogue(mode, v, gpre[j], upre[j]);
            }
        }
        __syncthreads();   // the next unit reuses the LDS regions
    }
}

// Solo region forward: every group of GL lanes owns a whole unit (one FPA
// region, or one chunk of a split region) and walks all of its boxes, so a
// wavefront advances 64 / GL units side by side (neighbours in the
// work-sorted unit list, so of about equal length; a group whose list has
// ended loads zeros); no cross-group or cross-wave reduction, no workgroup
// barrier, each group parks its region in its window area and writes it row
// by row.  For batches of many short regions, where the cooperative
// kernel's set-up and reductions outweigh a unit's few passes.
template <int B, int SH>
__global__ void __launch_bounds__(64 * kSoloWaves) k_forward_region_solo(
    const int4 *__restrict__ meta, const int4 *__restrict__ items, const int stride, const int n_units,
    const float *__restrict__ box_wf, const int n_wf, const float *__restrict__ fp, const int fp_floats,
    const float *__restrict__ g, const float *__restrict__ uaux, float *__restrict__ out,
    float *__restrict__ partials, const int mode) {
    using Wn = RWin<B, SH>;
    constexpr int RX = Wn::RX, GL = Wn::GL, NG = Wn::GROUPS, NPIX = Wn::NPIX;
    static_assert(Wn::REG >= NPIX, "a group parks its region in its window area");
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int gi = lane / GL, gl = lane % GL, lx = gl % Wn::GX, ly = gl / Wn::GX;
    float *S = lds + wv * Wn::WAVE + gi * Wn::GREG;
    const __amdgpu_buffer_rsrc_t fr = rsrc(fp, fp_floats);
    const __amdgpu_buffer_rsrc_t wr = rsrc(box_wf, n_wf);

    const int nv = solo_groups(n_units, nw * NG);
    for (int v = blockIdx.x; v < nv; v += gridDim.x) {
        const int first = solo_unit(v, wv * NG, nw * NG);
        if (first >= n_units) continue;   // so are the wave's other groups
        const int unit = solo_unit(v, wv * NG + gi, nw * NG);
        const bool active = unit < n_units;
        const int u = active ? unit : first;   // a valid unit for the loads; its results are dropped
        const int4 *list = items + (size_t)u * stride;
        const int4 m0 = meta[3 * u], m1 = meta[3 * u + 1], m2 = meta[3 * u + 2];
        const int gamma = m1.z, xi = m1.w;
        unsigned poff[Wn::NT];
        region_piece_offsets<B, SH>(poff, gl, m2.z);
        const int kend = active ? stride : 0;   // an inactive group reads empty records
        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = 0.0f;

        int k = 0;
        int4 rec0 = record(list, k, kend);
        int4 rec1 = record(list, k + 1, kend);
        RPend<B, SH> pa;
        load_region<B, SH>(pa, fr, wr, rec0, gl, poff);
        while (__builtin_amdgcn_ballot_w64(rec0.w >= 0) != 0) {
            store_region<B, SH>(S, pa, gl);
            wave_lds_sync();
            k += 1;
            const int4 rec3 = record(list, k + 1, kend);
            load_region<B, SH>(pa, fr, wr, rec1, gl, poff);
            correlate<B, Wn::SXP, Wn::REG>(acc, S, lx, ly);
            wave_lds_sync();
            rec0 = rec1;
            rec1 = rec3;
        }
        // the group's region, parked row-major in its window area, leaves
        // row by row (contiguous stores of the group's lanes)
#pragma unroll
        for (int kq = 0; kq < 4; ++kq)
            *reinterpret_cast<float4 *>(S + (4 * ly + kq) * RX + 4 * lx) =
                make_float4(acc[kq][0], acc[kq][1], acc[kq][2], acc[kq][3]);
        wave_lds_sync();
        if (active) {
            const int r0 = m0.x, c0 = m0.y;
            const bool whole = m0.z == 1;
#pragma unroll
            for (int j = 0; j < NPIX / GL; ++j) {
                const int o = gl + GL * j;
                const float v = S[o];
                if (!whole) {   // a chunk of a split region: its partial region
                    partials[(size_t)m0.w * kRegionPixels + o] = v;
                    continue;
                }
                const int r = r0 + o % RX, c = c0 + o / RX;
                if (r < gamma && c < xi) {
                    const size_t i = (size_t)r + (size_t)gamma * c;
                    const float gv = mode != kFwdPlain ? g[(size_t)m2.x + i] : 0.0f;
                    const float uv = fwd_aux(mode) ? uaux[fwd_aux_off(mode, m2.x, m2.y) + i] : 0.0f;
                    out[(size_t)m2.y + i] = fwd_epilogue(mode, v, gv, uv);
                }
            }
        }
        wave_lds_sync();   // the next unit's first window overwrites the parked region
    }
}

// Sum the partial regions (rx x ry pixels, slots of kRegionPixels floats) of
// every split FPA region in chunk order and apply the forward epilogue.  One
// workgroup (a thread per slot float) per split region.
__global__ void __launch_bounds__(kRegionPixels) k_finish_regions(const int4 *__restrict__ split_meta,
                                                                  const float *__restrict__ partials,
                                                                  const float *__restrict__ g,
                                                                  const float *__restrict__ uaux,
                                                                  float *__restrict__ out, int mode, int rx, int ry) {
    const int o = threadIdx.x;
    if (o >= rx * ry) return;
    const int4 s0 = split_meta[2 * blockIdx.x], s1 = split_meta[2 * blockIdx.x + 1];
    const int r = s0.x + o % rx, c = s0.y + o / rx;
    if (r >= s1.x || c >= s1.y) return;
    const size_t i = (size_t)r + (size_t)s1.x * c;
    const float gv = mode != kFwdPlain ? g[(size_t)s1.z + i] : 0.0f;
    const float uv = fwd_aux(mode) ? uaux[fwd_aux_off(mode, s1.z, s1.w) + i] : 0.0f;
    float v = 0.0f;
    for (int ch = 0; ch < s0.z; ++ch) v += partials[((size_t)s0.w + ch) * kRegionPixels + o];
    out[(size_t)s1.w + i] = fwd_epilogue(mode, v, gv, uv);
}

// x[0, n) = v (grid-strided); a kernel rather than a memset so that a
// captured graph replays it like any other node.
__global__ void __launch_bounds__(256) k_fill(float *__restrict__ x, const int64_t n, const float v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = v;
}

// Zero-bordered copy of x for the region forward.  Block b = (x offset,
// padded offset, a, alpha) of one (frame, wavelength); workgroup (row, b)
// writes padded row `row` (rows 0 .. alpha + 2 hy - 1, pitch a + 2 hx):
// element (X, Y) of the block, X in [-hx, a + hx), Y in [-hy, alpha + hy),
// holds x_s(X, Y) inside the field stop and 0 outside.
__global__ void __launch_bounds__(256) k_pad(const int4 *__restrict__ blocks, const float *__restrict__ x,
                                             float *__restrict__ fp, const int hx, const int hy) {
    const int4 bl = blocks[blockIdx.y];
    const int a = bl.z, alpha = bl.w, P = a + 2 * hx;
    const int row = blockIdx.x;
    if (row >= alpha + 2 * hy) return;
    const int Y = row - hy;
    const bool yin = Y >= 0 && Y < alpha;
    float *dst = fp + (size_t)bl.y + (size_t)P * row;
    const float *src = x + (size_t)bl.x + (size_t)a * (yin ? Y : 0);
    for (int e = threadIdx.x; e < P; e += blockDim.x) {
        const int X = e - hx;
        dst[e] = (yin && X >= 0 && X < a) ? src[X] : 0.0f;
    }
}

// Back projection (+ EM update).  Units: (frame, wavelength, field-stop tile).
template <int B, bool D4>
__global__ void __launch_bounds__(64 * Win<B>::MAXW) k_adjoint(const int4 *__restrict__ meta,
                                                               const int4 *__restrict__ items, const int stride,
                                                               const int n_units, const float *__restrict__ box_w,
                                                               const float *__restrict__ hsum,
                                                               const float *__restrict__ u, const float *in1,
                                                               const float *__restrict__ in2, float *out,
                                                               float *__restrict__ out2, float *__restrict__ flux,
                                                               const int mode, float *__restrict__ fpad,
                                                               const int hx, const int hy, const float relax) {
    using Wn = Win<B>;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    float *S = lds + wv * Wn::WREG;
    const int lx = lane & 15, ly = lane >> 4;

    for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
        const int4 m0 = meta[3 * unit], m1 = meta[3 * unit + 1], m2 = meta[3 * unit + 2];
        const int4 *list = items + (size_t)m0.z * stride;
        int k = wv;
        int4 rec0 = record(list, k, stride);
        int4 rec1 = record(list, k + nw, stride);
                const Geo geo{m1.x, m1.y, m1.z, m1.w};
        const int x0 = m0.x, y0 = m0.y;
        const __amdgpu_buffer_rsrc_t ur = rsrc(u + (size_t)(unsigned)m2.x, geo.gamma * geo.xi);
        const int x = x0 + lane;
        const size_t sb = (size_t)(unsigned)m0.w;

        // operands of the epilogue (in1: f or y; in2: f or zeta), fetched up front
        float p1[kRowsPerWave], p2[kRowsPerWave];
        FOR_OWN_ROWS(j, row) {
            const int y = y0 + row;
            const bool in = x < geo.a && y < geo.alpha;
            const size_t o = sb + (size_t)x + (size_t)geo.a * y;
            p1[j] = (in && mode != kAdjPlain) ? in1[o] : 0.0f;
            p2[j] = (in && (mode == kAdjVjpPre || mode == kAdjVjpGrad)) ? in2[o] : 0.0f;
        }
        const float hs = hsum[m0.z];

        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = 0.0f;

        // byte offsets of this lane's extra window slots (column 64 + e, row
        // yy) within a direct window; with D4 (every box of the list direct)
        // the offsets of its 16-byte pieces instead
        unsigned xo[Wn::NXT > 0 ? Wn::NXT : 1];
        unsigned voff[Pending4<B>::NQ];
        if constexpr (D4) {
            adjoint_piece_offsets<B>(voff, lane, geo.gamma);
        } else {
#pragma unroll
            for (int t = 0; t < Wn::NXT; ++t) {
                const int kk = lane + 64 * t;
                xo[t] = kk < Wn::E * Wn::SY ? 4u * (unsigned)(TX + kk % Wn::ED) + 4u * (unsigned)geo.gamma *
                                                                                       (unsigned)(kk / Wn::ED)
                                            : 0u;
            }
        }

        Pending<B> pa;
        Pending4<B> pq;
        auto fetch = [&](int4 rec) {
            if (rec.w < 0) return;
            if constexpr (D4)
                load_adjoint_direct4<B>(pq, ur, box_w, geo, rec.x + x0, rec.y + y0, rec.w, lane, voff);
            else if (rec.z)
                load_adjoint_direct<B>(pa, ur, box_w, geo, rec.x + x0, rec.y + y0, rec.w, lane, xo);
            else
                load_adjoint<B>(pa, ur, box_w, geo, rec.x + x0, rec.y + y0, rec.w, lane);
        };
        fetch(rec0);
        while (rec0.w >= 0) {
            if constexpr (D4)
                store_window4<B>(S, pq, lane);
            else
                store_window<B>(S, pa, lane);
            wave_lds_sync();
            k += nw;
            const int4 rec3 = record(list, k + nw, stride);
            fetch(rec1);
            correlate<B, Win<B>::SXP, Win<B>::REG>(acc, S, lx, ly);
            wave_lds_sync();
            rec0 = rec1;
            rec1 = rec3;
        }

        park_tile(acc, lds, wv, lx, ly);
        float fl = 0.0f;   // this lane's share of sum b zeta (kAdjVjpPre)
        FOR_OWN_ROWS(j, row) {
            const int y = y0 + row;
            const float v = row_sum(lds, nw, row, lane);
            if (x < geo.a && y < geo.alpha) {
                const size_t o = sb + (size_t)x + (size_t)geo.a * y;
                if (mode == kAdjPlain) {
                    out[o] = v;
                } else if (adj_updates(mode)) {
                    const float nf = adj_update(mode, p1[j], v, hs, relax);
                    out[o] = nf;
                    // the padded copy of f the region forward reads (block offset
                    // m2.y, row pitch m2.z)
                    if (fpad) fpad[(size_t)m2.y + (size_t)(x + hx) + (size_t)m2.z * (size_t)(y + hy)] = nf;
                } else if (mode == kAdjVjpPre) {
                    const float bj = hs != 0.0f ? (p1[j] * p2[j]) / hs : 0.0f;
                    out[o] = v;
                    out2[o] = bj;
                    fl = __builtin_fmaf(bj, v, fl);
                } else {
                    out[o] = (hs != 0.0f ? (p1[j] * p2[j]) / hs : 0.0f) + v;
                }
            }
        }
        if (mode == kAdjVjpPre) {
            // sum over the unit: wavefront butterfly, then the waves in order
            fl = wave_sum(fl);
            float *red = lds + nw * (TX * TY);   // past the parked tiles
            if (lane == 0) red[wv] = fl;
            __syncthreads();
            if (threadIdx.x == 0) {
                float t = 0.0f;
                for (int w2 = 0; w2 < nw; ++w2) t += red[w2];
                flux[unit] = t;
            }
        }
        __syncthreads();   // the next unit reuses the LDS regions
    }
}

// ---------------------------------------------------------------------------
// Solo variants of the tile kernels: every wavefront owns a whole work unit
// (one FPA tile, or one wavelength's field-stop tile) and walks all its boxes
// with one window in flight; no cross-wave reduction, no workgroup barrier.
// The wave parks its tile in its own window area and writes it row by row.  For batches of many small units
// (few boxes each), where splitting a unit's boxes over the waves of a
// workgroup leaves each wave too few items to hide a window load.

// Micro-tile element (k, q) of lane (lx, ly) is output (tx, ty) = (4 lx + q,
// 4 ly + k) of the 64 x 16 tile.
template <int B>
__global__ void __launch_bounds__(256) k_forward_solo(const int4 *__restrict__ meta,
                                                      const int4 *__restrict__ items, const int stride,
                                                      const int n_units, const float *__restrict__ box_wf,
                                                      const float *__restrict__ f, const float *__restrict__ g,
                                                      const float *__restrict__ uaux, float *__restrict__ out,
                                                      float *__restrict__ partials, const int mode) {
    using Wn = Win<B>;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    float *S = lds + wv * Wn::WREG;
    const int lx = lane & 15, ly = lane >> 4;

    unsigned xs[Wn::NXT > 0 ? Wn::NXT : 1];
#pragma unroll
    for (int t = 0; t < Wn::NXT; ++t) {
        const int kk = lane + 64 * t;
        xs[t] = kk < Wn::E * Wn::SY ? (unsigned)(kk % Wn::ED) + 64u * (unsigned)(kk / Wn::ED) : ~0u;
    }

    const int nv = solo_groups(n_units, nw);
    for (int v = blockIdx.x; v < nv; v += gridDim.x) {
        const int unit = solo_unit(v, wv, nw);
        if (unit >= n_units) continue;
        const int4 *list = items + (size_t)unit * stride;
        const int4 m0 = meta[3 * unit], m1 = meta[3 * unit + 1], m2 = meta[3 * unit + 2];
        const Geo geo{m1.x, m1.y, m1.z, m1.w};
        const int r0 = m0.x, c0 = m0.y;
        const bool whole = m0.z == 1;
        int k = 0;
        int4 rec0 = record(list, 0, stride);
        int4 rec1 = record(list, 1, stride);

        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = 0.0f;

        Pending<B> pa;
        if (rec0.w >= 0) {
            if (rec0.z & kDirectFlag)
                load_forward_direct<B>(pa, f, box_wf, geo, rec0, lane, xs);
            else
                load_forward<B>(pa, f, box_wf, geo, rec0, lane);
        }
        while (rec0.w >= 0) {
            store_window<B>(S, pa, lane);
            wave_lds_sync();
            k += 1;
            const int4 rec3 = record(list, k + 1, stride);
            if (rec1.w >= 0) {
                if (rec1.z & kDirectFlag)
                    load_forward_direct<B>(pa, f, box_wf, geo, rec1, lane, xs);
                else
                    load_forward<B>(pa, f, box_wf, geo, rec1, lane);
            }
            correlate<B, Win<B>::SXP, Win<B>::REG>(acc, S, lx, ly);
            wave_lds_sync();
            rec0 = rec1;
            rec1 = rec3;
        }

        // the tile, parked row-major in the wave's window area, leaves row by
        // row (256-byte stores)
#pragma unroll
        for (int kq = 0; kq < 4; ++kq)
            *reinterpret_cast<float4 *>(S + (4 * ly + kq) * TX + 4 * lx) =
                make_float4(acc[kq][0], acc[kq][1], acc[kq][2], acc[kq][3]);
        wave_lds_sync();
        const int r = r0 + lane;
#pragma unroll
        for (int ty = 0; ty < TY; ++ty) {
            const float v = S[ty * TX + lane];
            if (!whole) {
                partials[(size_t)m0.w * (TX * TY) + ty * TX + lane] = v;
                continue;
            }
            const int c = c0 + ty;
            if (r < geo.gamma && c < geo.xi) {
                const size_t i = (size_t)r + (size_t)geo.gamma * c;
                const float gv = mode != kFwdPlain ? g[(size_t)m2.x + i] : 0.0f;
                const float uv = fwd_aux(mode) ? uaux[fwd_aux_off(mode, m2.x, m2.y) + i] : 0.0f;
                out[(size_t)m2.y + i] = fwd_epilogue(mode, v, gv, uv);
            }
        }
        wave_lds_sync();   // the next unit's first window overwrites the parked tile
    }
}

template <int B, bool D4>
__global__ void __launch_bounds__(256) k_adjoint_solo(const int4 *__restrict__ meta,
                                                      const int4 *__restrict__ items, const int stride,
                                                      const int n_units, const float *__restrict__ box_w,
                                                      const float *__restrict__ hsum, const float *__restrict__ u,
                                                      const float *in1, const float *__restrict__ in2, float *out,
                                                      float *__restrict__ out2, float *__restrict__ flux,
                                                      const int mode, float *__restrict__ fpad, const int hx,
                                                      const int hy, const float relax) {
    using Wn = Win<B>;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    float *S = lds + wv * Wn::WREG;
    const int lx = lane & 15, ly = lane >> 4;

    const int nv = solo_groups(n_units, nw);
    for (int v = blockIdx.x; v < nv; v += gridDim.x) {
        const int unit = solo_unit(v, wv, nw);
        if (unit >= n_units) continue;
        const int4 m0 = meta[3 * unit], m1 = meta[3 * unit + 1], m2 = meta[3 * unit + 2];
        const int4 *list = items + (size_t)m0.z * stride;
        const Geo geo{m1.x, m1.y, m1.z, m1.w};
        const int x0 = m0.x, y0 = m0.y;
        const __amdgpu_buffer_rsrc_t ur = rsrc(u + (size_t)(unsigned)m2.x, geo.gamma * geo.xi);
        const size_t sb = (size_t)(unsigned)m0.w;
        const float hs = hsum[m0.z];
        int k = 0;
        int4 rec0 = record(list, 0, stride);
        int4 rec1 = record(list, 1, stride);

        unsigned xo[Wn::NXT > 0 ? Wn::NXT : 1];
        unsigned voff[Pending4<B>::NQ];
        if constexpr (D4) {
            adjoint_piece_offsets<B>(voff, lane, geo.gamma);
        } else {
#pragma unroll
            for (int t = 0; t < Wn::NXT; ++t) {
                const int kk = lane + 64 * t;
                xo[t] = kk < Wn::E * Wn::SY ? 4u * (unsigned)(TX + kk % Wn::ED) + 4u * (unsigned)geo.gamma *
                                                                                       (unsigned)(kk / Wn::ED)
                                            : 0u;
            }
        }

        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][q] = 0.0f;

        Pending<B> pa;
        Pending4<B> pq;
        auto fetch = [&](int4 rec) {
            if (rec.w < 0) return;
            if constexpr (D4)
                load_adjoint_direct4<B>(pq, ur, box_w, geo, rec.x + x0, rec.y + y0, rec.w, lane, voff);
            else if (rec.z)
                load_adjoint_direct<B>(pa, ur, box_w, geo, rec.x + x0, rec.y + y0, rec.w, lane, xo);
            else
                load_adjoint<B>(pa, ur, box_w, geo, rec.x + x0, rec.y + y0, rec.w, lane);
        };
        fetch(rec0);
        while (rec0.w >= 0) {
            if constexpr (D4)
                store_window4<B>(S, pq, lane);
            else
                store_window<B>(S, pa, lane);
            wave_lds_sync();
            k += 1;
            const int4 rec3 = record(list, k + 1, stride);
            fetch(rec1);
            correlate<B, Win<B>::SXP, Win<B>::REG>(acc, S, lx, ly);
            wave_lds_sync();
            rec0 = rec1;
            rec1 = rec3;
        }

#pragma unroll
        for (int kq = 0; kq < 4; ++kq)
            *reinterpret_cast<float4 *>(S + (4 * ly + kq) * TX + 4 * lx) =
                make_float4(acc[kq][0], acc[kq][1], acc[kq][2], acc[kq][3]);
        wave_lds_sync();
        float fl = 0.0f;   // this lane's share of sum b zeta (kAdjVjpPre)
        const int x = x0 + lane;
#pragma unroll
        for (int ty = 0; ty < TY; ++ty) {
            const int y = y0 + ty;
            if (x < geo.a && y < geo.alpha) {
                const size_t o = sb + (size_t)x + (size_t)geo.a * y;
                const float v = S[ty * TX + lane];
                if (mode == kAdjPlain) {
                    out[o] = v;
                } else if (adj_updates(mode)) {
                    const float nf = adj_update(mode, in1[o], v, hs, relax);
                    out[o] = nf;
                    if (fpad) fpad[(size_t)m2.y + (size_t)(x + hx) + (size_t)m2.z * (size_t)(y + hy)] = nf;
                } else if (mode == kAdjVjpPre) {
                    const float bj = hs != 0.0f ? (in1[o] * in2[o]) / hs : 0.0f;
                    out[o] = v;
                    out2[o] = bj;
                    fl = __builtin_fmaf(bj, v, fl);
                } else {
                    out[o] = (hs != 0.0f ? (in1[o] * in2[o]) / hs : 0.0f) + v;
                }
            }
        }
        if (mode == kAdjVjpPre) {
            fl = wave_sum(fl);
            if (lane == 0) flux[unit] = fl;
        }
        wave_lds_sync();   // the next unit's first window overwrites the parked tile
    }
}

// ---------------------------------------------------------------------------
// Derivatives with respect to the calibration values.
//
// For box (rA, cA) of wavelength s and its slot (dr, dc), the entry at FPA
// position p = (rA + dr) + gamma (cA + dc) is the H entry of voxel (x, y) at
// pixel (p + x + gamma y) mod n, so its derivative gathers
//   sum over voxels of  u(p + x + gamma y) b(x, y) + e(p + x + gamma y) f(x, y).
// Units are the back-projection units (frame, wavelength, field-stop tile):
// each wave takes boxes of the wavelength in turn, stages the u and e windows
// of the box over the tile (the back projection's windows), correlates them
// with the lane's 4 x 4 voxels of b and f for every slot, sums each slot over
// the wavefront, and writes one partial per (unit, box, slot).

constexpr int kVgWaves = 4;

// u and e windows of one (field-stop tile, box) pair, at the same addresses
// as the back projection's window.  Slots that meet no voxel inside the field
// stop (xx >= xlim or yy >= ylim) load 0: the buffers hold no defined values
// outside the pixels the forward kernels write.
template <int B>
__device__ __forceinline__ void load_pair(Pending<B> &pu, Pending<B> &pe, __amdgpu_buffer_rsrc_t ur,
                                          __amdgpu_buffer_rsrc_t er, const Geo &p, int Xs, int Ys, int xlim,
                                          int ylim, int lane) {
    using Wn = Win<B>;
    int q0, xr, yq, y0;
    floor_divmod(Xs, p.gamma, q0, xr);
    floor_divmod(Ys + q0, p.xi, yq, y0);
    int xm = xr + lane, y = y0;
    while (xm >= p.gamma) {
        xm -= p.gamma;
        y = step_mod(y, p.xi);
    }
    if (p.xi >= Wn::SY) {
        const bool vx = lane < xlim;
        const unsigned o0 = (unsigned)(xm + p.gamma * y) * 4u;
        const unsigned step = 4u * (unsigned)p.gamma, wrap = 4u * (unsigned)(p.gamma * p.xi);
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) {
            const unsigned o = o0 + step * (unsigned)yy;
            const unsigned off = (vx && yy < ylim) ? min(o, o - wrap) : kOutOfRange;
            pu.v[yy] = bload(ur, off);
            pe.v[yy] = bload(er, off);
        }
    } else {
#pragma unroll
        for (int yy = 0; yy < Wn::SY; ++yy) {
            const unsigned off = (lane < xlim && yy < ylim) ? (unsigned)(xm + p.gamma * y) * 4u : kOutOfRange;
            pu.v[yy] = bload(ur, off);
            pe.v[yy] = bload(er, off);
            y = step_mod(y, p.xi);
        }
    }
#pragma unroll
    for (int t = 0; t < Wn::NXT; ++t) {
        const int k = lane + 64 * t;
        unsigned off = kOutOfRange;
        if (k < Wn::E * Wn::SY) {
            const int e = k % Wn::ED, yy = k / Wn::ED;
            if (TX + e < xlim && yy < ylim) {
                int xe = xr + TX + e, ye = y0;
                while (xe >= p.gamma) {
                    xe -= p.gamma;
                    ye = step_mod(ye, p.xi);
                }
                ye += yy;
                while (ye >= p.xi) ye -= p.xi;
                off = (unsigned)(xe + p.gamma * ye) * 4u;
            }
        }
        pu.x[t] = bload(ur, off);
        pe.x[t] = bload(er, off);
    }
}

// acc[j*B + i] += sum_{k,q < 4} bq[k][q] * Su[(4ly+k+j)*SXP + 4lx+q+i]
//                             + fq[k][q] * Se[(4ly+k+j)*SXP + 4lx+q+i]
template <int B>
__device__ __forceinline__ void correlate_values(float (&acc)[B * B], const float *Su, const float *Se,
                                                 const float (&bq)[4][4], const float (&fq)[4][4], int lx, int ly) {
    using Wn = Win<B>;
#pragma unroll
    for (int row = 0; row < Wn::NR; ++row) {
        float su[4 * Wn::NV], se[4 * Wn::NV];
        const float4 *pu = reinterpret_cast<const float4 *>(Su + (4 * ly + row) * Wn::SXP + 4 * lx);
        const float4 *pe = reinterpret_cast<const float4 *>(Se + (4 * ly + row) * Wn::SXP + 4 * lx);
#pragma unroll
        for (int v = 0; v < Wn::NV; ++v) {
            const float4 a = pu[v], c = pe[v];
            su[4 * v + 0] = a.x;
            su[4 * v + 1] = a.y;
            su[4 * v + 2] = a.z;
            su[4 * v + 3] = a.w;
            se[4 * v + 0] = c.x;
            se[4 * v + 1] = c.y;
            se[4 * v + 2] = c.z;
            se[4 * v + 3] = c.w;
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int k = row - j;
            if (k < 0 || k >= 4) continue;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                float t = acc[j * B + i];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    t = __builtin_fmaf(bq[k][q], su[q + i], t);
                    t = __builtin_fmaf(fq[k][q], se[q + i], t);
                }
                acc[j * B + i] = t;
            }
        }
    }
}

template <int B>
__global__ void __launch_bounds__(64 * kVgWaves) k_value_grad(const int4 *__restrict__ meta,
                                                              const int4 *__restrict__ items, const int stride,
                                                              const int n_units, const float *__restrict__ u,
                                                              const float *__restrict__ e,
                                                              const float *__restrict__ b,
                                                              const float *__restrict__ f,
                                                              float *__restrict__ part) {
    using Wn = Win<B>;
    constexpr int BB = B * B;
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    float *Su = lds + wv * (2 * Wn::REG);
    float *Se = Su + Wn::REG;
    const int lx = lane & 15, ly = lane >> 4;

    for (int unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
        const int4 m0 = meta[3 * unit], m1 = meta[3 * unit + 1], m2 = meta[3 * unit + 2];
        const int4 *list = items + (size_t)m0.z * stride;
        const Geo geo{m1.x, m1.y, m1.z, m1.w};
        const int x0 = m0.x, y0 = m0.y;
        const int n = geo.gamma * geo.xi;
        const __amdgpu_buffer_rsrc_t ur = rsrc(u + (size_t)(unsigned)m2.x, n);
        const __amdgpu_buffer_rsrc_t er = rsrc(e + (size_t)(unsigned)m2.x, n);
        const size_t sb = (size_t)(unsigned)m0.w;
        const int xlim = geo.a - x0 + B - 1, ylim = geo.alpha - y0 + B - 1;

        // this lane's 4 x 4 voxels of b and f (0 outside the field stop)
        float bq[4][4], fq[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int x = x0 + 4 * lx + q, y = y0 + 4 * ly + k;
                const bool in = x < geo.a && y < geo.alpha;
                const size_t o = sb + (size_t)x + (size_t)geo.a * y;
                bq[k][q] = in ? b[o] : 0.0f;
                fq[k][q] = in ? f[o] : 0.0f;
            }

        int k = wv;
        int4 rec = record(list, k, stride);
        Pending<B> pu, pe;
        if (rec.w >= 0) load_pair<B>(pu, pe, ur, er, geo, rec.x + x0, rec.y + y0, xlim, ylim, lane);
        while (rec.w >= 0) {
            store_window<B, false>(Su, pu, lane);
            store_window<B, false>(Se, pe, lane);
            wave_lds_sync();
            const int4 nxt = record(list, k + nw, stride);
            if (nxt.w >= 0) load_pair<B>(pu, pe, ur, er, geo, nxt.x + x0, nxt.y + y0, xlim, ylim, lane);
            float acc[BB];
#pragma unroll
            for (int t = 0; t < BB; ++t) acc[t] = 0.0f;
            correlate_values<B>(acc, Su, Se, bq, fq, lx, ly);
            wave_lds_sync();
            float mine = 0.0f;
#pragma unroll
            for (int t = 0; t < BB; ++t) {
                const float tot = wave_sum(acc[t]);
                if (lane == t) mine = tot;
            }
            if (lane < BB) part[((size_t)unit * stride + k) * BB + lane] = mine;
            k += nw;
            rec = nxt;
        }
    }
}

// Per calibration entry (one wavefront each, lanes over the units): its
// slot's partials over every unit of its wavelength (all frames sharing the
// plan), minus (sum of b zeta) / h_s; sums in double, butterfly order fixed.
__global__ void __launch_bounds__(256) k_value_finish(const int32_t *__restrict__ entry_slot,
                                                      const int32_t *__restrict__ box_lam,
                                                      const int32_t *__restrict__ lam_box0,
                                                      const int32_t *__restrict__ lam_units_ptr,
                                                      const int32_t *__restrict__ lam_units, const int stride,
                                                      const int BB, const float *__restrict__ part,
                                                      const float *__restrict__ flux, const float *__restrict__ hsum,
                                                      float *__restrict__ dv, const long long entry0,
                                                      const long long n, const int accumulate) {
    const int lane = threadIdx.x & 63;
    const long long t = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= n) return;   // the whole wavefront leaves together
    const int slot = entry_slot[entry0 + t];
    float v = 0.0f;
    if (slot >= 0) {
        const int gb = slot / BB, k = slot - gb * BB;
        const int gl = box_lam[gb], j = gb - lam_box0[gl];
        double s = 0.0, fl = 0.0;
        for (int p = lam_units_ptr[gl] + lane; p < lam_units_ptr[gl + 1]; p += 64) {
            const int un = lam_units[p];
            s += (double)part[((size_t)un * stride + j) * BB + k];
            fl += (double)flux[un];
        }
        s = wave_sum(s);
        fl = wave_sum(fl);
        const float hs = hsum[gl];
        v = (float)(s - (hs != 0.0f ? fl / (double)hs : 0.0));
    }
    if (lane == 0) dv[t] = accumulate ? dv[t] + v : v;
}

// New calibration values: one workgroup per wavelength [lam0 + blockIdx.x];
// every slot of its boxes gets the sum (double) of its entries' values, and
// h_s the sum (double) of the slots.
__global__ void __launch_bounds__(256) k_set_values(const float *__restrict__ values, const long long entry0,
                                                    const int32_t *__restrict__ slot_entries_ptr,
                                                    const int32_t *__restrict__ slot_entries,
                                                    const int32_t *__restrict__ lam_box0, const int lam0,
                                                    const int BB, float *__restrict__ box_w,
                                                    float *__restrict__ box_wf, float *__restrict__ hsum) {
    __shared__ double red[256];
    const int gl = lam0 + blockIdx.x;
    const int s0 = lam_box0[gl] * BB, s1 = lam_box0[gl + 1] * BB;
    double part = 0.0;
    for (int slot = s0 + (int)threadIdx.x; slot < s1; slot += blockDim.x) {
        double acc = 0.0;
        for (int p = slot_entries_ptr[slot]; p < slot_entries_ptr[slot + 1]; ++p)
            acc += (double)values[(long long)slot_entries[p] - entry0];
        const float v = (float)acc;
        const int gb = slot / BB, k = slot - gb * BB;
        box_w[slot] = v;
        box_wf[gb * BB + (BB - 1 - k)] = v;   // the forward kernel's reversed copy
        part += (double)v;
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) hsum[gl] = (float)red[0];
}

// ---------------------------------------------------------------------------
// EM diagnostics of one frame (Sec. 2: the column sums h below eq. (em) and
// the Poisson likelihood EM increases, Shepp and Vardi): flux sum_j h_j f_j,
// sum_i g_i, log-likelihood sum_i (g_i log ghat_i - ghat_i) with a g_i = 0
// term contributing -ghat_i, and the count of pixels with g_i > 0 but
// ghat_i <= 0 (the likelihood is then -inf).  Accumulated in double;
// atomic-free and deterministic: every workgroup of k_diag_partial reduces a
// fixed slice (thread-strided, then a fixed tree) into diag partial b, and
// k_diag_final sums the partials in order.
constexpr int kDiagBlocks = kDiagParts;

__device__ __forceinline__ void block_sum4(double (&v)[4], double *red) {
#pragma unroll
    for (int k = 0; k < 4; ++k) red[4 * threadIdx.x + k] = v[k];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[4 * threadIdx.x + k] += red[4 * (threadIdx.x + o) + k];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = red[k];
}

__global__ void __launch_bounds__(256) k_diag_partial(const float *__restrict__ g, const float *__restrict__ ghat,
                                                      const float *__restrict__ f, const float *__restrict__ hsum,
                                                      const long long n, const long long m, const long long ell,
                                                      double *__restrict__ part) {
    __shared__ double red[4 * 256];
    const long long b = blockIdx.x, nb = gridDim.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};   // flux, sum g, log-likelihood, bad pixels
    const long long p0 = n * b / nb, p1 = n * (b + 1) / nb;
    for (long long i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
        const double gi = g[i], gh = ghat[i];
        v[1] += gi;
        if (gi > 0.0) {
            if (gh > 0.0)
                v[2] += gi * log(gh) - gh;
            else
                v[3] += 1.0;
        } else {
            v[2] -= gh;
        }
    }
    const long long j0 = m * b / nb, j1 = m * (b + 1) / nb;
    for (long long j = j0 + threadIdx.x; j < j1; j += blockDim.x) v[0] += (double)hsum[j / ell] * (double)f[j];
    block_sum4(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) part[4 * b + k] = v[k];
}

__global__ void __launch_bounds__(256) k_diag_final(const double *__restrict__ part, const int nparts,
                                                    double *__restrict__ out) {
    __shared__ double red[4 * 256];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nparts; p += blockDim.x)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += part[4 * p + k];
    block_sum4(v, red);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = v[1];
        out[2] = v[3] > 0.0 ? -HUGE_VAL : v[2];
        out[3] = v[3];
    }
}

template <int B>
int enable_large_lds() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, []() {
        const int bytes = Win<B>::MAXW * Win<B>::WREG * (int)sizeof(float);
        err = hipFuncSetAttribute((const void *)k_forward<B>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (err == hipSuccess)
            err = hipFuncSetAttribute((const void *)k_adjoint<B, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      bytes);
        if (err == hipSuccess)
            err = hipFuncSetAttribute((const void *)k_adjoint<B, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      bytes);
    });
    return (int)err;
}

int device_cus() {
    static std::once_flag once;
    static int cus = 256;
    std::call_once(once, []() {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
            prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    });
    return cus;
}

// Grid of a launch over n_units work units.  By default one workgroup per
// unit: the hardware dispatcher then hands the next unit to whichever compute
// unit frees first.  With `persistent`, only as many workgroups as fit on
// the chip at once (by LDS and waves per CU) are launched and each walks the
// unit list with a grid stride.
int grid_for(int n_units, size_t lds_bytes, int waves, bool persistent) {
    if (!persistent) return std::max(1, n_units);
    const int by_lds = lds_bytes ? (int)std::min<size_t>(8, (160 * 1024) / lds_bytes) : 8;
    const int by_waves = std::max(1, 32 / waves);
    const int resident = std::max(1, std::min(by_lds, by_waves));
    return std::max(1, std::min(n_units, device_cus() * resident));
}

template <int B>
int forward_B(const DevWork &w, const float *x, const float *g, const float *u, float *out, int mode, void *workspace,
              hipStream_t st) {
    const DevList &L = mode == kFwdPlain ? w.fwd_full : w.fwd_em;
    if (L.n_units == 0) return 0;
    if (L.waves == 1) {   // solo: four units per workgroup, a wave each
        float *partials = (mode != kFwdPlain && w.n_split > 0) ? (float *)((char *)workspace + w.partials_off) : nullptr;
        const size_t lds = (size_t)kSoloWaves * Win<B>::WREG * sizeof(float);
        const int groups = solo_groups(L.n_units, kSoloWaves);
        hipLaunchKernelGGL(k_forward_solo<B>, dim3(grid_for(groups, lds, kSoloWaves, w.persistent)),
                           dim3(64 * kSoloWaves), lds, st, L.meta, L.items, L.stride, L.n_units, w.box_wf, x, g, u,
                           out, partials, mode);
        if (partials) {
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return (int)e;
            hipLaunchKernelGGL(k_finish_split, dim3(w.n_split), dim3(256), 0, st, w.split_meta,
                               (const float *)partials, g, u, out, mode);
        }
        return (int)hipGetLastError();
    }
    const size_t lds = (size_t)L.waves * Win<B>::WREG * sizeof(float);
    if (lds > 65536) {
        const int e = enable_large_lds<B>();
        if (e) return e;
    }
    float *partials = (mode != kFwdPlain && w.n_split > 0) ? (float *)((char *)workspace + w.partials_off) : nullptr;
    hipLaunchKernelGGL(k_forward<B>, dim3(grid_for(L.n_units, lds, L.waves, w.persistent)), dim3(64 * L.waves), lds, st,
                       L.meta, L.items, L.stride, L.n_units, w.box_wf, x, g, u, out, partials, mode);
    if (partials) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(k_finish_split, dim3(w.n_split), dim3(256), 0, st, w.split_meta, (const float *)partials,
                           g, u, out, mode);
    }
    return (int)hipGetLastError();
}

template <int B, int SH>
int forward_region_B(const DevWork &w, const float *g, const float *u, float *out, int mode, void *workspace,
                     hipStream_t st) {
    using Wn = RWin<B, SH>;
    const DevList &L = w.fwd_pad;
    if (L.n_units == 0) return 0;
    const int waves = w.region_solo ? kSoloWaves : L.waves;
    const size_t lds = (size_t)waves * Wn::WAVE * sizeof(float);
    if (lds > 65536) {   // both kernels may ask for more than 64 KiB of LDS (small regions, large B)
        static std::once_flag once;
        static hipError_t err = hipSuccess;
        std::call_once(once, []() {
            err = hipFuncSetAttribute((const void *)k_forward_region<B, SH>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      Wn::MAXW * Wn::WAVE * (int)sizeof(float));
            if (err == hipSuccess)
                err = hipFuncSetAttribute((const void *)k_forward_region_solo<B, SH>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          kSoloWaves * Wn::WAVE * (int)sizeof(float));
        });
        if (err != hipSuccess) return (int)err;
    }
    const float *fp = (const float *)((const char *)workspace + w.fp_off);
    float *partials = w.n_rsplit > 0 ? (float *)((char *)workspace + w.rpartials_off) : nullptr;
    if (w.region_solo) {   // a lane group per unit, 64 / GL units per wave
        const int groups = solo_groups(L.n_units, Wn::GROUPS * kSoloWaves);
        hipLaunchKernelGGL((k_forward_region_solo<B, SH>), dim3(grid_for(groups, lds, kSoloWaves, w.persistent)),
                           dim3(64 * kSoloWaves), lds, st, L.meta, L.items, L.stride, L.n_units, w.box_wf, w.n_wf,
                           fp, w.fp_floats, g, u, out, partials, mode);
    } else {
        hipLaunchKernelGGL((k_forward_region<B, SH>), dim3(grid_for(L.n_units, lds, L.waves, w.persistent)),
                           dim3(64 * L.waves), lds, st, L.meta, L.items, L.stride, L.n_units, w.box_wf, w.n_wf, fp,
                           w.fp_floats, g, u, out, partials, mode);
    }
    if (partials) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(k_finish_regions, dim3(w.n_rsplit), dim3(kRegionPixels), 0, st, w.rsplit_meta,
                           (const float *)partials, g, u, out, mode, Wn::RX, Wn::RY);
    }
    return (int)hipGetLastError();
}

template <int B>
int forward_region_shape(const DevWork &w, const float *g, const float *u, float *out, int mode, void *workspace,
                         hipStream_t st) {
    switch (w.region_shape) {
        case 1: return forward_region_B<B, 1>(w, g, u, out, mode, workspace, st);
        case 2: return forward_region_B<B, 2>(w, g, u, out, mode, workspace, st);
        case 3: return forward_region_B<B, 3>(w, g, u, out, mode, workspace, st);
        case 4: return forward_region_B<B, 4>(w, g, u, out, mode, workspace, st);
        case 5: return forward_region_B<B, 5>(w, g, u, out, mode, workspace, st);
        case 6: return forward_region_B<B, 6>(w, g, u, out, mode, workspace, st);
    }
    return (int)hipErrorInvalidValue;
}

template <int B>
int adjoint_B(const DevWork &w, const float *r, const float *in1, const float *in2, float *out, float *out2,
              float *flux, int mode, hipStream_t st, float *fpad, float relax) {
    const DevList &L = w.adj;
    if (L.n_units == 0) return 0;
    if (L.waves == 1) {   // solo: four units per workgroup, a wave each
        const size_t lds = (size_t)kSoloWaves * Win<B>::WREG * sizeof(float);
        const int groups = solo_groups(L.n_units, kSoloWaves);
        auto kern = w.adj_direct ? k_adjoint_solo<B, true> : k_adjoint_solo<B, false>;
        hipLaunchKernelGGL(kern, dim3(grid_for(groups, lds, kSoloWaves, w.persistent)),
                           dim3(64 * kSoloWaves), lds, st, L.meta, L.items, L.stride, L.n_units, w.box_w, w.h, r, in1,
                           in2, out, out2, flux, mode, fpad, w.halo_x, w.halo_y, relax);
        return (int)hipGetLastError();
    }
    const size_t lds = (size_t)L.waves * Win<B>::WREG * sizeof(float);
    if (lds > 65536) {
        const int e = enable_large_lds<B>();
        if (e) return e;
    }
    auto kern = w.adj_direct ? k_adjoint<B, true> : k_adjoint<B, false>;
    hipLaunchKernelGGL(kern, dim3(grid_for(L.n_units, lds, L.waves, w.persistent)), dim3(64 * L.waves), lds, st,
                       L.meta, L.items, L.stride, L.n_units, w.box_w, w.h, r, in1, in2, out, out2, flux, mode, fpad,
                       w.halo_x, w.halo_y, relax);
    return (int)hipGetLastError();
}

template <int B>
int value_grad_B(const DevWork &w, const float *u, const float *e, const float *b, const float *f, float *part,
                 hipStream_t st) {
    const DevList &L = w.adj;
    if (L.n_units == 0) return 0;
    const size_t lds = (size_t)kVgWaves * 2 * Win<B>::REG * sizeof(float);
    static_assert((size_t)kVgWaves * 2 * Win<8>::REG * sizeof(float) <= 65536, "value kernel LDS");
    hipLaunchKernelGGL(k_value_grad<B>, dim3(L.n_units), dim3(64 * kVgWaves), lds, st, L.meta, L.items, L.stride,
                       L.n_units, u, e, b, f, part);
    return (int)hipGetLastError();
}

}  // namespace

int max_waves(int B) { return B <= 5 ? Win<1>::MAXW : Win<8>::MAXW; }
int min_waves() { return kMinWaves; }

int launch_forward(const DevWork &w, const float *x, const float *g, const float *u, float *out, int mode,
                   void *workspace, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (w.B) {
        case 1: return forward_B<1>(w, x, g, u, out, mode, workspace, st);
        case 2: return forward_B<2>(w, x, g, u, out, mode, workspace, st);
        case 3: return forward_B<3>(w, x, g, u, out, mode, workspace, st);
        case 4: return forward_B<4>(w, x, g, u, out, mode, workspace, st);
        case 5: return forward_B<5>(w, x, g, u, out, mode, workspace, st);
        case 6: return forward_B<6>(w, x, g, u, out, mode, workspace, st);
        case 7: return forward_B<7>(w, x, g, u, out, mode, workspace, st);
        case 8: return forward_B<8>(w, x, g, u, out, mode, workspace, st);
    }
    return (int)hipErrorInvalidValue;
}

int launch_adjoint(const DevWork &w, const float *r, const float *in1, const float *in2, float *out, float *out2,
                   float *flux, int mode, void *stream, void *fpad_ws, float relax) {
    hipStream_t st = (hipStream_t)stream;
    float *fpad = (fpad_ws && adj_updates(mode) && w.pad_ok) ? (float *)((char *)fpad_ws + w.fp_off) : nullptr;
    switch (w.B) {
        case 1: return adjoint_B<1>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
        case 2: return adjoint_B<2>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
        case 3: return adjoint_B<3>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
        case 4: return adjoint_B<4>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
        case 5: return adjoint_B<5>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
        case 6: return adjoint_B<6>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
        case 7: return adjoint_B<7>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
        case 8: return adjoint_B<8>(w, r, in1, in2, out, out2, flux, mode, st, fpad, relax);
    }
    return (int)hipErrorInvalidValue;
}

int launch_fill(float *x, int64_t n, float v, void *stream) {
    if (n <= 0) return 0;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65535);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, (hipStream_t)stream, x, n, v);
    return (int)hipGetLastError();
}

int launch_pad(const DevWork &w, const float *x, void *workspace, void *stream) {
    if (!w.pad_ok || w.n_pad_blocks == 0) return (int)hipErrorInvalidValue;
    float *fp = (float *)((char *)workspace + w.fp_off);
    hipLaunchKernelGGL(k_pad, dim3((unsigned)w.pad_rows, (unsigned)w.n_pad_blocks), dim3(256), 0,
                       (hipStream_t)stream, w.pad_blocks, x, fp, w.halo_x, w.halo_y);
    return (int)hipGetLastError();
}

int launch_forward_pad(const DevWork &w, const float *g, const float *u, float *out, int mode, void *workspace,
                       void *stream) {
    if (!w.pad_ok) return (int)hipErrorInvalidValue;
    hipStream_t st = (hipStream_t)stream;
    switch (w.B) {
        case 1: return forward_region_shape<1>(w, g, u, out, mode, workspace, st);
        case 2: return forward_region_shape<2>(w, g, u, out, mode, workspace, st);
        case 3: return forward_region_shape<3>(w, g, u, out, mode, workspace, st);
        case 4: return forward_region_shape<4>(w, g, u, out, mode, workspace, st);
        case 5: return forward_region_shape<5>(w, g, u, out, mode, workspace, st);
        case 6: return forward_region_shape<6>(w, g, u, out, mode, workspace, st);
        case 7: return forward_region_shape<7>(w, g, u, out, mode, workspace, st);
        case 8: return forward_region_shape<8>(w, g, u, out, mode, workspace, st);
    }
    return (int)hipErrorInvalidValue;
}

int launch_value_grad(const DevWork &w, const float *u, const float *e, const float *b, const float *f, float *part,
                      void *stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (w.B) {
        case 1: return value_grad_B<1>(w, u, e, b, f, part, st);
        case 2: return value_grad_B<2>(w, u, e, b, f, part, st);
        case 3: return value_grad_B<3>(w, u, e, b, f, part, st);
        case 4: return value_grad_B<4>(w, u, e, b, f, part, st);
        case 5: return value_grad_B<5>(w, u, e, b, f, part, st);
        case 6: return value_grad_B<6>(w, u, e, b, f, part, st);
        case 7: return value_grad_B<7>(w, u, e, b, f, part, st);
        case 8: return value_grad_B<8>(w, u, e, b, f, part, st);
    }
    return (int)hipErrorInvalidValue;
}

int launch_value_finish(const DevWork &w, const float *part, const float *flux, float *dv, int64_t entry0,
                        int64_t n_entries, bool accumulate, void *stream) {
    if (n_entries <= 0) return 0;
    const int64_t blocks = (n_entries + 3) / 4;   // 4 entries (wavefronts) per workgroup
    hipLaunchKernelGGL(k_value_finish, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, w.entry_slot,
                       w.box_lam, w.lam_box0, w.lam_units_ptr, w.lam_units, w.adj.stride, w.B * w.B, part, flux,
                       (const float *)w.h, dv, (long long)entry0, (long long)n_entries, accumulate ? 1 : 0);
    return (int)hipGetLastError();
}

int launch_diagnostics(const float *g, const float *ghat, const float *f, const float *hsum, int64_t n, int64_t m,
                       int64_t ell, double *part, double *out, void *stream) {
    hipLaunchKernelGGL(k_diag_partial, dim3(kDiagBlocks), dim3(256), 0, (hipStream_t)stream, g, ghat, f, hsum,
                       (long long)n, (long long)m, (long long)ell, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, (hipStream_t)stream, (const double *)part, kDiagBlocks,
                       out);
    return (int)hipGetLastError();
}

int launch_set_values(const DevWork &w, const float *values, int64_t entry0, int32_t lam0, int32_t lam1,
                      void *stream) {
    if (lam1 <= lam0) return 0;
    hipLaunchKernelGGL(k_set_values, dim3((unsigned)(lam1 - lam0)), dim3(256), 0, (hipStream_t)stream, values,
                       (long long)entry0, w.slot_entries_ptr, w.slot_entries, w.lam_box0, lam0, w.B * w.B, w.box_w,
                       w.box_wf, w.h);
    return (int)hipGetLastError();
}

}  // namespace ctis
