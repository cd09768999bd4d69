// Internal types shared by the host plan builder, the C ABI glue and the HIP
// kernels of libctis.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ctis.h"

#ifndef __HIP_PLATFORM_AMD__
#define __HIP_PLATFORM_AMD__
#endif
#include <hip/hip_runtime_api.h>

namespace ctis {

// Tile shape of both kernels: a wavefront covers 64 x 16 outputs (fast x slow
// axis) with a 4 x 4 register micro-tile per lane (16 lanes x 4 lanes).
constexpr int kTileFast = 64;
constexpr int kTileSlow = 16;
constexpr int kMaxBox = 8;
// 32-bit buffer offsets (in bytes) address the FPA and one wavelength block
constexpr int64_t kMaxPixels = (int64_t(1) << 29) - 1;

// One forward launch: a list of work units, one workgroup each.  A unit is a
// chunk of the boxes that meet one FPA tile; a tile with more boxes than the
// chunk size is split over several units, whose partial tiles a second,
// small kernel sums.
struct FwdList {
    const int4 *unit_meta;   // n_units: (tile, chunk, n_chunks, partial slot of chunk 0)
    const int4 *items;       // n_units * stride records (X, Y, s, box), X, Y = window
                             //   origin (r0 - (B-1) - rA, c0 - (B-1) - cA); box = -1 ends
    int32_t n_units = 0, stride = 1, waves = 4;
};

// Device-side tables of a plan (one allocation, pointers into it).
struct DevTables {
    FwdList fwd_full;           // every FPA tile, one unit each (plain projection)
    FwdList fwd_em;             // FPA tiles with boxes, heavy tiles split (EM)
    const int4 *split_meta;     // n_split_tiles: (tile, n_chunks, partial slot of chunk 0, 0)
    const int4 *adj_items;      // w * adj_stride: per wavelength, its boxes with
                                //   X, Y = the anchor (rA, cA)
    const float *box_w;         // nb*B*B, [dc*B + dr]
    const float *box_wf;        // nb*B*B, flipped: [(B-1-dc)*B + (B-1-dr)]
    const float *h;             // w: column sums per wavelength
};

// Scalar kernel parameters (passed by value).
struct KParams {
    int32_t a, alpha, w, gamma, xi;
    int32_t ell, n;
    int32_t ntr;        // FPA tiles along the fast axis
    int32_t nbx, nby;   // field-stop tiles along x and y
    int32_t adj_stride; // records per wavelength (max boxes of one wavelength)
};

struct HostList {
    std::vector<int32_t> unit_meta, items;   // int4 records, flattened
    int32_t n_units = 0, stride = 1, waves = 4;
};

struct HostTables {
    int32_t B = 1;
    std::vector<int32_t> box_rc, box_lambda, lambda_box_ptr;
    std::vector<float> box_w, box_wf, h;
    std::vector<int32_t> tile_order, tile_item_ptr, item_box;
    int32_t ntr = 0, ntc = 0, n_tiles = 0, n_active = 0;
    int32_t nbx = 0, nby = 0;
    int64_t nnz = 0, n_support = 0;
    bool nonneg = true;
    HostList fwd_full, fwd_em;
    int32_t chunk = 64;          // max boxes per forward unit in EM
    int32_t partial_slots = 0;   // 64x16 partial tiles of split FPA tiles
    int32_t n_split_tiles = 0;
    std::vector<int32_t> split_meta;
};

}  // namespace ctis

struct ctis_plan {
    int32_t a, alpha, w, gamma, xi;
    int64_t n, ell, m;
    ctis::HostTables ht;
    int32_t device = -1;
    void *dev_mem = nullptr;    // one allocation holding every table
    ctis::DevTables dt{};
    ctis::KParams kp{};
    int32_t waves_adj = 4;
    size_t workspace_bytes = 0;
    size_t ws_partials = 0;      // byte offset of the partial tiles in the EM workspace
};

namespace ctis {

void set_error(const std::string &msg);
ctis_status fail(ctis_status st, const std::string &msg);

// host plan builder (plan.cpp)
ctis_status build_host_tables(ctis_plan *p, const int64_t *lambda_ptr, const int32_t *fpa_index,
                              const float *value, int forced_box);
ctis_status upload_tables(ctis_plan *p);

// kernel launchers (kernels.hip); return hipError_t as int
int max_waves(int box);
int min_waves();
int launch_forward(const ctis_plan *p, const float *f, const float *g, float *out, bool em_ratio,
                   void *workspace, void *stream);
int launch_adjoint(const ctis_plan *p, const float *u, const float *fin, float *out, bool em_update,
                   void *stream);

}  // namespace ctis
