// Internal types shared by the host plan builder, the C ABI glue and the HIP
// kernels of libctis.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ctis.h"

namespace ctis {

// Tile shape of both kernels: a wavefront covers 64 x 16 outputs (fast x slow
// axis) with a 4 x 4 register micro-tile per lane (16 lanes x 4 lanes).
constexpr int kTileFast = 64;
constexpr int kTileSlow = 16;
constexpr int kMaxBox = 8;

// Device-side tables of a plan (one allocation, pointers into it).
struct DevTables {
    const int32_t *box_rc;          // 2*nb: anchor (r, c) of each box
    const int32_t *box_lambda;      // nb
    const float *box_w;             // nb*B*B, [dc*B + dr]
    const float *box_wf;            // nb*B*B, flipped: [(B-1-dc)*B + (B-1-dr)]
    const int32_t *lambda_box_ptr;  // w+1
    const float *h;                 // w
    const int32_t *tile_order;      // n_tiles: active tiles (heaviest first), then the rest
    const int32_t *tile_item_ptr;   // n_tiles+1, indexed by tile id
    const int32_t *item_box;        // n_items
};

// Scalar kernel parameters (passed by value).
struct KParams {
    int32_t a, alpha, w, gamma, xi;
    int32_t ell, n;
    int32_t ntr;        // FPA tiles along the fast axis
    int32_t nbx, nby;   // field-stop tiles along x and y
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
    int32_t waves_fwd = 4;
    int32_t waves_adj = 4;
    size_t workspace_bytes = 0;
};

namespace ctis {

void set_error(const std::string &msg);
ctis_status fail(ctis_status st, const std::string &msg);

// host plan builder (plan.cpp)
ctis_status build_host_tables(ctis_plan *p, const int64_t *lambda_ptr, const int32_t *fpa_index,
                              const float *value, int forced_box);
ctis_status upload_tables(ctis_plan *p);

// kernel launchers (kernels.hip); return hipError_t as int
int launch_forward(const ctis_plan *p, const float *f, const float *g, float *out, bool em_ratio,
                   void *stream);
int launch_adjoint(const ctis_plan *p, const float *u, const float *fin, float *out, bool em_update,
                   void *stream);

}  // namespace ctis
