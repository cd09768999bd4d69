// Host side of a plan: validation, merging of the calibration entries,
// grouping of each wavelength's nonzeros into dense B x B boxes, support
// statistics, the forward work list, and the upload of the tables.
//
// The operator is the paper's: column j = (x, y, s) of H is the calibration
// image c_s shifted cyclically by q = x + gamma*y over the vectorised FPA
// (Sec. 2 calibration + shift-invariance; Sec. 3 H_s = C_s E and its index
// map).  Grouping the nonzeros into boxes does not change the operator: a box
// anchored at FPA position (rA, cA) holds the entries at (rA + dr, cA + dc),
// and the 1-D index of such an entry is exactly rA + dr + gamma*(cA + dc), so
// the kernels' cyclic address arithmetic stays the paper's.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_set>

#include "ctis_internal.h"

namespace ctis {

namespace {

struct Entry {
    int64_t idx;
    int32_t r, c;
    float v;
};

struct Dsu {
    std::vector<int32_t> p;
    explicit Dsu(size_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int32_t find(int32_t x) {
        while (p[x] != x) {
            p[x] = p[p[x]];
            x = p[x];
        }
        return x;
    }
    void unite(int32_t a, int32_t b) {
        a = find(a);
        b = find(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

struct Component {
    int32_t rmin, rmax, cmin, cmax;
    std::vector<int32_t> members;   // indices into the wavelength's entry list
};

// 8-connected components of one wavelength's nonzero positions (decoded 2-D
// FPA coordinates; no wrap -- grouping is a layout choice only).
std::vector<Component> components(const std::vector<Entry> &e, int32_t gamma, int32_t xi) {
    const int32_t k = (int32_t)e.size();
    Dsu d(k);
    // entries are sorted by 1-D index: binary search for neighbours
    auto find_idx = [&](int64_t idx) -> int32_t {
        auto it = std::lower_bound(e.begin(), e.end(), idx,
                                   [](const Entry &a, int64_t v) { return a.idx < v; });
        if (it != e.end() && it->idx == idx) return (int32_t)(it - e.begin());
        return -1;
    };
    for (int32_t t = 0; t < k; ++t) {
        for (int dc = -1; dc <= 1; ++dc)
            for (int dr = -1; dr <= 1; ++dr) {
                if (!dr && !dc) continue;
                int32_t r = e[t].r + dr, c = e[t].c + dc;
                if (r < 0 || r >= gamma || c < 0 || c >= xi) continue;
                int32_t o = find_idx((int64_t)r + (int64_t)gamma * c);
                if (o >= 0) d.unite(t, o);
            }
    }
    std::vector<int32_t> root_to_comp(k, -1);
    std::vector<Component> out;
    for (int32_t t = 0; t < k; ++t) {
        int32_t rt = d.find(t);
        if (root_to_comp[rt] < 0) {
            root_to_comp[rt] = (int32_t)out.size();
            out.push_back(Component{e[t].r, e[t].r, e[t].c, e[t].c, {}});
        }
        Component &cp = out[root_to_comp[rt]];
        cp.rmin = std::min(cp.rmin, e[t].r);
        cp.rmax = std::max(cp.rmax, e[t].r);
        cp.cmin = std::min(cp.cmin, e[t].c);
        cp.cmax = std::max(cp.cmax, e[t].c);
        cp.members.push_back(t);
    }
    return out;
}

// distinct B x B cells (aligned at the component's bounding-box corner) that
// hold at least one member, as (cell_r, cell_c) pairs in ascending order
std::vector<std::pair<int32_t, int32_t>> cells(const Component &cp, const std::vector<Entry> &e, int B) {
    std::vector<std::pair<int32_t, int32_t>> v;
    v.reserve(cp.members.size());
    for (int32_t t : cp.members) v.emplace_back((e[t].r - cp.rmin) / B, (e[t].c - cp.cmin) / B);
    std::sort(v.begin(), v.end(), [](auto a, auto b) {
        return a.second != b.second ? a.second < b.second : a.first < b.first;
    });
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t floor_div(int64_t a, int64_t b) {
    const int64_t q = a / b;
    return (a % b != 0 && (a < 0) != (b < 0)) ? q - 1 : q;
}

int64_t floor_mod(int64_t a, int64_t b) {
    const int64_t r = a % b;
    return r < 0 ? r + b : r;
}

// count of set entries of the circular sliding OR along a sequence
// get(k), k in [0, len), window `win` ending at k (k - win + 1 .. k, mod len)
template <class Get, class Set>
void circular_window_or(int64_t len, int64_t win, Get get, Set set) {
    int64_t cnt = 0;
    for (int64_t x = 0; x < win; ++x) cnt += get(((0 - x) % len + len) % len);
    set(0, cnt > 0);
    for (int64_t k = 1; k < len; ++k) {
        cnt += get(k);
        cnt -= get(((k - win) % len + len) % len);
        set(k, cnt > 0);
    }
}

}  // namespace

// Forward work list on a grid of tf x ts FPA cells: the cells met by the
// dilated image of every box, i.e. the pixels (A + X + gamma*Y) mod n for X <
// a + B - 1, Y < alpha + B - 1 (the exact 1-D shift, including runs that
// continue in the next FPA column or wrap round the FPA).
ctis_status build_grid(HostTables &T, const ctis_plan *p, int32_t tf, int32_t ts, WorkGrid &G) {
    const int64_t gamma = p->gamma, xi = p->xi;
    const int B = T.B;
    G = WorkGrid{};
    G.tf = tf;
    G.ts = ts;
    const int64_t ntr = ceil_div(gamma, tf), ntc = ceil_div(xi, ts);
    if (ntr * ntc > INT32_MAX) return fail(CTIS_E_TOO_LARGE, "too many FPA cells");
    G.ntr = (int32_t)ntr;
    G.ntc = (int32_t)ntc;
    G.n_cells = (int32_t)(ntr * ntc);
    const int32_t nb = (int32_t)T.box_lambda.size();
    std::vector<int32_t> stamp((size_t)G.n_cells, -1);
    std::vector<std::pair<int32_t, int32_t>> pairs;   // (cell, box)
    const int64_t L0 = (int64_t)p->a + B - 1, rows = (int64_t)p->alpha + B - 1;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t rA = T.box_rc[2 * (size_t)b], cA = T.box_rc[2 * (size_t)b + 1];
        for (int64_t Y = 0; Y < rows; ++Y) {
            // pixels (A + X + gamma*Y) mod n, X in [0, L0): a run along the fast
            // axis starting at (rA, cA + Y), continuing in the next FPA column
            int64_t r = rA, c = (cA + Y) % xi, L = L0;
            while (L > 0) {
                const int64_t seg = std::min<int64_t>(L, gamma - r);
                const int64_t tc = c / ts;
                for (int64_t tr = r / tf; tr <= (r + seg - 1) / tf; ++tr) {
                    const int32_t cell = (int32_t)(tr + ntr * tc);
                    if (stamp[(size_t)cell] != b) {
                        stamp[(size_t)cell] = b;
                        pairs.emplace_back(cell, b);
                    }
                }
                L -= seg;
                r = 0;
                c = (c + 1) % xi;
            }
        }
    }
    if ((int64_t)pairs.size() > INT32_MAX) return fail(CTIS_E_TOO_LARGE, "forward work list too long");
    std::sort(pairs.begin(), pairs.end());
    G.item_ptr.assign((size_t)G.n_cells + 1, 0);
    G.item_box.resize(pairs.size());
    for (size_t k = 0; k < pairs.size(); ++k) {
        G.item_ptr[(size_t)pairs[k].first + 1]++;
        G.item_box[k] = pairs[k].second;
    }
    for (int32_t t = 0; t < G.n_cells; ++t) G.item_ptr[(size_t)t + 1] += G.item_ptr[(size_t)t];
    G.order.resize((size_t)G.n_cells);
    std::iota(G.order.begin(), G.order.end(), 0);
    auto count = [&](int32_t t) { return G.item_ptr[(size_t)t + 1] - G.item_ptr[(size_t)t]; };
    std::stable_sort(G.order.begin(), G.order.end(), [&](int32_t x, int32_t y) { return count(x) > count(y); });
    int64_t active_items = 0;
    for (int32_t t = 0; t < G.n_cells; ++t) {
        G.n_active += count(t) > 0;
        G.max_items = std::max(G.max_items, count(t));
        active_items += count(t);
    }
    // EM chunk: a cell is split over several workgroups only when it holds
    // more than 64 boxes and more than twice the boxes an average compute
    // unit gets (256 CUs); otherwise splitting only adds the partial pass
    G.chunk = (int32_t)std::max<int64_t>(64, 2 * ((active_items + 255) / 256));
    return CTIS_OK;
}

ctis_status build_host_tables(ctis_plan *p, const int64_t *lambda_ptr, const int32_t *fpa_index,
                              const float *value, int forced_box, bool keep_zeros, int region_shape) {
    HostTables &T = p->ht;
    const int32_t w = p->w, gamma = p->gamma, xi = p->xi, a = p->a, alpha = p->alpha;
    const int64_t n = p->n;

    // -- 1. merge duplicates (sum in double), drop exact zeros unless the
    //       structure is to be kept (positions, whatever their values) ---------
    std::vector<std::vector<Entry>> ent(w);
    T.nonneg = true;
    T.nnz = 0;
    T.n_in = lambda_ptr[w];
    T.dropped = false;
    std::vector<int32_t> in_merged((size_t)T.n_in, -1);   // input entry -> merged entry of its wavelength
    for (int32_t s = 0; s < w; ++s) {
        const int64_t b = lambda_ptr[s], e = lambda_ptr[s + 1];
        std::vector<std::pair<int64_t, int64_t>> order;   // (index, position)
        order.reserve((size_t)(e - b));
        for (int64_t t = b; t < e; ++t) order.emplace_back((int64_t)fpa_index[t], t);
        std::sort(order.begin(), order.end());
        auto &out = ent[s];
        for (size_t k = 0; k < order.size();) {
            size_t k2 = k;
            double acc = 0.0;
            while (k2 < order.size() && order[k2].first == order[k].first) {
                acc += (double)value[order[k2].second];
                ++k2;
            }
            const float v = (float)acc;
            if (v != 0.0f || keep_zeros) {
                const int64_t idx = order[k].first;
                for (size_t kk = k; kk < k2; ++kk) in_merged[(size_t)order[kk].second] = (int32_t)out.size();
                out.push_back(Entry{idx, (int32_t)(idx % gamma), (int32_t)(idx / gamma), v});
                if (v < 0.0f) T.nonneg = false;
            } else {
                T.dropped = true;
            }
            k = k2;
        }
        T.nnz += (int64_t)out.size();
    }

    // -- 2. components and the box side B --------------------------------------
    std::vector<std::vector<Component>> comps(w);
    for (int32_t s = 0; s < w; ++s) comps[s] = components(ent[s], gamma, xi);
    int B = forced_box;
    if (B == 0) {
        double best = 0.0;
        for (int cand = 1; cand <= kMaxBox; ++cand) {
            int64_t nb = 0;
            for (int32_t s = 0; s < w; ++s)
                for (const auto &cp : comps[s]) nb += (int64_t)cells(cp, ent[s], cand).size();
            // per box and output: B*B multiply-adds plus staging of its window,
            // which costs about as much as 12 multiply-adds per output
            const double cost = (double)nb * (double)(cand * cand + 12);
            if (B == 0 || cost < best) {
                best = cost;
                B = cand;
            }
        }
    }
    T.B = B;

    // -- 3. boxes (per wavelength, sorted by anchor index) ----------------------
    T.box_rc.clear();
    T.box_lambda.clear();
    T.box_w.clear();
    T.box_wf.clear();
    T.lambda_box_ptr.assign((size_t)w + 1, 0);
    const int BB = B * B;
    T.entry_slot.assign((size_t)T.n_in, -1);
    for (int32_t s = 0; s < w; ++s) {
        struct Box {
            int32_t r, c;
            std::vector<float> v;
            std::vector<std::pair<int32_t, int32_t>> members;   // (merged entry, slot in the box)
        };
        std::vector<Box> boxes;
        for (const auto &cp : comps[s]) {
            auto cl = cells(cp, ent[s], B);
            const size_t base = boxes.size();
            for (auto [ci, cj] : cl) boxes.push_back(Box{cp.rmin + B * ci, cp.cmin + B * cj,
                                                          std::vector<float>((size_t)BB, 0.0f), {}});
            for (int32_t t : cp.members) {
                const int32_t ci = (ent[s][t].r - cp.rmin) / B, cj = (ent[s][t].c - cp.cmin) / B;
                auto it = std::lower_bound(cl.begin(), cl.end(), std::make_pair(ci, cj), [](auto x, auto y) {
                    return x.second != y.second ? x.second < y.second : x.first < y.first;
                });
                Box &bx = boxes[base + (size_t)(it - cl.begin())];
                const int32_t k = (ent[s][t].c - bx.c) * B + (ent[s][t].r - bx.r);
                bx.v[(size_t)k] = ent[s][t].v;
                bx.members.emplace_back(t, k);
            }
        }
        std::sort(boxes.begin(), boxes.end(), [&](const Box &x, const Box &y) {
            return (int64_t)x.r + (int64_t)gamma * x.c < (int64_t)y.r + (int64_t)gamma * y.c;
        });
        // slot of every merged entry: global box id * B*B + position in the box
        std::vector<int64_t> merged_slot(ent[s].size(), -1);
        for (const auto &bx : boxes) {
            const int64_t gb = (int64_t)T.box_lambda.size();
            if ((gb + 1) * BB > INT32_MAX) return fail(CTIS_E_TOO_LARGE, "too many calibration boxes");
            for (auto [t, k] : bx.members) merged_slot[(size_t)t] = gb * BB + k;
            T.box_rc.push_back(bx.r);
            T.box_rc.push_back(bx.c);
            T.box_lambda.push_back(s);
            for (int k = 0; k < BB; ++k) T.box_w.push_back(bx.v[(size_t)k]);
            for (int dc = 0; dc < B; ++dc)
                for (int dr = 0; dr < B; ++dr)
                    T.box_wf.push_back(bx.v[(size_t)((B - 1 - dc) * B + (B - 1 - dr))]);
        }
        T.lambda_box_ptr[(size_t)s + 1] = (int32_t)T.box_lambda.size();
        for (int64_t t = lambda_ptr[s]; t < lambda_ptr[s + 1]; ++t)
            if (in_merged[(size_t)t] >= 0) T.entry_slot[(size_t)t] = (int32_t)merged_slot[(size_t)in_merged[(size_t)t]];
    }

    // -- 4. column sums per wavelength (sum of c_s, in double) ------------------
    T.h.assign((size_t)w, 0.0f);
    for (int32_t s = 0; s < w; ++s) {
        double acc = 0.0;
        for (const auto &e : ent[s]) acc += (double)e.v;
        T.h[(size_t)s] = (float)acc;
    }

    // -- 5. support: FPA pixels in the image of some nonzero --------------------
    {
        std::vector<uint8_t> M((size_t)n, 0), D1((size_t)n, 0), D2((size_t)n, 0);
        for (int32_t s = 0; s < w; ++s)
            for (const auto &e : ent[s]) M[(size_t)e.idx] = 1;
        // shift along the vectorised FPA by x in [0, a)
        circular_window_or(n, a, [&](int64_t k) { return (int64_t)M[(size_t)k]; },
                           [&](int64_t k, bool v) { D1[(size_t)k] = v; });
        // shift by gamma*y, y in [0, alpha): a circular window along each residue class
        for (int64_t rho = 0; rho < gamma; ++rho)
            circular_window_or(xi, alpha, [&](int64_t k) { return (int64_t)D1[(size_t)(rho + gamma * k)]; },
                               [&](int64_t k, bool v) { D2[(size_t)(rho + gamma * k)] = v; });
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) cnt += D2[(size_t)i];
        T.n_support = cnt;
    }

    // -- 6. forward work lists: FPA tiles and regions met by each box's dilated
    //       image, and whether the region path's padded copy of f is exact --
    ctis_status st = build_grid(T, p, kTileFast, kTileSlow, T.tiles);
    if (st != CTIS_OK) return st;
    T.region_shape = region_shape ? region_shape : kDefaultRegionShape;
    st = build_grid(T, p, region_fast(T.region_shape), region_slow(T.region_shape), T.regions);
    if (st != CTIS_OK) return st;
    T.pad_ok = (int64_t)gamma - a >= halo_fast(T.region_shape, B) && (int64_t)xi - alpha >= halo_slow(T.region_shape, B);

    // -- 7. field-stop tiling of the back projection ----------------------------
    T.nbx = (int32_t)ceil_div(a, kTileFast);
    T.nby = (int32_t)ceil_div(alpha, kTileSlow);
    if ((int64_t)T.nbx * T.nby * w > INT32_MAX) return fail(CTIS_E_TOO_LARGE, "too many field-stop tiles");

    int32_t max_boxes = 0;
    for (int32_t s = 0; s < w; ++s)
        max_boxes = std::max(max_boxes, T.lambda_box_ptr[(size_t)s + 1] - T.lambda_box_ptr[(size_t)s]);
    T.max_boxes = max_boxes;
    return CTIS_OK;
}

namespace {

int32_t waves_for(int32_t work, int B) {
    // one wavefront per box of the heaviest unit, up to the workgroup's cap:
    // every window of the unit is in flight at once (measured on a 128^2 FPA
    // frame with ~17 boxes per tile: 16 waves 10.9 us per EM iteration, 11
    // waves 11.3 us)
    return std::max(min_waves(), std::min(max_waves(B), work));
}

// Back projection: while its units fit on the chip at once (one workgroup
// per compute unit of the MI355X's 256), the launch is latency-bound and
// every box of a wavelength gets its own wavefront (all windows in flight
// together); with more units than compute units the fewest waves per
// workgroup keep the most units resident.  Both measured on the c2 and c3
// shapes.
constexpr int64_t kChipCUs = 256;

int32_t adjoint_waves(int64_t units, int32_t boxes, int B) {
    if (units > kChipCUs) return min_waves();
    return std::max(min_waves(), std::min(max_waves(B), boxes));
}

// Forward: in the latency-bound regime (units fit on the chip) one wave per
// box of the heaviest unit; with more units than compute units about
// one wave per four boxes of the average unit (measured: a 1024^2 frame with
// ~62 boxes per tile runs fastest with 16 waves, 64 uneven frames with ~16
// boxes per tile with 4).
int32_t forward_waves(int64_t units, int64_t items, int32_t max_items, int B) {
    if (units <= kChipCUs) return waves_for(max_items, B);
    const int64_t avg = units > 0 ? (items + units / 2) / units : 0;
    return std::max(min_waves(), std::min<int32_t>(max_waves(B), (int32_t)((avg + 2) / 4)));
}

// Region forward: a wave takes G boxes of its region at a time (one per
// lane group; G = 4 for regions of 256 pixels), so a workgroup of W waves
// takes G W per pass.  In the latency-bound regime (the units fit on the
// chip at once) enough waves for the heaviest unit's boxes in one pass, up to
// the workgroup's cap (a 128^2 frame with up to 17 boxes per 16 x 16 region:
// 2 waves 10.6 us per EM iteration, 4 waves 10.0 us, 6 waves 9.7 us).
// Otherwise about one wave per 5 G / 4 boxes of the average unit, 1 to 4:
// more waves per workgroup leave fewer workgroups resident per compute unit
// (measured on the 512^2 and 1024^2 frames with 15 and 46 boxes per 16 x 16
// region: 3 and 4 waves best, 5 or more a third slower).
int32_t region_waves(int64_t units, int64_t items, int32_t max_items, int shape) {
    const int64_t g = 64 / region_gl(shape);
    if (units <= kChipCUs)
        return (int32_t)std::max<int64_t>(1, std::min<int64_t>(kFwdMaxWaves, (max_items + g - 1) / g));
    const int64_t avg = units > 0 ? (items + units - 1) / units : 0;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(4, (4 * avg + 5 * g - 1) / (5 * g)));
}

void push4(std::vector<int32_t> &v, int32_t a, int32_t b, int32_t c, int32_t d) {
    v.push_back(a);
    v.push_back(b);
    v.push_back(c);
    v.push_back(d);
}

// A window of sx x sy positions at the (undecoded, possibly negative) origin
// (Xs, Ys) of E f_s reads exactly what a 2-D window over f_s bordered with
// zeros reads, when no position of it lies past the FPA's last column or
// row, and every position the 1-D cyclic shift carries into the previous
// FPA column (a negative column) or round the end of the FPA (a negative row)
// lands on a column at or past a, or a row at or past alpha, where E f_s is
// 0: Xs > a - gamma and Ys > alpha - xi.
bool direct_2d(int64_t Xs, int64_t Ys, int64_t a, int64_t alpha, int64_t gamma, int64_t xi, int64_t sx, int64_t sy) {
    return Xs > a - gamma && Xs + sx <= gamma && Ys > alpha - xi && Ys + sy <= xi;
}

struct UnitRef {
    int32_t frame, tile, chunk, n_chunks, slot, work;
};

// XCD-aware unit order for batches.  The MI355X deals workgroups to its 8
// XCDs (each with its own L2) round-robin by workgroup index, so unit
// position p runs on XCD p mod 8 (also under the persistent grid, whose size
// is a multiple of 8).  Frames read only their own f, g and u, so each frame
// is given one XCD -- greedily by work, largest frame first to the least
// loaded XCD -- and position 8k + x takes the next unit of XCD x's frames (in
// their incoming order); a position whose list has run out takes the last
// unit of the fullest remaining list, trading that unit's locality for
// balance.  With fewer frames than XCDs the order is left as it is.
constexpr int kXcds = 8;

template <class Unit, class FrameOf, class WorkOf>
std::vector<Unit> xcd_order(const std::vector<Unit> &units, size_t n_frames, FrameOf frame_of, WorkOf work_of) {
    if (n_frames < (size_t)kXcds) return units;
    std::vector<int64_t> fwork(n_frames, 0);
    for (const Unit &u : units) fwork[(size_t)frame_of(u)] += work_of(u);
    std::vector<size_t> order(n_frames);
    std::iota(order.begin(), order.end(), size_t(0));
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return fwork[x] > fwork[y]; });
    std::vector<int64_t> load(kXcds, 0);
    std::vector<int> frame_xcd(n_frames, 0);
    for (size_t f : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        frame_xcd[f] = x;
        load[(size_t)x] += fwork[f];
    }
    std::vector<std::vector<Unit>> bins(kXcds);
    for (const Unit &u : units) bins[(size_t)frame_xcd[(size_t)frame_of(u)]].push_back(u);
    std::vector<size_t> head(kXcds, 0), tail(kXcds);
    for (int x = 0; x < kXcds; ++x) tail[(size_t)x] = bins[(size_t)x].size();
    std::vector<Unit> out;
    out.reserve(units.size());
    while (out.size() < units.size()) {
        for (int x = 0; x < kXcds && out.size() < units.size(); ++x) {
            if (head[(size_t)x] < tail[(size_t)x]) {
                out.push_back(bins[(size_t)x][head[(size_t)x]++]);
                continue;
            }
            size_t best = 0;
            int src = -1;
            for (int y = 0; y < kXcds; ++y)
                if (tail[(size_t)y] - head[(size_t)y] > best) {
                    best = tail[(size_t)y] - head[(size_t)y];
                    src = y;
                }
            out.push_back(bins[(size_t)src][--tail[(size_t)src]]);
        }
    }
    return out;
}

}  // namespace

ctis_status build_work(const std::vector<FrameRef> &frames, bool with_full, HostWork &hw) {
    hw = HostWork{};
    if (frames.empty()) return fail(CTIS_E_ARG, "no frames");
    hw.B = frames[0].plan->ht.B;
    const int B = hw.B;
    const int BB = B * B;
    // distinct plans in order of first appearance; frames that share a plan
    // share its boxes, wavelengths and values
    std::vector<const ctis_plan *> dplans;
    int32_t box_base = 0, lambda_base = 0, max_chunk_items = 0, max_full_items = 0, max_boxes = 0;
    int64_t entry_base = 0;
    for (size_t k = 0; k < frames.size(); ++k) {
        const ctis_plan *pl = frames[k].plan;
        const HostTables &T = pl->ht;
        if (T.B != B) return fail(CTIS_E_ARG, "all frames of a batch need the same box side B");
        const auto it = std::find(dplans.begin(), dplans.end(), pl);
        if (it != dplans.end()) {
            hw.frame_plan.push_back((int32_t)(it - dplans.begin()));
        } else {
            hw.frame_plan.push_back((int32_t)dplans.size());
            dplans.push_back(pl);
            hw.plan_box0.push_back(box_base);
            hw.plan_lam0.push_back(lambda_base);
            hw.plan_entry0.push_back(entry_base);
            if ((int64_t)box_base + (int64_t)T.box_lambda.size() > INT32_MAX / BB ||
                (int64_t)lambda_base + pl->w > INT32_MAX || entry_base + T.n_in > INT32_MAX)
                return fail(CTIS_E_TOO_LARGE, "too many boxes, wavelengths or entries");
            box_base += (int32_t)T.box_lambda.size();
            lambda_base += pl->w;
            entry_base += T.n_in;
            hw.box_w.insert(hw.box_w.end(), T.box_w.begin(), T.box_w.end());
            hw.box_wf.insert(hw.box_wf.end(), T.box_wf.begin(), T.box_wf.end());
            hw.h.insert(hw.h.end(), T.h.begin(), T.h.end());
            hw.dropped = hw.dropped || T.dropped;
        }
        max_boxes = std::max(max_boxes, T.max_boxes);
        hw.u_floats = std::max<int64_t>(hw.u_floats, frames[k].u_base + pl->n);
        hw.g_floats = std::max<int64_t>(hw.g_floats, frames[k].g_base + pl->n);
        hw.f_floats = std::max<int64_t>(hw.f_floats, frames[k].f_base + pl->m);
    }
    std::vector<int32_t> fbox(frames.size()), flam(frames.size());
    for (size_t k = 0; k < frames.size(); ++k) {
        fbox[k] = hw.plan_box0[(size_t)hw.frame_plan[k]];
        flam[k] = hw.plan_lam0[(size_t)hw.frame_plan[k]];
    }

    // padded copy of f for the region path: per frame and wavelength a block
    // of (a + 2 Hx) x (alpha + 2 Hy) floats, frames back to back.  The path
    // needs every frame to allow it, with one region shape.
    const int shape = frames[0].plan->ht.region_shape;
    const int Hx = halo_fast(shape, B), Hy = halo_slow(shape, B);
    hw.region_shape = shape;
    hw.halo_x = Hx;
    hw.halo_y = Hy;
    std::vector<int64_t> fp_base(frames.size(), 0);
    hw.pad_ok = true;
    for (size_t k = 0; k < frames.size(); ++k) {
        const ctis_plan *pl = frames[k].plan;
        hw.pad_ok = hw.pad_ok && pl->ht.pad_ok && pl->ht.region_shape == shape;
        fp_base[k] = hw.fp_floats;
        hw.fp_floats += (int64_t)pl->w * (pl->a + 2 * Hx) * (pl->alpha + 2 * Hy);
        hw.pad_rows = std::max(hw.pad_rows, pl->alpha + 2 * Hy);
    }
    if (hw.fp_floats > kMaxPixels) hw.pad_ok = false;

    // forward lists: units of every frame, heaviest first (a stable order).
    // Tile records (tile path): (window origin Xs, Ys, f offset of the box's
    // wavelength block, global box).  Region records (region path): (float
    // offset of the window origin in the padded copy, 0, 0, global box).
    auto build_fwd = [&](HostList &L, bool region, bool em, int32_t stride, std::vector<int32_t> &smeta,
                         int32_t &n_split, int32_t &slots) -> ctis_status {
        std::vector<UnitRef> units;
        for (size_t k = 0; k < frames.size(); ++k) {
            const HostTables &T = frames[k].plan->ht;
            const WorkGrid &G = region ? T.regions : T.tiles;
            const int32_t ntl = em ? G.n_active : G.n_cells;
            for (int32_t u = 0; u < ntl; ++u) {
                const int32_t tile = G.order[(size_t)u];
                const int32_t cnt = G.item_ptr[(size_t)tile + 1] - G.item_ptr[(size_t)tile];
                const int32_t nch = em ? std::max(1, (cnt + stride - 1) / stride) : 1;
                const int32_t slot0 = nch > 1 ? slots : -1;
                if (nch > 1) {
                    push4(smeta, (tile % G.ntr) * G.tf, (tile / G.ntr) * G.ts, nch, slot0);
                    push4(smeta, frames[k].plan->gamma, frames[k].plan->xi, (int32_t)frames[k].g_base,
                          (int32_t)frames[k].u_base);
                    slots += nch;
                    n_split++;
                }
                for (int32_t c = 0; c < nch; ++c)
                    units.push_back(UnitRef{(int32_t)k, tile, c, nch, nch > 1 ? slot0 + c : -1,
                                            std::min(stride, cnt - c * stride)});
            }
        }
        std::stable_sort(units.begin(), units.end(), [](const UnitRef &x, const UnitRef &y) { return x.work > y.work; });
        units = xcd_order(units, frames.size(), [](const UnitRef &u) { return u.frame; },
                          [](const UnitRef &u) { return (int64_t)u.work; });
        L.stride = std::max(1, stride);
        L.meta.clear();
        L.items.clear();
        for (const UnitRef &ur : units) {
            const FrameRef &fr = frames[(size_t)ur.frame];
            const ctis_plan *pl = fr.plan;
            const HostTables &T = pl->ht;
            const WorkGrid &G = region ? T.regions : T.tiles;
            const int32_t r0 = (ur.tile % G.ntr) * G.tf, c0 = (ur.tile / G.ntr) * G.ts;
            const int64_t P = (int64_t)pl->a + 2 * Hx, PB = P * ((int64_t)pl->alpha + 2 * Hy);
            push4(L.meta, r0, c0, ur.n_chunks, ur.slot);
            push4(L.meta, pl->a, pl->alpha, pl->gamma, pl->xi);
            push4(L.meta, (int32_t)fr.g_base, em ? (int32_t)fr.u_base : (int32_t)fr.g_base, region ? (int32_t)P : 0, 0);
            const int32_t b0 = G.item_ptr[(size_t)ur.tile];
            const int32_t cnt = G.item_ptr[(size_t)ur.tile + 1] - b0;
            for (int32_t k = 0; k < L.stride; ++k) {
                const int32_t idx = ur.chunk * L.stride + k;
                if (!(k < ur.work && idx < cnt)) {
                    push4(L.items, 0, 0, 0, -1);
                    continue;
                }
                const int32_t b = G.item_box[(size_t)(b0 + idx)];
                const int32_t s = T.box_lambda[(size_t)b];
                const int64_t Xs = (int64_t)r0 - (B - 1) - T.box_rc[2 * (size_t)b];
                const int64_t Ys = (int64_t)c0 - (B - 1) - T.box_rc[2 * (size_t)b + 1];
                if (!region) {
                    // decoded origin; direct if the window's columns do not carry
                    // into the next FPA column and its rows do not wrap
                    const int64_t q0 = floor_div(Xs, pl->gamma);
                    const int64_t xr = Xs - q0 * pl->gamma, y0 = floor_mod(Ys + q0, pl->xi);
                    const int32_t foff = (int32_t)(fr.f_base + (int64_t)s * pl->ell);
                    if (xr + kTileFast + B - 1 <= pl->gamma && y0 + kTileSlow + B - 1 <= pl->xi)
                        push4(L.items, (int32_t)xr, (int32_t)y0, foff | kDirectFlag, fbox[(size_t)ur.frame] + b);
                    else if (direct_2d(Xs, Ys, pl->a, pl->alpha, pl->gamma, pl->xi, kTileFast + B - 1,
                                       kTileSlow + B - 1))
                        push4(L.items, (int32_t)Xs, (int32_t)Ys, foff | kDirectFlag, fbox[(size_t)ur.frame] + b);
                    else
                        push4(L.items, (int32_t)Xs, (int32_t)Ys, foff, fbox[(size_t)ur.frame] + b);
                    continue;
                }
                // The window's slot (xx, yy) holds fE((Xs + xx) + gamma*(Ys + yy) mod n).
                // Write its origin as X + gamma*Y with X in [-Hx, a) and Y in [-Hy,
                // alpha): the window then lies inside the padded block, whose value
                // at (X', Y') is fE(X' + gamma*Y' mod n) because the FPA leaves Hx
                // and Hy pixels beside the field stop.  From the canonical origin
                // (qf, qs): X = qf, or qf - gamma with qs + 1 if the window starts
                // within Hx of the FPA's last row; likewise Y = qs or qs - xi.  (A
                // window meeting the image of its box holds a voxel of the field
                // stop, so one of the two fits.)
                const int64_t q = floor_mod(Xs + (int64_t)pl->gamma * Ys, pl->n);
                int64_t X = q % pl->gamma, Y = q / pl->gamma;
                if (X >= pl->a) {
                    if (X < (int64_t)pl->gamma - Hx) return fail(CTIS_E_ARG, "region window outside the field stop");
                    X -= pl->gamma;
                    Y = (Y + 1) % pl->xi;
                }
                if (Y >= pl->alpha) {
                    if (Y < (int64_t)pl->xi - Hy) return fail(CTIS_E_ARG, "region window outside the field stop");
                    Y -= pl->xi;
                }
                const int64_t poff = fp_base[(size_t)ur.frame] + (int64_t)s * PB + (X + Hx) + P * (Y + Hy);
                push4(L.items, (int32_t)poff, 0, 0, fbox[(size_t)ur.frame] + b);
            }
            if (L.items.size() > (size_t)INT32_MAX) return fail(CTIS_E_TOO_LARGE, "forward work list too large");
        }
        L.n_units = (int32_t)(L.meta.size() / 12);
        return CTIS_OK;
    };
    int32_t chunk = 1 << 30, rchunk = 1 << 30;
    for (const FrameRef &fr : frames) {
        chunk = std::min(chunk, fr.plan->ht.tiles.chunk);
        rchunk = std::min(rchunk, fr.plan->ht.regions.chunk);
    }
    for (const FrameRef &fr : frames) {
        const HostTables &T = fr.plan->ht;
        max_chunk_items = std::max(max_chunk_items, std::min(T.tiles.max_items, chunk));
        max_full_items = std::max(max_full_items, T.tiles.max_items);
    }
    auto count_items = [](const HostList &L) {
        int64_t n = 0;
        for (size_t k = 3; k < L.items.size(); k += 4) n += L.items[k] >= 0;
        return n;
    };
    auto max_unit_items = [](const HostList &L) {   // most boxes of one unit
        int32_t best = 0;
        const size_t per = 4 * (size_t)L.stride;
        for (size_t u = 0; u + per <= L.items.size(); u += per) {
            int32_t n = 0;
            for (size_t k = u + 3; k < u + per; k += 4) n += L.items[k] >= 0;
            best = std::max(best, n);
        }
        return best;
    };
    ctis_status st = CTIS_OK;
    if (with_full) {
        std::vector<int32_t> no_split;
        int32_t n0 = 0, s0 = 0;
        st = build_fwd(hw.fwd_full, false, false, std::max(1, max_full_items), no_split, n0, s0);
        if (st != CTIS_OK) return st;
        hw.fwd_full.waves = forward_waves(hw.fwd_full.n_units, count_items(hw.fwd_full), max_full_items, B);
    }
    st = build_fwd(hw.fwd_em, false, true, chunk, hw.split_meta, hw.n_split, hw.partial_slots);
    if (st != CTIS_OK) return st;
    hw.fwd_em.waves = forward_waves(hw.fwd_em.n_units, count_items(hw.fwd_em), max_chunk_items, B);
    if (hw.pad_ok) {
        st = build_fwd(hw.fwd_pad, true, true, rchunk, hw.rsplit_meta, hw.n_rsplit, hw.rpartial_slots);
        if (st != CTIS_OK) return st;
        hw.fwd_pad.waves = region_waves(hw.fwd_pad.n_units, count_items(hw.fwd_pad), max_unit_items(hw.fwd_pad), shape);
        for (size_t k = 0; k < frames.size(); ++k) {
            const ctis_plan *pl = frames[k].plan;
            const int64_t PB = (int64_t)(pl->a + 2 * Hx) * (pl->alpha + 2 * Hy);
            for (int32_t s = 0; s < pl->w; ++s)
                push4(hw.pad_blocks, (int32_t)(frames[k].f_base + (int64_t)s * pl->ell),
                      (int32_t)(fp_base[k] + (int64_t)s * PB), pl->a, pl->alpha);
        }
    }

    // adjoint: units (frame, wavelength, field-stop tile); records per global wavelength
    HostList &A = hw.adj;
    A.stride = std::max(1, max_boxes);
    A.items.assign((size_t)4 * lambda_base * A.stride, 0);
    for (size_t d = 0; d < dplans.size(); ++d) {
        const ctis_plan *pl = dplans[d];
        const HostTables &T = pl->ht;
        for (int32_t s = 0; s < pl->w; ++s) {
            const int32_t gs = hw.plan_lam0[d] + s;
            const int32_t b0 = T.lambda_box_ptr[(size_t)s], b1 = T.lambda_box_ptr[(size_t)s + 1];
            for (int32_t j = 0; j < A.stride; ++j) {
                int32_t *rec = &A.items[(size_t)4 * ((size_t)gs * A.stride + j)];
                if (b0 + j < b1) {
                    rec[0] = T.box_rc[2 * (size_t)(b0 + j)];
                    rec[1] = T.box_rc[2 * (size_t)(b0 + j) + 1];
                    // direct: what the voxels inside the field stop read stays inside
                    // the FPA (the box's image of the dilated field stop neither
                    // carries into the next FPA column nor wraps round the FPA's
                    // end), and the last tile's whole window ends inside u (the
                    // loader's row offset is a scalar offset, which is kept in
                    // bounds rather than left to the range check).  Lanes of a
                    // tile past a or alpha may then read other pixels of u; their
                    // outputs are never written.
                    const int64_t last = (int64_t)rec[0] + (int64_t)T.nbx * kTileFast + B - 2 +
                                         (int64_t)pl->gamma * ((int64_t)rec[1] + (int64_t)T.nby * kTileSlow + B - 2);
                    rec[2] = ((int64_t)rec[0] + pl->a + B - 1 <= pl->gamma &&
                              (int64_t)rec[1] + pl->alpha + B - 1 <= pl->xi && last < (int64_t)pl->n) ? 1 : 0;
                    rec[3] = hw.plan_box0[d] + b0 + j;
                } else {
                    rec[3] = -1;
                }
            }
        }
    }
    struct AdjRef {
        int32_t frame, s, vt, work;
    };
    std::vector<AdjRef> adj_units;
    for (size_t k = 0; k < frames.size(); ++k) {
        const ctis_plan *pl = frames[k].plan;
        const HostTables &T = pl->ht;
        for (int32_t s = 0; s < pl->w; ++s) {
            const int32_t nb = T.lambda_box_ptr[(size_t)s + 1] - T.lambda_box_ptr[(size_t)s];
            for (int32_t vt = 0; vt < T.nbx * T.nby; ++vt) adj_units.push_back(AdjRef{(int32_t)k, s, vt, nb});
        }
    }
    if (adj_units.size() > (size_t)INT32_MAX / ((size_t)A.stride * BB))
        return fail(CTIS_E_TOO_LARGE, "too many back-projection units");
    hw.adj_direct = true;
    for (size_t r = 0; r < A.items.size(); r += 4)
        if (A.items[r + 3] >= 0 && A.items[r + 2] == 0) hw.adj_direct = false;
    adj_units = xcd_order(adj_units, frames.size(), [](const AdjRef &u) { return u.frame; },
                          [](const AdjRef &u) { return (int64_t)u.work; });
    std::vector<std::vector<int32_t>> units_of(lambda_base);
    for (const AdjRef &au : adj_units) {
        const FrameRef &fr = frames[(size_t)au.frame];
        const ctis_plan *pl = fr.plan;
        const HostTables &T = pl->ht;
        const int32_t gs = flam[(size_t)au.frame] + au.s;
        units_of[(size_t)gs].push_back((int32_t)(A.meta.size() / 12));
        push4(A.meta, (au.vt % T.nbx) * kTileFast, (au.vt / T.nbx) * kTileSlow, gs,
              (int32_t)(fr.f_base + (int64_t)au.s * pl->ell));
        push4(A.meta, pl->a, pl->alpha, pl->gamma, pl->xi);
        const int64_t P = (int64_t)pl->a + 2 * Hx, PB = P * ((int64_t)pl->alpha + 2 * Hy);
        push4(A.meta, (int32_t)fr.u_base, hw.pad_ok ? (int32_t)(fp_base[(size_t)au.frame] + (int64_t)au.s * PB) : 0,
              hw.pad_ok ? (int32_t)P : 0, 0);
    }
    A.n_units = (int32_t)(A.meta.size() / 12);
    A.waves = adjoint_waves(A.n_units, max_boxes, B);

    // value tables
    hw.box_lam.resize((size_t)box_base);
    hw.lam_box0.assign((size_t)lambda_base + 1, box_base);
    hw.entry_slot.reserve((size_t)entry_base);
    for (size_t d = 0; d < dplans.size(); ++d) {
        const HostTables &T = dplans[d]->ht;
        for (size_t b = 0; b < T.box_lambda.size(); ++b)
            hw.box_lam[(size_t)hw.plan_box0[d] + b] = hw.plan_lam0[d] + T.box_lambda[b];
        for (int32_t s = 0; s < dplans[d]->w; ++s)
            hw.lam_box0[(size_t)(hw.plan_lam0[d] + s)] = hw.plan_box0[d] + T.lambda_box_ptr[(size_t)s];
        for (int32_t slot : T.entry_slot) hw.entry_slot.push_back(slot < 0 ? -1 : hw.plan_box0[d] * BB + slot);
    }
    hw.lam_units_ptr.assign(1, 0);
    for (const auto &v : units_of) {
        hw.lam_units.insert(hw.lam_units.end(), v.begin(), v.end());
        hw.lam_units_ptr.push_back((int32_t)hw.lam_units.size());
    }
    const size_t n_slots = (size_t)box_base * BB;
    hw.slot_entries_ptr.assign(n_slots + 1, 0);
    for (int32_t slot : hw.entry_slot)
        if (slot >= 0) hw.slot_entries_ptr[(size_t)slot + 1]++;
    for (size_t k = 0; k < n_slots; ++k) hw.slot_entries_ptr[k + 1] += hw.slot_entries_ptr[k];
    hw.slot_entries.resize((size_t)hw.slot_entries_ptr[n_slots]);
    {
        std::vector<int32_t> pos(hw.slot_entries_ptr.begin(), hw.slot_entries_ptr.end() - 1);
        for (size_t t = 0; t < hw.entry_slot.size(); ++t)
            if (hw.entry_slot[t] >= 0) hw.slot_entries[(size_t)pos[(size_t)hw.entry_slot[t]]++] = (int32_t)t;
    }
    return CTIS_OK;
}

Layout layout_for(const HostWork &hw) {
    auto up256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    Layout L{};
    L.partials_off = up256((size_t)hw.u_floats * sizeof(float));
    L.rpartials_off = L.partials_off + up256((size_t)hw.partial_slots * kTileFast * kTileSlow * sizeof(float));
    L.fp_off = L.rpartials_off + up256((size_t)hw.rpartial_slots * kRegionPixels * sizeof(float));
    L.diag_off = L.fp_off + up256(hw.pad_ok ? (size_t)hw.fp_floats * sizeof(float) : 0);
    L.em_bytes = L.diag_off + (size_t)kDiagParts * 4 * sizeof(double);
    L.e_off = up256(L.em_bytes);
    L.zeta_off = L.e_off + up256((size_t)hw.u_floats * sizeof(float));
    L.b_off = L.zeta_off + up256((size_t)hw.f_floats * sizeof(float));
    L.hpart_off = L.b_off + up256((size_t)hw.f_floats * sizeof(float));
    L.vg_off = L.hpart_off + up256((size_t)hw.adj.n_units * sizeof(float));
    L.vjp_bytes = L.vg_off + up256((size_t)hw.adj.n_units * hw.adj.stride * hw.B * hw.B * sizeof(float));
    L.solve_r_off = L.e_off;
    L.solve_ones_off = L.solve_r_off + up256((size_t)hw.g_floats * sizeof(float));
    L.solve_bytes = L.solve_ones_off + up256((size_t)hw.f_floats * sizeof(float));
    return L;
}

ctis_status upload_work(const HostWork &hw, DevWork &dw) {
    struct Part {
        const void *src;
        size_t bytes;
        size_t off;
    };
    std::vector<Part> parts = {
        {hw.fwd_full.meta.data(), hw.fwd_full.meta.size() * 4, 0},
        {hw.fwd_full.items.data(), hw.fwd_full.items.size() * 4, 0},
        {hw.fwd_em.meta.data(), hw.fwd_em.meta.size() * 4, 0},
        {hw.fwd_em.items.data(), hw.fwd_em.items.size() * 4, 0},
        {hw.split_meta.data(), hw.split_meta.size() * 4, 0},
        {hw.adj.meta.data(), hw.adj.meta.size() * 4, 0},
        {hw.adj.items.data(), hw.adj.items.size() * 4, 0},
        {hw.box_w.data(), hw.box_w.size() * 4, 0},
        {hw.box_wf.data(), hw.box_wf.size() * 4, 0},
        {hw.h.data(), hw.h.size() * 4, 0},
        {hw.entry_slot.data(), hw.entry_slot.size() * 4, 0},
        {hw.box_lam.data(), hw.box_lam.size() * 4, 0},
        {hw.lam_box0.data(), hw.lam_box0.size() * 4, 0},
        {hw.lam_units_ptr.data(), hw.lam_units_ptr.size() * 4, 0},
        {hw.lam_units.data(), hw.lam_units.size() * 4, 0},
        {hw.slot_entries_ptr.data(), hw.slot_entries_ptr.size() * 4, 0},
        {hw.slot_entries.data(), hw.slot_entries.size() * 4, 0},
        {hw.fwd_pad.meta.data(), hw.fwd_pad.meta.size() * 4, 0},
        {hw.fwd_pad.items.data(), hw.fwd_pad.items.size() * 4, 0},
        {hw.rsplit_meta.data(), hw.rsplit_meta.size() * 4, 0},
        {hw.pad_blocks.data(), hw.pad_blocks.size() * 4, 0},
    };
    size_t total = 0;
    for (auto &pt : parts) {
        pt.off = total;
        total += (std::max<size_t>(pt.bytes, 4) + 255) & ~(size_t)255;
    }
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, total);
    if (e != hipSuccess) return fail(CTIS_E_NOMEM, std::string("hipMalloc of work tables: ") + hipGetErrorString(e));
    for (const auto &pt : parts) {
        if (!pt.bytes) continue;
        e = hipMemcpy((char *)mem + pt.off, pt.src, pt.bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(mem);
            return fail(CTIS_E_HIP, std::string("hipMemcpy of work tables: ") + hipGetErrorString(e));
        }
    }
    auto at = [&](int k) { return (const void *)((const char *)mem + parts[(size_t)k].off); };
    auto list = [&](DevList &L, const HostList &H, int k0) {
        L.meta = (const int4 *)at(k0);
        L.items = (const int4 *)at(k0 + 1);
        L.n_units = H.n_units;
        L.stride = H.stride;
        L.waves = H.waves;
    };
    dw = DevWork{};
    dw.B = hw.B;
    list(dw.fwd_full, hw.fwd_full, 0);
    list(dw.fwd_em, hw.fwd_em, 2);
    dw.split_meta = (const int4 *)at(4);
    dw.n_split = hw.n_split;
    dw.adj.meta = (const int4 *)at(5);
    dw.adj.items = (const int4 *)at(6);
    dw.adj.n_units = hw.adj.n_units;
    dw.adj.stride = hw.adj.stride;
    dw.adj.waves = hw.adj.waves;
    dw.box_w = (float *)at(7);
    dw.box_wf = (float *)at(8);
    dw.h = (float *)at(9);
    dw.entry_slot = (const int32_t *)at(10);
    dw.box_lam = (const int32_t *)at(11);
    dw.lam_box0 = (const int32_t *)at(12);
    dw.lam_units_ptr = (const int32_t *)at(13);
    dw.lam_units = (const int32_t *)at(14);
    dw.slot_entries_ptr = (const int32_t *)at(15);
    dw.slot_entries = (const int32_t *)at(16);
    dw.pad_ok = hw.pad_ok;
    dw.region_shape = hw.region_shape;
    dw.halo_x = hw.halo_x;
    dw.halo_y = hw.halo_y;
    if (hw.pad_ok) {
        list(dw.fwd_pad, hw.fwd_pad, 17);
        dw.rsplit_meta = (const int4 *)at(19);
        dw.n_rsplit = hw.n_rsplit;
        dw.pad_blocks = (const int4 *)at(20);
        dw.n_pad_blocks = (int32_t)(hw.pad_blocks.size() / 4);
        dw.pad_rows = hw.pad_rows;
        dw.fp_floats = (int32_t)hw.fp_floats;
    }
    dw.f_floats = (int32_t)hw.f_floats;
    dw.n_wf = (int32_t)hw.box_wf.size();
    dw.n_entries = (int64_t)hw.entry_slot.size();
    dw.n_lambda = (int32_t)hw.h.size();
    dw.n_boxes = (int32_t)hw.box_lam.size();
    const Layout L = layout_for(hw);
    dw.partials_off = L.partials_off;
    dw.rpartials_off = L.rpartials_off;
    dw.fp_off = L.fp_off;
    dw.diag_off = L.diag_off;
    dw.workspace_bytes = L.em_bytes;
    dw.e_off = L.e_off;
    dw.zeta_off = L.zeta_off;
    dw.b_off = L.b_off;
    dw.hpart_off = L.hpart_off;
    dw.vg_off = L.vg_off;
    dw.vjp_workspace_bytes = L.vjp_bytes;
    dw.adj_direct = hw.adj_direct;
    dw.solve_r_off = L.solve_r_off;
    dw.solve_ones_off = L.solve_ones_off;
    dw.solve_workspace_bytes = L.solve_bytes;
    dw.mem = mem;
    return CTIS_OK;
}

void free_work(DevWork &dw) {
    if (dw.mem) (void)hipFree(dw.mem);
    dw = DevWork{};
}

}  // namespace ctis
