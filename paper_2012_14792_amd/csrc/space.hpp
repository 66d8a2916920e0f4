// Candidate-space plan: host-built tables that let the GPU enumerate every TRS candidate
// of a frame geometry in canonical rank order, and the device-side views of them.
//
// A candidate (Section 1 and Section 2.3 of the paper, with the explicit space of the
// design notes) is a c x r tile grid with column boundaries X and row boundaries Y, plus,
// per tile, a slice count k and split offsets Z, with sum of k = N.  For a fixed shape and
// Y, the list of per-tile choices ("combinations") does not depend on X, so the space is
// stored as: per shape, the X list and the Y list; per (shape, Y), its combinations, each
// a vector of per-tile option indices; per tile height h, the option list (k ascending,
// then Z lexicographic).  Canonical rank = shape base + xi * sum_Y M(Y) + prefix_M(yi) + m.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "trs.h"

namespace trs {

constexpr int kMaxRS = TRS_MAX_RS;
constexpr int kMaxGrid = 256;        // CTU columns / rows
constexpr int kRecCap = 2048;        // tile-option records staged in LDS per work item
constexpr int kSpanCap = 255;        // distinct column spans per work item
constexpr int64_t kComboCap = int64_t(1) << 28;   // u16 entries in all combination tables
constexpr int64_t kSpaceCap = int64_t(1) << 40;

// One tile-grid shape (c, r).
struct ShapeDev {
    int32_t c, r, T, kcap;     // kcap = min(Kmax, N - (T - 1)): largest k any tile can take
    int64_t nX, nY, SM;        // |X|, |Y|, sum over Y of M(Y)
    int64_t rank_base;         // rank of this shape's first candidate
    int64_t x_off, y_off;      // u16 offsets of the X and Y tables (rows of c+1 / r+1)
    int64_t yinfo_off;         // offset into the per-Y arrays
};

// A unit of GPU work: area-feasible candidates of one (shape, Y), from X = xa onwards.
// The area rule depends only on the geometry, so it is applied when the plan is built and
// an item lists only the candidates that pass it.  Entry e of the item is candidate
// f = (x - xa) * M + m; its tile t uses tile-option record ent_rid[rid_off + t * n_ent + e];
// record i of the item is described by rdesc[2 * (rec_off + i)]: word 0 = column span start
// | span end << 9 | tile-row start << 18 (CTUs), word 1 = option index.
struct ItemDev {
    int64_t rank0;             // rank of (X = xa, Y = yi, m = 0)
    int64_t combo_off;         // u16 offset of this (shape, Y)'s combination table, [T][M]
    int64_t SM;                // rank stride between consecutive X: sum over Y of M(Y)
    int64_t y_row;             // u16 offset of this item's Y vector (r + 1 entries)
    int64_t ent_off;           // first entry in ent_f
    int64_t rid_off;           // first record index in ent_rid
    int64_t rec_off;           // first record descriptor
    int32_t shape, yi, xa, M, n_ent, n_rec, c, r, T, pad;
};

// Device pointers into the uploaded plan (passed to kernels by value).
struct SpaceView {
    const int32_t *colpx, *rowpx;      // pixel prefix sums of CTU widths / heights
    const int32_t *opt_base;           // [H + 1]: first option of height h
    const int32_t *opt_kcnt;           // [(H + 1) * (Kmax + 1)]: options of height h with k <= kk
    const uint8_t *opt_k;              // per option: k
    const uint16_t *opt_z;             // per option: Kmax + 1 offsets z_0 = 0 .. z_k = h
    const ShapeDev *shapes;
    const uint16_t *xtab, *ytab;
    const int64_t *y_prefM, *y_combo;
    const int32_t *y_M;
    const uint16_t *combos;
    const ItemDev *items;
    const uint32_t *ent_f;             // per entry: (x - xa) * M + m
    const uint16_t *ent_rid;           // per item [T][n_ent] record indices
    const uint32_t *rdesc;             // per record: two words (see ItemDev)
    const uint32_t *rdesc4;            // per record: four words, the split rows inline (see Plan)
    const int32_t *unif_rs;            // [n_unif * 4]
    int32_t W, H, N, Km, n_items, n_shapes, n_unif, pad;
    int32_t cu, ru;                    // uniform grid shape
    int32_t rec_max;                   // largest per-item record count
    int32_t rid_max;                   // largest per-item n_ent * T, rounded up to 8
    int32_t compact, pad3;             // 1: rdesc4 holds every record
    int64_t total, uniform_rank, n_feasible;
};

struct Plan {
    // key
    int32_t device, width, height, cs, N, Cm, Rm, Km, dtile_req, drs_req, item_target;
    int64_t budget;
    // geometry and space
    int32_t W = 0, H = 0, dt = 0, dr = 0;
    int64_t total = 0;
    std::vector<int32_t> colpx, rowpx, opt_base, opt_kcnt;
    std::vector<uint8_t> opt_k;
    std::vector<uint16_t> opt_z;
    std::vector<ShapeDev> shapes;
    std::vector<uint16_t> xtab, ytab;
    std::vector<int64_t> y_prefM, y_combo;
    std::vector<int32_t> y_M;
    std::vector<uint16_t> combos;
    std::vector<ItemDev> items;
    std::vector<uint32_t> ent_f;
    std::vector<uint16_t> ent_rid;
    std::vector<uint32_t> rdesc;
    // Per record, four words: word 0 as in rdesc; words 1..3 the slice count k (low byte)
    // and the split rows z_1 .. z_k of the option (one byte each, z_k = tile height).
    // Filled only when every record has k <= 11 and tile heights <= 255 (compact = 1).
    std::vector<uint32_t> rdesc4;
    int32_t compact = 0;
    int32_t cu = 0, ru = 0, n_unif = 0;
    std::vector<int32_t> unif_rs;
    int64_t uniform_rank = -1;
    int32_t rec_max = 0;               // largest record count of an item (LDS records)
    int32_t rid_max = 0;               // largest n_ent * T of an item, rounded up to 8
    int64_t n_feasible = 0;            // area-feasible candidates
    int64_t tile_lookups = 0, records = 0, record_slices = 0;
    // device copy
    void *dblob = nullptr;
    size_t dbytes = 0;
    SpaceView view{};
};

// Validates the geometry/parameters that the space depends on.
trs_status check_space_args(const trs_frame *f, const trs_search_params *p);

// Ladder rule and |C| without building tables.
trs_status space_size(int W, int H, const trs_search_params *p, int64_t *n, int32_t *dt,
                      int32_t *dr);

// Builds the host tables (no device work).
trs_status build_plan(const trs_frame *f, const trs_search_params *p, Plan &plan);

// Host decode of a rank.
trs_status decode_rank(const Plan &plan, int64_t rank, trs_result *out);

}  // namespace trs
