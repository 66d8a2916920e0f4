// Internal launch interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "space.hpp"

namespace trs {

// Search workspace header (device), followed by the SATs and per-item arrays.
struct WsHeader {
    unsigned long long tmin;        // T~min (Eq. 3)
    unsigned long long bound;       // floor(T~min (den + num) / den), the Eq. 4 bound
    int n_live;                     // items whose step-1 minimum is within the bound
    int pad0;
    unsigned long long pad[5];
};

// One work item's step-2 winner (q = UINT64_MAX when it has none) and the number of
// candidates it scored in step 2 (0 when skipped).
struct Partial {
    unsigned long long q, t;
    long long rank;
    int32_t item, f, n, pad;
};

struct WsLayout {
    size_t header, satT, satS1, satS2, item_min, live, partial, total;
};

WsLayout ws_layout(const Plan &pl);

struct SearchArgs {
    SpaceView sp;
    const uint32_t *cost, *s1;
    const uint64_t *s2;
    char *ws;
    WsLayout lay;
    trs_result *out;
    int lam_num, lam_den;             // lam_num < 0: infinite
    int block;                        // work-group size of the search kernels
    int dt, dr;
    hipEvent_t ev[4];                 // optional timing events (all null when not profiling)
};

// ---- batched form: many frames of mixed sizes and parameters, one launch per stage ----

// Per-frame descriptor on the device.  o_* are byte offsets of the frame's arrays in the
// batch workspace.
struct BatchFrameDev {
    const uint16_t *luma;
    long long stride;
    const uint32_t *prev;
    uint32_t a, b, wp, pad0;
    int w, h, W, H;
    int plan, lam_num, lam_den, dt;
    int dr, ctu_base, item_base, n_items;
    int brief_base, pad1;             // first ItemBrief of this frame's plan
    long long o_s1, o_grad, o_tex, o_mean, o_var, o_s2, o_cost, o_hdr, o_satT, o_satS1, o_satS2;
};

// Frame-inner step-1 work unit: one item of one plan for a chunk of up to kChunk frames
// that share the plan.  It carries what the kernel needs of the item, so one load starts it.
constexpr int kChunk = 8;
struct UnitDev {
    const uint16_t *rids;             // the item's record indices [T][n_ent], 16-byte aligned
    const uint32_t *rdesc4;           // the item's compact record descriptors
    int n_ent, n_rec, T, S;           // S = W + 1, the SAT row length
    int item, chunk, pad0, pad1;
};
// What the batched step 2 needs of one item of one plan (one load per live entry).
struct ItemBrief {
    const uint16_t *rids;             // record indices [T][n_ent], 16-byte aligned
    const uint32_t *rdesc4;           // compact record descriptors
    const uint32_t *ent_f;            // candidates' local indices
    long long rank0, SM;              // rank = rank0 + (f / M) * SM + f % M
    int n_ent, n_rec, T, M;
};
// One frame slot of a chunk: its SAT of predicted times (byte offset in the workspace) and
// its first item in the flat item list (-1: empty slot, which reads the chunk's first frame).
struct ChunkSlot {
    long long o_sat;
    int item_base, pad;
};

struct BatchLaunch {
    const SpaceView *plans;           // device
    const BatchFrameDev *frames;      // device
    const int *ctu_frame, *item_frame;
    const UnitDev *units;             // device; null: step 1 runs per (frame, item)
    const ChunkSlot *slots;           // device, kChunk per chunk
    const ItemBrief *briefs;          // device, per (plan, item); null with units
    int n_frames, total_ctus, total_items, cs;
    int block, grid1, grid2, rec_max;
    int n_units, grid_u, rid_max, pad;
    long long o_item_min, o_part;     // byte offsets in the workspace
    long long o_live, o_live_n;       // step-2 list of live (frame << 32 | item) entries, its length
};

// Dynamic LDS of the frame-inner step-1 kernel, or 0 when the records and record indices
// of the largest item do not fit.
int unit_lds_bytes(int rec_max, int rid_max);
int unit_occupancy(int block, int rec_max, int rid_max);
// Dynamic LDS and occupancy of the batched step-2 kernel over the live list.
int step2_lds_bytes(int rec_max, int rid_max);
int step2_occupancy(int block, int rec_max, int rid_max);

// Byte layout of one frame's region and its size (W x H CTUs).
long long batch_frame_region(int W, int H, BatchFrameDev *fr, long long base);
int batch_lds_bytes(int rec_max, bool step2);
// Work-groups per CU the batched search kernels can keep resident.
int batch_occupancy(int block, int rec_max, bool step2);
// stages: the feature launch, the five launches after it (cost map to result), or both.
// ev (nullable, with both stages): 7 events recorded before the first launch and after each
// of the six.
constexpr int kStageFeatures = 1, kStageSearch = 2;
hipError_t launch_batch(const BatchLaunch &b, char *ws, trs_result *out, hipStream_t s,
                        const hipEvent_t *ev = nullptr, int stages = kStageFeatures | kStageSearch);

hipError_t launch_features(int w, int h, int cs, const uint16_t *luma, int64_t stride,
                           const trs_feat &out, hipStream_t s);
hipError_t launch_cost_map(int n, const uint32_t *tex, const uint32_t *prev, trs_blend b,
                           uint32_t *cost, uint32_t *flags, hipStream_t s);
hipError_t launch_search(const SearchArgs &a, hipStream_t s);
// Cost map (from tex, prev, blend) followed by the search, with the cost map fused into the
// prefix-sum kernel when the grid fits in LDS.
hipError_t launch_partition_tail(const SearchArgs &a, const uint32_t *tex, const uint32_t *prev,
                                 trs_blend b, uint32_t *cost, uint32_t *flags, hipStream_t s);

}  // namespace trs
