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
