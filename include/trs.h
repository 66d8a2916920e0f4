/*
 * trs.h -- C ABI of the MI355X (gfx950) dynamic tile + rectangular-slice (TRS) frame
 * partitioning library (libtrs.so).
 *
 * Method: Amestoy, Hamidouche, Bergeron, Menard, "Quality-driven Dynamic VVC Frame
 * Partitioning for efficient Parallel Processing", ICIP 2020.  Before a frame is encoded
 * by N threads, one rectangular slice (RS) per thread, the frame is cut into a tile grid and
 * each tile into runs of whole CTU rows (Section 1).  Step 1 finds the smallest predicted
 * parallel time T~min (Eq. 1, Eq. 3) from per-CTU time predictions; step 2 picks, among
 * partitions with T~(P) <= T~min (1 + lambda) (Eq. 4), the one with the least within-RS luma
 * squared error (Eq. 2).  Only partitions with k A_min(P) > A_max(P) are searched
 * (Section 2.3, k = 3).
 *
 * Conventions shared by every entry point
 *   - Pointers named *_dev (and every array argument of the launch calls) are device
 *     pointers owned by the caller; the library never frees them.  Host pointers are marked.
 *   - Launch calls are asynchronous on the given HIP stream: they validate their scalar
 *     arguments on the host, enqueue kernels and return.  A negative status means nothing
 *     was enqueued and no output was written.  Data-dependent outcomes (no feasible
 *     partition, cost overflow) are reported in device memory (trs_result.status, the cost
 *     flag word) once the stream reaches them.
 *   - Per-CTU arrays are in raster order (row of CTUs after row), W = ceil(width / ctu),
 *     H = ceil(height / ctu); right and bottom CTUs may be partial.
 *   - The first search on a given (frame geometry, search parameters) pair builds the
 *     candidate-space tables on the host and uploads them to the current device
 *     (synchronous, allocated once and kept until trs_release_plans() or process exit).
 *     Later calls with the same pair only enqueue kernels.
 *   - Thread safety: calls may come from several host threads; plan construction is
 *     serialised internally.  Two searches that share one workspace must be ordered by the
 *     caller (same stream or events).
 */
#ifndef TRS_H
#define TRS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum trs_status {
    TRS_OK = 0,
    TRS_ENOFEASIBLE = 1,   /* warning: no area-feasible partition; the uniform one is returned */
    TRS_EINVAL = -1,       /* invalid argument */
    TRS_ERANGE = -2,       /* overflow guard tripped */
    TRS_ENOSPACE = -3,     /* candidate space empty, above 2^40, or beyond table limits */
    TRS_EWORKSPACE = -4,   /* workspace missing or smaller than trs_search_workspace() */
    TRS_EDEVICE = -5,      /* a HIP runtime call failed */
    TRS_ENOTIMPL = -6
} trs_status;

/* Frame geometry.  width, height in [1, 8192]; ctu_size in {32, 64, 128} (VVC uses 128);
 * bit_depth in [8, 12].  Sample values above 2^bit_depth - 1 are the caller's contract. */
typedef struct trs_frame {
    int32_t width, height, ctu_size, bit_depth;
} trs_frame;

/* Per-CTU features, device arrays of W*H entries (Section 2.2 needs the RS luma sums S1, S2
 * that Eq. 2 expands to; tex/mean/var describe the texture for time models).
 *   s1   = sum of samples, s2 = sum of squared samples, grad = G, the sum over samples
 *          (x, y) of the CTU of |p(x+1,y) - p(x,y)| + |p(x,y+1) - p(x,y)|, each term taken
 *          only when the neighbour lies inside the frame (it may lie in the next CTU);
 *   tex  = floor(G / n), mean = floor(s1 / n), var = floor((n s2 - s1^2) / n^2),
 *          with n the CTU's sample count. */
typedef struct trs_feat {
    uint32_t *s1, *grad, *tex, *mean, *var;
    uint64_t *s2;
} trs_feat;

/* Time-map blend (Section 2.1: the predicted time of a CTU is the measured time of the
 * co-located CTU in the previous frame of the same temporal layer, w_prev = 256).
 * cost = floor((w_prev prev + (256 - w_prev) (a + b tex) + 128) / 256) when prev is given,
 * a + b tex otherwise.  w_prev in [0, 256]. */
typedef struct trs_blend {
    uint32_t a, b, w_prev;
} trs_blend;

/* Search parameters.
 *   n_threads       N, the number of RS (= encoding threads), 1..64;
 *   max_tile_cols/rows, max_rs_per_tile: bounds Cmax, Rmax, Kmax of the candidate space;
 *   area_k          k of the balance rule k A_min > A_max (Section 2.3); 0 disables it;
 *   lambda_num/den  lambda = num / den of Eq. 4, 0 <= num <= 65535, 1 <= den <= 65535;
 *                   num < 0 means lambda = infinity (pure Eq. 2 clustering);
 *   dtile, drs      window (in CTUs) of tile boundaries around the uniform positions and of
 *                   RS split offsets inside a tile; -1 = unbounded; both -2 = ladder rule:
 *                   the first of (inf,inf), (3,1), (2,1), (1,1), (1,0), (0,0) whose space
 *                   holds at most space_budget candidates (else (0,0));
 *   space_budget    ladder budget, <= 0 means 2^24;
 *   sched_block     work-group size for the search kernels (64, 128, 256, 512; 0 = 256);
 *   sched_item      target area-feasible candidates per work item (0 = 512).  The schedule
 *                   changes speed only, never the result;
 *   prune           extra geometric rules, off by default (0), from the authors' pruning notes
 *                   left as comments in the paper's source: bit 0 (TRS_PRUNE_HEIGHTS) drops a
 *                   candidate with a tile whose largest slice height (pixels) exceeds twice its
 *                   smallest; bit 1 (TRS_PRUNE_MEANS) drops a candidate with a tile whose mean
 *                   slice area is above 1.5 times, or below 1/1.5 of, the mean area of the other
 *                   tiles' slices.  Like the area rule, they apply in both steps;
 *   min_rs          smallest RS count of a candidate, 0..N; 0 (default) means N.  With
 *                   min_rs < N the space holds partitions into n RS for every n in
 *                   [min_rs, N], leaving N - n threads idle (Section 1 cites work in which
 *                   fewer tiles than cores lower the coding loss); T~(P) is still the slowest
 *                   RS (Eq. 1).  A shape (c, r) is valid when c r <= N and min_rs <= Kmax c r;
 *                   the canonical order is unchanged, over tile choices whose k sum to any n
 *                   in [min_rs, N];
 *   span_tiles      1: besides runs of CTU rows inside one tile, an RS may be a block of two or
 *                   more complete tiles stacked in one tile column (Section 2.3 allows an RS of
 *                   several complete tiles forming a rectangle; blocks across tile columns are
 *                   not covered).  Only trs_literal_search takes it (TRS_ENOTIMPL elsewhere);
 *                   0 (default) keeps every RS inside one tile. */
#define TRS_PRUNE_HEIGHTS 1
#define TRS_PRUNE_MEANS 2
typedef struct trs_search_params {
    int32_t n_threads, max_tile_cols, max_tile_rows, max_rs_per_tile;
    int32_t area_k, lambda_num, lambda_den;
    int32_t dtile, drs;
    int32_t sched_block, sched_item;
    int32_t prune;
    int32_t min_rs;
    int32_t span_tiles;
    int64_t space_budget;
} trs_search_params;

#define TRS_MAX_RS 64

/* Result of one search (written to device memory by trs_search).
 *   rank          canonical rank of the chosen partition (order: tile-grid shape (c, r)
 *                 ascending, column boundaries X, row boundaries Y lexicographic, then the
 *                 per-tile (k, split offsets) choices with the first tile in raster order
 *                 most significant); -1 if the fallback uniform grid is outside the space;
 *   t_min         T~min of Eq. 3 (-1 when nothing is feasible);
 *   t_sel, q_sel  T~(P) (Eq. 1) and Q(P) = sum over RS of S2 - floor(S1^2 / n) (Eq. 2 in
 *                 exact integers) of the chosen partition; ties in Q are broken by smaller
 *                 T~(P), then by smaller rank;
 *   n_enumerated  |C|; n_feasible: candidates passing the area rule;
 *   n_step2       candidates scored in step 2: a work item whose step-1 minimum already
 *                 exceeds the Eq. 4 bound cannot hold a step-2 candidate and is skipped
 *                 (a work count: it depends on the schedule, unlike every other field);
 *   uniform_rank, t_unif, q_unif: rank and scores of the uniform c_u x r_u grid
 *                 (c_u r_u = N, most square, c_u >= r_u, one RS per tile);
 *   status        TRS_OK or TRS_ENOFEASIBLE;
 *   col_bd/row_bd tile boundaries in CTUs (tile_cols + 1 and tile_rows + 1 entries);
 *   rs[i]         RS rectangles {x0, y0, x1, y1} in CTUs (half open), tiles in raster
 *                 order, top to bottom inside a tile; rs_time[i] its predicted time.
 * Every byte is written: entries past tile_cols + 1, tile_rows + 1 and n_rs are zero. */
typedef struct trs_result {
    int64_t rank, t_min, t_sel, q_sel, n_enumerated, n_feasible, n_step2, uniform_rank, t_unif,
            q_unif;
    int32_t status, tile_cols, tile_rows, n_rs, dtile_used, drs_used;
    int32_t col_bd[TRS_MAX_RS + 1], row_bd[TRS_MAX_RS + 1];
    int32_t rs[TRS_MAX_RS][4];
    int64_t rs_time[TRS_MAX_RS];
} trs_result;

/* Per-CTU luma features (inputs of Eq. 2; Section 2.2).  luma: device, uint16 samples,
 * row r at luma + r * stride_elems; stride_elems >= width, a multiple of 8, and luma
 * 16-byte aligned.  out: device arrays of W*H entries each (all six required).
 * Errors: TRS_EINVAL (geometry, alignment, null), TRS_EDEVICE (launch failure). */
trs_status trs_features(const trs_frame *frame, const uint16_t *luma, int64_t stride_elems,
                        trs_feat out, hipStream_t stream);

/* Predicted per-CTU time map T~(c) (Section 2.1).  tex, prev, cost: device, W*H entries;
 * prev may be NULL (first frame: texture model only).  flags_dev: NULL or a device uint32
 * that the kernel ORs with 1 when a value exceeds 2^31 - 1 (the value is then clamped).
 * Errors: TRS_EINVAL, TRS_EDEVICE. */
trs_status trs_cost_map(const trs_frame *frame, const uint32_t *tex, const uint32_t *prev,
                        trs_blend blend, uint32_t *cost, uint32_t *flags_dev,
                        hipStream_t stream);

/* Host: workspace bytes trs_search needs for this geometry and parameters (builds the
 * candidate-space plan if it does not exist yet).  Errors: TRS_EINVAL, TRS_ENOSPACE. */
trs_status trs_search_workspace(const trs_frame *frame, const trs_search_params *params,
                                size_t *bytes);

/* The two-step search (Eq. 3, then Eq. 2 under Eq. 4, area rule of Section 2.3) over the
 * candidate space, exhaustive and exact.  cost: T~ per CTU (u32); s1, s2: per-CTU luma sums
 * from trs_features; workspace: device, at least trs_search_workspace() bytes, 256-byte
 * aligned, contents need not be initialised; out_dev: device trs_result.
 * Returns TRS_ENOFEASIBLE (a warning: the output, the uniform partition, is still written)
 * when no candidate of the space passes the area rule, which depends on the geometry only.
 * Errors: TRS_EINVAL, TRS_ENOSPACE, TRS_EWORKSPACE, TRS_EDEVICE. */
trs_status trs_search(const trs_frame *frame, const trs_search_params *params,
                      const uint32_t *cost, const uint32_t *s1, const uint64_t *s2,
                      void *workspace, size_t ws_bytes, trs_result *out_dev,
                      hipStream_t stream);

/* Exact two-step search over the literal space, in which every CTU boundary may be a tile
 * boundary and a split row (the space of Section 2.3 without windows: params->dtile and
 * params->drs must both be -1).  Same decision rule as trs_search (Eq. 3, then Eq. 2 under
 * Eq. 4, area rule of Section 2.3), solved without listing the candidates: the area rule is
 * split into windows [a, k a) over the possible smallest RS areas a, and inside a window the
 * least largest RS time and the least (Q, T~(P)) follow from dynamic programs over split rows,
 * tiles and column boundaries.  Among partitions with equal (Q, T~(P)) it returns the first in
 * the order (window, r, row boundaries, c) of that decomposition, not the smallest canonical
 * rank: rank, n_feasible and uniform_rank are -1, n_step2 is the number of (window, row
 * boundaries) units searched (those whose tile-row bands can hold N RS by area and slice
 * count), n_enumerated the size of the literal space; status in the result is
 * TRS_ENOFEASIBLE (uniform grid returned) when nothing passes the area rule.  Inputs as in
 * trs_search; workspace: device, at least trs_literal_workspace() bytes, 256-byte aligned.
 * With params->span_tiles = 1 an RS may also be a block of two or more complete tiles stacked
 * in one tile column (n_enumerated then counts that wider space).
 * Limits: W <= 64 and H <= 40 CTUs, N <= 32, at most 2^24 units, and the per-unit DP tables
 * within the 160 KB of LDS a gfx950 work-group may use (TRS_ENOTIMPL / TRS_ENOSPACE beyond);
 * prune must be 0 and min_rs 0 or N (TRS_ENOTIMPL).
 * Returns TRS_OK once enqueued.  Errors: TRS_EINVAL, TRS_ENOTIMPL, TRS_ENOSPACE,
 * TRS_EWORKSPACE, TRS_EDEVICE. */
trs_status trs_literal_workspace(const trs_frame *frame, const trs_search_params *params,
                                 size_t *bytes);
trs_status trs_literal_search(const trs_frame *frame, const trs_search_params *params,
                              const uint32_t *cost, const uint32_t *s1, const uint64_t *s2,
                              void *workspace, size_t ws_bytes, trs_result *out_dev,
                              hipStream_t stream);

/* Per-stage durations (ms, summed) of the trs_literal_search calls made while profiling was
 * on (trs_profile_enable), then forgets them: ms[0] prefix sums and rectangle values, ms[1]
 * step-1 tile tables, ms[2] step-1 units, ms[3] step-2 tile tables, ms[4] step-2 units,
 * ms[5] unit reduction, ms[6] rebuild and result; *runs = number of searches; relax[0] and
 * relax[1] = DP relaxations (pair combinations, counted from the loop bounds) of the units that
 * step 1 and step 2 ran, the units skipped by a bound left out.  Each profiled search holds 16
 * bytes of device memory until this call.  Waits for the last recorded event.
 * Errors: TRS_EINVAL, TRS_EDEVICE. */
trs_status trs_profile_read_literal(double *ms, int64_t *runs, int64_t *relax);

/* The whole per-frame path in one call (Fig. 3 of the paper: current-frame luma and the
 * co-located previous times in, partition out): trs_features, trs_cost_map and trs_search
 * enqueued on one stream, with the cost map fused into the prefix-sum kernel when the CTU
 * grid is small.  Arguments as in those three calls; feat and cost are written as they
 * would be.  Returns as trs_search. */
trs_status trs_partition(const trs_frame *frame, const trs_search_params *params,
                         const uint16_t *luma, int64_t stride_elems, const uint32_t *prev,
                         trs_blend blend, trs_feat feat, uint32_t *cost, uint32_t *flags_dev,
                         void *workspace, size_t ws_bytes, trs_result *out_dev,
                         hipStream_t stream);

/* ---- Batched form: many frames, each with its own geometry and parameters ----
 * One description per frame: geometry, search parameters, its luma (device, layout as in
 * trs_features), its previous-frame CTU times (device, nullable) and blend. */
typedef struct trs_batch_frame {
    trs_frame frame;
    trs_search_params params;
    const uint16_t *luma;
    int64_t stride_elems;
    const uint32_t *prev;
    trs_blend blend;
} trs_batch_frame;

typedef struct trs_batch_s *trs_batch;

/* Host: build (or reuse) each frame's candidate-space plan and upload the batch's frame
 * descriptors and work list to the current device (allocates; synchronous).  The luma and
 * prev pointers are recorded: trs_batch_run reads them as they are when it runs.  All frames
 * share one ctu_size, and each frame's CTU grid must satisfy (W + 1) (H + 1) <= 2304.
 * block: work-group size of the search kernels (0 = 256); wgs_per_cu: resident work-groups
 * per CU of the persistent search kernels (0 = as many as fit).
 * Errors: TRS_EINVAL, TRS_ENOSPACE, TRS_ENOTIMPL (grid too large), TRS_EDEVICE. */
trs_status trs_batch_create(const trs_batch_frame *frames, int32_t n_frames, int32_t block,
                            int32_t wgs_per_cu, trs_batch *out);

/* Host: workspace bytes trs_batch_run needs (256-byte aligned device memory). */
trs_status trs_batch_workspace(trs_batch batch, size_t *bytes);

/* The whole path for every frame of the batch (per-CTU features, time maps, prefix sums,
 * both search steps, decode), enqueued on `stream` as six launches for the whole batch, with
 * the two search steps as persistent kernels over all frames' work items.  Frame f's result
 * (as trs_search's) goes to out_dev[f].  Capturable in a HIP graph.
 * Errors: TRS_EINVAL, TRS_EWORKSPACE, TRS_EDEVICE. */
trs_status trs_batch_run(trs_batch batch, void *workspace, size_t ws_bytes, trs_result *out_dev,
                         hipStream_t stream);

/* trs_batch_run in two parts on the caller's streams: trs_batch_features enqueues the
 * per-CTU features of every frame into the workspace (one launch); trs_batch_search enqueues
 * the other five launches, which read them.  The caller orders the two (same stream, or an
 * event); between them the features kernel of one batch can overlap another batch's search.
 * Errors: as trs_batch_run. */
trs_status trs_batch_features(trs_batch batch, void *workspace, size_t ws_bytes, hipStream_t stream);
trs_status trs_batch_search(trs_batch batch, void *workspace, size_t ws_bytes, trs_result *out_dev,
                            hipStream_t stream);

/* Host: device pointers of frame `frame`'s per-CTU features and time map inside a batch
 * workspace (valid after trs_batch_run on that workspace).  Errors: TRS_EINVAL. */
trs_status trs_batch_frame_arrays(trs_batch batch, void *workspace, int32_t frame,
                                  trs_feat *feat, uint32_t **cost);

/* Host: free the batch's device tables (plans stay cached). */
void trs_batch_destroy(trs_batch batch);

/* ---- Learned per-CTU time predictor (stands in for the previous-frame estimator of
 * Section 2.1; the paper's conclusion names a better CTU time estimator as future work) ----
 * A 10 -> 64 -> 64 -> 1 perceptron with exact GELU (0.5 x (1 + erf(x / sqrt 2))), FP32.
 * Inputs per CTU (raw, before normalisation): texture, variance, mean; the textures of the
 * left, right, upper and lower neighbours (own value at the frame edge); the previous time;
 * the mean of the 4 neighbours' previous times (own value at the edge); n / ctu_size^2.
 * Output: the predicted time in milliseconds.  Weights are row-major [out][in], device. */
#define TRS_MLP_IN 10
#define TRS_MLP_HIDDEN 64

typedef struct trs_mlp {
    const float *w1, *b1, *w2, *b2, *w3, *b3;   /* [64][10], [64], [64][64], [64], [64], [1] */
} trs_mlp;

typedef struct trs_mlp_grads {
    float *w1, *b1, *w2, *b2, *w3, *b3;
} trs_mlp_grads;

/* Input normalisation x' = (x - mean) inv_std, and the training range [lo, hi] per input:
 * trs_mlp_cost falls back to the plain blend for a CTU with an input outside it. */
typedef struct trs_mlp_norm {
    float mean[TRS_MLP_IN], inv_std[TRS_MLP_IN], lo[TRS_MLP_IN], hi[TRS_MLP_IN];
} trs_mlp_norm;

/* Raw inputs x[c][10] for every CTU from trs_features outputs and the previous times
 * (device).  Errors: TRS_EINVAL, TRS_EDEVICE. */
trs_status trs_mlp_inputs(const trs_frame *frame, const uint32_t *tex, const uint32_t *var,
                          const uint32_t *mean, const uint32_t *prev, float *x,
                          hipStream_t stream);

/* y[s] for n samples x[s][10] (device); z1, z2 (device [64][n], nullable) keep the hidden
 * pre-activations for trs_mlp_backward.  Errors: TRS_EINVAL, TRS_EDEVICE. */
trs_status trs_mlp_forward(const trs_mlp *mlp, const trs_mlp_norm *norm, const float *x,
                           int64_t n, float *y, float *z1, float *z2, hipStream_t stream);

/* Host: workspace bytes trs_mlp_backward needs for n samples. */
trs_status trs_mlp_backward_workspace(int64_t n, size_t *bytes);

/* Gradients of sum_s dy[s] y[s] with respect to every weight and bias, written (not
 * accumulated) to grads; z1, z2 from trs_mlp_forward on the same x.  Summation order is
 * fixed, so results repeat exactly.  Errors: TRS_EINVAL, TRS_EWORKSPACE, TRS_EDEVICE. */
trs_status trs_mlp_backward(const trs_mlp *mlp, const trs_mlp_norm *norm, const float *x,
                            const float *z1, const float *z2, const float *dy, int64_t n,
                            trs_mlp_grads grads, void *workspace, size_t ws_bytes,
                            hipStream_t stream);

/* Time map from predictions: cost = rint(1000 y) clamped to [1, 2^31 - 1] where y is finite
 * and every input lies in [lo, hi]; elsewhere the plain blend of trs_cost_map (tex, prev,
 * blend), and *n_fallback_dev (nullable) counts those CTUs.  Errors: TRS_EINVAL, TRS_EDEVICE. */
trs_status trs_mlp_cost(const trs_frame *frame, const float *y, const float *x,
                        const trs_mlp_norm *norm, const uint32_t *tex, const uint32_t *prev,
                        trs_blend blend, uint32_t *cost, uint32_t *n_fallback_dev,
                        hipStream_t stream);

/* Host: the lambda of Eq. 4 that Table 1 pairs with the frame's resolution and thread count:
 * frames up to 1080 lines take the FHD column, taller ones the UHD column; n_threads takes the
 * nearest of the table's rows n = 4 (n <= 5), 8 (6 <= n <= 9) and 12 (n >= 10).  FHD: 0, 3/10,
 * 1/10; UHD: 0, 1/10, 1/10.  Writes lambda = num / den.  Errors: TRS_EINVAL. */
trs_status trs_lambda_policy(const trs_frame *frame, int32_t n_threads, int32_t *lambda_num,
                             int32_t *lambda_den);

/* Host: which earlier frame's CTU times predict each frame of a random-access sequence
 * (Section 2.1: in RA coding the co-located CTU of the previously coded frame of the same
 * temporal layer, the co-TL frame, predicts better than the closest frame in time).
 * gop_size G: a power of two, 1..256; frames 0 .. n_frames - 1 in display order, n_frames in
 * 1 .. 2^24.  Dyadic hierarchy: frame p is in temporal layer 0 when G divides p, else
 * log2(G) - (trailing zero bits of p).  Coding order: frame 0, then per GOP its last frame and,
 * depth first, the midpoint of each open interval before its left and then its right half;
 * frames past the end are skipped.  Outputs (host arrays of n_frames entries, caller-owned):
 * coding_order[i] = frame coded i-th; layer[p]; cotl_ref[p] = the frame of layer[p] coded
 * last before p, or -1; closest_ref[p] = the frame coded before p nearest to it in display
 * order (ties: the earlier one), or -1 for frame 0.  Errors: TRS_EINVAL. */
trs_status trs_ra_schedule(int32_t gop_size, int32_t n_frames, int32_t *coding_order,
                           int32_t *layer, int32_t *cotl_ref, int32_t *closest_ref);

/* Host: |C| and the windows (dtile, drs) the ladder rule picks.  No device work.
 * Errors: TRS_EINVAL. */
trs_status trs_space_size(const trs_frame *frame, const trs_search_params *params,
                          int64_t *n, int32_t *dtile, int32_t *drs);

/* Work done by one trs_search for this geometry and these parameters (host only; builds
 * the plan if needed).  candidates = |C|; feasible = candidates passing the area rule (the
 * rule depends only on the geometry, so the plan applies it once and each search scores
 * only these); tile_lookups = sum over feasible candidates of their tile count; items =
 * work items (one work-group each); records / record_slices = tile-option records built per
 * step and the slices they sum; records_max = largest record count of one item;
 * entries_max = largest (candidates x tiles) of one item, rounded up to 8; table_bytes =
 * size of the device tables.  Errors: as trs_search_workspace. */
typedef struct trs_plan_stats {
    int64_t candidates, feasible, tile_lookups, items, records, record_slices, table_bytes;
    int32_t dtile, drs, records_max, entries_max;
} trs_plan_stats;

trs_status trs_search_stats(const trs_frame *frame, const trs_search_params *params,
                            trs_plan_stats *out);

/* Host: decode a canonical rank into the tile grid and RS rectangles (out_host fields
 * rank, tile_cols, tile_rows, col_bd, row_bd, n_rs, rs, dtile_used, drs_used,
 * n_enumerated; times and scores are left 0).  Errors: TRS_EINVAL (rank out of range),
 * TRS_ENOSPACE. */
trs_status trs_decode(const trs_frame *frame, const trs_search_params *params, int64_t rank,
                      trs_result *out_host);

/* Kernel timing.  While enabled (on != 0), every trs_search records HIP events on its
 * stream around its step-1 kernel and around its step-2 kernel, and every trs_batch_run
 * records events between its six launches.  trs_profile_read waits for the recorded search
 * events, returns the summed milliseconds of the step-1 and step-2 kernels and the number of
 * searches timed, and clears that record.  trs_profile_read_batch does the same for batch
 * runs: ms[0..5] = features, cost map + prefix sums, step 1, T~min, step 2, result.  Enabling
 * is for eager (not graph-captured) launches.  Host only; returns TRS_EDEVICE if an event
 * call fails. */
void trs_profile_enable(int on);
trs_status trs_profile_read(double *ms_step1, double *ms_step2, int64_t *searches);
trs_status trs_profile_read_batch(double *ms, int64_t *runs);

/* Host: drop every cached candidate-space plan and free its device tables.  Batches created
 * before this call must be destroyed, not run, afterwards. */
void trs_release_plans(void);

/* Static description of a status code. */
const char *trs_strerror(trs_status status);

#ifdef __cplusplus
}
#endif

#endif /* TRS_H */
