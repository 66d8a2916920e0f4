// C ABI of libtrs.so (declarations and contracts in include/trs.h).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <array>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "mlp.hpp"
#include "space.hpp"
#include "trs.h"

namespace trs {
namespace lit {
void release_all();   // literal-space plans (literal.hip)
void profile_enable(bool on);
}
}  // namespace trs

namespace {

using trs::Plan;

struct PlanEntry {
    std::unique_ptr<Plan> plan;
    std::map<int, std::pair<void *, trs::SpaceView>> dev;   // per device: blob and view
};

using PlanKey = std::array<int64_t, 14>;

std::mutex g_mu;
std::map<PlanKey, PlanEntry> g_plans;
std::atomic<uint64_t> g_generation{1};      // bumped when plans are released

// Per-thread memo of the last plan used, so repeated searches skip the lock and the map.
struct FastPlan {
    uint64_t generation = 0;
    int device = -1;
    PlanKey key{};
    trs::SpaceView view{};
    trs::WsLayout lay{};
    int dt = 0, dr = 0;
};
thread_local FastPlan t_fast;

// Timing events recorded by trs_search while profiling is on (guarded by g_prof_mu).
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::array<hipEvent_t, 4>> g_prof_events;
// Batch-run events and the launch stages they cover (trs::kStageFeatures / kStageSearch).
std::vector<std::pair<std::array<hipEvent_t, 7>, int>> g_prof_batch;

PlanKey plan_key(const trs_frame *f, const trs_search_params *p)
{
    return {f->width, f->height, f->ctu_size, p->n_threads, p->max_tile_cols, p->max_tile_rows,
            p->max_rs_per_tile, p->dtile, p->drs, p->area_k,
            p->space_budget > 0 ? p->space_budget : (int64_t(1) << 24), p->sched_item, p->prune,
            p->min_rs > 0 ? p->min_rs : p->n_threads};
}

// Host tables for (f, p), built once.  Caller holds g_mu.
trs_status host_plan(const trs_frame *f, const trs_search_params *p, PlanEntry **out)
{
    auto key = plan_key(f, p);
    auto it = g_plans.find(key);
    if (it == g_plans.end()) {
        auto pl = std::make_unique<Plan>();
        trs_status st = trs::build_plan(f, p, *pl);
        if (st != TRS_OK) return st;
        it = g_plans.emplace(key, PlanEntry{std::move(pl), {}}).first;
    }
    *out = &it->second;
    return TRS_OK;
}

template <typename T>
size_t add_array(std::vector<std::tuple<const void *, size_t, size_t>> &parts, size_t &off,
                 const std::vector<T> &v)
{
    off = (off + 255) & ~size_t(255);
    size_t at = off;
    size_t bytes = v.size() * sizeof(T);
    parts.emplace_back(v.data(), bytes, at);
    off += bytes ? bytes : 1;
    return at;
}

// Device copy of the plan on the current device.  Caller holds g_mu.
trs_status device_view(PlanEntry &e, trs::SpaceView *view)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TRS_EDEVICE;
    auto it = e.dev.find(dev);
    if (it != e.dev.end()) {
        *view = it->second.second;
        return TRS_OK;
    }
    const Plan &pl = *e.plan;
    std::vector<std::tuple<const void *, size_t, size_t>> parts;
    size_t off = 0;
    size_t o_colpx = add_array(parts, off, pl.colpx);
    size_t o_rowpx = add_array(parts, off, pl.rowpx);
    size_t o_obase = add_array(parts, off, pl.opt_base);
    size_t o_okcnt = add_array(parts, off, pl.opt_kcnt);
    size_t o_ok = add_array(parts, off, pl.opt_k);
    size_t o_oz = add_array(parts, off, pl.opt_z);
    size_t o_shapes = add_array(parts, off, pl.shapes);
    size_t o_xtab = add_array(parts, off, pl.xtab);
    size_t o_ytab = add_array(parts, off, pl.ytab);
    size_t o_prefM = add_array(parts, off, pl.y_prefM);
    size_t o_ycombo = add_array(parts, off, pl.y_combo);
    size_t o_yM = add_array(parts, off, pl.y_M);
    size_t o_combos = add_array(parts, off, pl.combos);
    size_t o_items = add_array(parts, off, pl.items);
    size_t o_entf = add_array(parts, off, pl.ent_f);
    size_t o_entr = add_array(parts, off, pl.ent_rid);
    size_t o_rdesc = add_array(parts, off, pl.rdesc);
    size_t o_rdesc4 = add_array(parts, off, pl.rdesc4);
    size_t o_unif = add_array(parts, off, pl.unif_rs);
    const size_t bytes = (off + 255) & ~size_t(255);
    std::vector<char> host(bytes, 0);
    for (auto &pt : parts)
        if (std::get<1>(pt)) std::memcpy(host.data() + std::get<2>(pt), std::get<0>(pt), std::get<1>(pt));
    void *blob = nullptr;
    if (hipMalloc(&blob, bytes) != hipSuccess) return TRS_EDEVICE;
    if (hipMemcpy(blob, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(blob);
        return TRS_EDEVICE;
    }
    char *b = static_cast<char *>(blob);
    trs::SpaceView v{};
    v.colpx = reinterpret_cast<const int32_t *>(b + o_colpx);
    v.rowpx = reinterpret_cast<const int32_t *>(b + o_rowpx);
    v.opt_base = reinterpret_cast<const int32_t *>(b + o_obase);
    v.opt_kcnt = reinterpret_cast<const int32_t *>(b + o_okcnt);
    v.opt_k = reinterpret_cast<const uint8_t *>(b + o_ok);
    v.opt_z = reinterpret_cast<const uint16_t *>(b + o_oz);
    v.shapes = reinterpret_cast<const trs::ShapeDev *>(b + o_shapes);
    v.xtab = reinterpret_cast<const uint16_t *>(b + o_xtab);
    v.ytab = reinterpret_cast<const uint16_t *>(b + o_ytab);
    v.y_prefM = reinterpret_cast<const int64_t *>(b + o_prefM);
    v.y_combo = reinterpret_cast<const int64_t *>(b + o_ycombo);
    v.y_M = reinterpret_cast<const int32_t *>(b + o_yM);
    v.combos = reinterpret_cast<const uint16_t *>(b + o_combos);
    v.items = reinterpret_cast<const trs::ItemDev *>(b + o_items);
    v.ent_f = reinterpret_cast<const uint32_t *>(b + o_entf);
    v.ent_rid = reinterpret_cast<const uint16_t *>(b + o_entr);
    v.rdesc = reinterpret_cast<const uint32_t *>(b + o_rdesc);
    v.rdesc4 = reinterpret_cast<const uint32_t *>(b + o_rdesc4);
    v.compact = pl.compact;
    v.unif_rs = reinterpret_cast<const int32_t *>(b + o_unif);
    v.W = pl.W;
    v.H = pl.H;
    v.N = pl.N;
    v.Km = pl.Km;
    v.n_items = (int32_t)pl.items.size();
    v.n_shapes = (int32_t)pl.shapes.size();
    v.n_unif = pl.n_unif;
    v.rec_max = pl.rec_max;
    v.rid_max = pl.rid_max;
    v.n_feasible = pl.n_feasible;
    v.cu = pl.cu;
    v.ru = pl.ru;
    v.total = pl.total;
    v.uniform_rank = pl.uniform_rank;
    e.dev[dev] = {blob, v};
    *view = v;
    return TRS_OK;
}

bool frame_ok(const trs_frame *f)
{
    return f && f->width >= 1 && f->height >= 1 && f->width <= 8192 && f->height <= 8192 &&
           (f->ctu_size == 32 || f->ctu_size == 64 || f->ctu_size == 128) &&
           f->bit_depth >= 8 && f->bit_depth <= 12;
}

// Validation, plan lookup (building and uploading it on first use), workspace check and
// optional timing events for one search.
trs_status prepare_search(const trs_frame *frame, const trs_search_params *params,
                          void *workspace, size_t ws_bytes, trs::SearchArgs &a)
{
    trs_status st = trs::check_space_args(frame, params);
    if (st != TRS_OK) return st;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256) return TRS_EWORKSPACE;
    int dev = -1;
    const bool have_dev = hipGetDevice(&dev) == hipSuccess;
    const PlanKey key = plan_key(frame, params);
    FastPlan &fp = t_fast;
    if (!(have_dev && fp.generation == g_generation.load(std::memory_order_acquire) &&
          fp.device == dev && fp.key == key)) {
        std::lock_guard<std::mutex> lk(g_mu);
        PlanEntry *e = nullptr;
        st = host_plan(frame, params, &e);
        if (st != TRS_OK) return st;
        if (ws_bytes < trs::ws_layout(*e->plan).total) return TRS_EWORKSPACE;
        if (!have_dev) return TRS_EDEVICE;
        trs::SpaceView v{};
        st = device_view(*e, &v);
        if (st != TRS_OK) return st;
        fp.generation = g_generation.load(std::memory_order_acquire);
        fp.device = dev;
        fp.key = key;
        fp.view = v;
        fp.lay = trs::ws_layout(*e->plan);
        fp.dt = e->plan->dt;
        fp.dr = e->plan->dr;
    }
    if (ws_bytes < fp.lay.total) return TRS_EWORKSPACE;
    a.sp = fp.view;
    a.lay = fp.lay;
    a.dt = fp.dt;
    a.dr = fp.dr;
    a.ws = static_cast<char *>(workspace);
    a.lam_num = params->lambda_num < 0 ? -1 : params->lambda_num;
    a.lam_den = params->lambda_den;
    a.block = params->sched_block ? params->sched_block : 256;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof_on) {
        std::array<hipEvent_t, 4> ev{};
        for (auto &x : ev)
            if (hipEventCreate(&x) != hipSuccess) return TRS_EDEVICE;
        g_prof_events.push_back(ev);
        for (int i = 0; i < 4; i++) a.ev[i] = ev[i];
    }
    return TRS_OK;
}

}  // namespace

struct trs_batch_s {
    int device = -1;
    trs::BatchLaunch launch{};
    size_t ws_bytes = 0;
    void *blob = nullptr;
    std::vector<trs::BatchFrameDev> frames;
};

namespace {

// The batch's launches for `stages`, with profiling events when enabled.
trs_status batch_launch(trs_batch batch, void *workspace, size_t ws_bytes, trs_result *out_dev,
                        hipStream_t stream, int stages)
{
    if (!batch) return TRS_EINVAL;
    if (!workspace || ws_bytes < batch->ws_bytes || reinterpret_cast<uintptr_t>(workspace) % 256)
        return TRS_EWORKSPACE;
    std::array<hipEvent_t, 7> ev{};
    bool prof = false;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (g_prof_on) {
            for (auto &x : ev)
                if (hipEventCreate(&x) != hipSuccess) return TRS_EDEVICE;
            g_prof_batch.emplace_back(ev, stages);
            prof = true;
        }
    }
    return trs::launch_batch(batch->launch, static_cast<char *>(workspace), out_dev, stream,
                             prof ? ev.data() : nullptr, stages) == hipSuccess
               ? TRS_OK
               : TRS_EDEVICE;
}

}  // namespace

extern "C" {

trs_status trs_features(const trs_frame *frame, const uint16_t *luma, int64_t stride_elems,
                        trs_feat out, hipStream_t stream)
{
    if (!frame_ok(frame) || !luma) return TRS_EINVAL;
    if (stride_elems < frame->width || stride_elems % 8 != 0) return TRS_EINVAL;
    if (reinterpret_cast<uintptr_t>(luma) % 16 != 0) return TRS_EINVAL;
    if (!out.s1 || !out.s2 || !out.grad || !out.tex || !out.mean || !out.var) return TRS_EINVAL;
    hipError_t e = trs::launch_features(frame->width, frame->height, frame->ctu_size, luma,
                                        stride_elems, out, stream);
    return e == hipSuccess ? TRS_OK : TRS_EDEVICE;
}

trs_status trs_cost_map(const trs_frame *frame, const uint32_t *tex, const uint32_t *prev,
                        trs_blend blend, uint32_t *cost, uint32_t *flags_dev, hipStream_t stream)
{
    if (!frame_ok(frame) || !tex || !cost || blend.w_prev > 256) return TRS_EINVAL;
    const int cs = frame->ctu_size;
    const int n = ((frame->width + cs - 1) / cs) * ((frame->height + cs - 1) / cs);
    hipError_t e = trs::launch_cost_map(n, tex, prev, blend, cost, flags_dev, stream);
    return e == hipSuccess ? TRS_OK : TRS_EDEVICE;
}

trs_status trs_lambda_policy(const trs_frame *frame, int32_t n_threads, int32_t *lambda_num,
                             int32_t *lambda_den)
{
    if (!frame_ok(frame) || n_threads < 1 || !lambda_num || !lambda_den) return TRS_EINVAL;
    static const int32_t kNum[2][3] = {{0, 3, 1}, {0, 1, 1}};      // Table 1: [FHD, UHD][n = 4, 8, 12]
    const int col = frame->height <= 1080 ? 0 : 1;
    const int row = n_threads <= 5 ? 0 : n_threads <= 9 ? 1 : 2;
    *lambda_num = kNum[col][row];
    *lambda_den = 10;
    return TRS_OK;
}

trs_status trs_space_size(const trs_frame *frame, const trs_search_params *params, int64_t *n,
                          int32_t *dtile, int32_t *drs)
{
    if (!n || !dtile || !drs) return TRS_EINVAL;
    trs_status st = trs::check_space_args(frame, params);
    if (st != TRS_OK) return st;
    const int cs = frame->ctu_size;
    return trs::space_size((frame->width + cs - 1) / cs, (frame->height + cs - 1) / cs, params,
                           n, dtile, drs);
}

trs_status trs_search_workspace(const trs_frame *frame, const trs_search_params *params,
                                size_t *bytes)
{
    if (!bytes) return TRS_EINVAL;
    trs_status st = trs::check_space_args(frame, params);
    if (st != TRS_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    PlanEntry *e = nullptr;
    st = host_plan(frame, params, &e);
    if (st != TRS_OK) return st;
    *bytes = trs::ws_layout(*e->plan).total;
    return TRS_OK;
}

trs_status trs_search(const trs_frame *frame, const trs_search_params *params,
                      const uint32_t *cost, const uint32_t *s1, const uint64_t *s2,
                      void *workspace, size_t ws_bytes, trs_result *out_dev, hipStream_t stream)
{
    if (!cost || !s1 || !s2 || !out_dev) {
        trs_status st = trs::check_space_args(frame, params);
        return st != TRS_OK ? st : TRS_EINVAL;
    }
    trs::SearchArgs a{};
    trs_status st = prepare_search(frame, params, workspace, ws_bytes, a);
    if (st != TRS_OK) return st;
    a.cost = cost;
    a.s1 = s1;
    a.s2 = s2;
    a.out = out_dev;
    if (trs::launch_search(a, stream) != hipSuccess) return TRS_EDEVICE;
    return a.sp.n_feasible == 0 ? TRS_ENOFEASIBLE : TRS_OK;
}

trs_status trs_partition(const trs_frame *frame, const trs_search_params *params,
                         const uint16_t *luma, int64_t stride_elems, const uint32_t *prev,
                         trs_blend blend, trs_feat feat, uint32_t *cost, uint32_t *flags_dev,
                         void *workspace, size_t ws_bytes, trs_result *out_dev,
                         hipStream_t stream)
{
    trs_status st = trs::check_space_args(frame, params);
    if (st != TRS_OK) return st;
    if (!luma || stride_elems < frame->width || stride_elems % 8 != 0 ||
        reinterpret_cast<uintptr_t>(luma) % 16 != 0)
        return TRS_EINVAL;
    if (!feat.s1 || !feat.s2 || !feat.grad || !feat.tex || !feat.mean || !feat.var || !cost ||
        !out_dev || blend.w_prev > 256)
        return TRS_EINVAL;
    trs::SearchArgs a{};
    st = prepare_search(frame, params, workspace, ws_bytes, a);
    if (st != TRS_OK) return st;
    a.cost = cost;
    a.s1 = feat.s1;
    a.s2 = feat.s2;
    a.out = out_dev;
    if (trs::launch_features(frame->width, frame->height, frame->ctu_size, luma, stride_elems, feat,
                             stream) != hipSuccess)
        return TRS_EDEVICE;
    if (trs::launch_partition_tail(a, feat.tex, prev, blend, cost, flags_dev, stream) != hipSuccess)
        return TRS_EDEVICE;
    return a.sp.n_feasible == 0 ? TRS_ENOFEASIBLE : TRS_OK;
}

void trs_profile_enable(int on)
{
    trs::lit::profile_enable(on != 0);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
}

trs_status trs_profile_read(double *ms_step1, double *ms_step2, int64_t *searches)
{
    if (!ms_step1 || !ms_step2 || !searches) return TRS_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double a = 0, b = 0;
    trs_status st = TRS_OK;
    for (auto &ev : g_prof_events) {
        float x = 0, y = 0;
        if (hipEventSynchronize(ev[3]) != hipSuccess || hipEventElapsedTime(&x, ev[0], ev[1]) != hipSuccess ||
            hipEventElapsedTime(&y, ev[2], ev[3]) != hipSuccess)
            st = TRS_EDEVICE;
        a += x;
        b += y;
    }
    *ms_step1 = a;
    *ms_step2 = b;
    *searches = (int64_t)g_prof_events.size();
    for (auto &ev : g_prof_events)
        for (auto &x : ev) (void)hipEventDestroy(x);
    g_prof_events.clear();
    return st;
}

trs_status trs_profile_read_batch(double *ms, int64_t *runs)
{
    if (!ms || !runs) return TRS_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    trs_status st = TRS_OK;
    int64_t n = 0;
    for (int k = 0; k < 6; k++) ms[k] = 0.0;
    for (auto &rec : g_prof_batch) {
        const auto &ev = rec.first;
        const bool feat = rec.second & trs::kStageFeatures, srch = rec.second & trs::kStageSearch;
        if (hipEventSynchronize(ev[srch ? 6 : 1]) != hipSuccess) st = TRS_EDEVICE;
        for (int k = feat ? 0 : 1; k < (srch ? 6 : 1); k++) {
            float x = 0;
            if (hipEventElapsedTime(&x, ev[k], ev[k + 1]) != hipSuccess) st = TRS_EDEVICE;
            ms[k] += x;
        }
        n += srch;
    }
    *runs = n;
    for (auto &rec : g_prof_batch)
        for (auto &x : rec.first) (void)hipEventDestroy(x);
    g_prof_batch.clear();
    return st;
}

trs_status trs_search_stats(const trs_frame *frame, const trs_search_params *params,
                            trs_plan_stats *out)
{
    if (!out) return TRS_EINVAL;
    trs_status st = trs::check_space_args(frame, params);
    if (st != TRS_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    PlanEntry *e = nullptr;
    st = host_plan(frame, params, &e);
    if (st != TRS_OK) return st;
    const Plan &pl = *e->plan;
    out->candidates = pl.total;
    out->tile_lookups = pl.tile_lookups;
    out->items = (int64_t)pl.items.size();
    out->records = pl.records;
    out->record_slices = pl.record_slices;
    out->table_bytes = (int64_t)(pl.combos.size() * 2 + pl.xtab.size() * 2 + pl.ytab.size() * 2 +
                                 pl.items.size() * sizeof(trs::ItemDev) + pl.ent_f.size() * 4 +
                                 pl.ent_rid.size() * 2 + pl.rdesc.size() * 4 + pl.rdesc4.size() * 4 +
                                 pl.opt_z.size() * 2);
    out->feasible = pl.n_feasible;
    out->dtile = pl.dt;
    out->drs = pl.dr;
    out->records_max = pl.rec_max;
    out->entries_max = pl.rid_max;
    return TRS_OK;
}

trs_status trs_decode(const trs_frame *frame, const trs_search_params *params, int64_t rank,
                      trs_result *out_host)
{
    if (!out_host) return TRS_EINVAL;
    trs_status st = trs::check_space_args(frame, params);
    if (st != TRS_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    PlanEntry *e = nullptr;
    st = host_plan(frame, params, &e);
    if (st != TRS_OK) return st;
    std::memset(out_host, 0, sizeof(*out_host));
    return trs::decode_rank(*e->plan, rank, out_host);
}

trs_status trs_batch_create(const trs_batch_frame *frames, int32_t n_frames, int32_t block,
                            int32_t wgs_per_cu, trs_batch *out)
{
    if (!frames || n_frames < 1 || !out || wgs_per_cu < 0) return TRS_EINVAL;
    if (block != 0 && block != 64 && block != 128 && block != 256 && block != 512) return TRS_EINVAL;
    const int cs = frames[0].frame.ctu_size;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TRS_EDEVICE;
    auto b = std::make_unique<trs_batch_s>();
    b->device = dev;
    std::vector<trs::SpaceView> views;
    std::vector<const PlanEntry *> plan_of_view;
    std::vector<int> ctu_frame, item_frame;
    long long off = 0;
    int rec_max = 0, rid_max = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (int f = 0; f < n_frames; f++) {
            const trs_batch_frame &bf = frames[f];
            trs_status st = trs::check_space_args(&bf.frame, &bf.params);
            if (st != TRS_OK) return st;
            if (bf.frame.ctu_size != cs || !bf.luma || bf.stride_elems < bf.frame.width ||
                bf.stride_elems % 8 != 0 || reinterpret_cast<uintptr_t>(bf.luma) % 16 != 0 ||
                bf.blend.w_prev > 256)
                return TRS_EINVAL;
            const int W = (bf.frame.width + cs - 1) / cs, H = (bf.frame.height + cs - 1) / cs;
            if ((W + 1) * (H + 1) > 2304) return TRS_ENOTIMPL;
            PlanEntry *e = nullptr;
            st = host_plan(&bf.frame, &bf.params, &e);
            if (st != TRS_OK) return st;
            trs::SpaceView v{};
            st = device_view(*e, &v);
            if (st != TRS_OK) return st;
            int pi = -1;
            for (size_t q = 0; q < plan_of_view.size(); q++)
                if (plan_of_view[q] == e) pi = (int)q;
            if (pi < 0) {
                pi = (int)views.size();
                views.push_back(v);
                plan_of_view.push_back(e);
            }
            rec_max = std::max(rec_max, v.rec_max);
            rid_max = std::max(rid_max, v.rid_max);
            trs::BatchFrameDev fd{};
            fd.luma = bf.luma;
            fd.stride = bf.stride_elems;
            fd.prev = bf.prev;
            fd.a = bf.blend.a;
            fd.b = bf.blend.b;
            fd.wp = bf.blend.w_prev;
            fd.w = bf.frame.width;
            fd.h = bf.frame.height;
            fd.W = W;
            fd.H = H;
            fd.plan = pi;
            fd.lam_num = bf.params.lambda_num < 0 ? -1 : bf.params.lambda_num;
            fd.lam_den = bf.params.lambda_den;
            fd.dt = e->plan->dt;
            fd.dr = e->plan->dr;
            fd.ctu_base = (int)ctu_frame.size();
            fd.item_base = (int)item_frame.size();
            fd.n_items = (int)e->plan->items.size();
            off = trs::batch_frame_region(W, H, &fd, off);
            ctu_frame.insert(ctu_frame.end(), (size_t)W * H, f);
            item_frame.insert(item_frame.end(), (size_t)fd.n_items, f);
            if (item_frame.size() > (size_t)INT32_MAX / 2) return TRS_ENOSPACE;
            b->frames.push_back(fd);
        }
    }
    const long long total_items = (long long)item_frame.size();
    auto up = [](long long v) { return (v + 255) & ~255ll; };
    b->launch.o_item_min = up(off);
    b->launch.o_part = b->launch.o_item_min + up(8 * total_items);
    b->launch.o_live = b->launch.o_part + up((long long)sizeof(trs::Partial) * total_items);
    b->launch.o_live_n = b->launch.o_live + up(8 * total_items);
    b->ws_bytes = (size_t)(b->launch.o_live_n + 256);
    // frame-inner step-1 units: frames grouped by plan into chunks of kChunk, units ordered
    // item-major so one work-group's range revisits an item's tables chunk after chunk
    std::vector<trs::UnitDev> units;
    std::vector<trs::ChunkSlot> slots;
    std::vector<trs::ItemBrief> briefs;
    bool use_units = trs::unit_lds_bytes(rec_max, rid_max) > 0;
    for (const trs::SpaceView &v : views) use_units = use_units && v.compact;
    if (use_units) {
        for (int p = 0; p < (int)views.size(); p++) {
            std::vector<int> fl;
            for (int f = 0; f < n_frames; f++)
                if (b->frames[f].plan == p) fl.push_back(f);
            const int c0 = (int)(slots.size() / trs::kChunk);
            const int nc = ((int)fl.size() + trs::kChunk - 1) / trs::kChunk;
            for (int c = 0; c < nc; c++)
                for (int j = 0; j < trs::kChunk; j++) {
                    const int q = c * trs::kChunk + j;
                    const bool in = q < (int)fl.size();
                    const trs::BatchFrameDev &fd = b->frames[in ? fl[q] : fl[c * trs::kChunk]];
                    slots.push_back(trs::ChunkSlot{fd.o_satT, in ? fd.item_base : -1, 0});
                }
            const trs::Plan &pl = *plan_of_view[p]->plan;
            const trs::SpaceView &v = views[p];
            const int bb = (int)briefs.size();
            for (int f : fl) b->frames[f].brief_base = bb;
            for (int i = 0; i < (int)pl.items.size(); i++) {
                const trs::ItemDev &it = pl.items[i];
                for (int c = 0; c < nc; c++)
                    units.push_back(trs::UnitDev{v.ent_rid + it.rid_off, v.rdesc4 + 4 * it.rec_off, it.n_ent,
                                                 it.n_rec, it.T, pl.W + 1, i, c0 + c, 0, 0});
                briefs.push_back(trs::ItemBrief{v.ent_rid + it.rid_off, v.rdesc4 + 4 * it.rec_off,
                                                v.ent_f + it.ent_off, it.rank0, it.SM, it.n_ent, it.n_rec,
                                                it.T, it.M});
            }
        }
        if (units.size() > (size_t)INT32_MAX / 2) return TRS_ENOSPACE;
    }
    // device copy of views, frames and the index lists
    std::vector<std::tuple<const void *, size_t, size_t>> parts;
    size_t boff = 0;
    size_t o_views = add_array(parts, boff, views);
    size_t o_frames = add_array(parts, boff, b->frames);
    size_t o_cf = add_array(parts, boff, ctu_frame);
    size_t o_if = add_array(parts, boff, item_frame);
    size_t o_units = add_array(parts, boff, units);
    size_t o_briefs = add_array(parts, boff, briefs);
    size_t o_slots = add_array(parts, boff, slots);
    const size_t bytes = (boff + 255) & ~size_t(255);
    std::vector<char> host(bytes, 0);
    for (auto &pt : parts)
        if (std::get<1>(pt)) std::memcpy(host.data() + std::get<2>(pt), std::get<0>(pt), std::get<1>(pt));
    if (hipMalloc(&b->blob, bytes) != hipSuccess) return TRS_EDEVICE;
    if (hipMemcpy(b->blob, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(b->blob);
        return TRS_EDEVICE;
    }
    char *bp = static_cast<char *>(b->blob);
    trs::BatchLaunch &L = b->launch;
    L.plans = reinterpret_cast<const trs::SpaceView *>(bp + o_views);
    L.frames = reinterpret_cast<const trs::BatchFrameDev *>(bp + o_frames);
    L.ctu_frame = reinterpret_cast<const int *>(bp + o_cf);
    L.item_frame = reinterpret_cast<const int *>(bp + o_if);
    L.units = use_units ? reinterpret_cast<const trs::UnitDev *>(bp + o_units) : nullptr;
    L.slots = use_units ? reinterpret_cast<const trs::ChunkSlot *>(bp + o_slots) : nullptr;
    L.briefs = use_units ? reinterpret_cast<const trs::ItemBrief *>(bp + o_briefs) : nullptr;
    L.n_units = (int)units.size();
    L.n_frames = n_frames;
    L.total_ctus = (int)ctu_frame.size();
    L.total_items = (int)total_items;
    L.cs = cs;
    L.block = block ? block : 256;
    L.rec_max = rec_max;
    L.rid_max = rid_max;
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
        n_cu = 256;
    const int occ1 = wgs_per_cu ? wgs_per_cu : trs::batch_occupancy(L.block, rec_max, false);
    const int occ2 = wgs_per_cu ? wgs_per_cu : trs::batch_occupancy(L.block, rec_max, true);
    L.grid1 = (int)std::max<long long>(1, std::min<long long>(total_items, (long long)n_cu * occ1));
    L.grid2 = (int)std::max<long long>(1, std::min<long long>(total_items, (long long)n_cu * occ2));
    if (use_units) {
        const int occ2u = wgs_per_cu ? wgs_per_cu : trs::step2_occupancy(L.block, rec_max, rid_max);
        L.grid2 = (int)std::max<long long>(1, std::min<long long>(total_items, (long long)n_cu * occ2u));
        const int occu = wgs_per_cu ? wgs_per_cu : trs::unit_occupancy(L.block, rec_max, rid_max);
        L.grid_u = (int)std::max<long long>(1, std::min<long long>(L.n_units, (long long)n_cu * occu));
    }
    *out = b.release();
    return TRS_OK;
}

trs_status trs_batch_workspace(trs_batch batch, size_t *bytes)
{
    if (!batch || !bytes) return TRS_EINVAL;
    *bytes = batch->ws_bytes;
    return TRS_OK;
}

trs_status trs_batch_run(trs_batch batch, void *workspace, size_t ws_bytes, trs_result *out_dev,
                         hipStream_t stream)
{
    if (!out_dev) return TRS_EINVAL;
    return batch_launch(batch, workspace, ws_bytes, out_dev, stream, trs::kStageFeatures | trs::kStageSearch);
}

trs_status trs_batch_features(trs_batch batch, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    return batch_launch(batch, workspace, ws_bytes, nullptr, stream, trs::kStageFeatures);
}

trs_status trs_batch_search(trs_batch batch, void *workspace, size_t ws_bytes, trs_result *out_dev,
                            hipStream_t stream)
{
    if (!out_dev) return TRS_EINVAL;
    return batch_launch(batch, workspace, ws_bytes, out_dev, stream, trs::kStageSearch);
}

trs_status trs_batch_frame_arrays(trs_batch batch, void *workspace, int32_t frame, trs_feat *feat,
                                  uint32_t **cost)
{
    if (!batch || !workspace || frame < 0 || frame >= (int32_t)batch->frames.size()) return TRS_EINVAL;
    char *ws = static_cast<char *>(workspace);
    const trs::BatchFrameDev &fd = batch->frames[frame];
    if (feat) {
        feat->s1 = reinterpret_cast<uint32_t *>(ws + fd.o_s1);
        feat->grad = reinterpret_cast<uint32_t *>(ws + fd.o_grad);
        feat->tex = reinterpret_cast<uint32_t *>(ws + fd.o_tex);
        feat->mean = reinterpret_cast<uint32_t *>(ws + fd.o_mean);
        feat->var = reinterpret_cast<uint32_t *>(ws + fd.o_var);
        feat->s2 = reinterpret_cast<uint64_t *>(ws + fd.o_s2);
    }
    if (cost) *cost = reinterpret_cast<uint32_t *>(ws + fd.o_cost);
    return TRS_OK;
}

void trs_batch_destroy(trs_batch batch)
{
    if (!batch) return;
    if (batch->blob) (void)hipFree(batch->blob);
    delete batch;
}

static bool mlp_ok(const trs_mlp *m)
{
    return m && m->w1 && m->b1 && m->w2 && m->b2 && m->w3 && m->b3;
}

trs_status trs_mlp_inputs(const trs_frame *frame, const uint32_t *tex, const uint32_t *var,
                          const uint32_t *mean, const uint32_t *prev, float *x, hipStream_t stream)
{
    if (!frame_ok(frame) || !tex || !var || !mean || !prev || !x) return TRS_EINVAL;
    const int cs = frame->ctu_size;
    const int W = (frame->width + cs - 1) / cs, H = (frame->height + cs - 1) / cs;
    return trs::launch_mlp_inputs(W, H, cs, frame->width, frame->height, tex, var, mean, prev, x,
                                  stream) == hipSuccess ? TRS_OK : TRS_EDEVICE;
}

trs_status trs_mlp_forward(const trs_mlp *mlp, const trs_mlp_norm *norm, const float *x,
                           int64_t n, float *y, float *z1, float *z2, hipStream_t stream)
{
    if (!mlp_ok(mlp) || !norm || !x || !y || n < 1 || n > (int64_t(1) << 31) || (!z1) != (!z2))
        return TRS_EINVAL;
    return trs::launch_mlp_forward(*mlp, *norm, x, n, y, z1, z2, stream) == hipSuccess ? TRS_OK
                                                                                       : TRS_EDEVICE;
}

trs_status trs_mlp_backward_workspace(int64_t n, size_t *bytes)
{
    if (!bytes || n < 1 || n > (int64_t(1) << 31)) return TRS_EINVAL;
    *bytes = trs::mlp_backward_workspace(n);
    return TRS_OK;
}

trs_status trs_mlp_backward(const trs_mlp *mlp, const trs_mlp_norm *norm, const float *x,
                            const float *z1, const float *z2, const float *dy, int64_t n,
                            trs_mlp_grads grads, void *workspace, size_t ws_bytes,
                            hipStream_t stream)
{
    if (!mlp_ok(mlp) || !norm || !x || !z1 || !z2 || !dy || n < 1 || n > (int64_t(1) << 31))
        return TRS_EINVAL;
    if (!grads.w1 || !grads.b1 || !grads.w2 || !grads.b2 || !grads.w3 || !grads.b3) return TRS_EINVAL;
    if (!workspace || ws_bytes < trs::mlp_backward_workspace(n) ||
        reinterpret_cast<uintptr_t>(workspace) % 256)
        return TRS_EWORKSPACE;
    return trs::launch_mlp_backward(*mlp, *norm, x, z1, z2, dy, n, grads,
                                    static_cast<char *>(workspace), stream) == hipSuccess
               ? TRS_OK
               : TRS_EDEVICE;
}

trs_status trs_mlp_cost(const trs_frame *frame, const float *y, const float *x,
                        const trs_mlp_norm *norm, const uint32_t *tex, const uint32_t *prev,
                        trs_blend blend, uint32_t *cost, uint32_t *n_fallback_dev,
                        hipStream_t stream)
{
    if (!frame_ok(frame) || !y || !x || !norm || !tex || !cost || blend.w_prev > 256) return TRS_EINVAL;
    const int cs = frame->ctu_size;
    const long long n = (long long)((frame->width + cs - 1) / cs) * ((frame->height + cs - 1) / cs);
    return trs::launch_mlp_cost(n, y, x, *norm, tex, prev, blend, cost, n_fallback_dev, stream) ==
                   hipSuccess
               ? TRS_OK
               : TRS_EDEVICE;
}

void trs_release_plans(void)
{
    trs::lit::release_all();
    std::lock_guard<std::mutex> lk(g_mu);
    g_generation.fetch_add(1, std::memory_order_acq_rel);
    for (auto &kv : g_plans)
        for (auto &d : kv.second.dev) (void)hipFree(d.second.first);
    g_plans.clear();
}

const char *trs_strerror(trs_status s)
{
    switch (s) {
    case TRS_OK: return "ok";
    case TRS_ENOFEASIBLE: return "no area-feasible partition; uniform partition returned";
    case TRS_EINVAL: return "invalid argument";
    case TRS_ERANGE: return "value out of range";
    case TRS_ENOSPACE: return "candidate space empty or beyond table limits";
    case TRS_EWORKSPACE: return "workspace missing, misaligned or too small";
    case TRS_EDEVICE: return "HIP runtime error";
    case TRS_ENOTIMPL: return "not implemented";
    }
    return "unknown status";
}

}  // extern "C"
