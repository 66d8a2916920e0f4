// gfx950 kernels of the TRS partitioning path.
//
//   k_features  per-CTU luma statistics: one work-group per CTU, 16-byte row loads
//               (HBM-bound: every sample is read once; the 1-sample right halo and the
//               1-row bottom halo come from cache)
//   k_cost      per-CTU predicted time map (elementwise)
//   k_sat       inclusive 2D prefix sums of T~, S1, S2: wave-level scans along rows, then
//               along columns, one work-group
//   k_search    step 1 (P2 = false) and step 2 (P2 = true) over the candidate space: one
//               work item per work-group; tile-option records built in LDS, then one
//               candidate per lane, wave and work-group min-reductions
//   k_final     work-group reduction of the step-2 partials and decode of the winner
#include "kernels.hpp"

#include <climits>

namespace trs {
namespace {

constexpr int kWave = 64;
constexpr unsigned long long kNone = ~0ull;
constexpr unsigned long long kCostLimit = (1ull << 31) - 1;

__device__ __forceinline__ unsigned long long shfl_xor64(unsigned long long v, int m)
{
    unsigned lo = __shfl_xor((unsigned)v, m, kWave);
    unsigned hi = __shfl_xor((unsigned)(v >> 32), m, kWave);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ long long shfl_up64(long long v, int d)
{
    unsigned lo = __shfl_up((unsigned)(unsigned long long)v, d, kWave);
    unsigned hi = __shfl_up((unsigned)((unsigned long long)v >> 32), d, kWave);
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ long long shfl64(long long v, int src)
{
    unsigned lo = __shfl((unsigned)(unsigned long long)v, src, kWave);
    unsigned hi = __shfl((unsigned)((unsigned long long)v >> 32), src, kWave);
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ long long wave_incl_scan(long long v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        long long t = shfl_up64(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

// ---------------------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------------------

template <int CS>
__global__ void __launch_bounds__((CS / 8) * 16)
k_features(const uint16_t *__restrict__ luma, long long stride, int w, int h, int W,
           uint32_t *__restrict__ o_s1, unsigned long long *__restrict__ o_s2,
           uint32_t *__restrict__ o_g, uint32_t *__restrict__ o_tex,
           uint32_t *__restrict__ o_mean, uint32_t *__restrict__ o_var)
{
    constexpr int CH = CS / 8;           // 8-sample chunks per CTU row
    constexpr int NT = CH * 16;          // threads: CH chunks x 16 row groups
    constexpr int R = CS / 16;           // rows per row group
    const int cx = blockIdx.x, cy = blockIdx.y, tid = threadIdx.x;
    const int chunk = tid % CH, grp = tid / CH;
    const int x0 = cx * CS + chunk * 8;
    const int ybase = cy * CS + grp * R;
    uint32_t a1 = 0, a2 = 0, ag = 0;
    if (x0 < w && ybase < h) {
        const int nv = min(8, w - x0);
        const bool has_right = x0 + 8 < w;
        uint32_t prev[8];
#pragma unroll
        for (int r = 0; r <= R; r++) {
            const int y = ybase + r;
            if (y >= h) break;
            const uint16_t *row = luma + (long long)y * stride + x0;
            const uint4 v = *reinterpret_cast<const uint4 *>(row);
            uint32_t p[8] = {v.x & 0xffffu, v.x >> 16, v.y & 0xffffu, v.y >> 16,
                             v.z & 0xffffu, v.z >> 16, v.w & 0xffffu, v.w >> 16};
            if (r < R) {
                const uint32_t right = has_right ? (uint32_t)row[8] : 0u;
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    if (j < nv) {
                        a1 += p[j];
                        a2 += p[j] * p[j];
                        if (j + 1 < nv) ag += absdiff(p[j + 1], p[j]);
                        else if (j == 7 && has_right) ag += absdiff(right, p[7]);
                    }
                }
            }
            if (r >= 1) {
#pragma unroll
                for (int j = 0; j < 8; j++)
                    if (j < nv) ag += absdiff(p[j], prev[j]);
            }
#pragma unroll
            for (int j = 0; j < 8; j++) prev[j] = p[j];
        }
    }
    unsigned long long s2 = a2;
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) {
        a1 += __shfl_xor(a1, m, kWave);
        ag += __shfl_xor(ag, m, kWave);
        s2 += shfl_xor64(s2, m);
    }
    constexpr int NW = (NT + kWave - 1) / kWave;
    __shared__ uint32_t r1[NW], rg[NW];
    __shared__ unsigned long long r2[NW];
    const int lane = tid % kWave, wv = tid / kWave;
    if (lane == 0) { r1[wv] = a1; rg[wv] = ag; r2[wv] = s2; }
    __syncthreads();
    if (tid == 0) {
        uint32_t t1 = 0, tg = 0;
        unsigned long long t2 = 0;
        for (int i = 0; i < NW; i++) { t1 += r1[i]; tg += rg[i]; t2 += r2[i]; }
        const unsigned long long cw = min(CS, w - cx * CS), ch = min(CS, h - cy * CS);
        const unsigned long long n = cw * ch;
        const int c = cy * W + cx;
        o_s1[c] = t1;
        o_s2[c] = t2;
        o_g[c] = tg;
        o_tex[c] = (uint32_t)(tg / n);
        o_mean[c] = (uint32_t)(t1 / n);
        o_var[c] = (uint32_t)((n * t2 - (unsigned long long)t1 * t1) / (n * n));
    }
}

// ---------------------------------------------------------------------------------------
// Cost map
// ---------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_cost(int n, const uint32_t *__restrict__ tex, const uint32_t *__restrict__ prev, uint32_t a,
       uint32_t b, uint32_t wp, uint32_t *__restrict__ cost, uint32_t *flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // a + b tex <= (2^32 - 1) + (2^32 - 1)^2 < 2^64
    const unsigned long long model = (unsigned long long)a + (unsigned long long)b * tex[i];
    unsigned long long v;
    if (prev == nullptr) {
        v = model;
    } else if (wp == 256u) {
        v = prev[i];
    } else if (model >= (1ull << 40)) {
        v = kNone;                       // (256 - wp) model / 256 >= 2^32: out of range
    } else {
        v = ((unsigned long long)wp * prev[i] + (unsigned long long)(256u - wp) * model + 128ull) >> 8;
    }
    if (v > kCostLimit) {
        v = kCostLimit;
        if (flags) atomicOr(flags, 1u);
    }
    cost[i] = (uint32_t)v;
}

// ---------------------------------------------------------------------------------------
// Summed-area tables (int64, (H+1) x (W+1), zero first row and column)
// ---------------------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_sat(int W, int H, const uint32_t *__restrict__ cost, const uint32_t *__restrict__ s1,
      const unsigned long long *__restrict__ s2, long long *satT, long long *satS1,
      long long *satS2, WsHeader *hdr)
{
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, nw = blockDim.x / kWave;
    const int S = W + 1;
    if (tid == 0) {
        hdr->tmin = kNone;
        hdr->nfeas = 0;
        hdr->pruned = 0;
        hdr->step2 = 0;
    }
    for (int x = tid; x <= W; x += blockDim.x) satT[x] = satS1[x] = satS2[x] = 0;
    for (int y = wv; y < H; y += nw) {
        long long cT = 0, c1 = 0, c2 = 0;
        if (lane == 0) satT[(y + 1) * S] = satS1[(y + 1) * S] = satS2[(y + 1) * S] = 0;
        for (int xb = 0; xb < W; xb += kWave) {
            const int x = xb + lane;
            long long vT = x < W ? (long long)cost[y * W + x] : 0;
            long long v1 = x < W ? (long long)s1[y * W + x] : 0;
            long long v2 = x < W ? (long long)s2[y * W + x] : 0;
            vT = wave_incl_scan(vT, lane);
            v1 = wave_incl_scan(v1, lane);
            v2 = wave_incl_scan(v2, lane);
            if (x < W) {
                satT[(y + 1) * S + x + 1] = vT + cT;
                satS1[(y + 1) * S + x + 1] = v1 + c1;
                satS2[(y + 1) * S + x + 1] = v2 + c2;
            }
            cT += shfl64(vT, kWave - 1);
            c1 += shfl64(v1, kWave - 1);
            c2 += shfl64(v2, kWave - 1);
        }
    }
    __syncthreads();
    for (int x = 1 + wv; x <= W; x += nw) {
        long long cT = 0, c1 = 0, c2 = 0;
        for (int yb = 1; yb <= H; yb += kWave) {
            const int y = yb + lane;
            long long vT = y <= H ? satT[y * S + x] : 0;
            long long v1 = y <= H ? satS1[y * S + x] : 0;
            long long v2 = y <= H ? satS2[y * S + x] : 0;
            vT = wave_incl_scan(vT, lane);
            v1 = wave_incl_scan(v1, lane);
            v2 = wave_incl_scan(v2, lane);
            if (y <= H) {
                satT[y * S + x] = vT + cT;
                satS1[y * S + x] = v1 + c1;
                satS2[y * S + x] = v2 + c2;
            }
            cT += shfl64(vT, kWave - 1);
            c1 += shfl64(v1, kWave - 1);
            c2 += shfl64(v2, kWave - 1);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Search
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ long long rect(const long long *__restrict__ sat, int S, int x0, int y0,
                                          int x1, int y1)
{
    return sat[y1 * S + x1] - sat[y0 * S + x1] - sat[y1 * S + x0] + sat[y0 * S + x0];
}

// floor(s1^2 / n) for 0 <= s1 < 2^38 and 1 <= n < 2^27.  The quotient is at most the
// region's sum of squares (< 2^50), so a double estimate is within one unit; the exact
// remainder in wrapping 64-bit arithmetic corrects it.
__device__ __forceinline__ unsigned long long floor_sq_div(unsigned long long s1, unsigned n)
{
    const double d = (double)s1;
    unsigned long long q = (unsigned long long)((d * d) / (double)n);
    long long rem = (long long)(s1 * s1 - q * (unsigned long long)n);
    while (rem < 0) { q--; rem += n; }
    while (rem >= (long long)n) { q++; rem -= n; }
    return q;
}

__device__ __forceinline__ int kcnt(const SpaceView &sp, int h, int kk)
{
    return sp.opt_kcnt[h * (sp.Km + 1) + min(kk, sp.Km)];
}

// Work-group index -> item: consecutive items (which share combination tables and spans)
// go to the same XCD, whose L2 then serves them.  Work-groups are dispatched to the 8 XCDs
// round-robin.
__device__ __forceinline__ int xcd_item(int b, int G)
{
    const int xcd = b & 7, local = b >> 3, q = G >> 3, rm = G & 7;
    return xcd * q + min(xcd, rm) + local;
}

struct Key2 {
    unsigned long long q, t;
    long long rank;
    int f;
};

__device__ __forceinline__ bool key_less(const Key2 &a, const Key2 &b)
{
    if (a.q != b.q) return a.q < b.q;
    if (a.t != b.t) return a.t < b.t;
    return a.rank < b.rank;
}

template <int BS, bool P2>
__global__ void __launch_bounds__(BS)
k_search(SpaceView sp, const long long *__restrict__ satT, const long long *__restrict__ satS1,
         const long long *__restrict__ satS2, WsHeader *hdr,
         unsigned long long *__restrict__ item_min, Partial *__restrict__ part, int area_k,
         int lam_num, int lam_den)
{
    __shared__ unsigned long long recT[kRecCap];
    __shared__ unsigned long long recA[kRecCap];           // A_min | A_max << 32
    __shared__ unsigned long long recQ[P2 ? kRecCap : 1];
    __shared__ uint8_t smap[kMapCap];
    __shared__ int srowoff[kMaxRS + 1];
    __shared__ int sY[kMaxRS + 1];
    constexpr int NW = BS / kWave;
    __shared__ unsigned long long redq[NW], redt[NW];
    __shared__ long long redr[NW];
    __shared__ int redf[NW];

    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const ItemDev it = sp.items[item];
    const ShapeDev sd = sp.shapes[it.shape];

    unsigned long long bound = kNone;
    if (P2) {
        const unsigned long long tmin = hdr->tmin;
        if (lam_num >= 0)
            bound = tmin * (unsigned long long)(lam_den + lam_num) / (unsigned long long)lam_den;
        const unsigned long long imin = item_min[item];
        if (imin == kNone || imin > bound) {         // nothing here can pass Eq. 4
            if (tid == 0) {
                part[item] = Partial{kNone, kNone, LLONG_MAX, item, -1};
                atomicAdd(&hdr->pruned, 1ull);
            }
            return;
        }
    }

    const int c = sd.c, r = sd.r, T = sd.T, kcap = sd.kcap;
    const int S = sp.W + 1;
    const uint16_t *Yg = sp.ytab + sd.y_off + (long long)it.yi * (r + 1);
    for (int i = tid; i <= r; i += BS) sY[i] = Yg[i];
    for (int i = tid; i < it.xcount * c; i += BS) smap[i] = sp.spanmap[it.map_off + i];
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int j = 0; j < r; j++) {
            srowoff[j] = acc;
            const int h = sY[j + 1] - sY[j];
            acc += kcnt(sp, h, min(kcap, h));
        }
        srowoff[r] = acc;
    }
    __syncthreads();

    // Tile-option records: for (column span s, tile row j, option o) the option's largest
    // slice time, smallest and largest slice area and (step 2) summed ceil-SSE.
    const int rrow = it.rrow;
    const int nrec = it.nspans * rrow;
    for (int rid = tid; rid < nrec; rid += BS) {
        const int s = rid / rrow;
        const int rem = rid - s * rrow;
        int j = 0;
        while (j + 1 < r && srowoff[j + 1] <= rem) j++;
        const int o = rem - srowoff[j];
        const int xa = sp.spans[2 * (it.span_off + s)];
        const int xb = sp.spans[2 * (it.span_off + s) + 1];
        const int y0 = sY[j], h = sY[j + 1] - y0;
        const int opt = sp.opt_base[h] + o;
        const int k = sp.opt_k[opt];
        const uint16_t *z = sp.opt_z + (long long)opt * (sp.Km + 1);
        const unsigned wpx = (unsigned)(sp.colpx[xb] - sp.colpx[xa]);
        unsigned long long tmax = 0, qs = 0;
        unsigned amin = ~0u, amax = 0;
        for (int q = 0; q < k; q++) {
            const int ya = y0 + z[q], yb = y0 + z[q + 1];
            const unsigned long long tsum = (unsigned long long)rect(satT, S, xa, ya, xb, yb);
            const unsigned area = wpx * (unsigned)(sp.rowpx[yb] - sp.rowpx[ya]);
            tmax = max(tmax, tsum);
            amin = min(amin, area);
            amax = max(amax, area);
            if (P2) {
                const unsigned long long s1 = (unsigned long long)rect(satS1, S, xa, ya, xb, yb);
                const unsigned long long s2 = (unsigned long long)rect(satS2, S, xa, ya, xb, yb);
                qs += s2 - floor_sq_div(s1, area);
            }
        }
        recT[rid] = tmax;
        recA[rid] = (unsigned long long)amin | ((unsigned long long)amax << 32);
        if (P2) recQ[rid] = qs;
    }
    __syncthreads();

    // One candidate per lane: combine the T tile records of combination m for X = xa + xl.
    const int M = it.M;
    const int total = it.xcount * M;
    const uint16_t *__restrict__ cmb = sp.combos + it.combo_off;
    const float invM = 1.0f / (float)M;
    const unsigned long long ak = (unsigned long long)area_k;
    unsigned long long tbest = kNone, cnt = 0;
    Key2 best{kNone, kNone, LLONG_MAX, -1};
    for (int f = tid; f < total; f += BS) {
        int xl = (int)((float)f * invM);
        int m = f - xl * M;
        if (m < 0) { xl--; m += M; } else if (m >= M) { xl++; m -= M; }
        const uint8_t *mp = smap + xl * c;
        unsigned long long tmax = 0, qsum = 0;
        unsigned amin = ~0u, amax = 0;
        int t = 0;
        for (int j = 0; j < r; j++) {
            const int ro = srowoff[j];
            for (int i = 0; i < c; i++, t++) {
                const int rid = (int)mp[i] * rrow + ro + (int)cmb[(long long)t * M + m];
                tmax = max(tmax, recT[rid]);
                const unsigned long long A = recA[rid];
                amin = min(amin, (unsigned)A);
                amax = max(amax, (unsigned)(A >> 32));
                if (P2) qsum += recQ[rid];
            }
        }
        const bool feas = area_k == 0 || ak * amin > (unsigned long long)amax;
        if (!P2) {
            if (feas) {
                cnt++;
                tbest = min(tbest, tmax);
            }
        } else if (feas && tmax <= bound) {
            const Key2 cand{qsum, tmax, it.rank0 + (long long)xl * sd.SM + m, f};
            if (key_less(cand, best)) best = cand;
        }
    }
    (void)T;

    if (!P2) {
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) {
            tbest = min(tbest, shfl_xor64(tbest, m));
            cnt += shfl_xor64(cnt, m);
        }
        if (lane == 0) { redt[wv] = tbest; redq[wv] = cnt; }
        __syncthreads();
        if (tid == 0) {
            unsigned long long bt = kNone, bc = 0;
            for (int i = 0; i < NW; i++) { bt = min(bt, redt[i]); bc += redq[i]; }
            item_min[item] = bt;
            if (bt != kNone) atomicMin(&hdr->tmin, bt);
            if (bc) atomicAdd(&hdr->nfeas, bc);
        }
    } else {
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) {
            Key2 o;
            o.q = shfl_xor64(best.q, m);
            o.t = shfl_xor64(best.t, m);
            o.rank = (long long)shfl_xor64((unsigned long long)best.rank, m);
            o.f = __shfl_xor(best.f, m, kWave);
            if (key_less(o, best)) best = o;
        }
        if (lane == 0) { redq[wv] = best.q; redt[wv] = best.t; redr[wv] = best.rank; redf[wv] = best.f; }
        __syncthreads();
        if (tid == 0) {
            Key2 b{redq[0], redt[0], redr[0], redf[0]};
            for (int i = 1; i < NW; i++) {
                const Key2 o{redq[i], redt[i], redr[i], redf[i]};
                if (key_less(o, b)) b = o;
            }
            part[item] = Partial{b.q, b.t, b.rank, item, b.f};
            atomicAdd(&hdr->step2, (unsigned long long)total);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Final reduction and decode
// ---------------------------------------------------------------------------------------

__device__ void score_rect(const SpaceView &sp, const long long *satT, const long long *satS1,
                           const long long *satS2, int x0, int y0, int x1, int y1,
                           long long *t, long long *q)
{
    const int S = sp.W + 1;
    *t = rect(satT, S, x0, y0, x1, y1);
    const unsigned area = (unsigned)(sp.colpx[x1] - sp.colpx[x0]) * (unsigned)(sp.rowpx[y1] - sp.rowpx[y0]);
    const unsigned long long s1 = (unsigned long long)rect(satS1, S, x0, y0, x1, y1);
    const unsigned long long s2 = (unsigned long long)rect(satS2, S, x0, y0, x1, y1);
    *q = (long long)(s2 - floor_sq_div(s1, area));
}

__global__ void __launch_bounds__(256)
k_final(SpaceView sp, const Partial *__restrict__ part, int n_items, const WsHeader *hdr,
        const long long *satT, const long long *satS1, const long long *satS2,
        trs_result *out, int dt, int dr)
{
    constexpr int NW = 256 / kWave;
    __shared__ unsigned long long redq[NW], redt[NW];
    __shared__ long long redr[NW];
    __shared__ int redf[NW], redi[NW];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    for (int i = tid; i <= kMaxRS; i += 256) {
        out->col_bd[i] = 0;
        out->row_bd[i] = 0;
    }
    for (int i = tid; i < kMaxRS; i += 256) {
        for (int e = 0; e < 4; e++) out->rs[i][e] = 0;
        out->rs_time[i] = 0;
    }
    Key2 best{kNone, kNone, LLONG_MAX, -1};
    int bitem = -1;
    for (int i = tid; i < n_items; i += 256) {
        const Partial p = part[i];
        const Key2 k{p.q, p.t, p.rank, p.f};
        if (p.q != kNone && key_less(k, best)) { best = k; bitem = p.item; }
    }
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) {
        Key2 o;
        o.q = shfl_xor64(best.q, m);
        o.t = shfl_xor64(best.t, m);
        o.rank = (long long)shfl_xor64((unsigned long long)best.rank, m);
        o.f = __shfl_xor(best.f, m, kWave);
        const int oi = __shfl_xor(bitem, m, kWave);
        if (key_less(o, best)) { best = o; bitem = oi; }
    }
    if (lane == 0) { redq[wv] = best.q; redt[wv] = best.t; redr[wv] = best.rank; redf[wv] = best.f; redi[wv] = bitem; }
    __syncthreads();
    if (tid != 0) return;
    Key2 b{redq[0], redt[0], redr[0], redf[0]};
    int bi = redi[0];
    for (int i = 1; i < NW; i++) {
        const Key2 o{redq[i], redt[i], redr[i], redf[i]};
        if (key_less(o, b)) { b = o; bi = redi[i]; }
    }

    out->n_enumerated = sp.total;
    out->n_feasible = (long long)hdr->nfeas;
    out->n_step2 = (long long)hdr->step2;
    out->dtile_used = dt;
    out->drs_used = dr;
    out->uniform_rank = sp.uniform_rank;
    long long ut = -1, uq = -1;
    if (sp.n_unif > 0) {
        ut = 0;
        uq = 0;
        for (int i = 0; i < sp.n_unif; i++) {
            long long t, q;
            score_rect(sp, satT, satS1, satS2, sp.unif_rs[4 * i], sp.unif_rs[4 * i + 1],
                       sp.unif_rs[4 * i + 2], sp.unif_rs[4 * i + 3], &t, &q);
            ut = max(ut, t);
            uq += q;
        }
    }
    out->t_unif = ut;
    out->q_unif = uq;
    const int S = sp.W + 1;
    if (hdr->nfeas == 0 || b.q == kNone) {
        out->status = TRS_ENOFEASIBLE;
        out->rank = sp.uniform_rank;
        out->t_min = -1;
        out->t_sel = ut;
        out->q_sel = uq;
        int cu = 0, ru = 0;
        for (int i = 0; i < sp.n_unif; i++) {
            if (sp.unif_rs[4 * i + 1] == 0) cu++;
            if (sp.unif_rs[4 * i] == 0) ru++;
        }
        out->tile_cols = sp.n_unif ? cu : 0;
        out->tile_rows = sp.n_unif ? ru : 0;
        out->n_rs = sp.n_unif;
        for (int i = 0; i < cu; i++) out->col_bd[i] = sp.unif_rs[4 * i];
        if (cu) out->col_bd[cu] = sp.W;
        for (int j = 0; j < ru; j++) out->row_bd[j] = sp.unif_rs[4 * (j * cu) + 1];
        if (ru) out->row_bd[ru] = sp.H;
        for (int i = 0; i < sp.n_unif; i++) {
            for (int e = 0; e < 4; e++) out->rs[i][e] = sp.unif_rs[4 * i + e];
            out->rs_time[i] = rect(satT, S, sp.unif_rs[4 * i], sp.unif_rs[4 * i + 1],
                                   sp.unif_rs[4 * i + 2], sp.unif_rs[4 * i + 3]);
        }
        return;
    }
    out->status = TRS_OK;
    out->rank = b.rank;
    out->t_min = (long long)hdr->tmin;
    out->t_sel = (long long)b.t;
    out->q_sel = (long long)b.q;
    const ItemDev it = sp.items[bi];
    const ShapeDev sd = sp.shapes[it.shape];
    const int xl = b.f / it.M, m = b.f % it.M;
    const uint16_t *X = sp.xtab + sd.x_off + (long long)(it.xa + xl) * (sd.c + 1);
    const uint16_t *Y = sp.ytab + sd.y_off + (long long)it.yi * (sd.r + 1);
    out->tile_cols = sd.c;
    out->tile_rows = sd.r;
    for (int i = 0; i <= sd.c; i++) out->col_bd[i] = X[i];
    for (int j = 0; j <= sd.r; j++) out->row_bd[j] = Y[j];
    int n = 0;
    for (int t = 0; t < sd.T; t++) {
        const int i = t % sd.c, j = t / sd.c;
        const int h = Y[j + 1] - Y[j];
        const int opt = sp.opt_base[h] + sp.combos[it.combo_off + (long long)t * it.M + m];
        const int k = sp.opt_k[opt];
        const uint16_t *z = sp.opt_z + (long long)opt * (sp.Km + 1);
        for (int q = 0; q < k; q++) {
            out->rs[n][0] = X[i];
            out->rs[n][1] = Y[j] + z[q];
            out->rs[n][2] = X[i + 1];
            out->rs[n][3] = Y[j] + z[q + 1];
            out->rs_time[n] = rect(satT, S, X[i], Y[j] + z[q], X[i + 1], Y[j] + z[q + 1]);
            n++;
        }
    }
    out->n_rs = n;
}

template <int BS>
hipError_t launch_passes(const SearchArgs &a, long long *satT, long long *satS1, long long *satS2,
                         WsHeader *hdr, unsigned long long *imin, Partial *part, hipStream_t s)
{
    const int G = a.sp.n_items;
    if (a.ev[0] && hipEventRecord(a.ev[0], s) != hipSuccess) return hipErrorUnknown;
    hipLaunchKernelGGL((k_search<BS, false>), dim3(G), dim3(BS), 0, s, a.sp, satT, satS1, satS2,
                       hdr, imin, part, a.area_k, a.lam_num, a.lam_den);
    if (a.ev[1] && hipEventRecord(a.ev[1], s) != hipSuccess) return hipErrorUnknown;
    hipLaunchKernelGGL((k_search<BS, true>), dim3(G), dim3(BS), 0, s, a.sp, satT, satS1, satS2,
                       hdr, imin, part, a.area_k, a.lam_num, a.lam_den);
    if (a.ev[2] && hipEventRecord(a.ev[2], s) != hipSuccess) return hipErrorUnknown;
    return hipGetLastError();
}

}  // namespace

WsLayout ws_layout(const Plan &pl)
{
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    WsLayout l{};
    const size_t sat = sizeof(long long) * (size_t)(pl.W + 1) * (pl.H + 1);
    l.header = 0;
    l.satT = up(sizeof(WsHeader));
    l.satS1 = l.satT + up(sat);
    l.satS2 = l.satS1 + up(sat);
    l.item_min = l.satS2 + up(sat);
    l.partial = l.item_min + up(sizeof(unsigned long long) * pl.items.size());
    l.total = l.partial + up(sizeof(Partial) * pl.items.size());
    return l;
}

hipError_t launch_features(int w, int h, int cs, const uint16_t *luma, int64_t stride,
                           const trs_feat &o, hipStream_t s)
{
    const dim3 grid((w + cs - 1) / cs, (h + cs - 1) / cs);
    const int W = grid.x;
    switch (cs) {
    case 128:
        hipLaunchKernelGGL(k_features<128>, grid, dim3(256), 0, s, luma, (long long)stride, w, h, W,
                           o.s1, (unsigned long long *)o.s2, o.grad, o.tex, o.mean, o.var);
        break;
    case 64:
        hipLaunchKernelGGL(k_features<64>, grid, dim3(128), 0, s, luma, (long long)stride, w, h, W,
                           o.s1, (unsigned long long *)o.s2, o.grad, o.tex, o.mean, o.var);
        break;
    default:
        hipLaunchKernelGGL(k_features<32>, grid, dim3(64), 0, s, luma, (long long)stride, w, h, W,
                           o.s1, (unsigned long long *)o.s2, o.grad, o.tex, o.mean, o.var);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_cost_map(int n, const uint32_t *tex, const uint32_t *prev, trs_blend b,
                           uint32_t *cost, uint32_t *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_cost, dim3((n + 255) / 256), dim3(256), 0, s, n, tex, prev, b.a, b.b,
                       b.w_prev, cost, flags);
    return hipGetLastError();
}

hipError_t launch_search(const SearchArgs &a, hipStream_t s)
{
    auto *hdr = reinterpret_cast<WsHeader *>(a.ws + a.lay.header);
    auto *satT = reinterpret_cast<long long *>(a.ws + a.lay.satT);
    auto *satS1 = reinterpret_cast<long long *>(a.ws + a.lay.satS1);
    auto *satS2 = reinterpret_cast<long long *>(a.ws + a.lay.satS2);
    auto *imin = reinterpret_cast<unsigned long long *>(a.ws + a.lay.item_min);
    auto *part = reinterpret_cast<Partial *>(a.ws + a.lay.partial);
    hipLaunchKernelGGL(k_sat, dim3(1), dim3(256), 0, s, a.sp.W, a.sp.H, a.cost, a.s1,
                       (const unsigned long long *)a.s2, satT, satS1, satS2, hdr);
    hipError_t e;
    switch (a.block) {
    case 64: e = launch_passes<64>(a, satT, satS1, satS2, hdr, imin, part, s); break;
    case 128: e = launch_passes<128>(a, satT, satS1, satS2, hdr, imin, part, s); break;
    case 512: e = launch_passes<512>(a, satT, satS1, satS2, hdr, imin, part, s); break;
    default: e = launch_passes<256>(a, satT, satS1, satS2, hdr, imin, part, s); break;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, a.sp, part, a.sp.n_items, hdr, satT,
                       satS1, satS2, a.out, a.dt, a.dr);
    return hipGetLastError();
}

}  // namespace trs
