// Exact two-step search over the literal candidate space: every CTU boundary may serve as a
// tile boundary and as a split row (the space of Section 2.3 with no window around the uniform
// positions).  At 4K it holds 5.4e9 candidates, so instead of scoring them one by one the
// search is split into exact parts:
//
//   area windows  a partition passes the area rule k A_min > A_max iff all its RS areas lie in
//                 [a, k a) for a = its smallest area; the feasible set is the union over the
//                 windows [a, k a), a running over the distinct RS areas with
//                 N a <= A_total < k N a (host-side list); inside a window the rule is a
//                 condition on each RS alone;
//   k_lit_tiles   per (window, column strip): for every row range and slice count k, the best
//                 split of the tile's rows into k slices, one DP level per k (step 1: least
//                 largest slice time, Eq. 1; step 2: least (Q, T~) with every slice time
//                 within the Eq. 4 bound);
//   k_lit_units   per (window, row boundaries Y) unit kept by the host (its tile-row bands can
//                 hold N RS by area and slice count): a DP over column boundaries whose state
//                 is (tile columns used, RS used); the value of a column strip holding K RS
//                 comes from a DP over its r tiles.  One work-group per unit (one wave in step
//                 1, four in step 2), a wavefront over the right edge x of the strips, all state
//                 in LDS; step 2 on packed (Q, T~) keys when they fit 64 bits;
//   k_lit_pick    the best unit: step 1 by an atomic minimum of T~min, step 2 by a reduction
//                 over (Q, T~(P), unit);
//   k_lit_final   one work-group redoes the winning unit keeping the argmins, rebuilds boundaries
//                 and splits, and writes the trs_result.
// Ties follow the order (window, r, Y lexicographic, c) and the first minimising choice in
// ascending loop order inside each DP.  The canonical rank is not computed (-1), nor the count
// of feasible candidates (-1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "intmath.hpp"
#include "space.hpp"
#include "trs.h"

namespace trs {
namespace lit {
namespace {

constexpr long long kInf = LLONG_MAX;
constexpr unsigned long long kNone = ~0ull;
constexpr int kMaxW = 64, kMaxH = 40, kMaxN = 32;
constexpr size_t kLdsLimit = 160 * 1024;    // LDS per work-group on gfx950
constexpr long long kUnitCap = 1ll << 24;

// Device view of the host tables (by value).
struct LitView {
    int W, H, N, Cm, Rm, Km, S, R2, n_win, nY, n_units, n_wlive, karea, lam_num, lam_den, yrow, span;
    long long n_enumerated;
    const int *colpx, *rowpx;           // pixel prefix sums
    const long long *win;               // window lower bounds a (upper bound k a, or none)
    const unsigned char *ytab;          // per Y: r, then Y_0 .. Y_r (yrow bytes per entry)
    const unsigned char *strip_xy;      // per strip: x0, x1
    const unsigned char *row_yy;        // per row pair: y0, y1
    const int *ulist;                   // units kept (index window * nY + Y), ascending
    const int *dorder;                  // positions in ulist in dispatch order
    const int *wlive;                   // windows holding a kept unit, ascending
    unsigned long long *work;           // while profiling: relaxations of the units run, per step
    long long relaxA, relaxB;           // a unit of r tile rows has r relaxA + relaxB of them
};

struct LitWs {
    unsigned long long *hdr;            // [0] T~min, [1] winning unit, [2] its column count,
                                        // [3] least Q of a unit so far (step-2 pruning bound),
                                        // [4] 1 when the frame's total time is below 2^32 - 1,
                                        // [5] 1 when some rectangle has q < 0
    long long *sat;                     // 3 inclusive prefix sums, (H + 1) x (W + 1) each
    long long *rA, *rT, *rQ;            // per rectangle [S][R2]: area, time, q
    long long *tT, *tQ;                 // per [window][strip][row pair][k - 1]
    long long *uQ, *uT;                 // per unit: best (Q, T~) of step 2
    int *uC;                            // per unit: its column count
    long long *wT;                      // per window: least step-1 result of its units
};

__host__ __device__ __forceinline__ int sidx(int x0, int x1, int W)
{
    return x0 * W - x0 * (x0 - 1) / 2 + (x1 - x0 - 1);
}

__host__ __device__ __forceinline__ int ridx(int y0, int y1, int H)
{
    return y0 * H - y0 * (y0 - 1) / 2 + (y1 - y0 - 1);
}

__device__ __forceinline__ unsigned long long eq4_bound(unsigned long long tmin, int num, int den)
{
    if (num < 0) return kNone;
    return tmin * (unsigned long long)(den + num) / (unsigned long long)den;
}

// Quotient and remainder by a small divisor d (1 <= d <= 4096) for e < 2^16 without a divide:
// m = ceil(2^16 / d) overshoots e / d by less than one, which one correction step removes.
struct SmallDiv {
    unsigned d, m;
    __device__ explicit SmallDiv(unsigned dd) : d(dd), m((65536u + dd - 1) / dd) {}
    __device__ __forceinline__ void divmod(unsigned e, unsigned &q, unsigned &rr) const
    {
        q = (e * m) >> 16;
        if (q * d > e) q--;
        rr = e - q * d;
    }
};

// Step-2 values compare by Q, then T~; step 1 by T~ alone (q stays 0).
template <int STEP>
__device__ __forceinline__ bool better(long long aq, long long at, long long bq, long long bt)
{
    if (STEP == 1) return at < bt;
    return aq < bq || (aq == bq && at < bt);
}

// ---------------------------------------------------------------------------------------
// Prefix sums of T~, S1, S2 (one work-group, scanned in LDS: rows, then columns) and the
// header.
__global__ void __launch_bounds__(256)
k_lit_sat(LitView v, LitWs w, const uint32_t *__restrict__ cost, const uint32_t *__restrict__ s1,
          const uint64_t *__restrict__ s2)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    long long *sh = reinterpret_cast<long long *>(lds_raw);      // [3][(H + 1) x (W + 1)]
    const int W = v.W, H = v.H, P = (W + 1) * (H + 1);
    if (threadIdx.x == 0) {
        w.hdr[0] = kNone;
        w.hdr[1] = kNone;
        w.hdr[2] = 0;
        w.hdr[3] = kNone;
        w.hdr[5] = 0;
        if (v.work) { v.work[0] = 0; v.work[1] = 0; }
    }
    for (int i = threadIdx.x; i < v.n_win; i += blockDim.x) w.wT[i] = kInf;
    for (int e = threadIdx.x; e < 3 * P; e += blockDim.x) {
        const int a = e / P, rem = e - a * P, y = rem / (W + 1), x = rem - y * (W + 1);
        long long val = 0;
        if (x > 0 && y > 0) {
            const size_t c = (size_t)(y - 1) * W + (x - 1);
            val = a == 0 ? (long long)cost[c] : a == 1 ? (long long)s1[c] : (long long)s2[c];
        }
        sh[e] = val;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * (H + 1); t += blockDim.x) {           // rows: along x
        long long *row = sh + (size_t)(t / (H + 1)) * P + (size_t)(t % (H + 1)) * (W + 1);
        for (int x = 1; x <= W; x++) row[x] += row[x - 1];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * (W + 1); t += blockDim.x) {           // columns: along y
        long long *col = sh + (size_t)(t / (W + 1)) * P + (t % (W + 1));
        for (int y = 1; y <= H; y++) col[(size_t)y * (W + 1)] += col[(size_t)(y - 1) * (W + 1)];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * P; e += blockDim.x) w.sat[e] = sh[e];
    if (threadIdx.x == 0) w.hdr[4] = sh[P - 1] < 0xffffffffll;          // every time sum fits 32 bits
}

// Area, time and q = S2 - floor(S1^2 / n) of every rectangle.
__global__ void __launch_bounds__(256)
k_lit_rects(LitView v, LitWs w)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.S * v.R2) return;
    const int s = i / v.R2, p = i % v.R2;
    const int x0 = v.strip_xy[2 * s], x1 = v.strip_xy[2 * s + 1];
    const int y0 = v.row_yy[2 * p], y1 = v.row_yy[2 * p + 1];
    const int S = v.W + 1, P = (v.W + 1) * (v.H + 1);
    auto rect = [&](const long long *t) {
        return t[y1 * S + x1] - t[y0 * S + x1] - t[y1 * S + x0] + t[y0 * S + x0];
    };
    const long long A = (long long)(v.colpx[x1] - v.colpx[x0]) * (v.rowpx[y1] - v.rowpx[y0]);
    const long long a1 = rect(w.sat + P), a2 = rect(w.sat + 2 * (size_t)P);
    w.rA[i] = A;
    w.rT[i] = rect(w.sat);
    const long long q = a2 - (long long)floor_sq_div((unsigned long long)a1, (unsigned)A);
    w.rQ[i] = q;
    if (q < 0) w.hdr[5] = 1;            // statistics no real pixels have (S1^2 > n S2)
}

// ---------------------------------------------------------------------------------------
// Tile tables: one work-group per (window, strip).  Threads take row pairs (y0, y); level q
// holds the best split of rows [y0, y) into q slices.
// BS threads: 128 in step 1, 256 in step 2 (measured best of 64, 128 and 256 for each).  BUF:
// every level of the DP is kept in LDS, [row pair][k] as in the table, and the table block is
// written at the end in one coalesced pass (when 8 R2 (2 + Km) bytes, 8 R2 (3 + 2 Km) with Q,
// fit); else two levels are kept and each level is written as it is computed.
template <int STEP, bool BUF, int BS = STEP == 1 ? 128 : 256>
__global__ void __launch_bounds__(BS)
k_lit_tiles(LitView v, LitWs w)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int R2 = v.R2, H = v.H, Km = v.Km;
    const int wi = v.wlive[blockIdx.x / v.S], s = blockIdx.x % v.S;
    long long *sA = reinterpret_cast<long long *>(lds_raw);
    long long *sT = sA + R2;
    long long *sQ = sT + (STEP == 2 ? R2 : 0);
    long long *fT = sQ + R2;            // BUF: R2 x Km levels; else two levels of R2 entries
    long long *fQ = fT + (BUF ? (size_t)R2 * Km : 2 * (size_t)R2);
    unsigned long long tau = kNone;
    if (STEP == 2) {
        const unsigned long long tmin = w.hdr[0];
        if (tmin == kNone) return;
        tau = eq4_bound(tmin, v.lam_num, v.lam_den);
        // no unit of this window reaches step 2 (each unit's step-1 result is exact whenever it
        // is within the bound step 1 pruned with, which is at least tau)
        if (v.lam_num >= 0 && (unsigned long long)w.wT[wi] > tau) return;
    }
    const long long lo = v.win[wi];
    const long long hi = v.karea ? (long long)v.karea * lo : kInf;
    const size_t rbase = (size_t)s * R2;
    for (int p = threadIdx.x; p < R2; p += blockDim.x) {
        sA[p] = w.rA[rbase + p];
        sT[p] = w.rT[rbase + p];
        if (STEP == 2) sQ[p] = w.rQ[rbase + p];
    }
    __syncthreads();
    auto ok = [&](int p) {
        return sA[p] >= lo && sA[p] < hi && (STEP == 1 || (unsigned long long)sT[p] <= tau);
    };
    // level q of pair p
    auto cur = [&](long long *f, int p, int q) -> long long & {
        return BUF ? f[(size_t)p * Km + (q - 1)] : f[(size_t)(q & 1) * R2 + p];
    };
    const size_t tbase = ((size_t)wi * v.S + s) * R2;
    for (int q = 1; q <= Km; q++) {
        for (int p = threadIdx.x; p < R2; p += blockDim.x) {
            const int y0 = v.row_yy[2 * p], y = v.row_yy[2 * p + 1];
            long long bt = kInf, bq = kInf;
            if (q == 1) {
                if (ok(p)) { bt = sT[p]; bq = STEP == 2 ? sQ[p] : 0; }
            } else {
                for (int yp = y0 + q - 1; yp < y; yp++) {
                    const int pp = ridx(y0, yp, H), ps = ridx(yp, y, H);
                    const long long pt = cur(fT, pp, q - 1);
                    if (pt == kInf || !ok(ps)) continue;
                    const long long t = pt > sT[ps] ? pt : sT[ps];
                    const long long qq = STEP == 2 ? cur(fQ, pp, q - 1) + sQ[ps] : 0;
                    if (better<STEP>(qq, t, bq, bt)) { bt = t; bq = qq; }
                }
            }
            cur(fT, p, q) = bt;
            if (STEP == 2) cur(fQ, p, q) = bq;
            if (!BUF) {
                w.tT[(tbase + p) * Km + (q - 1)] = bt;
                if (STEP == 2) w.tQ[(tbase + p) * Km + (q - 1)] = bq;
            }
        }
        __syncthreads();
    }
    if (BUF)
        for (size_t e = threadIdx.x; e < (size_t)R2 * Km; e += blockDim.x) {
            w.tT[tbase * Km + e] = fT[e];
            if (STEP == 2) w.tQ[tbase * Km + e] = fQ[e];
        }
}

// ---------------------------------------------------------------------------------------
// The column DP of one unit (window, Y), serial per state: step 2 and the rebuild when (Q, T~)
// does not fit one 64-bit key.  LDS: strip values hs[x'][K] for the
// strips ending at the current x, the DP table F[i][x][n], a flag per hs row and per (i, x) row
// telling whether it holds a finite value, and with REC the argmins.
//
// Pruning (exact): a state whose T~ exceeds bt, or whose Q exceeds bq, becomes infinite.  Step
// 1 passes the Eq. 4 bound of the best T~min found so far (or that T~min when lambda is
// infinite), so every unit whose own minimum is within the final bound still reports it exactly;
// step 2 passes the best Q found so far when every rectangle has q >= 0 (Q of a partial
// partition then only grows), else none.  A partition through a pruned state cannot be the optimum.  REC (the rebuild) prunes
// nothing, so its argmins are those of the full DP.
struct UnitLds {
    long long *hsT, *hsQ, *FT, *FQ;
    long long *tvT, *tvQ;               // tile values of the strips ending at the current x
    unsigned *hsOk, *FOk;
    unsigned char *AX, *AK;
};

__host__ __device__ inline size_t unit_lds_bytes(int W, int N, int Cm, int Rm, int Km, int step, bool rec,
                                                 int span)
{
    const size_t hs = (size_t)W * (span ? Rm + 1 : 1) * (N + 1), F = (size_t)(Cm + 1) * (W + 1) * (N + 1);
    const size_t tv = (size_t)W * Rm * Km;
    size_t b = 8 * (hs + F + tv) * (step == 2 ? 2 : 1) + 4 * ((size_t)W + (size_t)(Cm + 1) * (W + 1));
    if (rec) b += 2 * F;
    return (b + 15) & ~size_t(15);
}

__device__ inline UnitLds unit_lds(unsigned char *raw, int W, int N, int Cm, int Rm, int Km, int step,
                                   bool rec, int span)
{
    const size_t hs = (size_t)W * (span ? Rm + 1 : 1) * (N + 1), F = (size_t)(Cm + 1) * (W + 1) * (N + 1);
    const size_t tv = (size_t)W * Rm * Km;
    UnitLds L{};
    long long *p = reinterpret_cast<long long *>(raw);
    L.hsT = p; p += hs;
    if (step == 2) { L.hsQ = p; p += hs; }
    L.FT = p; p += F;
    if (step == 2) { L.FQ = p; p += F; }
    L.tvT = p; p += tv;
    if (step == 2) { L.tvQ = p; p += tv; }
    unsigned *o = reinterpret_cast<unsigned *>(p);
    L.hsOk = o; o += W;
    L.FOk = o; o += (size_t)(Cm + 1) * (W + 1);
    unsigned char *c = reinterpret_cast<unsigned char *>(o);
    if (rec) { L.AX = c; L.AK = c + F; }
    return L;
}

template <int STEP, bool REC, bool SPAN>
__device__ void unit_dp(const LitView &v, const LitWs &w, int u, const UnitLds &L, int *Yl, int &r,
                        long long bt, long long bq)
{
    const int lane = threadIdx.x;
    const int W = v.W, N = v.N, Cm = v.Cm, Km = v.Km, S = v.S, R2 = v.R2;
    const int wi = u / v.nY, yi = u % v.nY;
    const unsigned char *yt = v.ytab + (size_t)yi * v.yrow;
    r = yt[0];
    for (int j = lane; j <= r; j += blockDim.x) Yl[j] = yt[1 + j];
    const size_t F = (size_t)(Cm + 1) * (W + 1) * (N + 1);
    for (size_t e = lane; e < F; e += blockDim.x) {
        L.FT[e] = kInf;
        if (STEP == 2) L.FQ[e] = kInf;
    }
    for (int e = lane; e < (Cm + 1) * (W + 1); e += blockDim.x) L.FOk[e] = e == 0;
    __syncthreads();
    if (lane == 0) {
        L.FT[0] = 0;
        if (STEP == 2) L.FQ[0] = 0;
    }
    auto fi = [&](int i, int x, int n) { return ((size_t)i * (W + 1) + x) * (N + 1) + n; };
    auto keep = [&](long long t, long long q) { return t <= bt && (STEP == 1 || q <= bq); };
    const int Rm = v.Rm, RR = SPAN ? Rm + 1 : 1;
    const long long lo = v.win[wi];
    const long long hi = v.karea ? (long long)v.karea * lo : kInf;
    const unsigned long long tau = STEP == 2 ? eq4_bound(w.hdr[0], v.lam_num, v.lam_den) : kNone;
    for (int x = 1; x <= W; x++) {
        // tile values (k = 1 .. Km) of the r tiles of every strip [x', x), loaded together
        for (int e = lane; e < x * r; e += blockDim.x) {
            const int xp = e / r, j = e % r;
            const size_t tb = (((size_t)wi * S + sidx(xp, x, W)) * R2 + ridx(Yl[j], Yl[j + 1], v.H)) * Km;
            const size_t lb = ((size_t)xp * Rm + j) * Km;
            for (int k = 0; k < Km; k++) {
                L.tvT[lb + k] = w.tT[tb + k];
                if (STEP == 2) L.tvQ[lb + k] = w.tQ[tb + k];
            }
        }
        __syncthreads();
        // strips [x', x): DP over the r tile-row levels.  With blocks of tiles allowed every
        // level has its own row of hs (a block ending at level b starts from a level a <= b - 2);
        // otherwise one row is updated in place, K descending.  Tiles are tried first (k
        // ascending), then blocks (a ascending), as in the oracle.
        for (int xp = lane; xp < x; xp += blockDim.x) {
            long long *baseT = L.hsT + (size_t)xp * RR * (N + 1);
            long long *baseQ = STEP == 2 ? L.hsQ + (size_t)xp * RR * (N + 1) : nullptr;
            auto rowT = [&](int b) { return baseT + (size_t)(SPAN ? b : 0) * (N + 1); };
            auto rowQ = [&](int b) { return baseQ + (size_t)(SPAN ? b : 0) * (N + 1); };
            for (int K = 0; K <= N; K++) {
                rowT(0)[K] = K == 0 ? 0 : kInf;
                if (STEP == 2) rowQ(0)[K] = K == 0 ? 0 : kInf;
            }
            const size_t rs0 = (size_t)sidx(xp, x, W) * R2;
            bool any = true;
            for (int b = 1; b <= r && (any || SPAN); b++) {
                const long long *tvT = L.tvT + ((size_t)xp * Rm + (b - 1)) * Km;
                const long long *tvQ = STEP == 2 ? L.tvQ + ((size_t)xp * Rm + (b - 1)) * Km : nullptr;
                const long long *sT = rowT(b - 1), *sQ = STEP == 2 ? rowQ(b - 1) : nullptr;
                long long *dT = rowT(b), *dQ = STEP == 2 ? rowQ(b) : nullptr;
                for (int K = N; K >= 0; K--) {
                    long long ct = kInf, cq = kInf;
                    for (int k = 1; k <= Km && k <= K; k++) {
                        const long long at = sT[K - k], tt = tvT[k - 1];
                        if (at == kInf || tt == kInf) continue;
                        const long long t = at > tt ? at : tt;
                        const long long q = STEP == 2 ? sQ[K - k] + tvQ[k - 1] : 0;
                        if (better<STEP>(q, t, cq, ct)) { ct = t; cq = q; }
                    }
                    dT[K] = ct;
                    if (STEP == 2) dQ[K] = cq;
                }
                // blocks of tiles a .. b - 1 as one RS, after the single tiles (the same order
                // per K as taking every choice for one K before the next K)
                if (SPAN)
                    for (int a = 0; a + 2 <= b; a++) {
                        const size_t ri = rs0 + ridx(Yl[a], Yl[b], v.H);
                        const long long A = w.rA[ri], bT = w.rT[ri];
                        if (A < lo || A >= hi || (STEP == 2 && (unsigned long long)bT > tau)) continue;
                        const long long bQ = STEP == 2 ? w.rQ[ri] : 0;
                        const long long *aT = rowT(a), *aQ = STEP == 2 ? rowQ(a) : nullptr;
                        for (int K = 1; K <= N; K++) {
                            const long long at = aT[K - 1];
                            if (at == kInf) continue;
                            const long long t = at > bT ? at : bT;
                            const long long q = STEP == 2 ? aQ[K - 1] + bQ : 0;
                            if (better<STEP>(q, t, STEP == 2 ? dQ[K] : 0, dT[K])) {
                                dT[K] = t;
                                if (STEP == 2) dQ[K] = q;
                            }
                        }
                    }
                any = false;
                for (int K = 0; K <= N; K++) {
                    if (dT[K] != kInf && !REC && !keep(dT[K], STEP == 2 ? dQ[K] : 0)) {
                        dT[K] = kInf;
                        if (STEP == 2) dQ[K] = kInf;
                    }
                    any |= dT[K] != kInf;
                }
            }
            if (!any)
                for (int K = 0; K <= N; K++) rowT(SPAN ? r : 0)[K] = kInf;
            L.hsOk[xp] = any;
        }
        __syncthreads();
        // states (i, n) at x
        for (int st = lane; st < Cm * N; st += blockDim.x) {
            const int i = 1 + st / N, n = 1 + st % N;
            if (i > x) continue;
            long long ct = kInf, cq = kInf;
            int ax = -1, ak = -1;
            for (int xp = i - 1; xp < x; xp++) {
                if (!L.hsOk[xp] || !L.FOk[(i - 1) * (W + 1) + xp]) continue;
                const size_t hrow = ((size_t)xp * RR + (SPAN ? r : 0)) * (N + 1);
                const long long *hT = L.hsT + hrow;
                for (int K = 1; K <= n; K++) {
                    const size_t fp = fi(i - 1, xp, n - K);
                    const long long at = L.FT[fp], tt = hT[K];
                    if (at == kInf || tt == kInf) continue;
                    const long long t = at > tt ? at : tt;
                    const long long q = STEP == 2 ? L.FQ[fp] + L.hsQ[hrow + K] : 0;
                    if (better<STEP>(q, t, cq, ct)) { ct = t; cq = q; ax = xp; ak = K; }
                }
            }
            if (ct != kInf && !REC && !keep(ct, cq)) ct = cq = kInf;
            const size_t f = fi(i, x, n);
            L.FT[f] = ct;
            if (STEP == 2) L.FQ[f] = cq;
            if (REC) { L.AX[f] = (unsigned char)ax; L.AK[f] = (unsigned char)ak; }
            if (ct != kInf) L.FOk[i * (W + 1) + x] = 1;
        }
        __syncthreads();
    }
}

// Step-2 values as one 64-bit key Q 2^tb + T~ (T~ < 2^tb): keys order as the pairs (Q, T~) do
// lexicographically, and joining two disjoint parts (Q adds, T~ takes the larger) is
// a + b - min(a mod 2^tb, b mod 2^tb).  It applies when every key stays below 2^61: the Q of a
// partial partition is at most the frame's S2 (q = S2 - floor(S1^2 / n) of an RS lies in
// [0, S2] by Cauchy-Schwarz when the statistics are those of real pixels, which k_lit_rects
// checks), and every T~ is at most the Eq. 4 bound and the frame's total.  kBig = 2^62 is
// "none"; a join involving it lands at or above kBig without wrapping (at most 2^63), and every
// stored value is either a key or exactly kBig.
constexpr unsigned long long kBig = 1ull << 62;

struct Pack {
    unsigned tb;
    unsigned long long mask;
    __device__ unsigned long long key(long long q, long long t) const
    {
        return t == kInf ? kBig : ((unsigned long long)q << tb) | (unsigned long long)t;
    }
};

__device__ bool pack_for(const LitView &v, const LitWs &w, Pack &p)
{
    if (w.hdr[5] != 0) return false;                     // some rectangle has q < 0
    const size_t P = (size_t)(v.W + 1) * (v.H + 1);
    const unsigned long long Ttot = (unsigned long long)w.sat[P - 1];
    const unsigned long long S2 = (unsigned long long)w.sat[3 * P - 1];
    unsigned long long cap = eq4_bound(w.hdr[0], v.lam_num, v.lam_den);
    cap = cap < Ttot ? cap : Ttot;
    int tb = 64 - __clzll(cap);                          // cap < 2^tb
    tb = tb < 1 ? 1 : tb;
    if (tb > 60 || S2 >= (1ull << (61 - tb))) return false;
    p.tb = (unsigned)tb;
    p.mask = (1ull << tb) - 1;
    return true;
}

// Step 1 (V: 32- or 64-bit T~) and step 2 (V: 64-bit keys) balanced over the lanes: the strip
// DP takes one (x', K) pair per lane (rows of hs double-buffered per tile), the column DP one
// (i, x') pair per lane, each folding its candidates for every n into F[i][x][n] with an LDS
// atomic minimum.  Same values as unit_dp: the minimum of a set does not depend on the order it
// is taken in.  In step 1 the largest value of V is "none" (a frame whose total time is below
// 2^32 - 1 runs with 32-bit values: every region sum fits), which max() propagates and min()
// ignores.  REC (step 2 only) keeps argmins equal to the serial DP's first minimum in ascending
// (x', K) order: once F[.][x][.] is final, each (i, x') pair finds its first K that reaches the
// value, and an atomic minimum of x' 64 + K picks the first pair.
template <class V, int NB, bool SPAN, int STEP, bool REC>
__device__ void unit_dp1(const LitView &v, const LitWs &w, int u, unsigned char *raw, int *Yl, int &r,
                         long long bound, const Pack &pk, unsigned char *AX, unsigned char *AK,
                         unsigned *AXK, long long *result, int *result_c)
{
    constexpr V kNo = STEP == 1 ? ~V(0) : V(kBig);
    // step 1: a value maps to the sentinel when it is infinite or does not fit below it
    auto narrow = [&](long long t) {
        return (t == kInf || (unsigned long long)t >= (unsigned long long)kNo) ? kNo : (V)t;
    };
    auto join = [&](V a, V b) -> V {
        if constexpr (STEP == 1) return a > b ? a : b;
        else {
            const V ta = a & pk.mask, tb = b & pk.mask;
            return a + b - (ta < tb ? ta : tb);
        }
    };
    V bt;                                                // values above it are pruned
    if constexpr (STEP == 1)
        bt = bound == kInf ? V(kNo - 1) : (narrow(bound) == kNo ? V(kNo - 1) : (V)bound);
    else
        bt = bound == kInf || (unsigned long long)bound >= (kBig >> pk.tb) ? V(kNo - 1)
                                                                          : (((V)bound << pk.tb) | pk.mask);
    const int lane = threadIdx.x;
    const int W = v.W, N = v.N, Cm = v.Cm, Km = v.Km, S = v.S, R2 = v.R2, Rm = v.Rm, NP = N + 1;
    const int wi = u / v.nY, yi = u % v.nY;
    const size_t F = (size_t)(Cm + 1) * (W + 1) * NP;
    // strip rows [level][x'][K]: all r + 1 tile-row levels when blocks of tiles are allowed (a
    // block ending at level b starts from level a <= b - 2), else two levels used in turn
    const int NPR = SPAN ? Rm * (Rm - 1) / 2 : 0;
    const int RR = SPAN ? Rm + 1 : 2;
    auto rowi = [&](int b) { return SPAN ? b : (b & 1); };
    V *FT = reinterpret_cast<V *>(raw);
    V *hs = FT + F;
    V *tv = hs + (size_t)W * RR * NP;
    V *bv = tv + (size_t)W * Rm * Km;                       // block values [x'][pair (a, b)]
    unsigned *FOk = reinterpret_cast<unsigned *>(bv + (size_t)W * NPR);
    unsigned *hsOk = FOk + (size_t)(Cm + 1) * (W + 1);
    const long long lo = SPAN ? v.win[wi] : 0;
    const long long hi = SPAN && v.karea ? (long long)v.karea * lo : kInf;
    const unsigned long long tau = STEP == 2 ? eq4_bound(w.hdr[0], v.lam_num, v.lam_den) : kNone;
    const unsigned char *yt = v.ytab + (size_t)yi * v.yrow;
    r = yt[0];
    for (int j = lane; j <= r; j += blockDim.x) Yl[j] = yt[1 + j];
    for (size_t e = lane; e < F; e += blockDim.x) FT[e] = e == 0 ? V(0) : kNo;
    for (int e = lane; e < (Cm + 1) * (W + 1); e += blockDim.x) FOk[e] = e == 0;
    if constexpr (REC)
        for (int e = lane; e < (Cm + 1) * NP; e += blockDim.x) AXK[e] = ~0u;
    __syncthreads();
    const SmallDiv divR((unsigned)r), divNP((unsigned)NP);
    for (int x = 1; x <= W; x++) {
        for (int e = lane; e < x * r; e += blockDim.x) {
            unsigned xp, j;
            divR.divmod((unsigned)e, xp, j);
            const size_t tb = (((size_t)wi * S + sidx(xp, x, W)) * R2 + ridx(Yl[j], Yl[j + 1], v.H)) * Km;
            const size_t lb = ((size_t)xp * Rm + j) * Km;
            for (int k = 0; k < Km; k++) {
                if constexpr (STEP == 1) tv[lb + k] = narrow(w.tT[tb + k]);
                else tv[lb + k] = pk.key(w.tQ[tb + k], w.tT[tb + k]);
            }
        }
        if constexpr (SPAN) {
            const int npair = r * (r - 1) / 2;
            for (int e = lane; e < x * npair; e += blockDim.x) {
                const int xp = e / npair;
                int pr = e - xp * npair, b = 2;
                while (pr >= b - 1) { pr -= b - 1; b++; }        // pair index (b-2)(b-1)/2 + a
                const size_t ri = (size_t)sidx(xp, x, W) * R2 + ridx(Yl[pr], Yl[b], v.H);
                const long long A = w.rA[ri];
                V val = kNo;
                if (A >= lo && A < hi) {
                    if constexpr (STEP == 1) val = narrow(w.rT[ri]);
                    else if ((unsigned long long)w.rT[ri] <= tau) val = pk.key(w.rQ[ri], w.rT[ri]);
                }
                bv[(size_t)xp * NPR + (e - xp * npair)] = val;
            }
        }
        for (int e = lane; e < x * NP; e += blockDim.x) {
            unsigned xp, K;
            divNP.divmod((unsigned)e, xp, K);
            hs[((size_t)rowi(0) * W + xp) * NP + K] = K == 0 ? V(0) : kNo;
        }
        for (int xp = lane; xp < x; xp += blockDim.x) hsOk[xp] = 0;
        __syncthreads();
        for (int b = 1; b <= r; b++) {
            for (int e = lane; e < x * NP; e += blockDim.x) {
                unsigned xp, K;
                divNP.divmod((unsigned)e, xp, K);
                const V *tj = tv + ((size_t)xp * Rm + (b - 1)) * Km;
                const V *row = hs + ((size_t)rowi(b - 1) * W + xp) * NP;
                V best = kNo;
                const int kmax = (int)K < Km ? (int)K : Km;
                for (int k = 1; k <= kmax; k++) {
                    const V t = join(row[K - k], tj[k - 1]);
                    best = t < best ? t : best;
                }
                if constexpr (SPAN)
                    for (int a = 0; a + 2 <= b && K >= 1; a++) {    // tiles a .. b - 1 as one RS
                        const V s0 = hs[((size_t)a * W + xp) * NP + K - 1];
                        const V c = bv[(size_t)xp * NPR + (b - 2) * (b - 1) / 2 + a];
                        const V t = join(s0, c);
                        best = t < best ? t : best;
                    }
                if (best > bt) best = kNo;
                hs[((size_t)rowi(b) * W + xp) * NP + K] = best;
                if (b == r && best != kNo) hsOk[xp] = 1;
            }
            __syncthreads();
        }
        // column DP: one (i, x') pair per lane, all n at once (x' varies fastest across lanes:
        // measured faster than i fastest, whose scattered row reads cost more than the atomic
        // conflicts it removes)
        const SmallDiv divX((unsigned)x);
        for (int e = lane; e < Cm * x; e += blockDim.x) {
            unsigned i1, xpu;
            divX.divmod((unsigned)e, i1, xpu);
            const int i = 1 + (int)i1, xp = (int)xpu;
            if (xp < i - 1 || !hsOk[xp] || !FOk[(i - 1) * (W + 1) + xp]) continue;
            const V *h = hs + ((size_t)rowi(r) * W + xp) * NP;
            const V *f = FT + ((size_t)(i - 1) * (W + 1) + xp) * NP;
            // both rows in registers (NB >= N, entries past N are "none"), loops unrolled
            V fr[NB + 1], hr[NB + 1];
#pragma unroll
            for (int q = 0; q <= NB; q++) {
                fr[q] = q <= N ? f[q] : kNo;
                hr[q] = q <= N ? h[q] : kNo;
            }
            bool any = false;
#pragma unroll
            for (int n = 1; n <= NB; n++) {
                V best = kNo;
#pragma unroll
                for (int K = 1; K <= n; K++) {
                    const V t = join(fr[n - K], hr[K]);
                    best = t < best ? t : best;
                }
                if (n <= N && best <= bt) {
                    atomicMin(FT + ((size_t)i * (W + 1) + x) * NP + n, best);
                    any = true;
                }
            }
            if (any) FOk[i * (W + 1) + x] = 1;
        }
        __syncthreads();
        if constexpr (REC) {
            for (int e = lane; e < Cm * x; e += blockDim.x) {
                unsigned i1, xpu;
                divX.divmod((unsigned)e, i1, xpu);
                const int i = 1 + (int)i1, xp = (int)xpu;
                if (xp < i - 1 || !hsOk[xp] || !FOk[(i - 1) * (W + 1) + xp]) continue;
                const V *h = hs + ((size_t)rowi(r) * W + xp) * NP;
                const V *f = FT + ((size_t)(i - 1) * (W + 1) + xp) * NP;
                const V *g = FT + ((size_t)i * (W + 1) + x) * NP;
                for (int n = 1; n <= N; n++) {
                    const V target = g[n];
                    if (target == kNo) continue;
                    for (int K = 1; K <= n; K++)
                        if (join(f[n - K], h[K]) == target) {
                            atomicMin(AXK + i * NP + n, (unsigned)(xp * 64 + K));
                            break;
                        }
                }
            }
            __syncthreads();
            for (int e = lane; e < Cm * NP; e += blockDim.x) {
                const int i = 1 + e / NP, n = e % NP;
                const unsigned c = AXK[i * NP + n];
                const size_t fo = ((size_t)i * (W + 1) + x) * NP + n;
                AX[fo] = c == ~0u ? 0xff : (unsigned char)(c / 64);
                AK[fo] = c == ~0u ? 0xff : (unsigned char)(c % 64);
                AXK[i * NP + n] = ~0u;
            }
            __syncthreads();
        }
    }
    if (lane == 0) {
        V best = kNo;
        int bc = 0;
        for (int c = 1; c <= Cm; c++) {
            const V t = FT[((size_t)c * (W + 1) + W) * NP + N];
            if (t < best) { best = t; bc = c; }
        }
        if constexpr (STEP == 1) {
            result[0] = best == kNo ? kInf : (long long)best;
        } else {
            result[0] = best == kNo ? kInf : (long long)(best >> pk.tb);
            result[1] = best == kNo ? kInf : (long long)(best & pk.mask);
        }
        *result_c = best == kNo ? 0 : bc;
    }
}

__host__ __device__ inline size_t unit1_lds_bytes(int W, int N, int Cm, int Rm, int Km, int vbytes, int span)
{
    const size_t F = (size_t)(Cm + 1) * (W + 1) * (N + 1);
    const size_t RR = span ? Rm + 1 : 2, NPR = span ? (size_t)Rm * (Rm - 1) / 2 : 0;
    return vbytes * (F + RR * W * (N + 1) + (size_t)W * Rm * Km + W * NPR) +
           4 * ((size_t)(Cm + 1) * (W + 1) + W);
}

// LDS of step 2: the serial DP's layout, or the packed one when the keys fit (decided at run
// time, so both must fit).
__host__ __device__ inline size_t unit2_lds_bytes(int W, int N, int Cm, int Rm, int Km, int span)
{
    const size_t a = unit_lds_bytes(W, N, Cm, Rm, Km, 2, false, span), b = unit1_lds_bytes(W, N, Cm, Rm, Km, 8, span);
    return a > b ? a : b;
}

// LDS of the rebuild's DP: the serial DP with argmins, or the packed DP followed by its argmin
// bytes and the per-x atomic scratch.
__host__ __device__ inline size_t rec_lds_bytes(int W, int N, int Cm, int Rm, int Km, int span)
{
    const size_t F = (size_t)(Cm + 1) * (W + 1) * (N + 1);
    const size_t a = unit_lds_bytes(W, N, Cm, Rm, Km, 2, true, span);
    const size_t b = ((unit1_lds_bytes(W, N, Cm, Rm, Km, 8, span) + 15) & ~size_t(15)) + ((2 * F + 15) & ~size_t(15)) +
                     4 * (size_t)(Cm + 1) * (N + 1);
    return ((a > b ? a : b) + 15) & ~size_t(15);
}

// True when unit u cannot hold any partition whose RS times are all <= bound (kInf: no time
// limit), so the unit can be skipped exactly.  Without blocks of tiles the RS of tile row j
// partition that full-width band, so they number at least ceil(A_j / (k a - 1)) (each RS area is
// below k a), at most floor(A_j / a) (each is at least a), at most Cm min(Kmax, h_j) (c <= Cm
// tiles of at most min(Kmax, h_j) slices), and at least ceil(T_j / bound); the bands' ranges
// must hold N.  One lane per band, sums across the wave; every wave computes the same answer.
__device__ bool unit_infeasible(const LitView &v, const LitWs &w, int u, long long bound)
{
    const int lane = threadIdx.x & 63;
    const int wi = u / v.nY, yi = u % v.nY;
    const unsigned char *yt = v.ytab + (size_t)yi * v.yrow;
    const int r = yt[0];
    const long long a = v.win[wi], k = v.karea;
    long long lo = 0, hi = 0;
    for (int j = lane; j < r; j += 64) {
        const int y0 = yt[1 + j], y1 = yt[2 + j];
        const long long A = (long long)v.colpx[v.W] * (v.rowpx[y1] - v.rowpx[y0]);
        long long mn = 1, mx = (long long)v.Cm * (v.Km < y1 - y0 ? v.Km : y1 - y0);
        if (k > 0) {
            const long long amax = k * a - 1;                      // largest area an RS may have
            const long long need = (A + amax - 1) / amax;
            mn = need > mn ? need : mn;
            mx = A / a < mx ? A / a : mx;
        }
        if (bound != kInf && bound > 0) {
            const long long T = w.rT[(size_t)sidx(0, v.W, v.W) * v.R2 + ridx(y0, y1, v.H)];
            const long long need = (T + bound - 1) / bound;
            mn = need > mn ? need : mn;
        }
        lo += mn;
        hi += mx < mn ? -(1ll << 40) : mx;                         // an empty range fails the test
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        lo += __shfl_xor(lo, m, 64);
        hi += __shfl_xor(hi, m, 64);
    }
    return lo > v.N || hi < v.N;
}

// One work-group of BS threads per unit: one wave in step 1 (many units run, throughput counts),
// four in step 2 (few units run, their latency counts).  NB: the register rows' length bucket
// (N <= NB), a template parameter of the kernel so that each launch is allocated the registers
// of its own bucket only.  The pruning bounds are read once and shared through LDS: the waves
// of a work-group must take the same branches around their barriers.
template <int STEP, class V1, int NB, int BS = STEP == 1 ? 64 : 256>
__global__ void __launch_bounds__(BS)
k_lit_units(LitView v, LitWs w)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int Yl[kMaxH + 1];
    __shared__ unsigned long long bound_sh;
    const int p = v.dorder[blockIdx.x];                 // position in the kept list
    const int u = v.ulist[p];                           // unit: window u / nY, row boundaries u % nY
    if (threadIdx.x == 0)
        bound_sh = __atomic_load_n(&w.hdr[STEP == 1 ? 0 : 3], __ATOMIC_RELAXED);
    __syncthreads();
    long long bt = kInf, bq = kInf;
    if (STEP == 1) {
        const unsigned long long best = bound_sh;
        if (best != kNone) bt = v.lam_num < 0 ? (long long)best : (long long)eq4_bound(best, v.lam_num, v.lam_den);
        if ((w.hdr[4] != 0) != (sizeof(V1) == 4)) return;     // the other launch takes this frame
        if (!v.span && unit_infeasible(v, w, u, bt)) {
            if (threadIdx.x == 0) w.uT[p] = kInf;
            return;
        }
    } else {
        const unsigned long long tmin = w.hdr[0];
        if (tmin == kNone) return;
        const unsigned long long tau = eq4_bound(tmin, v.lam_num, v.lam_den);
        if (v.lam_num >= 0 && (unsigned long long)w.uT[p] > tau) {       // no candidate within Eq. 4
            if (threadIdx.x == 0) { w.uQ[p] = kInf; w.uT[p] = kInf; w.uC[p] = 0; }
            return;
        }
        // the Q bound prunes exactly only while every q >= 0 (Q of a partial partition then
        // only grows)
        const unsigned long long qb = bound_sh;
        if (qb != kNone && w.hdr[5] == 0) bq = (long long)qb;
    }
    if (v.work && threadIdx.x == 0)
        atomicAdd(v.work + (STEP - 1), (unsigned long long)(v.ytab[(size_t)(u % v.nY) * v.yrow] * v.relaxA + v.relaxB));
    int r = 0;
    __shared__ long long res[2];
    __shared__ int res_c;
    const Pack none{};
    if (STEP == 1) {
        if (v.span) unit_dp1<V1, NB, true, 1, false>(v, w, u, lds_raw, Yl, r, bt, none, nullptr, nullptr, nullptr, res, &res_c);
        else unit_dp1<V1, NB, false, 1, false>(v, w, u, lds_raw, Yl, r, bt, none, nullptr, nullptr, nullptr, res, &res_c);
        __syncthreads();
        if (threadIdx.x != 0) return;
        w.uT[p] = res[0];                               // the unit's own minimum (kInf if pruned)
        if (res[0] != kInf) {
            atomicMin(w.hdr, (unsigned long long)res[0]);
            atomicMin(reinterpret_cast<unsigned long long *>(w.wT + u / v.nY), (unsigned long long)res[0]);
        }
        return;
    }
    Pack pk{};
    long long ct = kInf, cq = kInf;
    int bc = 0;
    if (pack_for(v, w, pk)) {
        using U = unsigned long long;
        if (v.span) unit_dp1<U, NB, true, 2, false>(v, w, u, lds_raw, Yl, r, bq, pk, nullptr, nullptr, nullptr, res, &res_c);
        else unit_dp1<U, NB, false, 2, false>(v, w, u, lds_raw, Yl, r, bq, pk, nullptr, nullptr, nullptr, res, &res_c);
        __syncthreads();
        if (threadIdx.x != 0) return;
        cq = res[0];
        ct = res[1];
        bc = res_c;
    } else {
        const UnitLds L = unit_lds(lds_raw, v.W, v.N, v.Cm, v.Rm, v.Km, STEP, false, v.span);
        if (v.span) unit_dp<STEP, false, true>(v, w, u, L, Yl, r, bt, bq);
        else unit_dp<STEP, false, false>(v, w, u, L, Yl, r, bt, bq);
        if (threadIdx.x != 0) return;
        for (int c = 1; c <= v.Cm; c++) {
            const size_t f = ((size_t)c * (v.W + 1) + v.W) * (v.N + 1) + v.N;
            const long long t = L.FT[f], q = STEP == 2 ? L.FQ[f] : 0;
            if (t != kInf && better<STEP>(q, t, cq, ct)) { ct = t; cq = q; bc = c; }
        }
    }
    w.uQ[p] = cq;
    w.uT[p] = ct;
    w.uC[p] = bc;
    if (ct != kInf) atomicMin(w.hdr + 3, (unsigned long long)cq);
}

// Lexicographic minimum of (Q, T~, unit) over the kept units (their list is in unit order, so
// the least position is the first unit).
__global__ void __launch_bounds__(1024)
k_lit_pick(LitView v, LitWs w)
{
    __shared__ long long sq[1024], st[1024];
    __shared__ int su[1024];
    if (w.hdr[0] == kNone) return;
    long long bq = kInf, bt = kInf;
    int bu = INT_MAX;
    // eight units per thread in flight (the comparison includes the position, so the order in
    // which a thread visits its units does not matter)
    constexpr int kPer = 8;
    for (int u0 = threadIdx.x; u0 < v.n_units; u0 += kPer * blockDim.x) {
        long long qv[kPer], tv[kPer];
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            const int u = u0 + j * (int)blockDim.x;
            qv[j] = u < v.n_units ? w.uQ[u] : kInf;
            tv[j] = u < v.n_units ? w.uT[u] : kInf;
        }
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            const int u = u0 + j * (int)blockDim.x;
            const long long q = qv[j], t = tv[j];
            if (q == kInf) continue;
            if (q < bq || (q == bq && (t < bt || (t == bt && u < bu)))) { bq = q; bt = t; bu = u; }
        }
    }
    sq[threadIdx.x] = bq;
    st[threadIdx.x] = bt;
    su[threadIdx.x] = bu;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const int o = threadIdx.x + h;
            const long long q = sq[o], t = st[o];
            const int uu = su[o];
            if (q < sq[threadIdx.x] || (q == sq[threadIdx.x] && (t < st[threadIdx.x] ||
                                                              (t == st[threadIdx.x] && uu < su[threadIdx.x])))) {
                sq[threadIdx.x] = q;
                st[threadIdx.x] = t;
                su[threadIdx.x] = uu;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && su[0] != INT_MAX) {
        w.hdr[1] = (unsigned long long)su[0];
        w.hdr[2] = (unsigned long long)w.uC[su[0]];
    }
}

// ---------------------------------------------------------------------------------------
// Rebuild the winner and write the result (four waves share the unit's DP; lane 0 walks the
// argmins back).
__host__ __device__ inline size_t final_lds_bytes(int W, int H, int N, int Cm, int Rm, int Km, int span)
{
    const size_t knap = (size_t)(Rm + 1) * (N + 1), tile = (size_t)(Km + 1) * (H + 1);
    return rec_lds_bytes(W, N, Cm, Rm, Km, span) + ((17 * knap + 15) & ~size_t(15)) + 20 * tile +
           (size_t)Rm * Cm + 16 + 24 * (size_t)(H + 1) * (H + 1) + 16;
}

constexpr int kFinalThreads = 256;

__global__ void __launch_bounds__(kFinalThreads)
k_lit_final(LitView v, LitWs w, trs_result *out)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int Yl[kMaxH + 1];
    __shared__ __align__(16) trs_result res;
    __shared__ int cx[kMaxW + 1], ck[kMaxW + 1];
    const int lane = threadIdx.x;
    const int W = v.W, H = v.H, N = v.N, Km = v.Km;
    {
        unsigned *z = reinterpret_cast<unsigned *>(&res);
        for (size_t e = lane; e < sizeof(trs_result) / 4; e += blockDim.x) z[e] = 0;
    }
    const UnitLds L = unit_lds(lds_raw, W, N, v.Cm, v.Rm, Km, 2, true, v.span);
    unsigned char *extra = lds_raw + rec_lds_bytes(W, N, v.Cm, v.Rm, Km, v.span);
    const size_t knap = (size_t)(v.Rm + 1) * (N + 1), tile = (size_t)(Km + 1) * (H + 1);
    long long *kT = reinterpret_cast<long long *>(extra), *kQ = kT + knap;
    unsigned char *kC = reinterpret_cast<unsigned char *>(kQ + knap);
    long long *fT = reinterpret_cast<long long *>(extra + ((17 * knap + 15) & ~size_t(15)));
    long long *fQ = fT + tile;
    int *fA = reinterpret_cast<int *>(fQ + tile);
    unsigned char *tcnt = reinterpret_cast<unsigned char *>(fA + tile);    // [row][column] slice counts
    __syncthreads();
    const unsigned long long tmin = w.hdr[0];
    const bool feasible = tmin != kNone && w.hdr[1] != kNone;
    int r = 0;
    // argmins of the column DP: the packed DP's when the keys fit, else the serial DP's
    const unsigned char *AX = L.AX, *AK = L.AK;
    if (feasible) {
        Pack pk{};
        if (pack_for(v, w, pk)) {
            const size_t F = (size_t)(v.Cm + 1) * (W + 1) * (N + 1);
            unsigned char *ax = lds_raw + ((unit1_lds_bytes(W, N, v.Cm, v.Rm, Km, 8, v.span) + 15) & ~size_t(15));
            unsigned char *ak = ax + F;
            unsigned *axk = reinterpret_cast<unsigned *>(ax + ((2 * F + 15) & ~size_t(15)));
            __shared__ long long res2[2];
            __shared__ int res2_c;
            using U = unsigned long long;
            const int u = v.ulist[(int)w.hdr[1]];
            if (v.span) {
                if (N <= 8) unit_dp1<U, 8, true, 2, true>(v, w, u, lds_raw, Yl, r, kInf, pk, ax, ak, axk, res2, &res2_c);
                else if (N <= 16) unit_dp1<U, 16, true, 2, true>(v, w, u, lds_raw, Yl, r, kInf, pk, ax, ak, axk, res2, &res2_c);
                else unit_dp1<U, kMaxN, true, 2, true>(v, w, u, lds_raw, Yl, r, kInf, pk, ax, ak, axk, res2, &res2_c);
            } else {
                if (N <= 8) unit_dp1<U, 8, false, 2, true>(v, w, u, lds_raw, Yl, r, kInf, pk, ax, ak, axk, res2, &res2_c);
                else if (N <= 16) unit_dp1<U, 16, false, 2, true>(v, w, u, lds_raw, Yl, r, kInf, pk, ax, ak, axk, res2, &res2_c);
                else unit_dp1<U, kMaxN, false, 2, true>(v, w, u, lds_raw, Yl, r, kInf, pk, ax, ak, axk, res2, &res2_c);
            }
            AX = ax;
            AK = ak;
        } else if (v.span) {
            unit_dp<2, true, true>(v, w, v.ulist[(int)w.hdr[1]], L, Yl, r, kInf, kInf);
        } else {
            unit_dp<2, true, false>(v, w, v.ulist[(int)w.hdr[1]], L, Yl, r, kInf, kInf);
        }
    }
    __syncthreads();
    if (lane == 0) {
        auto rect_at = [&](const long long *a, int x0, int x1, int y0, int y1) {
            return a[(size_t)sidx(x0, x1, W) * v.R2 + ridx(y0, y1, H)];
        };
        res.rank = -1;
        res.n_enumerated = v.n_enumerated;
        res.n_feasible = -1;
        res.n_step2 = v.n_units;
        res.uniform_rank = -1;
        res.dtile_used = -1;
        res.drs_used = -1;
        // uniform grid (Section 3.2): c_u r_u = N, most square, c_u >= r_u, one RS per tile
        int ru = 1;
        for (int d = 1; d * d <= N; d++) if (N % d == 0) ru = d;
        const int cu = N / ru;
        long long ut = -1, uq = -1;
        if (cu <= W && ru <= H) {
            ut = 0;
            uq = 0;
            for (int j = 0; j < ru; j++)
                for (int i = 0; i < cu; i++) {
                    const int x0 = i * W / cu, x1 = (i + 1) * W / cu, y0 = j * H / ru, y1 = (j + 1) * H / ru;
                    const long long t = rect_at(w.rT, x0, x1, y0, y1);
                    if (t > ut) ut = t;
                    uq += rect_at(w.rQ, x0, x1, y0, y1);
                }
        }
        res.t_unif = ut;
        res.q_unif = uq;
        if (!feasible) {
            res.status = TRS_ENOFEASIBLE;
            res.t_min = -1;
            res.t_sel = ut;
            res.q_sel = uq;
            if (ut >= 0) {
                res.tile_cols = cu;
                res.tile_rows = ru;
                for (int i = 0; i <= cu; i++) res.col_bd[i] = i * W / cu;
                for (int j = 0; j <= ru; j++) res.row_bd[j] = j * H / ru;
                int n = 0;
                for (int j = 0; j < ru; j++)
                    for (int i = 0; i < cu; i++, n++) {
                        res.rs[n][0] = res.col_bd[i];
                        res.rs[n][1] = res.row_bd[j];
                        res.rs[n][2] = res.col_bd[i + 1];
                        res.rs[n][3] = res.row_bd[j + 1];
                        res.rs_time[n] = rect_at(w.rT, res.rs[n][0], res.rs[n][2], res.rs[n][1], res.rs[n][3]);
                    }
                res.n_rs = n;
            }
        } else {
            const int c = (int)w.hdr[2];
            // column boundaries and RS count per strip, from the column DP's argmins
            int x = W, n = N;
            cx[c] = W;
            for (int i = c; i > 0; i--) {
                const size_t f = ((size_t)i * (W + 1) + x) * (N + 1) + n;
                cx[i - 1] = AX[f];
                ck[i - 1] = AK[f];
                x = cx[i - 1];
                n -= ck[i - 1];
            }
            res.tile_cols = c;
            res.tile_rows = r;
            for (int i = 0; i <= c; i++) res.col_bd[i] = cx[i];
            for (int j = 0; j <= r; j++) res.row_bd[j] = Yl[j];
        }
    }
    __syncthreads();
    // Tiles in raster order, slices top to bottom.  For a tile cut into slices, all lanes copy
    // its rectangles' area, time and q into LDS and redo the tile DP from there, then lane 0
    // emits the slices (a block of tiles is emitted at its top tile).
    if (feasible) {
        const int c = (int)w.hdr[2];
        const int wi = v.ulist[(int)w.hdr[1]] / v.nY;
        const unsigned long long tau = eq4_bound(tmin, v.lam_num, v.lam_den);
        const long long lo = v.win[wi];
        const long long hi = v.karea ? (long long)v.karea * lo : kInf;
        constexpr int kBlock = 100;                       // above every slice count (k <= H <= 40)
        auto rect_at = [&](const long long *a, int x0, int x1, int y0, int y1) {
            return a[(size_t)sidx(x0, x1, W) * v.R2 + ridx(y0, y1, H)];
        };
        auto ok = [&](int x0, int x1, int y0, int y1) {
            const long long A = rect_at(w.rA, x0, x1, y0, y1);
            return A >= lo && A < hi && (unsigned long long)rect_at(w.rT, x0, x1, y0, y1) <= tau;
        };
        // Every tile of a strip: its slice count k, or (blocks) kBlock + b on the top tile of a
        // block of tiles ending at tile row b and 0 inside it.  A DP over the tile-row levels,
        // strip by strip, the lanes taking the RS counts K of a level; per (level, K) tiles are
        // tried first (k ascending), then blocks (a ascending), first minimum kept.  Lane 0 walks
        // the choices back.
        for (int i = 0; i < c; i++) {
            const size_t sb = (size_t)wi * v.S + sidx(cx[i], cx[i + 1], W);
            for (int K = lane; K <= N; K += blockDim.x) {
                kT[K] = K == 0 ? 0 : kInf;
                kQ[K] = K == 0 ? 0 : kInf;
            }
            __syncthreads();
            for (int b = 1; b <= r; b++) {
                const size_t tb = (sb * v.R2 + ridx(Yl[b - 1], Yl[b], H)) * Km;
                for (int K = lane; K <= N; K += blockDim.x) {
                    long long bt = kInf, bq = kInf;
                    int bk = 0;
                    for (int k = 1; k <= Km && k <= K; k++) {
                        const long long at = kT[(b - 1) * (N + 1) + K - k], ct = w.tT[tb + k - 1];
                        if (at == kInf || ct == kInf) continue;
                        const long long t = at > ct ? at : ct;
                        const long long q = kQ[(b - 1) * (N + 1) + K - k] + w.tQ[tb + k - 1];
                        if (better<2>(q, t, bq, bt)) { bt = t; bq = q; bk = k; }
                    }
                    if (v.span && K >= 1)
                        for (int a = 0; a + 2 <= b; a++) {
                            if (!ok(cx[i], cx[i + 1], Yl[a], Yl[b])) continue;
                            const long long at = kT[a * (N + 1) + K - 1];
                            if (at == kInf) continue;
                            const long long bT = rect_at(w.rT, cx[i], cx[i + 1], Yl[a], Yl[b]);
                            const long long t = at > bT ? at : bT;
                            const long long q = kQ[a * (N + 1) + K - 1] + rect_at(w.rQ, cx[i], cx[i + 1], Yl[a], Yl[b]);
                            if (better<2>(q, t, bq, bt)) { bt = t; bq = q; bk = kBlock + a; }
                        }
                    kT[b * (N + 1) + K] = bt;
                    kQ[b * (N + 1) + K] = bq;
                    kC[b * (N + 1) + K] = (unsigned char)bk;
                }
                __syncthreads();
            }
            if (lane == 0) {
                for (int j = 0; j < r; j++) tcnt[j * v.Cm + i] = 0;
                for (int b = r, K = ck[i]; b > 0;) {
                    const int ch = kC[b * (N + 1) + K];
                    if (ch < kBlock) {
                        tcnt[(b - 1) * v.Cm + i] = (unsigned char)ch;
                        K -= ch;
                        b -= 1;
                    } else {
                        const int a = ch - kBlock;
                        tcnt[a * v.Cm + i] = (unsigned char)(kBlock + b);
                        K -= 1;
                        b = a;
                    }
                }
            }
            __syncthreads();                          // the next strip reuses the DP levels
        }
        long long *sA = reinterpret_cast<long long *>(                  // after tcnt
            (reinterpret_cast<uintptr_t>(tcnt + (size_t)v.Rm * v.Cm) + 15) & ~uintptr_t(15));
        const int HP = H + 1;
        long long *sT = sA + (size_t)HP * HP, *sQ = sT + (size_t)HP * HP;
        int nrs = 0;
        long long tsel = 0, qsel = 0;
        for (int j = 0; j < r; j++)
            for (int i = 0; i < c; i++) {
                const int kq = tcnt[j * v.Cm + i];
                if (kq == 0) continue;                                  // inside a block
                const int x0 = cx[i], x1 = cx[i + 1];
                if (kq >= kBlock) {                                     // a block of tiles j .. b - 1
                    if (lane == 0) {
                        const int yb = Yl[kq - kBlock];
                        const size_t ri = (size_t)sidx(x0, x1, W) * v.R2 + ridx(Yl[j], yb, H);
                        const long long t = w.rT[ri];
                        res.rs[nrs][0] = x0;
                        res.rs[nrs][1] = Yl[j];
                        res.rs[nrs][2] = x1;
                        res.rs[nrs][3] = yb;
                        res.rs_time[nrs] = t;
                        if (t > tsel) tsel = t;
                        qsel += w.rQ[ri];
                        nrs++;
                    }
                    continue;
                }
                const int y0 = Yl[j], y1 = Yl[j + 1], hh = y1 - y0;
                const size_t sb = (size_t)sidx(x0, x1, W) * v.R2;
                for (int e = lane; e < (hh + 1) * (hh + 1); e += blockDim.x) {
                    const int ya = y0 + e / (hh + 1), yb = y0 + e % (hh + 1);
                    if (ya >= yb) continue;
                    const size_t ri = sb + ridx(ya, yb, H);
                    sA[(ya - y0) * HP + (yb - y0)] = w.rA[ri];
                    sT[(ya - y0) * HP + (yb - y0)] = w.rT[ri];
                    sQ[(ya - y0) * HP + (yb - y0)] = w.rQ[ri];
                }
                // the tile's split DP, the lanes taking the end rows y of a level (first
                // minimum over the split rows yp in ascending order, as in the oracle)
                auto ok = [&](int ya, int yb) {
                    const long long A = sA[(ya - y0) * HP + (yb - y0)];
                    return A >= lo && A < hi && (unsigned long long)sT[(ya - y0) * HP + (yb - y0)] <= tau;
                };
                auto at = [&](int q, int y) { return (size_t)q * (H + 1) + y; };
                for (int e = lane; e < (kq + 1) * (hh + 1); e += blockDim.x) {
                    const int q = e / (hh + 1), y = y0 + e % (hh + 1);
                    const bool start = q == 0 && y == y0;
                    fT[at(q, y)] = start ? 0 : kInf;
                    fQ[at(q, y)] = start ? 0 : kInf;
                    fA[at(q, y)] = -1;
                }
                __syncthreads();
                for (int q = 1; q <= kq; q++) {
                    for (int y = y0 + q + lane; y <= y1; y += blockDim.x) {
                        long long bt = kInf, bq = kInf;
                        int ba = -1;
                        for (int yp = y0 + q - 1; yp < y; yp++) {
                            if (fT[at(q - 1, yp)] == kInf || !ok(yp, y)) continue;
                            const long long st = sT[(yp - y0) * HP + (y - y0)];
                            const long long t = fT[at(q - 1, yp)] > st ? fT[at(q - 1, yp)] : st;
                            const long long qq = fQ[at(q - 1, yp)] + sQ[(yp - y0) * HP + (y - y0)];
                            if (better<2>(qq, t, bq, bt)) { bt = t; bq = qq; ba = yp; }
                        }
                        fT[at(q, y)] = bt;
                        fQ[at(q, y)] = bq;
                        fA[at(q, y)] = ba;
                    }
                    __syncthreads();
                }
                if (lane == 0) {
                    int rows[kMaxH + 1];
                    rows[kq] = y1;
                    for (int q = kq, y = y1; q > 0; q--) { y = fA[at(q, y)]; rows[q - 1] = y; }
                    for (int q = 0; q < kq; q++) {
                        const long long t = sT[(rows[q] - y0) * HP + (rows[q + 1] - y0)];
                        res.rs[nrs][0] = x0;
                        res.rs[nrs][1] = rows[q];
                        res.rs[nrs][2] = x1;
                        res.rs[nrs][3] = rows[q + 1];
                        res.rs_time[nrs] = t;
                        if (t > tsel) tsel = t;
                        qsel += sQ[(rows[q] - y0) * HP + (rows[q + 1] - y0)];
                        nrs++;
                    }
                }
                __syncthreads();
            }
        if (lane == 0) {
            res.n_rs = nrs;
            res.status = TRS_OK;
            res.t_min = (long long)tmin;
            res.t_sel = tsel;
            res.q_sel = qsel;
        }
    }
    __syncthreads();
    const unsigned *src = reinterpret_cast<const unsigned *>(&res);
    unsigned *dst = reinterpret_cast<unsigned *>(out);
    for (size_t e = lane; e < sizeof(trs_result) / 4; e += blockDim.x) dst[e] = src[e];
}

// ---------------------------------------------------------------------------------------
// Host side: the plan (geometry, windows, row-boundary list), cached per geometry and
// parameters with one device copy per device, and the workspace layout.
struct LitPlan {
    int W = 0, H = 0, N = 0, Cm = 0, Rm = 0, Km = 0, S = 0, R2 = 0, karea = 0, yrow = 0, span = 0;
    long long n_win = 0, nY = 0, n_units = 0, n_enumerated = 0;
    std::vector<int> colpx, rowpx;
    std::vector<long long> win;
    std::vector<int> ulist, dorder, wlive;
    std::vector<unsigned char> ytab, strip_xy, row_yy;
    std::vector<char> blob;             // the tables above, packed for the device copy
    size_t o_col = 0, o_row = 0, o_win = 0, o_y = 0, o_sx = 0, o_ry = 0, o_ul = 0, o_do = 0, o_wl = 0;
    std::map<int, void *> dev;          // device copies of the tables
};

struct WsLayout {
    size_t hdr, sat, rA, rT, rQ, tT, tQ, uQ, uT, uC, wT, bytes;
};

std::mutex g_mu;
std::map<std::vector<long long>, LitPlan> g_plans;

// Stage timing while profiling is on: events around the launches of every search.
constexpr int kStages = 7;     // prefix sums + rectangles, tiles 1, units 1, tiles 2, units 2, pick, final
std::mutex g_prof_mu;
bool g_prof_on = false;
struct ProfRun {
    std::array<hipEvent_t, kStages + 1> ev;
    unsigned long long *work;           // device: relaxations run in step 1 and step 2
};
std::vector<ProfRun> g_prof_ev;

trs_status check_args(const trs_frame *f, const trs_search_params *p)
{
    trs_status st = check_space_args(f, p);
    if (st != TRS_OK) return st;
    if (p->dtile != -1 || p->drs != -1) return TRS_EINVAL;          // the literal space only
    if (p->prune != 0 || (p->min_rs != 0 && p->min_rs != p->n_threads)) return TRS_ENOTIMPL;
    // (span_tiles is taken: check_space_args has checked it is 0 or 1)
    const int W = (f->width + f->ctu_size - 1) / f->ctu_size, H = (f->height + f->ctu_size - 1) / f->ctu_size;
    if (W > kMaxW || H > kMaxH || p->n_threads > kMaxN) return TRS_ENOTIMPL;
    return TRS_OK;
}

unsigned long long sat_add(unsigned long long a, unsigned long long b)
{
    return a > ~0ull - b ? ~0ull : a + b;
}

unsigned long long sat_mul(unsigned long long a, unsigned long long b)
{
    return a && b > ~0ull / a ? ~0ull : a * b;
}

unsigned long long binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    unsigned __int128 c = 1;                                 // exact for n <= 64
    for (int i = 1; i <= k; i++) c = c * (unsigned)(n - k + i) / (unsigned)i;
    return c > ~0ull ? ~0ull : (unsigned long long)c;
}

// |C| of the literal space with blocks of tiles: for every row-boundary vector Y (the plan's
// list), cover(Y)[n] = ways to cover one tile column with n RS, levels taken one tile row at a
// time (a tile of h rows into k slices: C(h - 1, k - 1) ways) or as blocks of >= 2 tile rows;
// then sum over c of C(W - 1, c - 1) times the coefficient of z^N in cover(Y)^c.  Saturating.
long long span_count(const LitPlan &pl, int max_cols)
{
    const int N = pl.N, r_max = pl.Rm;
    unsigned long long total = 0;
    std::vector<unsigned long long> cov((size_t)(r_max + 1) * (N + 1)), pw(N + 1), nx(N + 1);
    for (long long yi = 0; yi < pl.nY; yi++) {
        const unsigned char *yt = &pl.ytab[(size_t)yi * pl.yrow];
        const int r = yt[0];
        std::fill(cov.begin(), cov.end(), 0ull);
        cov[0] = 1;
        for (int b = 1; b <= r; b++)
            for (int n = 0; n <= N; n++) {
                unsigned long long acc = 0;
                const int h = yt[1 + b] - yt[b];
                for (int k = 1; k <= pl.Km && k <= h && k <= n; k++)
                    acc = sat_add(acc, sat_mul(cov[(size_t)(b - 1) * (N + 1) + n - k], binom(h - 1, k - 1)));
                if (n >= 1)
                    for (int a = 0; a + 2 <= b; a++) acc = sat_add(acc, cov[(size_t)a * (N + 1) + n - 1]);
                cov[(size_t)b * (N + 1) + n] = acc;
            }
        std::fill(pw.begin(), pw.end(), 0ull);
        pw[0] = 1;
        for (int c = 1; c <= max_cols && c <= pl.W; c++) {
            std::fill(nx.begin(), nx.end(), 0ull);
            for (int a = 0; a <= N; a++)
                if (pw[a])
                    for (int b = 0; a + b <= N; b++)
                        nx[a + b] = sat_add(nx[a + b], sat_mul(pw[a], cov[(size_t)r * (N + 1) + b]));
            pw.swap(nx);
            total = sat_add(total, sat_mul(binom(pl.W - 1, c - 1), pw[N]));
        }
    }
    return total > (unsigned long long)LLONG_MAX ? LLONG_MAX : (long long)total;
}

trs_status build(const trs_frame *f, const trs_search_params *p, LitPlan &pl)
{
    const int cs = f->ctu_size;
    pl.W = (f->width + cs - 1) / cs;
    pl.H = (f->height + cs - 1) / cs;
    pl.N = p->n_threads;
    pl.Cm = std::min(p->max_tile_cols, pl.W);
    pl.Rm = std::min(p->max_tile_rows, pl.H);
    pl.Km = std::min(p->max_rs_per_tile, pl.H);
    pl.karea = p->area_k;
    pl.span = p->span_tiles;
    pl.S = pl.W * (pl.W + 1) / 2;
    pl.R2 = pl.H * (pl.H + 1) / 2;
    pl.colpx.assign(pl.W + 1, 0);
    pl.rowpx.assign(pl.H + 1, 0);
    for (int x = 0; x < pl.W; x++) pl.colpx[x + 1] = pl.colpx[x] + std::min(cs, f->width - x * cs);
    for (int y = 0; y < pl.H; y++) pl.rowpx[y + 1] = pl.rowpx[y] + std::min(cs, f->height - y * cs);
    pl.strip_xy.resize(2 * (size_t)pl.S);
    for (int x0 = 0; x0 < pl.W; x0++)
        for (int x1 = x0 + 1; x1 <= pl.W; x1++) {
            const int s = sidx(x0, x1, pl.W);
            pl.strip_xy[2 * s] = (unsigned char)x0;
            pl.strip_xy[2 * s + 1] = (unsigned char)x1;
        }
    pl.row_yy.resize(2 * (size_t)pl.R2);
    for (int y0 = 0; y0 < pl.H; y0++)
        for (int y1 = y0 + 1; y1 <= pl.H; y1++) {
            const int q = ridx(y0, y1, pl.H);
            pl.row_yy[2 * q] = (unsigned char)y0;
            pl.row_yy[2 * q + 1] = (unsigned char)y1;
        }
    if (unit2_lds_bytes(pl.W, pl.N, pl.Cm, pl.Rm, pl.Km, pl.span) > kLdsLimit - 1024 ||
        final_lds_bytes(pl.W, pl.H, pl.N, pl.Cm, pl.Rm, pl.Km, pl.span) > kLdsLimit - 4 * 1024 ||
        (size_t)7 * 8 * pl.R2 > kLdsLimit)
        return TRS_ENOTIMPL;
    // windows: distinct RS areas a with N a <= A_total < k N a (all areas when k = 0: one window)
    std::vector<long long> areas;
    for (int x0 = 0; x0 < pl.W; x0++)
        for (int x1 = x0 + 1; x1 <= pl.W; x1++)
            for (int y0 = 0; y0 < pl.H; y0++)
                for (int y1 = y0 + 1; y1 <= pl.H; y1++)
                    areas.push_back((long long)(pl.colpx[x1] - pl.colpx[x0]) * (pl.rowpx[y1] - pl.rowpx[y0]));
    std::sort(areas.begin(), areas.end());
    areas.erase(std::unique(areas.begin(), areas.end()), areas.end());
    const long long At = (long long)pl.colpx[pl.W] * pl.rowpx[pl.H], N = pl.N;
    pl.win.clear();
    if (pl.karea == 0) pl.win.push_back(0);
    else
        for (long long a : areas)
            if (N * a <= At && (long long)pl.karea * N * a > At) pl.win.push_back(a);
    pl.n_win = (long long)pl.win.size();
    // row boundaries: r = 1 .. Rm, each Y increasing from 0 to H, lexicographic
    pl.yrow = pl.Rm + 2;
    pl.ytab.clear();
    std::vector<int> Y(pl.Rm + 1);
    for (int r = 1; r <= pl.Rm; r++) {
        for (int j = 0; j < r; j++) Y[j] = j;
        Y[r] = pl.H;
        while (true) {
            pl.ytab.push_back((unsigned char)r);
            for (int j = 0; j <= r; j++) pl.ytab.push_back((unsigned char)Y[j]);
            for (int j = r + 1; j <= pl.Rm; j++) pl.ytab.push_back(0);
            if ((long long)pl.ytab.size() / pl.yrow * std::max<long long>(pl.n_win, 1) > kUnitCap)
                return TRS_ENOSPACE;
            int j = r - 1;
            while (j >= 1 && Y[j] >= pl.H - (r - j)) j--;
            if (j < 1) break;
            Y[j]++;
            for (int q = j + 1; q < r; q++) Y[q] = Y[q - 1] + 1;
        }
    }
    pl.nY = (long long)pl.ytab.size() / pl.yrow;
    if (pl.n_win * pl.nY > kUnitCap) return TRS_ENOSPACE;
    // Units kept: without blocks of tiles the RS of tile row j partition that full-width band of
    // area A_j, so they number at least max(1, ceil(A_j / (k a - 1))) and at most
    // min(Cm min(Km, h_j), floor(A_j / a)); a unit whose bands' ranges cannot hold N RS has no
    // candidate and is dropped here (this part of the test depends on the geometry alone; the
    // kernel adds the time bound).  With blocks every unit is kept.
    pl.ulist.clear();
    std::vector<long long> wstart(pl.n_win + 1, 0);
    for (long long wi = 0; wi < pl.n_win; wi++) {
        wstart[wi] = (long long)pl.ulist.size();
        const long long a = pl.win[wi], k = pl.karea;
        for (long long yi = 0; yi < pl.nY; yi++) {
            bool keep = true;
            if (!pl.span) {
                const unsigned char *yt = &pl.ytab[(size_t)yi * pl.yrow];
                long long lo = 0, hi = 0;
                for (int j = 0; j < yt[0]; j++) {
                    const int y0 = yt[1 + j], y1 = yt[2 + j];
                    const long long A = (long long)pl.colpx[pl.W] * (pl.rowpx[y1] - pl.rowpx[y0]);
                    long long mn = 1, mx = (long long)pl.Cm * std::min(pl.Km, y1 - y0);
                    if (k > 0) {
                        mn = std::max(mn, (A + k * a - 2) / (k * a - 1));
                        mx = std::min(mx, A / a);
                    }
                    lo += mn;
                    hi += mx < mn ? -(1ll << 40) : mx;
                }
                keep = lo <= N && hi >= N;
            }
            if (keep) pl.ulist.push_back((int)(wi * pl.nY + yi));
        }
    }
    wstart[pl.n_win] = (long long)pl.ulist.size();
    pl.n_units = (long long)pl.ulist.size();
    pl.wlive.clear();
    for (long long wi = 0; wi < pl.n_win; wi++)
        if (wstart[wi + 1] > wstart[wi]) pl.wlive.push_back((int)wi);
    // Dispatch order (speed only: ties are broken by unit order): windows nearest first to 3/4 of
    // the mean RS area, where the smallest area of a balanced partition tends to lie, so that the
    // pruning bounds tighten early; inside a window, unit order.
    {
        std::vector<int> wo(pl.n_win);
        for (long long i = 0; i < pl.n_win; i++) wo[i] = (int)i;
        const double target = 0.75 * (double)At / (double)N;
        auto dist = [&](int i) { return std::fabs(std::log(std::max<double>((double)pl.win[i], 1.0) / target)); };
        std::stable_sort(wo.begin(), wo.end(), [&](int x, int y) { return dist(x) < dist(y); });
        pl.dorder.clear();
        for (int wi : wo)
            for (long long q = wstart[wi]; q < wstart[wi + 1]; q++) pl.dorder.push_back((int)q);
    }
    if (pl.span) {
        pl.n_enumerated = span_count(pl, p->max_tile_cols);
        return TRS_OK;
    }
    trs_search_params lp = *p;
    int32_t dt, dr;
    int64_t n = 0;
    trs_status st = space_size(pl.W, pl.H, &lp, &n, &dt, &dr);
    if (st != TRS_OK) return st;
    pl.n_enumerated = n;
    return TRS_OK;
}

template <int STEP, class V1>
void launch_units(int N, dim3 grid, size_t lds, hipStream_t stream, const LitView &v, const LitWs &w)
{
    const dim3 block(STEP == 1 ? 64 : 256);
    if (N <= 8) hipLaunchKernelGGL((k_lit_units<STEP, V1, 8>), grid, block, lds, stream, v, w);
    else if (N <= 16) hipLaunchKernelGGL((k_lit_units<STEP, V1, 16>), grid, block, lds, stream, v, w);
    else hipLaunchKernelGGL((k_lit_units<STEP, V1, kMaxN>), grid, block, lds, stream, v, w);
}

WsLayout layout(const LitPlan &pl)
{
    WsLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off += (bytes + 255) & ~size_t(255); return at; };
    const size_t nrect = (size_t)pl.S * pl.R2, ntab = (size_t)pl.n_win * nrect * pl.Km;
    L.hdr = take(256);
    L.sat = take(3 * 8 * (size_t)(pl.W + 1) * (pl.H + 1));
    L.rA = take(8 * nrect);
    L.rT = take(8 * nrect);
    L.rQ = take(8 * nrect);
    L.tT = take(8 * ntab);
    L.tQ = take(8 * ntab);
    L.uQ = take(8 * (size_t)std::max<long long>(pl.n_units, 1));
    L.uT = take(8 * (size_t)std::max<long long>(pl.n_units, 1));
    L.uC = take(4 * (size_t)std::max<long long>(pl.n_units, 1));
    L.wT = take(8 * (size_t)std::max<long long>(pl.n_win, 1));
    L.bytes = off;
    return L;
}

std::vector<long long> key_of(const trs_frame *f, const trs_search_params *p)
{
    return {f->width, f->height, f->ctu_size, p->n_threads, p->max_tile_cols, p->max_tile_rows,
            p->max_rs_per_tile, p->area_k, p->span_tiles};
}

// Plan for (f, p); caller holds g_mu.
trs_status plan_for(const trs_frame *f, const trs_search_params *p, LitPlan **out)
{
    const auto key = key_of(f, p);
    auto it = g_plans.find(key);
    if (it == g_plans.end()) {
        LitPlan pl;
        trs_status st = build(f, p, pl);
        if (st != TRS_OK) return st;
        it = g_plans.emplace(key, std::move(pl)).first;
    }
    *out = &it->second;
    return TRS_OK;
}

template <class T>
size_t put(std::vector<char> &blob, const std::vector<T> &v)
{
    const size_t at = (blob.size() + 15) & ~size_t(15);
    blob.resize(at + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + at, v.data(), v.size() * sizeof(T));
    return at;
}

trs_status view_of(LitPlan &pl, const trs_search_params *p, LitView *v)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TRS_EDEVICE;
    if (pl.blob.empty()) {
        pl.o_col = put(pl.blob, pl.colpx);
        pl.o_row = put(pl.blob, pl.rowpx);
        pl.o_win = put(pl.blob, pl.win);
        pl.o_y = put(pl.blob, pl.ytab);
        pl.o_sx = put(pl.blob, pl.strip_xy);
        pl.o_ry = put(pl.blob, pl.row_yy);
        pl.o_ul = put(pl.blob, pl.ulist);
        pl.o_do = put(pl.blob, pl.dorder);
        pl.o_wl = put(pl.blob, pl.wlive);
    }
    auto it = pl.dev.find(dev);
    if (it == pl.dev.end()) {
        void *d = nullptr;
        if (hipMalloc(&d, std::max<size_t>(pl.blob.size(), 16)) != hipSuccess) return TRS_EDEVICE;
        if (hipMemcpy(d, pl.blob.data(), pl.blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return TRS_EDEVICE;
        }
        it = pl.dev.emplace(dev, d).first;
    }
    const char *d = static_cast<const char *>(it->second);
    *v = LitView{};
    v->W = pl.W; v->H = pl.H; v->N = pl.N; v->Cm = pl.Cm; v->Rm = pl.Rm; v->Km = pl.Km;
    v->S = pl.S; v->R2 = pl.R2; v->n_win = (int)pl.n_win; v->nY = (int)pl.nY;
    v->n_units = (int)pl.n_units; v->n_wlive = (int)pl.wlive.size(); v->karea = pl.karea; v->yrow = pl.yrow; v->span = pl.span;
    v->lam_num = p->lambda_num < 0 ? -1 : p->lambda_num;
    v->lam_den = p->lambda_den;
    v->n_enumerated = pl.n_enumerated;
    // loop bounds of one unit: the strip DP relaxes min(Km, K) pairs per (x' < x, tile row, K),
    // the column DP n pairs per (i <= min(x, Cm), x' in [i - 1, x), n)
    long long knap = 0, colB = 0;
    for (int K = 0; K <= pl.N; K++) knap += std::min(pl.Km, K);
    for (int x = 1; x <= pl.W; x++)
        for (int i = 1; i <= std::min(x, pl.Cm); i++) colB += (long long)(x - i + 1) * pl.N * (pl.N + 1) / 2;
    v->relaxA = knap * pl.W * (pl.W + 1) / 2;
    v->relaxB = colB;
    v->colpx = reinterpret_cast<const int *>(d + pl.o_col);
    v->rowpx = reinterpret_cast<const int *>(d + pl.o_row);
    v->win = reinterpret_cast<const long long *>(d + pl.o_win);
    v->ytab = reinterpret_cast<const unsigned char *>(d + pl.o_y);
    v->strip_xy = reinterpret_cast<const unsigned char *>(d + pl.o_sx);
    v->row_yy = reinterpret_cast<const unsigned char *>(d + pl.o_ry);
    v->ulist = reinterpret_cast<const int *>(d + pl.o_ul);
    v->dorder = reinterpret_cast<const int *>(d + pl.o_do);
    v->wlive = reinterpret_cast<const int *>(d + pl.o_wl);
    return TRS_OK;
}

}  // namespace

void profile_enable(bool on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on;
}

void release_all()
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_plans)
        for (auto &d : kv.second.dev) (void)hipFree(d.second);
    g_plans.clear();
}

}  // namespace lit
}  // namespace trs

extern "C" trs_status trs_literal_workspace(const trs_frame *frame, const trs_search_params *params,
                                            size_t *bytes)
{
    using namespace trs::lit;
    if (!bytes) return TRS_EINVAL;
    trs_status st = check_args(frame, params);
    if (st != TRS_OK) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    LitPlan *pl = nullptr;
    st = plan_for(frame, params, &pl);
    if (st != TRS_OK) return st;
    *bytes = layout(*pl).bytes;
    return TRS_OK;
}

extern "C" trs_status trs_literal_search(const trs_frame *frame, const trs_search_params *params,
                                         const uint32_t *cost, const uint32_t *s1, const uint64_t *s2,
                                         void *workspace, size_t ws_bytes, trs_result *out_dev,
                                         hipStream_t stream)
{
    using namespace trs::lit;
    trs_status st = check_args(frame, params);
    if (st != TRS_OK) return st;
    if (!cost || !s1 || !s2 || !out_dev) return TRS_EINVAL;
    LitView v{};
    WsLayout L{};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        LitPlan *pl = nullptr;
        st = plan_for(frame, params, &pl);
        if (st != TRS_OK) return st;
        st = view_of(*pl, params, &v);
        if (st != TRS_OK) return st;
        L = layout(*pl);
    }
    if (!workspace || ws_bytes < L.bytes || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return TRS_EWORKSPACE;
    char *ws = static_cast<char *>(workspace);
    LitWs w{};
    w.hdr = reinterpret_cast<unsigned long long *>(ws + L.hdr);
    w.sat = reinterpret_cast<long long *>(ws + L.sat);
    w.rA = reinterpret_cast<long long *>(ws + L.rA);
    w.rT = reinterpret_cast<long long *>(ws + L.rT);
    w.rQ = reinterpret_cast<long long *>(ws + L.rQ);
    w.tT = reinterpret_cast<long long *>(ws + L.tT);
    w.tQ = reinterpret_cast<long long *>(ws + L.tQ);
    w.uQ = reinterpret_cast<long long *>(ws + L.uQ);
    w.uT = reinterpret_cast<long long *>(ws + L.uT);
    w.uC = reinterpret_cast<int *>(ws + L.uC);
    w.wT = reinterpret_cast<long long *>(ws + L.wT);
    std::array<hipEvent_t, kStages + 1> ev{};
    bool prof = false;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof = g_prof_on;
    }
    unsigned long long *work = nullptr;
    if (prof) {
        bool ok = true;
        int made = 0;
        for (auto &e : ev) {
            if (hipEventCreate(&e) != hipSuccess) { ok = false; break; }
            made++;
        }
        if (ok && hipMalloc(&work, 2 * sizeof(unsigned long long)) != hipSuccess) ok = false;
        if (!ok) {                      // release what was made
            for (int i = 0; i < made; i++) (void)hipEventDestroy(ev[i]);
            return TRS_EDEVICE;
        }
        v.work = work;                  // cleared by k_lit_sat
    }
    auto mark = [&](int i) { if (prof) (void)hipEventRecord(ev[i], stream); };
    const int nrect = v.S * v.R2;
    mark(0);
    hipLaunchKernelGGL(k_lit_sat, dim3(1), dim3(256), (size_t)3 * 8 * (v.W + 1) * (v.H + 1), stream, v, w,
                       cost, s1, s2);
    hipLaunchKernelGGL(k_lit_rects, dim3((nrect + 255) / 256), dim3(256), 0, stream, v, w);
    mark(1);
    if (v.n_units > 0) {
        const size_t tl = (size_t)7 * 8 * v.R2;                    // two levels kept
        const size_t tb1 = (size_t)8 * v.R2 * (2 + v.Km), tb2 = (size_t)8 * v.R2 * (3 + 2 * v.Km);
        const dim3 gt((unsigned)(v.n_wlive * v.S)), gu((unsigned)v.n_units);
        if (tb1 <= kLdsLimit - 1024) hipLaunchKernelGGL((k_lit_tiles<1, true>), gt, dim3(128), tb1, stream, v, w);
        else hipLaunchKernelGGL((k_lit_tiles<1, false>), gt, dim3(128), tl, stream, v, w);
        mark(2);
        launch_units<1, unsigned>(v.N, gu, unit1_lds_bytes(v.W, v.N, v.Cm, v.Rm, v.Km, 4, v.span), stream, v, w);
        launch_units<1, unsigned long long>(v.N, gu, unit1_lds_bytes(v.W, v.N, v.Cm, v.Rm, v.Km, 8, v.span), stream, v, w);
        mark(3);
        if (tb2 <= kLdsLimit - 1024) hipLaunchKernelGGL((k_lit_tiles<2, true>), gt, dim3(256), tb2, stream, v, w);
        else hipLaunchKernelGGL((k_lit_tiles<2, false>), gt, dim3(256), tl, stream, v, w);
        mark(4);
        launch_units<2, unsigned long long>(v.N, gu, unit2_lds_bytes(v.W, v.N, v.Cm, v.Rm, v.Km, v.span), stream, v, w);
        mark(5);
        hipLaunchKernelGGL(k_lit_pick, dim3(1), dim3(1024), 0, stream, v, w);
        mark(6);
    } else {
        for (int i = 2; i <= 6; i++) mark(i);
    }
    hipLaunchKernelGGL(k_lit_final, dim3(1), dim3(kFinalThreads), final_lds_bytes(v.W, v.H, v.N, v.Cm, v.Rm, v.Km, v.span),
                       stream, v, w, out_dev);
    mark(7);
    if (prof) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_ev.push_back(ProfRun{ev, work});
    }
    return hipGetLastError() == hipSuccess ? TRS_OK : TRS_EDEVICE;
}

extern "C" trs_status trs_profile_read_literal(double *ms, int64_t *runs, int64_t *relax)
{
    using namespace trs::lit;
    if (!ms || !runs || !relax) return TRS_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < kStages; i++) ms[i] = 0;
    relax[0] = relax[1] = 0;
    trs_status st = TRS_OK;
    for (auto &run : g_prof_ev) {
        auto &ev = run.ev;
        if (hipEventSynchronize(ev[kStages]) != hipSuccess) st = TRS_EDEVICE;
        for (int i = 0; i < kStages && st == TRS_OK; i++) {
            float t = 0;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) st = TRS_EDEVICE;
            ms[i] += t;
        }
        unsigned long long n[2] = {0, 0};
        if (st == TRS_OK && hipMemcpy(n, run.work, sizeof(n), hipMemcpyDeviceToHost) != hipSuccess) st = TRS_EDEVICE;
        relax[0] += (int64_t)n[0];
        relax[1] += (int64_t)n[1];
        for (auto &e : ev) (void)hipEventDestroy(e);
        (void)hipFree(run.work);
    }
    *runs = (int64_t)g_prof_ev.size();
    g_prof_ev.clear();
    return st;
}
