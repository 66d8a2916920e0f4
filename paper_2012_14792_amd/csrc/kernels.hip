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

#include "intmath.hpp"

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

// Pointers read from device tables are generic; these views tell the compiler they address
// global memory, so loads through them are global (not flat) loads.
template <class T> using gptr = const __attribute__((address_space(1))) T *;
template <class T> __device__ __forceinline__ gptr<T> as_global(const T *p) { return (gptr<T>)p; }

__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t w) { return __builtin_bit_cast(u16x2, w); }

// ---------------------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------------------

// Work-group index -> item: consecutive items (which share combination tables, spans, or
// neighbouring CTU rows) go to the same XCD, whose L2 then serves them.  Work-groups are
// dispatched to the 8 XCDs round-robin.
__device__ __forceinline__ int xcd_item(int b, int G)
{
    const int xcd = b & 7, local = b >> 3, q = G >> 3, rm = G & 7;
    return xcd * q + min(xcd, rm) + local;
}

// Statistics of CTU `ctu` (raster index) of one frame, by the whole work-group of
// (CS / 8) * 16 threads.
template <int CS>
__device__ __forceinline__ void features_ctu(const uint16_t *__restrict__ luma, long long stride,
                                             int w, int h, int W, int ctu,
                                             uint32_t *__restrict__ o_s1,
                                             unsigned long long *__restrict__ o_s2,
                                             uint32_t *__restrict__ o_g, uint32_t *__restrict__ o_tex,
                                             uint32_t *__restrict__ o_mean,
                                             uint32_t *__restrict__ o_var)
{
    constexpr int CH = CS / 8;           // 8-sample chunks per CTU row
    constexpr int NT = CH * 16;          // threads: CH chunks x 16 row groups
    constexpr int R = CS / 16;           // rows per row group
    const int cy = ctu / W, cx = ctu - cy * W, tid = threadIdx.x;
    const int chunk = tid % CH, grp = tid / CH;
    const int x0 = cx * CS + chunk * 8;
    const int ybase = cy * CS + grp * R;
    uint32_t a1 = 0, a2 = 0, ag = 0;
    if (x0 < w && ybase < h) {
        const int nv = min(8, w - x0);
        const bool has_right = x0 + 8 < w;
        const int nrow = min(R + 1, h - ybase);         // rows present, incl. the halo row
        // issue every load of this thread before using any of them
        u32x4 v[R + 1];
        uint32_t right[R];
        const gptr<uint16_t> row0 = as_global(luma + (long long)ybase * stride + x0);
#pragma unroll
        for (int r = 0; r <= R; r++)
            v[r] = r < nrow ? *reinterpret_cast<const gptr<u32x4>>(row0 + (long long)r * stride)
                            : u32x4{0u, 0u, 0u, 0u};
        // the sample right of the chunk is the first sample of the next lane's chunk (lanes of
        // one CTU row form one 16-lane DPP row), except for the row's last chunk
        const bool last = chunk == CH - 1;
#pragma unroll
        for (int r = 0; r < R; r++) {
            uint32_t nb = 0;
            if (CH == 16) nb = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[r].x, 0x101, 0xf, 0xf, false) & 0xffffu;
            const bool load = CH != 16 || last;
            right[r] = (r < nrow && has_right) ? (load ? (uint32_t)row0[(long long)r * stride + 8] : nb) : 0u;
        }
        if (nv == 8) {
            // Full chunk: samples stay packed two per 32-bit word.  sad_u16 adds the
            // absolute differences of both 16-bit halves, udot2 the products of both halves.
            uint32_t s1 = 0, s2 = 0, g = 0;
#pragma unroll
            for (int r = 0; r <= R; r++) {
                if (r < nrow) {
                    const uint32_t w0 = v[r].x, w1 = v[r].y, w2 = v[r].z, w3 = v[r].w;
                    if (r < R) {
                        s1 = __builtin_amdgcn_sad_u16(w0, 0u, s1);
                        s1 = __builtin_amdgcn_sad_u16(w1, 0u, s1);
                        s1 = __builtin_amdgcn_sad_u16(w2, 0u, s1);
                        s1 = __builtin_amdgcn_sad_u16(w3, 0u, s1);
                        s2 = __builtin_amdgcn_udot2(as_u16x2(w0), as_u16x2(w0), s2, false);
                        s2 = __builtin_amdgcn_udot2(as_u16x2(w1), as_u16x2(w1), s2, false);
                        s2 = __builtin_amdgcn_udot2(as_u16x2(w2), as_u16x2(w2), s2, false);
                        s2 = __builtin_amdgcn_udot2(as_u16x2(w3), as_u16x2(w3), s2, false);
                        // (p1,p2), (p3,p4), (p5,p6), (p7,right): right = p7 at the frame edge
                        const uint32_t rw = has_right ? right[r] : (w3 >> 16);
                        g = __builtin_amdgcn_sad_u16(__builtin_amdgcn_alignbyte(w1, w0, 2), w0, g);
                        g = __builtin_amdgcn_sad_u16(__builtin_amdgcn_alignbyte(w2, w1, 2), w1, g);
                        g = __builtin_amdgcn_sad_u16(__builtin_amdgcn_alignbyte(w3, w2, 2), w2, g);
                        g = __builtin_amdgcn_sad_u16(__builtin_amdgcn_alignbyte(rw, w3, 2), w3, g);
                    }
                    if (r >= 1) {
                        g = __builtin_amdgcn_sad_u16(w0, v[r - 1].x, g);
                        g = __builtin_amdgcn_sad_u16(w1, v[r - 1].y, g);
                        g = __builtin_amdgcn_sad_u16(w2, v[r - 1].z, g);
                        g = __builtin_amdgcn_sad_u16(w3, v[r - 1].w, g);
                    }
                }
            }
            a1 = s1;
            a2 = s2;
            ag = g;
        } else {
        uint32_t prev[8];
#pragma unroll
        for (int r = 0; r <= R; r++) {
            if (r < nrow) {
                const uint32_t p[8] = {v[r].x & 0xffffu, v[r].x >> 16, v[r].y & 0xffffu, v[r].y >> 16,
                                       v[r].z & 0xffffu, v[r].z >> 16, v[r].w & 0xffffu, v[r].w >> 16};
                if (r < R) {
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        if (j < nv) {
                            a1 += p[j];
                            a2 += p[j] * p[j];
                            if (j + 1 < nv) ag += absdiff(p[j + 1], p[j]);
                            else if (j == 7 && has_right) ag += absdiff(right[r], p[7]);
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
        o_s1[ctu] = t1;
        o_s2[ctu] = t2;
        o_g[ctu] = tg;
        o_tex[ctu] = (uint32_t)(tg / n);
        o_mean[ctu] = (uint32_t)(t1 / n);
        o_var[ctu] = (uint32_t)((n * t2 - (unsigned long long)t1 * t1) / (n * n));
    }
}

template <int CS>
__global__ void __launch_bounds__((CS / 8) * 16)
k_features(const uint16_t *__restrict__ luma, long long stride, int w, int h, int W,
           uint32_t *__restrict__ o_s1, unsigned long long *__restrict__ o_s2,
           uint32_t *__restrict__ o_g, uint32_t *__restrict__ o_tex,
           uint32_t *__restrict__ o_mean, uint32_t *__restrict__ o_var)
{
    features_ctu<CS>(luma, stride, w, h, W, xcd_item(blockIdx.x, gridDim.x), o_s1, o_s2, o_g,
                     o_tex, o_mean, o_var);
}

// ---------------------------------------------------------------------------------------
// Cost map
// ---------------------------------------------------------------------------------------

// Predicted time of one CTU; sets *over when the value is clamped to 2^31 - 1.
__device__ __forceinline__ uint32_t cost_of(uint32_t tex, const uint32_t *prev, int i, uint32_t a,
                                            uint32_t b, uint32_t wp, bool *over)
{
    // a + b tex <= (2^32 - 1) + (2^32 - 1)^2 < 2^64
    const unsigned long long model = (unsigned long long)a + (unsigned long long)b * tex;
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
    *over = v > kCostLimit;
    return (uint32_t)(*over ? kCostLimit : v);
}

__global__ void __launch_bounds__(256)
k_cost(int n, const uint32_t *__restrict__ tex, const uint32_t *__restrict__ prev, uint32_t a,
       uint32_t b, uint32_t wp, uint32_t *__restrict__ cost, uint32_t *flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool over;
    cost[i] = cost_of(tex[i], prev, i, a, b, wp, &over);
    if (over && flags) atomicOr(flags, 1u);
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
    (void)hdr;
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

// The same tables for grids with (H+1)(W+1) <= kSatLds, by one work-group: the inputs are
// read into LDS by every thread at once (at entry (y + 1, x + 1) of the tables' layout), then
// one thread per CTU row and one per column keep running sums in LDS.
constexpr int kSatLds = 2304;

__global__ void __launch_bounds__(256)
k_sat_lds(int W, int H, const uint32_t *__restrict__ cost, const uint32_t *__restrict__ s1,
          const unsigned long long *__restrict__ s2, long long *satT, long long *satS1,
          long long *satS2, WsHeader *hdr)
{
    __shared__ long long lT[kSatLds], l1[kSatLds], l2[kSatLds];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int S = W + 1, n = W * H;
    (void)hdr;
    for (int i = tid; i < n; i += nt) {
        const int y = i / W, e = (y + 1) * S + (i - y * W) + 1;
        lT[e] = cost[i];
        l1[e] = s1[i];
        l2[e] = (long long)s2[i];
    }
    for (int y = tid; y <= H; y += nt) lT[y * S] = l1[y * S] = l2[y * S] = 0;
    for (int x = tid; x <= W; x += nt) lT[x] = l1[x] = l2[x] = 0;
    __syncthreads();
    for (int y = tid; y < H; y += nt) {
        long long aT = 0, a1 = 0, a2 = 0;
        const int e0 = (y + 1) * S + 1;
        for (int x = 0; x < W; x++) {
            aT += lT[e0 + x];
            a1 += l1[e0 + x];
            a2 += l2[e0 + x];
            lT[e0 + x] = aT;
            l1[e0 + x] = a1;
            l2[e0 + x] = a2;
        }
    }
    __syncthreads();
    for (int x = tid; x <= W; x += nt) {
        long long aT = 0, a1 = 0, a2 = 0;
        satT[x] = satS1[x] = satS2[x] = 0;
        for (int y = 1; y <= H; y++) {
            aT += lT[y * S + x];
            a1 += l1[y * S + x];
            a2 += l2[y * S + x];
            satT[y * S + x] = aT;
            satS1[y * S + x] = a1;
            satS2[y * S + x] = a2;
        }
    }
}

// Cost map fused with the LDS prefix sums (same grids as k_sat_lds), by one work-group.  All
// inputs are first read into LDS by every thread at once (in the tables' layout, at entry
// (y + 1, x + 1)), so the serial row and column sums touch LDS only.
__device__ void cost_sat_body(int W, int H, const uint32_t *__restrict__ tex,
                              const uint32_t *__restrict__ prev, uint32_t a, uint32_t b,
                              uint32_t wp, uint32_t *__restrict__ cost, uint32_t *flags,
                              const uint32_t *__restrict__ s1,
                              const unsigned long long *__restrict__ s2, long long *satT,
                              long long *satS1, long long *satS2)
{
    __shared__ long long lT[kSatLds], l1[kSatLds], l2[kSatLds];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int S = W + 1, n = W * H;
    bool any_over = false;
    for (int i = tid; i < n; i += nt) {
        bool over;
        const uint32_t v = cost_of(tex[i], prev, i, a, b, wp, &over);
        const int y = i / W, e = (y + 1) * S + (i - y * W) + 1;
        cost[i] = v;
        lT[e] = v;
        l1[e] = s1[i];
        l2[e] = (long long)s2[i];
        any_over |= over;
    }
    if (any_over && flags) atomicOr(flags, 1u);
    for (int y = tid; y <= H; y += nt) lT[y * S] = l1[y * S] = l2[y * S] = 0;
    for (int x = tid; x <= W; x += nt) lT[x] = l1[x] = l2[x] = 0;
    __syncthreads();
    for (int y = tid; y < H; y += nt) {                 // row sums in place
        long long aT = 0, a1 = 0, a2 = 0;
        const int e0 = (y + 1) * S + 1;
        for (int x = 0; x < W; x++) {
            aT += lT[e0 + x];
            a1 += l1[e0 + x];
            a2 += l2[e0 + x];
            lT[e0 + x] = aT;
            l1[e0 + x] = a1;
            l2[e0 + x] = a2;
        }
    }
    __syncthreads();
    for (int x = tid; x <= W; x += nt) {                // column sums, written out
        long long aT = 0, a1 = 0, a2 = 0;
        satT[x] = satS1[x] = satS2[x] = 0;
        for (int y = 1; y <= H; y++) {
            aT += lT[y * S + x];
            a1 += l1[y * S + x];
            a2 += l2[y * S + x];
            satT[y * S + x] = aT;
            satS1[y * S + x] = a1;
            satS2[y * S + x] = a2;
        }
    }
}

__global__ void __launch_bounds__(256)
k_cost_sat(int W, int H, const uint32_t *__restrict__ tex, const uint32_t *__restrict__ prev,
           uint32_t a, uint32_t b, uint32_t wp, uint32_t *__restrict__ cost, uint32_t *flags,
           const uint32_t *__restrict__ s1, const unsigned long long *__restrict__ s2,
           long long *satT, long long *satS1, long long *satS2, WsHeader *hdr)
{
    (void)hdr;
    cost_sat_body(W, H, tex, prev, a, b, wp, cost, flags, s1, s2, satT, satS1, satS2);
}

// ---------------------------------------------------------------------------------------
// Search
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ long long rect(const long long *__restrict__ sat, int S, int x0, int y0,
                                          int x1, int y1)
{
    return sat[y1 * S + x1] - sat[y0 * S + x1] - sat[y1 * S + x0] + sat[y0 * S + x0];
}

__device__ __forceinline__ int kcnt(const SpaceView &sp, int h, int kk)
{
    return sp.opt_kcnt[h * (sp.Km + 1) + min(kk, sp.Km)];
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

// Byte offsets of the search kernels' dynamic LDS arrays (-1: not present).
struct LdsMap {
    int recT, recQ, satT, satS1, satS2, bytes;
};

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

// Final reduction over the step-2 partials (one per live item) and decode of the winner
// into *out.  Run by one whole work-group of BS >= 64 threads.
template <int BS>
__device__ void final_block(const SpaceView &sp, const Partial *__restrict__ part, int n_part,
                            const WsHeader *hdr, const long long *satT, const long long *satS1,
                            const long long *satS2, trs_result *out, int dt, int dr)
{
    constexpr int NW = BS / kWave;
    __shared__ unsigned long long redq[NW], redt[NW], redn[NW];
    __shared__ long long redr[NW];
    __shared__ int redf[NW], redi[NW];
    __shared__ int sk[kMaxRS];                       // slices per tile of the winner
    __shared__ long long ut[kMaxRS], uq[kMaxRS];     // uniform slice scores
    __shared__ Key2 sbest;
    __shared__ int sbi;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int S = sp.W + 1;
    for (int i = tid; i <= kMaxRS; i += BS) {
        out->col_bd[i] = 0;
        out->row_bd[i] = 0;
    }
    for (int i = tid; i < kMaxRS; i += BS) {
        for (int e = 0; e < 4; e++) out->rs[i][e] = 0;
        out->rs_time[i] = 0;
    }
    for (int i = tid; i < sp.n_unif; i += BS)
        score_rect(sp, satT, satS1, satS2, sp.unif_rs[4 * i], sp.unif_rs[4 * i + 1],
                   sp.unif_rs[4 * i + 2], sp.unif_rs[4 * i + 3], &ut[i], &uq[i]);
    Key2 best{kNone, kNone, LLONG_MAX, -1};
    int bitem = -1;
    unsigned long long scored = 0;
    for (int i = tid; i < n_part; i += BS) {
        const Partial p = part[i];
        const Key2 k{p.q, p.t, p.rank, p.f};
        scored += (unsigned long long)p.n;
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
        scored += shfl_xor64(scored, m);
    }
    if (lane == 0) {
        redq[wv] = best.q; redt[wv] = best.t; redr[wv] = best.rank; redf[wv] = best.f;
        redi[wv] = bitem; redn[wv] = scored;
    }
    __syncthreads();
    if (tid == 0) {
        Key2 b{redq[0], redt[0], redr[0], redf[0]};
        int bi = redi[0];
        for (int i = 1; i < NW; i++) {
            const Key2 o{redq[i], redt[i], redr[i], redf[i]};
            if (key_less(o, b)) { b = o; bi = redi[i]; }
        }
        sbest = b;
        sbi = bi;
    }
    __syncthreads();
    const Key2 b = sbest;
    const bool none = sp.n_feasible == 0 || b.q == kNone;  // uniform over the block
    int ncols, nrows, nrs;
    if (none) {
        // no feasible candidate: the uniform grid
        ncols = sp.n_unif ? sp.cu : 0;
        nrows = sp.n_unif ? sp.ru : 0;
        nrs = sp.n_unif;
        for (int i = tid; i <= ncols && ncols; i += BS) out->col_bd[i] = (int)((long long)i * sp.W / sp.cu);
        for (int i = tid; i <= nrows && nrows; i += BS) out->row_bd[i] = (int)((long long)i * sp.H / sp.ru);
        for (int i = tid; i < nrs; i += BS) {
            for (int e = 0; e < 4; e++) out->rs[i][e] = sp.unif_rs[4 * i + e];
            out->rs_time[i] = ut[i];
        }
    } else {
        const ItemDev it = sp.items[sbi];
        const ShapeDev sd = sp.shapes[it.shape];
        const int xl = b.f / it.M, m = b.f - xl * it.M;
        const uint16_t *X = sp.xtab + sd.x_off + (long long)(it.xa + xl) * (sd.c + 1);
        const uint16_t *Y = sp.ytab + sd.y_off + (long long)it.yi * (sd.r + 1);
        ncols = sd.c;
        nrows = sd.r;
        for (int q = tid; q <= sd.c; q += BS) out->col_bd[q] = X[q];
        for (int q = tid; q <= sd.r; q += BS) out->row_bd[q] = Y[q];
        int opt = 0, i = 0, j = 0;
        if (tid < sd.T) {
            i = tid % sd.c;
            j = tid / sd.c;
            const int h = Y[j + 1] - Y[j];
            opt = sp.opt_base[h] + sp.combos[it.combo_off + (long long)tid * it.M + m];
            sk[tid] = sp.opt_k[opt];
        }
        __syncthreads();
        nrs = 0;
        for (int t = 0; t < sd.T; t++) nrs += sk[t];
        if (tid < sd.T) {
            int slot = 0;
            for (int t = 0; t < tid; t++) slot += sk[t];
            const uint16_t *z = sp.opt_z + (long long)opt * (sp.Km + 1);
            for (int q = 0; q < sk[tid]; q++, slot++) {
                const int y0 = Y[j] + z[q], y1 = Y[j] + z[q + 1];
                out->rs[slot][0] = X[i];
                out->rs[slot][1] = y0;
                out->rs[slot][2] = X[i + 1];
                out->rs[slot][3] = y1;
                out->rs_time[slot] = rect(satT, S, X[i], y0, X[i + 1], y1);
            }
        }
    }
    if (tid == 0) {
        long long tu = -1, qu = -1;
        if (sp.n_unif > 0) {
            tu = 0;
            qu = 0;
            for (int q = 0; q < sp.n_unif; q++) { tu = max(tu, ut[q]); qu += uq[q]; }
        }
        unsigned long long n2 = 0;
        for (int q = 0; q < NW; q++) n2 += redn[q];
        out->n_enumerated = sp.total;
        out->n_feasible = sp.n_feasible;
        out->n_step2 = (long long)n2;
        out->dtile_used = dt;
        out->drs_used = dr;
        out->uniform_rank = sp.uniform_rank;
        out->t_unif = tu;
        out->q_unif = qu;
        out->tile_cols = ncols;
        out->tile_rows = nrows;
        out->n_rs = nrs;
        if (none) {
            out->status = TRS_ENOFEASIBLE;
            out->rank = sp.uniform_rank;
            out->t_min = -1;
            out->t_sel = tu;
            out->q_sel = qu;
        } else {
            out->status = TRS_OK;
            out->rank = b.rank;
            out->t_min = (long long)hdr->tmin;
            out->t_sel = (long long)b.t;
            out->q_sel = (long long)b.q;
        }
    }
}

// Scores one work item with the whole work-group: phase 1 builds its tile-option records
// (recT, and recQ in step 2), phase 2 scores its candidates one per lane.  The result is
// valid in thread 0: the item's smallest T~(P) (step 1) or its best (Q, T~, rank) within
// `bound` (step 2).
template <int BS, bool P2>
__device__ __forceinline__ void search_item(const SpaceView &sp, const ItemDev &it,
                                            const long long *sT, const long long *s1t,
                                            const long long *s2t, unsigned long long bound,
                                            unsigned long long *recT, unsigned long long *recQ,
                                            unsigned long long &tbest_out, Key2 &best_out)
{
    constexpr int NW = BS / kWave;
    __shared__ unsigned long long redq[NW], redt[NW];
    __shared__ long long redr[NW];
    __shared__ int redf[NW];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int S = sp.W + 1;
    for (int rid = tid; rid < it.n_rec; rid += BS) {
        const uint32_t d0 = sp.rdesc[2 * (it.rec_off + rid)];
        const int opt = (int)sp.rdesc[2 * (it.rec_off + rid) + 1];
        const int xa = d0 & 511, xb = (d0 >> 9) & 511, y0 = (int)(d0 >> 18);
        const int k = sp.opt_k[opt];
        const uint16_t *z = sp.opt_z + (long long)opt * (sp.Km + 1);
        const unsigned wpx = (unsigned)(sp.colpx[xb] - sp.colpx[xa]);
        unsigned long long tmax = 0, qs = 0;
        for (int q = 0; q < k; q++) {
            const int ya = y0 + z[q], yb = y0 + z[q + 1];
            tmax = max(tmax, (unsigned long long)rect(sT, S, xa, ya, xb, yb));
            if (P2) {
                const unsigned area = wpx * (unsigned)(sp.rowpx[yb] - sp.rowpx[ya]);
                const unsigned long long a1 = (unsigned long long)rect(s1t, S, xa, ya, xb, yb);
                const unsigned long long a2 = (unsigned long long)rect(s2t, S, xa, ya, xb, yb);
                qs += a2 - floor_sq_div(a1, area);
            }
        }
        recT[rid] = tmax;
        if (P2) recQ[rid] = qs;
    }
    __syncthreads();

    const int n = it.n_ent, T = it.T;
    const uint16_t *__restrict__ rids = sp.ent_rid + it.rid_off;
    unsigned long long tbest = kNone;
    Key2 best{kNone, kNone, LLONG_MAX, -1};
    for (int e = tid; e < n; e += BS) {
        unsigned long long tmax = 0, qsum = 0;
#pragma unroll 4
        for (int t = 0; t < T; t++) {
            const int rr = rids[t * n + e];
            tmax = max(tmax, recT[rr]);
            if (P2) qsum += recQ[rr];
        }
        if (!P2) {
            tbest = min(tbest, tmax);
        } else if (tmax <= bound && (qsum < best.q || (qsum == best.q && tmax <= best.t))) {
            const int f = (int)sp.ent_f[it.ent_off + e];
            const int xl = f / it.M;
            const Key2 cand{qsum, tmax, it.rank0 + (long long)xl * it.SM + (f - xl * it.M), f};
            if (key_less(cand, best)) best = cand;
        }
    }

    if (!P2) {
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) tbest = min(tbest, shfl_xor64(tbest, m));
        if (lane == 0) redt[wv] = tbest;
        __syncthreads();
        if (tid == 0) {
            unsigned long long bt = kNone;
            for (int i = 0; i < NW; i++) bt = min(bt, redt[i]);
            tbest_out = bt;
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
            best_out = b;
        }
    }
}

// One work item per work-group.  Phase 1 builds the item's tile-option records in LDS: for
// a column span, tile row and (k, split offsets) option, the largest slice time (Eq. 1)
// and, in step 2, the summed per-slice ceil-SSE (Eq. 2).  Phase 2 scores the item's
// candidates, one per lane: T~(P) is the max of its tiles' record times, Q(P) the sum of
// their record sums.  STAGE: the prefix sums the records read are first copied to LDS.
//
// Step 1 writes each item's smallest T~(P); k_live turns those into T~min, the Eq. 4
// bound and the list of items that can hold a step-2 candidate; step 2 runs over that
// list only; k_final reduces its partials and decodes the winner.
template <int BS, bool P2, bool STAGE>
__global__ void __launch_bounds__(BS)
k_search(SpaceView sp, LdsMap L, const long long *__restrict__ satT,
         const long long *__restrict__ satS1, const long long *__restrict__ satS2,
         WsHeader *hdr, unsigned long long *__restrict__ item_min, int *__restrict__ live,
         Partial *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned long long *recT = reinterpret_cast<unsigned long long *>(lds + L.recT);
    unsigned long long *recQ = reinterpret_cast<unsigned long long *>(lds + (P2 ? L.recQ : L.recT));
    const int tid = threadIdx.x;
    const int S = sp.W + 1;
    int slot, item;
    if (P2) {
        const int n_live = hdr->n_live;
        if ((int)blockIdx.x >= n_live) return;      // the item list is shorter than the grid
        slot = xcd_item(blockIdx.x, n_live);
        item = live[slot];
    } else {
        slot = item = xcd_item(blockIdx.x, gridDim.x);
    }
    const long long *sT = satT, *s1t = satS1, *s2t = satS2;
    if (STAGE) {                       // independent of the item: overlaps its load latency
        long long *lT = reinterpret_cast<long long *>(lds + L.satT);
        long long *l1 = reinterpret_cast<long long *>(lds + (P2 ? L.satS1 : L.satT));
        long long *l2 = reinterpret_cast<long long *>(lds + (P2 ? L.satS2 : L.satT));
        const int n = S * (sp.H + 1);
        for (int e = tid; e < n; e += BS) {
            lT[e] = satT[e];
            if (P2) {
                l1[e] = satS1[e];
                l2[e] = satS2[e];
            }
        }
        sT = lT;
        s1t = l1;
        s2t = l2;
    }
    const ItemDev it = sp.items[item];
    const unsigned long long bound = P2 ? hdr->bound : kNone;
    if (STAGE) __syncthreads();

    unsigned long long tb;
    Key2 bk;
    search_item<BS, P2>(sp, it, sT, s1t, s2t, bound, recT, recQ, tb, bk);
    if (tid == 0) {
        if (!P2) item_min[item] = tb;
        else part[slot] = Partial{bk.q, bk.t, bk.rank, item, bk.f, it.n_ent, 0};
    }
}

// T~min (Eq. 3) over the step-1 item minima, the Eq. 4 bound, and the list of items whose
// minimum is within it (the only ones that can hold a step-2 candidate), in item order.
__global__ void __launch_bounds__(1024)
k_live(int n_items, const unsigned long long *__restrict__ item_min, int lam_num, int lam_den,
       WsHeader *hdr, int *__restrict__ live)
{
    constexpr int BS = 1024, NW = BS / kWave;
    __shared__ unsigned long long rt[NW];
    __shared__ int wcnt[NW];
    __shared__ int sbase;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    unsigned long long t = kNone;
    for (int i = tid; i < n_items; i += BS) t = min(t, item_min[i]);
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) t = min(t, shfl_xor64(t, m));
    if (lane == 0) rt[wv] = t;
    if (tid == 0) sbase = 0;
    __syncthreads();
    unsigned long long tmin = kNone;
    for (int i = 0; i < NW; i++) tmin = min(tmin, rt[i]);
    unsigned long long bnd = kNone;
    if (lam_num >= 0)
        bnd = tmin * (unsigned long long)(lam_den + lam_num) / (unsigned long long)lam_den;
    for (int i0 = 0; i0 < n_items; i0 += BS) {
        const int i = i0 + tid;
        const bool keep = i < n_items && item_min[i] <= bnd;
        const unsigned long long mask = __ballot(keep);
        if (lane == 0) wcnt[wv] = __popcll(mask);
        __syncthreads();
        int off = sbase;
        for (int q = 0; q < wv; q++) off += wcnt[q];
        if (keep) live[off + __popcll(mask & ((1ull << lane) - 1ull))] = i;
        __syncthreads();
        if (tid == 0) for (int q = 0; q < NW; q++) sbase += wcnt[q];
        __syncthreads();
    }
    if (tid == 0) {
        hdr->tmin = tmin;
        hdr->bound = bnd;
        hdr->n_live = sbase;
    }
}

// Winner over the step-2 partials of the live items (none for a plan without any
// area-feasible candidate), decoded into *out.
__global__ void __launch_bounds__(256)
k_final(SpaceView sp, const Partial *__restrict__ part, const WsHeader *hdr,
        const long long *satT, const long long *satS1, const long long *satS2, trs_result *out,
        int dt, int dr)
{
    final_block<256>(sp, part, sp.n_items ? hdr->n_live : 0, hdr, satT, satS1, satS2, out, dt, dr);
}

// LDS layout of a search kernel: records and (when staged) the prefix sums.
LdsMap lds_map(const SpaceView &sp, bool p2, bool stage)
{
    LdsMap L{-1, -1, -1, -1, -1, 0};
    int off = 0;
    auto take = [&](int bytes) { int at = off; off += (bytes + 15) & ~15; return at; };
    const int rec = sp.rec_max > 0 ? sp.rec_max : 1;
    L.recT = take(8 * rec);
    if (p2) L.recQ = take(8 * rec);
    if (stage) {
        const int n = (sp.W + 1) * (sp.H + 1);
        L.satT = take(8 * n);
        if (p2) {
            L.satS1 = take(8 * n);
            L.satS2 = take(8 * n);
        }
    }
    L.bytes = off;
    return L;
}

constexpr int kStageLimit = 24 * 1024;   // prefix sums copied to LDS only up to this size

struct WsPtrs {
    WsHeader *hdr;
    long long *satT, *satS1, *satS2;
    unsigned long long *imin;
    int *live;
    Partial *part;
};

WsPtrs ws_ptrs(const SearchArgs &a)
{
    return WsPtrs{reinterpret_cast<WsHeader *>(a.ws + a.lay.header),
                  reinterpret_cast<long long *>(a.ws + a.lay.satT),
                  reinterpret_cast<long long *>(a.ws + a.lay.satS1),
                  reinterpret_cast<long long *>(a.ws + a.lay.satS2),
                  reinterpret_cast<unsigned long long *>(a.ws + a.lay.item_min),
                  reinterpret_cast<int *>(a.ws + a.lay.live),
                  reinterpret_cast<Partial *>(a.ws + a.lay.partial)};
}

template <int BS, bool P2>
void launch_pass(const SearchArgs &a, const WsPtrs &w, hipStream_t s)
{
    const int G = a.sp.n_items;
    const int satb = 8 * (a.sp.W + 1) * (a.sp.H + 1) * (P2 ? 3 : 1);
    if (satb <= kStageLimit) {
        const LdsMap L = lds_map(a.sp, P2, true);
        hipLaunchKernelGGL((k_search<BS, P2, true>), dim3(G), dim3(BS), L.bytes, s, a.sp, L, w.satT,
                           w.satS1, w.satS2, w.hdr, w.imin, w.live, w.part);
    } else {
        const LdsMap L = lds_map(a.sp, P2, false);
        hipLaunchKernelGGL((k_search<BS, P2, false>), dim3(G), dim3(BS), L.bytes, s, a.sp, L, w.satT,
                           w.satS1, w.satS2, w.hdr, w.imin, w.live, w.part);
    }
}

template <int BS>
hipError_t launch_passes(const SearchArgs &a, const WsPtrs &w, hipStream_t s)
{
    if (a.sp.n_items > 0) {
        if (a.ev[0] && hipEventRecord(a.ev[0], s) != hipSuccess) return hipErrorUnknown;
        launch_pass<BS, false>(a, w, s);
        if (a.ev[1] && hipEventRecord(a.ev[1], s) != hipSuccess) return hipErrorUnknown;
        hipLaunchKernelGGL(k_live, dim3(1), dim3(1024), 0, s, a.sp.n_items, w.imin, a.lam_num,
                           a.lam_den, w.hdr, w.live);
        if (a.ev[2] && hipEventRecord(a.ev[2], s) != hipSuccess) return hipErrorUnknown;
        launch_pass<BS, true>(a, w, s);
        if (a.ev[3] && hipEventRecord(a.ev[3], s) != hipSuccess) return hipErrorUnknown;
    }
    hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, a.sp, w.part, w.hdr, w.satT, w.satS1,
                       w.satS2, a.out, a.dt, a.dr);
    return hipGetLastError();
}

hipError_t launch_after_sat(const SearchArgs &a, hipStream_t s)
{
    const WsPtrs w = ws_ptrs(a);
    switch (a.block) {
    case 64: return launch_passes<64>(a, w, s);
    case 128: return launch_passes<128>(a, w, s);
    case 512: return launch_passes<512>(a, w, s);
    default: return launch_passes<256>(a, w, s);
    }
}


// ---------------------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------------------

template <int CS>
__global__ void __launch_bounds__((CS / 8) * 16)
k_features_batch(const BatchFrameDev *__restrict__ frames, const int *__restrict__ ctu_frame,
                 char *ws)
{
    const int g = xcd_item(blockIdx.x, gridDim.x);
    const BatchFrameDev fr = frames[ctu_frame[g]];
    features_ctu<CS>(fr.luma, fr.stride, fr.w, fr.h, fr.W, g - fr.ctu_base,
                     reinterpret_cast<uint32_t *>(ws + fr.o_s1),
                     reinterpret_cast<unsigned long long *>(ws + fr.o_s2),
                     reinterpret_cast<uint32_t *>(ws + fr.o_grad),
                     reinterpret_cast<uint32_t *>(ws + fr.o_tex),
                     reinterpret_cast<uint32_t *>(ws + fr.o_mean),
                     reinterpret_cast<uint32_t *>(ws + fr.o_var));
}

// One work-group per frame: cost map (overflow flag in the frame's header) and SATs.  The
// first work-group also clears the step-2 list length.
__global__ void __launch_bounds__(256)
k_cost_sat_batch(const BatchFrameDev *__restrict__ frames, char *ws, int *live_n)
{
    const BatchFrameDev fr = frames[blockIdx.x];
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws + fr.o_hdr);
    if (threadIdx.x == 0) hdr->pad0 = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *live_n = 0;
    __syncthreads();
    cost_sat_body(fr.W, fr.H, reinterpret_cast<const uint32_t *>(ws + fr.o_tex), fr.prev, fr.a,
                  fr.b, fr.wp, reinterpret_cast<uint32_t *>(ws + fr.o_cost),
                  reinterpret_cast<uint32_t *>(&hdr->pad0),
                  reinterpret_cast<const uint32_t *>(ws + fr.o_s1),
                  reinterpret_cast<const unsigned long long *>(ws + fr.o_s2),
                  reinterpret_cast<long long *>(ws + fr.o_satT),
                  reinterpret_cast<long long *>(ws + fr.o_satS1),
                  reinterpret_cast<long long *>(ws + fr.o_satS2));
}

// Persistent search over every (frame, item) of the batch: work-group b takes a contiguous
// range of the flat item list (ranges of neighbouring b stay on one XCD).  Step 2 skips
// items whose step-1 minimum exceeds their frame's Eq. 4 bound.
//
// Step 1 (P2 false) walks the flat (frame, item) list; step 2 walks the list of live entries
// k_tmin_batch compacted, so its work spreads evenly over the grid.
template <int BS, bool P2>
__global__ void __launch_bounds__(BS)
k_search_batch(const SpaceView *__restrict__ plans, const BatchFrameDev *__restrict__ frames,
               const int *__restrict__ item_frame, int n_flat, char *ws,
               unsigned long long *__restrict__ item_min, Partial *__restrict__ part, int rec_max,
               const unsigned long long *__restrict__ live, const int *__restrict__ live_n)
{
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned long long *recT = reinterpret_cast<unsigned long long *>(lds);
    unsigned long long *recQ = recT + rec_max;
    const int tid = threadIdx.x;
    const int G = gridDim.x, b = xcd_item(blockIdx.x, G);
    const int total = P2 ? *live_n : n_flat;
    const int beg = (int)((long long)total * b / G), end = (int)((long long)total * (b + 1) / G);
    int cur = -1;
    BatchFrameDev fr{};
    for (int x = beg; x < end; x++) {
        const int g = P2 ? frames[(int)(live[x] >> 32)].item_base + (int)(unsigned)live[x] : x;
        const int f = item_frame[g];
        if (f != cur) {
            fr = frames[f];
            cur = f;
        }
        const SpaceView &sp = plans[fr.plan];
        const int i = g - fr.item_base;
        const unsigned long long bound = P2 ? reinterpret_cast<const WsHeader *>(ws + fr.o_hdr)->bound : kNone;
        const ItemDev it = sp.items[i];
        __syncthreads();                             // the previous item's records are read
        unsigned long long tb;
        Key2 bk;
        search_item<BS, P2>(sp, it, reinterpret_cast<const long long *>(ws + fr.o_satT),
                            reinterpret_cast<const long long *>(ws + fr.o_satS1),
                            reinterpret_cast<const long long *>(ws + fr.o_satS2), bound, recT,
                            recQ, tb, bk);
        if (tid == 0) {
            if (!P2) item_min[g] = tb;
            else part[g] = Partial{bk.q, bk.t, bk.rank, i, bk.f, it.n_ent, 0};
        }
    }
}

// One work-group per frame: T~min and the Eq. 4 bound from the frame's item minima; the
// frame's items within the bound are appended as (frame << 32 | item), in item order at a
// position reserved with one atomic, to the step-2 list, and the others get an empty partial.
__global__ void __launch_bounds__(256)
k_tmin_batch(const BatchFrameDev *__restrict__ frames,
             const unsigned long long *__restrict__ item_min, char *ws,
             Partial *__restrict__ part, unsigned long long *__restrict__ live, int *__restrict__ live_n)
{
    constexpr int NW = 256 / kWave, KR = 8;           // items per thread held in registers
    __shared__ unsigned long long rt[NW];
    __shared__ unsigned long long sbound;
    __shared__ int wcnt[NW];
    __shared__ int sbase;
    const BatchFrameDev fr = frames[blockIdx.x];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const unsigned long long *im = item_min + fr.item_base;
    const int n = fr.n_items;
    // item tid + 256 q of each 2048-item block; the first block stays in registers
    unsigned long long v[KR];
#pragma unroll
    for (int q = 0; q < KR; q++) v[q] = tid + 256 * q < n ? im[tid + 256 * q] : kNone;
    unsigned long long t = kNone;
#pragma unroll
    for (int q = 0; q < KR; q++) t = min(t, v[q]);
    for (int i = tid + 256 * KR; i < n; i += 256) t = min(t, im[i]);
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) t = min(t, shfl_xor64(t, m));
    if (lane == 0) rt[wv] = t;
    __syncthreads();
    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws + fr.o_hdr);
    if (tid == 0) {
        unsigned long long tmin = kNone;
        for (int i = 0; i < NW; i++) tmin = min(tmin, rt[i]);
        unsigned long long bnd = kNone;
        if (fr.lam_num >= 0 && tmin != kNone)
            bnd = tmin * (unsigned long long)(fr.lam_den + fr.lam_num) / (unsigned long long)fr.lam_den;
        hdr->tmin = tmin;
        hdr->bound = bnd;
        sbound = bnd;
    }
    __syncthreads();
    const unsigned long long bound = sbound;
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < KR; q++) cnt += tid + 256 * q < n && v[q] <= bound;
    for (int i = tid + 256 * KR; i < n; i += 256) cnt += im[i] <= bound;
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) cnt += __shfl_xor(cnt, m, kWave);
    if (lane == 0) wcnt[wv] = cnt;
    __syncthreads();
    if (tid == 0) {
        int c = 0;
        for (int i = 0; i < NW; i++) c += wcnt[i];
        hdr->n_live = c;
        sbase = c ? atomicAdd(live_n, c) : 0;
    }
    __syncthreads();
    int base = sbase;
    for (int i0 = 0; i0 < n; i0 += 256) {
        const int i = i0 + tid, q = i0 / 256;
        const bool in = i < n;
        unsigned long long val = kNone;
#pragma unroll
        for (int r = 0; r < KR; r++)
            if (r == q) val = v[r];
        if (q >= KR && in) val = im[i];
        const bool ok = in && val <= bound;
        if (in && !ok) part[fr.item_base + i] = Partial{kNone, kNone, LLONG_MAX, i, -1, 0, 0};
        const unsigned long long mask = __ballot(ok);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        __syncthreads();                               // wcnt of the previous chunk is read
        if (lane == 0) wcnt[wv] = __popcll(mask);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wv; w++) off += wcnt[w];
        if (ok) live[off + before] = ((unsigned long long)blockIdx.x << 32) | (unsigned)i;
        for (int w = 0; w < NW; w++) base += wcnt[w];
    }
}

// Frame-inner step 1 for a chunk of up to kChunk frames that share one plan: the item's
// records are built for every frame of the chunk into LDS as [record][frame] (a padded row
// per record), then each lane takes candidates, reads each tile's record index once and
// updates all frames' running maxima from that row.  Writes item_min for each frame.
constexpr int kRecRow = kChunk + 2;                     // u64 per record row (16-byte rows)


// Minimum over the work-group's wave of each of kChunk values per lane, reduce-scattered:
// after the three halving exchanges lane l holds the partial of value (l >> 3) & 7 over 8
// lanes, and three more exchanges finish it.  Returns that value's wave minimum (valid in
// lanes with l % 8 == 0).
__device__ __forceinline__ unsigned long long wave_min8(const unsigned long long (&v)[kChunk], int lane)
{
    static_assert(kChunk == 8, "reduce-scatter is written for 8 values");
    unsigned long long a[4], b2[2], c;
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const unsigned long long keep = h5 ? v[4 + i] : v[i], send = h5 ? v[i] : v[4 + i];
        a[i] = min(keep, shfl_xor64(send, 32));
    }
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const unsigned long long keep = h4 ? a[2 + i] : a[i], send = h4 ? a[i] : a[2 + i];
        b2[i] = min(keep, shfl_xor64(send, 16));
    }
    {
        const unsigned long long keep = h3 ? b2[1] : b2[0], send = h3 ? b2[0] : b2[1];
        c = min(keep, shfl_xor64(send, 8));
    }
#pragma unroll
    for (int m = 4; m >= 1; m >>= 1) c = min(c, shfl_xor64(c, m));
    return c;
}

template <int BS>
__global__ void __launch_bounds__(BS)
k_step1_units(const UnitDev *__restrict__ units, const ChunkSlot *__restrict__ slots, int n_units,
              int rec_max, char *ws, unsigned long long *__restrict__ item_min)
{
    constexpr int NW = BS / kWave;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned long long *rec = reinterpret_cast<unsigned long long *>(lds);
    uint16_t *srid = reinterpret_cast<uint16_t *>(lds + 8 * kRecRow * rec_max);
    __shared__ unsigned long long red[kChunk][NW];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int G = gridDim.x, b = xcd_item(blockIdx.x, G);
    const int beg = (int)((long long)n_units * b / G), end = (int)((long long)n_units * (b + 1) / G);
    if (beg >= end) return;
    UnitDev next = units[beg];
    for (int u = beg; u < end; u++) {
        const UnitDev ud = next;
        if (u + 1 < end) next = units[u + 1];           // used by the next iteration
        const int n = ud.n_ent, T = ud.T, S = ud.S;
        const ChunkSlot *sl = slots + ud.chunk * kChunk;
        __syncthreads();                                // the previous unit's LDS is read
        // the item's record indices go to LDS in 16-byte pieces (arrays are 16-byte aligned
        // and padded); each thread's first piece is stored after the record build
        const gptr<u32x4> rsrc = as_global(reinterpret_cast<const u32x4 *>(ud.rids));
        const int nv = (n * T + 7) >> 3;
        u32x4 piece = {0u, 0u, 0u, 0u};
        if (tid < nv) piece = rsrc[tid];
        // phase 1: one record per thread, all frames of the chunk; a record's corner loads
        // for every frame are issued before any is used
        const gptr<u32x4> rd = as_global(reinterpret_cast<const u32x4 *>(ud.rdesc4));
        for (int rid = tid; rid < ud.n_rec; rid += BS) {
            const u32x4 d = rd[rid];
            const int xa = d.x & 511, xb = (d.x >> 9) & 511, y0 = (int)(d.x >> 18);
            const int k = d.y & 255;
            unsigned long long tmax[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; j++) tmax[j] = 0;
            int ya = y0;
            for (int q = 0; q < k; q++) {
                const int zi = q + 1;                   // byte zi of words 1..3
                const uint32_t wsel = zi < 4 ? d.y : zi < 8 ? d.z : d.w;
                const int yb = y0 + (int)((wsel >> (8 * (zi & 3))) & 255);
                const int i00 = ya * S + xa, i01 = ya * S + xb, i10 = yb * S + xa, i11 = yb * S + xb;
                long long c[kChunk][4];
#pragma unroll
                for (int j = 0; j < kChunk; j++) {
                    const gptr<long long> st = as_global(reinterpret_cast<const long long *>(ws + sl[j].o_sat));
                    c[j][0] = st[i11];
                    c[j][1] = st[i01];
                    c[j][2] = st[i10];
                    c[j][3] = st[i00];
                }
#pragma unroll
                for (int j = 0; j < kChunk; j++)
                    tmax[j] = max(tmax[j], (unsigned long long)(c[j][0] - c[j][1] - c[j][2] + c[j][3]));
                ya = yb;
            }
#pragma unroll
            for (int j = 0; j < kChunk; j++) rec[rid * kRecRow + j] = tmax[j];
        }
        {
            u32x4 *dst = reinterpret_cast<u32x4 *>(srid);
            if (tid < nv) dst[tid] = piece;
            for (int v = tid + BS; v < nv; v += BS) dst[v] = rsrc[v];
        }
        __syncthreads();
        // phase 2: one candidate per lane, every frame of the chunk at once
        unsigned long long tmin[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; j++) tmin[j] = kNone;
        for (int e = tid; e < n; e += BS) {
            unsigned long long cur[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; j++) cur[j] = 0;
#pragma unroll 2
            for (int t = 0; t < T; t++) {
                const unsigned long long *row = rec + (int)srid[t * n + e] * kRecRow;
#pragma unroll
                for (int j = 0; j < kChunk; j++) cur[j] = max(cur[j], row[j]);
            }
#pragma unroll
            for (int j = 0; j < kChunk; j++) tmin[j] = min(tmin[j], cur[j]);
        }
        const unsigned long long v = wave_min8(tmin, lane);
        if ((lane & 7) == 0) red[(lane >> 3) & 7][wv] = v;
        __syncthreads();
        if (tid < kChunk) {
            const int base = sl[tid].item_base;
            if (base >= 0) {
                unsigned long long m = kNone;
                for (int w = 0; w < NW; w++) m = min(m, red[tid][w]);
                item_min[base + ud.item] = m;
            }
        }
    }
}

// One work-group per frame: the frame's winner over its items' partials, decoded.
__global__ void __launch_bounds__(256)
k_final_batch(const SpaceView *__restrict__ plans, const BatchFrameDev *__restrict__ frames,
              const Partial *__restrict__ part, char *ws, trs_result *out)
{
    const BatchFrameDev fr = frames[blockIdx.x];
    const SpaceView sp = plans[fr.plan];
    final_block<256>(sp, part + fr.item_base, fr.n_items,
                     reinterpret_cast<const WsHeader *>(ws + fr.o_hdr),
                     reinterpret_cast<const long long *>(ws + fr.o_satT),
                     reinterpret_cast<const long long *>(ws + fr.o_satS1),
                     reinterpret_cast<const long long *>(ws + fr.o_satS2), out + blockIdx.x,
                     fr.dt, fr.dr);
}

// Batched step 2 over the live list of (frame, item) entries, split evenly over the grid.
// Per entry: the item's record indices go to LDS in 16-byte pieces; each thread builds
// records from their compact descriptors with every corner load of the three SATs issued
// before use (pixel sizes come from the CTU grid: a column boundary x sits at min(x cs, w));
// lanes score candidates against the frame's Eq. 4 bound and keep the least (Q, T~, rank).
template <int BS>
__global__ void __launch_bounds__(BS)
k_step2_live(const BatchFrameDev *__restrict__ frames, const ItemBrief *__restrict__ briefs,
             const unsigned long long *__restrict__ live, const int *__restrict__ live_n, int cs,
             int rec_max, char *ws, Partial *__restrict__ part)
{
    constexpr int NW = BS / kWave;
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned long long *recT = reinterpret_cast<unsigned long long *>(lds);
    unsigned long long *recQ = recT + rec_max;
    uint16_t *srid = reinterpret_cast<uint16_t *>(recQ + rec_max);
    __shared__ unsigned long long redq[NW], redt[NW];
    __shared__ long long redr[NW];
    __shared__ int redf[NW];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int total = *live_n;
    const int G = gridDim.x, b = xcd_item(blockIdx.x, G);
    const int beg = (int)((long long)total * b / G), end = (int)((long long)total * (b + 1) / G);
    for (int x = beg; x < end; x++) {
        const unsigned long long en = live[x];
        const int f = (int)(en >> 32), i = (int)(unsigned)en;
        const BatchFrameDev &fr = frames[f];
        const ItemBrief ib = briefs[fr.brief_base + i];
        const int n = ib.n_ent, T = ib.T, S = fr.W + 1, w = fr.w, h = fr.h;
        const unsigned long long bound = reinterpret_cast<const WsHeader *>(ws + fr.o_hdr)->bound;
        const gptr<char> sT = as_global(ws + fr.o_satT), s1 = as_global(ws + fr.o_satS1);
        const gptr<char> s2 = as_global(ws + fr.o_satS2);
        __syncthreads();                                // the previous entry's LDS is read
        const gptr<u32x4> rsrc = as_global(reinterpret_cast<const u32x4 *>(ib.rids));
        const int nv = (n * T + 7) >> 3;
        u32x4 piece = {0u, 0u, 0u, 0u};
        if (tid < nv) piece = rsrc[tid];
        const gptr<u32x4> rd = as_global(reinterpret_cast<const u32x4 *>(ib.rdesc4));
        for (int rid = tid; rid < ib.n_rec; rid += BS) {
            const u32x4 d = rd[rid];
            const int xa = d.x & 511, xb = (d.x >> 9) & 511, y0 = (int)(d.x >> 18);
            const int k = d.y & 255;
            const unsigned wpx = (unsigned)(min(xb * cs, w) - xa * cs);
            unsigned long long tmax = 0, qs = 0;
            auto at = [](gptr<char> base, unsigned o) { return *(const gptr<long long>)(base + o); };
            // a slice's top corners are the previous slice's bottom corners
            const unsigned p00 = 8u * (unsigned)(y0 * S + xa), p01 = 8u * (unsigned)(y0 * S + xb);
            long long tt0 = at(sT, p00), tt1 = at(sT, p01), ta0 = at(s1, p00), ta1 = at(s1, p01);
            long long tb0 = at(s2, p00), tb1 = at(s2, p01);
            int ya = y0;
            for (int q = 0; q < k; q++) {
                const int zi = q + 1;
                const uint32_t wsel = zi < 4 ? d.y : zi < 8 ? d.z : d.w;
                const int yb = y0 + (int)((wsel >> (8 * (zi & 3))) & 255);
                const unsigned o10 = 8u * (unsigned)(yb * S + xa), o11 = 8u * (unsigned)(yb * S + xb);
                const long long bt0 = at(sT, o10), bt1 = at(sT, o11), ba0 = at(s1, o10), ba1 = at(s1, o11);
                const long long bb0 = at(s2, o10), bb1 = at(s2, o11);
                const unsigned hpx = (unsigned)(min(yb * cs, h) - ya * cs);
                tmax = max(tmax, (unsigned long long)(bt1 - tt1 - bt0 + tt0));
                qs += (unsigned long long)(bb1 - tb1 - bb0 + tb0) -
                      floor_sq_div((unsigned long long)(ba1 - ta1 - ba0 + ta0), wpx * hpx);
                tt0 = bt0; tt1 = bt1; ta0 = ba0; ta1 = ba1; tb0 = bb0; tb1 = bb1;
                ya = yb;
            }
            recT[rid] = tmax;
            recQ[rid] = qs;
        }
        {
            u32x4 *dst = reinterpret_cast<u32x4 *>(srid);
            if (tid < nv) dst[tid] = piece;
            for (int v = tid + BS; v < nv; v += BS) dst[v] = rsrc[v];
        }
        __syncthreads();
        Key2 best{kNone, kNone, LLONG_MAX, -1};
        for (int e = tid; e < n; e += BS) {
            unsigned long long tmax = 0, qsum = 0;
#pragma unroll 4
            for (int t = 0; t < T; t++) {
                const int rr = srid[t * n + e];
                tmax = max(tmax, recT[rr]);
                qsum += recQ[rr];
            }
            if (tmax <= bound && (qsum < best.q || (qsum == best.q && tmax <= best.t))) {
                const int fe = (int)as_global(ib.ent_f)[e];
                const int xl = fe / ib.M;
                const Key2 cand{qsum, tmax, ib.rank0 + (long long)xl * ib.SM + (fe - xl * ib.M), fe};
                if (key_less(cand, best)) best = cand;
            }
        }
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
            Key2 bk{redq[0], redt[0], redr[0], redf[0]};
            for (int q = 1; q < NW; q++) {
                const Key2 o{redq[q], redt[q], redr[q], redf[q]};
                if (key_less(o, bk)) bk = o;
            }
            part[fr.item_base + i] = Partial{bk.q, bk.t, bk.rank, i, bk.f, n, 0};
        }
    }
}

inline void mark(const hipEvent_t *ev, int i, hipStream_t s)
{
    if (ev) (void)hipEventRecord(ev[i], s);
}

template <int BS>
void launch_batch_search(const BatchLaunch &b, char *ws, hipStream_t s, const hipEvent_t *ev)
{
    auto *imin = reinterpret_cast<unsigned long long *>(ws + b.o_item_min);
    auto *part = reinterpret_cast<Partial *>(ws + b.o_part);
    auto *live = reinterpret_cast<unsigned long long *>(ws + b.o_live);
    auto *live_n = reinterpret_cast<int *>(ws + b.o_live_n);
    if (b.units)
        hipLaunchKernelGGL(k_step1_units<BS>, dim3(b.grid_u), dim3(BS), unit_lds_bytes(b.rec_max, b.rid_max),
                           s, b.units, b.slots, b.n_units, b.rec_max, ws, imin);
    else
        hipLaunchKernelGGL((k_search_batch<BS, false>), dim3(b.grid1), dim3(BS),
                           batch_lds_bytes(b.rec_max, false), s, b.plans, b.frames, b.item_frame,
                           b.total_items, ws, imin, part, b.rec_max, live, live_n);
    mark(ev, 3, s);
    hipLaunchKernelGGL(k_tmin_batch, dim3(b.n_frames), dim3(256), 0, s, b.frames, imin, ws, part,
                       live, live_n);
    mark(ev, 4, s);
    if (b.briefs)
        hipLaunchKernelGGL(k_step2_live<BS>, dim3(b.grid2), dim3(BS), step2_lds_bytes(b.rec_max, b.rid_max), s,
                           b.frames, b.briefs, live, live_n, b.cs, b.rec_max, ws, part);
    else
        hipLaunchKernelGGL((k_search_batch<BS, true>), dim3(b.grid2), dim3(BS),
                           batch_lds_bytes(b.rec_max, true), s, b.plans, b.frames, b.item_frame,
                           b.total_items, ws, imin, part, b.rec_max, live, live_n);
}

template <int BS>
int occupancy_of(int rec_max, bool step2)
{
    int n = 0;
    const int lds = batch_lds_bytes(rec_max, step2);
    hipError_t e = step2
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search_batch<BS, true>, BS, lds)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search_batch<BS, false>, BS, lds);
    return e == hipSuccess && n > 0 ? n : 1;
}

template <int BS>
int unit_occupancy_of(int lds)
{
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step1_units<BS>, BS, lds);
    return e == hipSuccess && n > 0 ? n : 1;
}
}  // namespace

int step2_lds_bytes(int rec_max, int rid_max)
{
    return 16 * (rec_max > 0 ? rec_max : 1) + 2 * ((rid_max + 7) & ~7);
}

int step2_occupancy(int block, int rec_max, int rid_max)
{
    const int lds = step2_lds_bytes(rec_max, rid_max);
    int n = 0;
    hipError_t e;
    switch (block) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step2_live<64>, 64, lds); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step2_live<128>, 128, lds); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step2_live<512>, 512, lds); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step2_live<256>, 256, lds); break;
    }
    return e == hipSuccess && n > 0 ? n : 1;
}

int unit_lds_bytes(int rec_max, int rid_max)
{
    const long long bytes = 8ll * kRecRow * (rec_max > 0 ? rec_max : 1) + 2ll * ((rid_max + 7) & ~7);
    return bytes <= 65536 ? (int)bytes : 0;
}

int unit_occupancy(int block, int rec_max, int rid_max)
{
    const int lds = unit_lds_bytes(rec_max, rid_max);
    switch (block) {
    case 64: return unit_occupancy_of<64>(lds);
    case 128: return unit_occupancy_of<128>(lds);
    case 512: return unit_occupancy_of<512>(lds);
    default: return unit_occupancy_of<256>(lds);
    }
}

WsLayout ws_layout(const Plan &pl)
{
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    WsLayout l{};
    const size_t sat = sizeof(long long) * (size_t)(pl.W + 1) * (pl.H + 1);
    const size_t n = pl.items.size();
    l.header = 0;
    l.satT = up(sizeof(WsHeader));
    l.satS1 = l.satT + up(sat);
    l.satS2 = l.satS1 + up(sat);
    l.item_min = l.satS2 + up(sat);
    l.live = l.item_min + up(sizeof(unsigned long long) * n);
    l.partial = l.live + up(sizeof(int) * n);
    l.total = l.partial + up(sizeof(Partial) * n);
    return l;
}

hipError_t launch_features(int w, int h, int cs, const uint16_t *luma, int64_t stride,
                           const trs_feat &o, hipStream_t s)
{
    const int W = (w + cs - 1) / cs;
    const dim3 grid(W * ((h + cs - 1) / cs));
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
    const WsPtrs w = ws_ptrs(a);
    if ((a.sp.W + 1) * (a.sp.H + 1) <= kSatLds)
        hipLaunchKernelGGL(k_sat_lds, dim3(1), dim3(256), 0, s, a.sp.W, a.sp.H, a.cost, a.s1,
                           (const unsigned long long *)a.s2, w.satT, w.satS1, w.satS2, w.hdr);
    else
        hipLaunchKernelGGL(k_sat, dim3(1), dim3(256), 0, s, a.sp.W, a.sp.H, a.cost, a.s1,
                           (const unsigned long long *)a.s2, w.satT, w.satS1, w.satS2, w.hdr);
    return launch_after_sat(a, s);
}

hipError_t launch_partition_tail(const SearchArgs &a, const uint32_t *tex, const uint32_t *prev,
                                 trs_blend b, uint32_t *cost, uint32_t *flags, hipStream_t s)
{
    const WsPtrs w = ws_ptrs(a);
    if ((a.sp.W + 1) * (a.sp.H + 1) <= kSatLds) {
        hipLaunchKernelGGL(k_cost_sat, dim3(1), dim3(256), 0, s, a.sp.W, a.sp.H, tex, prev, b.a,
                           b.b, b.w_prev, cost, flags, a.s1, (const unsigned long long *)a.s2,
                           w.satT, w.satS1, w.satS2, w.hdr);
        if (hipGetLastError() != hipSuccess) return hipErrorUnknown;
        return launch_after_sat(a, s);
    }
    const hipError_t e = launch_cost_map(a.sp.W * a.sp.H, tex, prev, b, cost, flags, s);
    if (e != hipSuccess) return e;
    return launch_search(a, s);
}

long long batch_frame_region(int W, int H, BatchFrameDev *fr, long long base)
{
    auto up = [](long long v) { return (v + 255) & ~255ll; };
    const long long n = (long long)W * H, sat = 8ll * (W + 1) * (H + 1);
    long long o = base;
    fr->o_s1 = o;   o += up(4 * n);
    fr->o_grad = o; o += up(4 * n);
    fr->o_tex = o;  o += up(4 * n);
    fr->o_mean = o; o += up(4 * n);
    fr->o_var = o;  o += up(4 * n);
    fr->o_s2 = o;   o += up(8 * n);
    fr->o_cost = o; o += up(4 * n);
    fr->o_hdr = o;  o += up(sizeof(WsHeader));
    fr->o_satT = o; o += up(sat);
    fr->o_satS1 = o; o += up(sat);
    fr->o_satS2 = o; o += up(sat);
    return o;
}

int batch_lds_bytes(int rec_max, bool step2)
{
    const int rec = rec_max > 0 ? rec_max : 1;
    return 8 * rec * (step2 ? 2 : 1);
}

int batch_occupancy(int block, int rec_max, bool step2)
{
    switch (block) {
    case 64: return occupancy_of<64>(rec_max, step2);
    case 128: return occupancy_of<128>(rec_max, step2);
    case 512: return occupancy_of<512>(rec_max, step2);
    default: return occupancy_of<256>(rec_max, step2);
    }
}

hipError_t launch_batch(const BatchLaunch &b, char *ws, trs_result *out, hipStream_t s,
                        const hipEvent_t *ev, int stages)
{
    mark(ev, 0, s);
    if (stages & kStageFeatures) switch (b.cs) {
    case 128:
        hipLaunchKernelGGL(k_features_batch<128>, dim3(b.total_ctus), dim3(256), 0, s, b.frames,
                           b.ctu_frame, ws);
        break;
    case 64:
        hipLaunchKernelGGL(k_features_batch<64>, dim3(b.total_ctus), dim3(128), 0, s, b.frames,
                           b.ctu_frame, ws);
        break;
    default:
        hipLaunchKernelGGL(k_features_batch<32>, dim3(b.total_ctus), dim3(64), 0, s, b.frames,
                           b.ctu_frame, ws);
        break;
    }
    mark(ev, 1, s);
    if (!(stages & kStageSearch)) return hipGetLastError();
    hipLaunchKernelGGL(k_cost_sat_batch, dim3(b.n_frames), dim3(256), 0, s, b.frames, ws,
                       reinterpret_cast<int *>(ws + b.o_live_n));
    mark(ev, 2, s);
    if (b.total_items > 0) {
        switch (b.block) {
        case 64: launch_batch_search<64>(b, ws, s, ev); break;
        case 128: launch_batch_search<128>(b, ws, s, ev); break;
        case 512: launch_batch_search<512>(b, ws, s, ev); break;
        default: launch_batch_search<256>(b, ws, s, ev); break;
        }
    } else {
        mark(ev, 3, s);
        hipLaunchKernelGGL(k_tmin_batch, dim3(b.n_frames), dim3(256), 0, s, b.frames,
                           reinterpret_cast<unsigned long long *>(ws + b.o_item_min), ws,
                           reinterpret_cast<Partial *>(ws + b.o_part),
                           reinterpret_cast<unsigned long long *>(ws + b.o_live),
                           reinterpret_cast<int *>(ws + b.o_live_n));
        mark(ev, 4, s);
    }
    mark(ev, 5, s);
    hipLaunchKernelGGL(k_final_batch, dim3(b.n_frames), dim3(256), 0, s, b.plans, b.frames,
                       reinterpret_cast<const Partial *>(ws + b.o_part), ws, out);
    mark(ev, 6, s);
    return hipGetLastError();
}

}  // namespace trs
