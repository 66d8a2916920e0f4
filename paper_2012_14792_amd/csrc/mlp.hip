// Learned per-CTU time predictor: a 10 -> 64 -> 64 -> 1 perceptron with exact (erf) GELU,
// FP32, standing in for the previous-frame time estimator of Section 2.1 (the paper's
// conclusion names a better CTU time estimator as future work).
//
//   k_mlp_inputs      the 10 raw inputs per CTU from the method's own features and times
//   k_mlp_fwd         four lanes per sample, weights in LDS; optionally keeps z1, z2
//   k_mlp_bwd_data    per sample (four lanes) dz2 = dy W3 * gelu'(z2), dz1 = (W2^T dz2) * gelu'(z1),
//                     and the activations gelu(z1), gelu(z2) from the same erf
//   k_mlp_bwd_w       weight gradients: each work-group sums its sample chunk into one
//                     partial (entries spread over threads, samples staged in LDS tiles)
//   k_mlp_reduce*     partials summed in two fixed-order passes, one thread per entry
//   k_mlp_cost        prediction -> u32 microseconds, or the plain blend per CTU when the
//                     prediction is not finite or an input is outside the training range
#include <hip/hip_runtime.h>

#include "mlp.hpp"

namespace trs {
namespace {

constexpr int kIn = kMlpIn, kHid = kMlpHid;
constexpr int kEntries = kHid * kIn + kHid + kHid * kHid + kHid + kHid + 1;   // 4929
constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * kInvSqrt2)); }

// gelu(x) and d/dx gelu(x) = Phi(x) + x phi(x) from one erf, with the same operations (and so
// the same values) as gelu() above
__device__ __forceinline__ void gelu_and_grad(float x, float &g, float &d)
{
    const float e = erff(x * kInvSqrt2);
    g = 0.5f * x * (1.0f + e);
    d = 0.5f * (1.0f + e) + x * kInvSqrt2Pi * expf(-0.5f * x * x);
}

struct Weights {
    const float *w1, *b1, *w2, *b2, *w3, *b3;
};

__global__ void __launch_bounds__(256)
k_mlp_inputs(int W, int H, int cs, int w, int h, const uint32_t *__restrict__ tex,
             const uint32_t *__restrict__ var, const uint32_t *__restrict__ mean,
             const uint32_t *__restrict__ prev, float *__restrict__ x)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= W * H) return;
    const int cy = c / W, cx = c - cy * W;
    const int l = cx > 0 ? c - 1 : c, r = cx + 1 < W ? c + 1 : c;
    const int u = cy > 0 ? c - W : c, d = cy + 1 < H ? c + W : c;
    const float n = (float)(min(cs, w - cx * cs) * min(cs, h - cy * cs));
    float *o = x + (long long)c * kIn;
    o[0] = (float)tex[c];
    o[1] = (float)var[c];
    o[2] = (float)mean[c];
    o[3] = (float)tex[l];
    o[4] = (float)tex[r];
    o[5] = (float)tex[u];
    o[6] = (float)tex[d];
    o[7] = (float)prev[c];
    o[8] = 0.25f * ((float)prev[l] + (float)prev[r] + (float)prev[u] + (float)prev[d]);
    o[9] = n / (float)(cs * cs);
}

// Lanes 4i .. 4i + 3 (one DPP quad) work on one sample; quarter q of the quad owns hidden units
// 16 q .. 16 q + 15 of each layer.  quad_from<m> returns the value of lane q ^ m of the quad.
constexpr int kLanes = 4, kQ = kHid / kLanes;

template <int M>
__device__ __forceinline__ float quad_from(float v)
{
    constexpr int ctrl = M == 1 ? 0xB1 : M == 2 ? 0x4E : 0x1B;   // quad_perm [1,0,3,2] [2,3,0,1] [3,2,1,0]
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF,
                                                                 0xF, false));
}

// Sum of one value per quad lane in the fixed order (v0 + v1) + (v2 + v3); every lane gets it.
__device__ __forceinline__ float quad_sum(float v, int q)
{
    const float o1 = quad_from<1>(v);
    const float pair = (q & 1) ? o1 + v : v + o1;                 // lanes 0,1: v0 + v1; 2,3: v2 + v3
    const float o2 = quad_from<2>(pair);
    return (q & 2) ? o2 + pair : pair + o2;
}

// LDS copies of W1 and W2 for the four-lane kernels: row r = 16 q + kk is stored at position
// 4 kk + q (the four quarters' rows side by side) and W2 rows are padded to 65 floats, so the
// four addresses one load instruction reads from a quad lie in four different banks.
constexpr int kW2Pitch = kHid + 1;

__device__ __forceinline__ int qrow(int r) { return (r % kQ) * kLanes + r / kQ; }

__device__ __forceinline__ void load_weights_q(const Weights &w, float *sW1, float *sb1, float *sW2,
                                               float *sb2, float *sW3, float *sb3)
{
    for (int i = threadIdx.x; i < kHid * kIn; i += blockDim.x) sW1[qrow(i / kIn) * kIn + i % kIn] = w.w1[i];
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x)
        sW2[qrow(i / kHid) * kW2Pitch + i % kHid] = w.w2[i];
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        sb1[i] = w.b1[i];
        sb2[i] = w.b2[i];
        sW3[i] = w.w3[i];
    }
    if (threadIdx.x == 0) sb3[0] = w.b3[0];
}

// Four lanes per sample: each evaluates its quarter of the first layer, the quad exchanges the
// quarters, each evaluates its quarter of the second layer and its share of the output, and the
// quad adds the shares in a fixed order.
__global__ void __launch_bounds__(256)
k_mlp_fwd(Weights wt, trs_mlp_norm nm, const float *__restrict__ x, long long n,
          float *__restrict__ y, float *__restrict__ z1o, float *__restrict__ z2o)
{
    __shared__ float sW1[kHid * kIn], sb1[kHid], sW2[kHid * kW2Pitch], sb2[kHid], sW3[kHid], sb3[1];
    load_weights_q(wt, sW1, sb1, sW2, sb2, sW3, sb3);
    __syncthreads();
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long s = g / kLanes;
    const int q = (int)(g % kLanes);
    const bool ok = s < n;                     // the four lanes of a quad agree
    const long long sc = ok ? s : 0;
    float xn[kIn];
#pragma unroll
    for (int i = 0; i < kIn; i++) xn[i] = (x[sc * kIn + i] - nm.mean[i]) * nm.inv_std[i];
    float mine[kQ], h1[kHid];
#pragma unroll
    for (int jj = 0; jj < kQ; jj++) {
        const int j = kQ * q + jj;
        float z = sb1[j];
#pragma unroll
        for (int i = 0; i < kIn; i++) z = fmaf(sW1[(jj * kLanes + q) * kIn + i], xn[i], z);
        if (z1o && ok) z1o[(long long)j * n + s] = z;
        mine[jj] = gelu(z);
    }
#pragma unroll
    for (int jj = 0; jj < kQ; jj++) {
        const float v[4] = {mine[jj], quad_from<1>(mine[jj]), quad_from<2>(mine[jj]), quad_from<3>(mine[jj])};
        // quarter Q comes from lane q ^ Q, i.e. v[q ^ Q]
#pragma unroll
        for (int Q = 0; Q < kLanes; Q++) {
            const int m = q ^ Q;
            h1[kQ * Q + jj] = m == 0 ? v[0] : m == 1 ? v[1] : m == 2 ? v[2] : v[3];
        }
    }
    float part = 0.0f;
    for (int kk = 0; kk < kQ; kk++) {
        const int k = kQ * q + kk;
        float z = sb2[k];
#pragma unroll
        for (int j = 0; j < kHid; j++) z = fmaf(sW2[(kk * kLanes + q) * kW2Pitch + j], h1[j], z);
        if (z2o && ok) z2o[(long long)k * n + s] = z;
        part = fmaf(sW3[k], gelu(z), part);
    }
    const float tot = quad_sum(part, q);
    if (ok && q == 0) y[s] = sb3[0] + tot;
}

// Four lanes per sample: the lane of quarter q owns dz2 for k in 16 q .. 16 q + 15, forms its
// share of W2^T dz2 for every j, and the quad adds the shares in a fixed order; each lane then
// writes dz1 (and the activations) for its quarter of j.
__global__ void __launch_bounds__(256)
k_mlp_bwd_data(Weights wt, const float *__restrict__ z1, const float *__restrict__ z2,
               const float *__restrict__ dy, long long n, float *__restrict__ dz1o,
               float *__restrict__ dz2o, float *__restrict__ h1o, float *__restrict__ h2o)
{
    __shared__ float sW1[kHid * kIn], sb1[kHid], sW2[kHid * kW2Pitch], sb2[kHid], sW3[kHid], sb3[1];
    load_weights_q(wt, sW1, sb1, sW2, sb2, sW3, sb3);
    __syncthreads();
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long s = g / kLanes;
    const int q = (int)(g % kLanes);
    const bool ok = s < n;
    const long long sc = ok ? s : 0;
    const float gy = dy[sc];
    float dz2[kQ];
#pragma unroll
    for (int kk = 0; kk < kQ; kk++) {
        const int k = kQ * q + kk;
        float gg, d;
        gelu_and_grad(z2[(long long)k * n + sc], gg, d);
        dz2[kk] = gy * sW3[k] * d;
        if (ok) {
            dz2o[(long long)k * n + s] = dz2[kk];
            h2o[(long long)k * n + s] = gg;
        }
    }
    for (int j = 0; j < kHid; j++) {
        float a = 0.0f;
#pragma unroll
        for (int kk = 0; kk < kQ; kk++) a = fmaf(sW2[(kk * kLanes + q) * kW2Pitch + j], dz2[kk], a);
        const float tot = quad_sum(a, q);
        if (ok && (j / kQ) == q) {
            float gg, d;
            gelu_and_grad(z1[(long long)j * n + s], gg, d);
            dz1o[(long long)j * n + s] = tot * d;
            h1o[(long long)j * n + s] = gg;
        }
    }
}

// Weight gradients of one sample chunk: sum over samples s of
//   dW1[j][i] += dz1[j] xn[i], db1 += dz1, dW2[k][j] += dz2[k] h1[j], db2 += dz2,
//   dW3[k] += dy h2[k], db3 += dy
// Samples are staged in LDS tiles.  Thread t owns 16 entries of dW2 (row k = t / 4, columns
// 16 (t % 4) ..) and up to 4 of the 833 other entries (dW1, db1, db2, dW3, db3 in that order).
constexpr int kTile = 32;
constexpr int kSmall = kHid * kIn + kHid + kHid + kHid + 1;          // 833
constexpr int kW2Off = kHid * kIn + kHid;                            // dW2 in the entry order

__device__ __forceinline__ int small_to_entry(int q)
{
    // small entries: dW1 (640), db1 (64), db2 (64), dW3 (64), db3 (1)
    return q < kHid * kIn + kHid ? q : q + kHid * kHid;
}

__global__ void __launch_bounds__(256)
k_mlp_bwd_w(trs_mlp_norm nm, const float *__restrict__ x, const float *__restrict__ h1,
            const float *__restrict__ h2, const float *__restrict__ dz1,
            const float *__restrict__ dz2, const float *__restrict__ dy, long long n,
            int chunk, float *__restrict__ partial)
{
    // rows padded by one float: the staging writes walk r (samples) fastest
    __shared__ float tx[kTile][kIn], th1[kTile][kHid + 1], th2[kTile][kHid + 1];
    __shared__ float tdz1[kTile][kHid + 1], tdz2[kTile][kHid + 1], tdy[kTile];
    const int tid = threadIdx.x;
    const int k2 = tid >> 2, j2 = (tid & 3) * 16;
    float a2[16];
#pragma unroll
    for (int q = 0; q < 16; q++) a2[q] = 0.0f;
    float as[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const long long s0 = (long long)blockIdx.x * chunk;
    const long long s1 = min(n, s0 + chunk);
    for (long long t0 = s0; t0 < s1; t0 += kTile) {
        const int nt = (int)min<long long>(kTile, s1 - t0);
        __syncthreads();
#pragma unroll 1
        for (int e = tid; e < kTile * kHid; e += blockDim.x) {
            // consecutive threads read consecutive samples of one row j of the [64][n] arrays
            const int j = e / kTile, r = e - j * kTile;
            const bool in = r < nt;
            const long long s = t0 + r;
            th1[r][j] = in ? h1[(long long)j * n + s] : 0.0f;
            th2[r][j] = in ? h2[(long long)j * n + s] : 0.0f;
            tdz1[r][j] = in ? dz1[(long long)j * n + s] : 0.0f;
            tdz2[r][j] = in ? dz2[(long long)j * n + s] : 0.0f;
        }
        for (int e = tid; e < kTile * kIn; e += blockDim.x) {
            const int r = e / kIn, i = e - r * kIn;
            tx[r][i] = r < nt ? (x[(t0 + r) * kIn + i] - nm.mean[i]) * nm.inv_std[i] : 0.0f;
        }
        for (int r = tid; r < kTile; r += blockDim.x) tdy[r] = r < nt ? dy[t0 + r] : 0.0f;
        __syncthreads();
#pragma unroll 2
        for (int r = 0; r < kTile; r++) {
            const float d = tdz2[r][k2];
#pragma unroll
            for (int q = 0; q < 16; q++) a2[q] = fmaf(d, th1[r][j2 + q], a2[q]);
        }
#pragma unroll 1
        for (int q = 0; q < 4; q++) {
            const int sidx = tid + q * 256;
            if (sidx >= kSmall) break;
            float a = as[q];
            if (sidx < kHid * kIn) {                         // dW1[j][i]
                const int j = sidx / kIn, i = sidx - j * kIn;
                for (int r = 0; r < kTile; r++) a = fmaf(tdz1[r][j], tx[r][i], a);
            } else if (sidx < kHid * kIn + kHid) {           // db1[j]
                const int j = sidx - kHid * kIn;
                for (int r = 0; r < kTile; r++) a += tdz1[r][j];
            } else if (sidx < kHid * kIn + 2 * kHid) {       // db2[k]
                const int k = sidx - kHid * kIn - kHid;
                for (int r = 0; r < kTile; r++) a += tdz2[r][k];
            } else if (sidx < kSmall - 1) {                  // dW3[k]
                const int k = sidx - kHid * kIn - 2 * kHid;
                for (int r = 0; r < kTile; r++) a = fmaf(tdy[r], th2[r][k], a);
            } else {                                         // db3
                for (int r = 0; r < kTile; r++) a += tdy[r];
            }
            as[q] = a;
        }
    }
    float *out = partial + (long long)blockIdx.x * kEntries;
#pragma unroll
    for (int q = 0; q < 16; q++) out[kW2Off + k2 * kHid + j2 + q] = a2[q];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int sidx = tid + q * 256;
        if (sidx < kSmall) out[small_to_entry(sidx)] = as[q];
    }
}

struct Grads {
    float *w1, *b1, *w2, *b2, *w3, *b3;
};

// The partials are summed in two fixed-order passes, one thread per gradient entry (lanes read
// consecutive entries of a partial, so loads are coalesced): pass 1 sums groups of kGroup
// consecutive partials, pass 2 the group sums in order.  The result repeats exactly.
constexpr int kGroup = 32;

__global__ void __launch_bounds__(256)
k_mlp_reduce_groups(const float *__restrict__ partial, int n_part, float *__restrict__ grp)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x, g = blockIdx.y;
    if (e >= kEntries) return;
    const int p1 = min(n_part, (g + 1) * kGroup);
    float a = 0.0f;
#pragma unroll 8
    for (int p = g * kGroup; p < p1; p++) a += partial[(long long)p * kEntries + e];
    grp[(long long)g * kEntries + e] = a;
}

__global__ void __launch_bounds__(256)
k_mlp_reduce(const float *__restrict__ grp, int n_grp, Grads g)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kEntries) return;
    float a = 0.0f;
#pragma unroll 8
    for (int q = 0; q < n_grp; q++) a += grp[(long long)q * kEntries + e];
    int o = e;
    if (o < kHid * kIn) { g.w1[o] = a; return; }
    o -= kHid * kIn;
    if (o < kHid) { g.b1[o] = a; return; }
    o -= kHid;
    if (o < kHid * kHid) { g.w2[o] = a; return; }
    o -= kHid * kHid;
    if (o < kHid) { g.b2[o] = a; return; }
    o -= kHid;
    if (o < kHid) { g.w3[o] = a; return; }
    g.b3[0] = a;
}

__global__ void __launch_bounds__(256)
k_mlp_cost(long long n, const float *__restrict__ y, const float *__restrict__ x,
           trs_mlp_norm nm, const uint32_t *__restrict__ tex, const uint32_t *__restrict__ prev,
           uint32_t a, uint32_t b, uint32_t wp, uint32_t *__restrict__ cost,
           uint32_t *__restrict__ n_fallback)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    bool ok = isfinite(y[c]);
    for (int i = 0; i < kIn; i++) {
        const float v = x[c * kIn + i];
        ok = ok && v >= nm.lo[i] && v <= nm.hi[i];
    }
    const float us = rintf(1000.0f * y[c]);
    if (ok) {
        // 2^31 is the first float above the clamp
        cost[c] = us < 1.0f ? 1u : us < 2147483648.0f ? (uint32_t)us : 0x7fffffffu;
        return;
    }
    // plain blend, as the cost map computes it (w = 256: the previous time)
    const unsigned long long model = (unsigned long long)a + (unsigned long long)b * tex[c];
    unsigned long long v;
    if (prev == nullptr) v = model;
    else if (wp == 256u) v = prev[c];
    else if (model >= (1ull << 40)) v = ~0ull;
    else v = ((unsigned long long)wp * prev[c] + (unsigned long long)(256u - wp) * model + 128ull) >> 8;
    cost[c] = (uint32_t)min(v, (unsigned long long)0x7fffffff);
    if (n_fallback) atomicAdd(n_fallback, 1u);
}

}  // namespace

hipError_t launch_mlp_inputs(int W, int H, int cs, int w, int h, const uint32_t *tex,
                             const uint32_t *var, const uint32_t *mean, const uint32_t *prev,
                             float *x, hipStream_t s)
{
    const int n = W * H;
    hipLaunchKernelGGL(k_mlp_inputs, dim3((n + 255) / 256), dim3(256), 0, s, W, H, cs, w, h, tex, var,
                       mean, prev, x);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const trs_mlp &m, const trs_mlp_norm &nm, const float *x, long long n,
                              float *y, float *z1, float *z2, hipStream_t s)
{
    const Weights w{m.w1, m.b1, m.w2, m.b2, m.w3, m.b3};
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((kLanes * n + 255) / 256)), dim3(256), 0, s, w, nm, x, n,
                       y, z1, z2);
    return hipGetLastError();
}

size_t mlp_backward_workspace(long long n)
{
    const long long chunk = mlp_chunk(n);
    const long long parts = (n + chunk - 1) / chunk, groups = (parts + kGroup - 1) / kGroup;
    return (size_t)(4 * kHid * n + (parts + groups) * kEntries) * sizeof(float) + 512;
}

long long mlp_chunk(long long n)
{
    // about 4 work-groups per CU for the weight-gradient kernel, at least one tile each
    long long c = (n + 1023) / 1024;
    c = (c + kTile - 1) / kTile * kTile;
    return c < kTile ? kTile : c;
}

hipError_t launch_mlp_backward(const trs_mlp &m, const trs_mlp_norm &nm, const float *x,
                               const float *z1, const float *z2, const float *dy, long long n,
                               const trs_mlp_grads &g, char *ws, hipStream_t s)
{
    const Weights w{m.w1, m.b1, m.w2, m.b2, m.w3, m.b3};
    float *dz1 = reinterpret_cast<float *>(ws);
    float *dz2 = dz1 + kHid * n;
    float *h1 = dz2 + kHid * n;
    float *h2 = h1 + kHid * n;
    float *part = h2 + kHid * n;
    const long long chunk = mlp_chunk(n);
    const int parts = (int)((n + chunk - 1) / chunk), groups = (parts + kGroup - 1) / kGroup;
    float *grp = part + (long long)parts * kEntries;
    hipLaunchKernelGGL(k_mlp_bwd_data, dim3((unsigned)((kLanes * n + 255) / 256)), dim3(256), 0, s, w, z1,
                       z2, dy, n, dz1, dz2, h1, h2);
    hipLaunchKernelGGL(k_mlp_bwd_w, dim3(parts), dim3(256), 0, s, nm, x, h1, h2, dz1, dz2, dy, n,
                       (int)chunk, part);
    const Grads gg{g.w1, g.b1, g.w2, g.b2, g.w3, g.b3};
    const unsigned eb = (unsigned)((kEntries + 255) / 256);
    hipLaunchKernelGGL(k_mlp_reduce_groups, dim3(eb, (unsigned)groups), dim3(256), 0, s, part, parts, grp);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(eb), dim3(256), 0, s, grp, groups, gg);
    return hipGetLastError();
}

hipError_t launch_mlp_cost(long long n, const float *y, const float *x, const trs_mlp_norm &nm,
                           const uint32_t *tex, const uint32_t *prev, trs_blend b, uint32_t *cost,
                           uint32_t *n_fallback, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_cost, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, y, x, nm, tex,
                       prev, b.a, b.b, b.w_prev, cost, n_fallback);
    return hipGetLastError();
}

}  // namespace trs
