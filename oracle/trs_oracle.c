/*
 * Plain CPU oracle for dynamic tile + rectangular-slice (TRS) frame partitioning.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library.  It shares no code, header, table or
 * constant with the GPU library; it is written to be read against the paper, not to be fast.
 *
 * What it computes (Amestoy et al., "Quality-driven Dynamic VVC Frame Partitioning for
 * efficient Parallel Processing", ICIP 2020):
 *   - per-CTU luma statistics (sample count n, sum S1, sum of squares S2, gradient G) and
 *     the derived texture / mean / variance;                     (inputs of Section 2.2)
 *   - the per-CTU predicted time map T~(c): the co-located CTU time of the previous frame
 *     of the same temporal layer, optionally blended with a texture model;   (Section 2.1)
 *   - step 1: T~min = min over partitions P of T~(P), with T~(P) the largest region sum of
 *     T~(c);                                                      (Eq. 1 and Eq. 3)
 *   - step 2: among partitions with T~(P) <= T~min (1 + lambda), the one minimising the
 *     within-region luma sum of squared errors;                   (Eq. 2 and Eq. 4)
 *   - both steps search only partitions with k * A_min(P) > A_max(P), k = 3.  (Section 2.3)
 *   - the same two steps over the literal space (every CTU boundary allowed), solved exactly
 *     by decomposition instead of enumeration (orc_literal_search; pinned to the exhaustive
 *     search of that space where it finishes).
 *
 * Readings of points the paper leaves open (each is also listed in the design notes):
 *   - the number of rectangular slices (RS) equals the thread count N;
 *   - an RS is a run of whole CTU rows inside one tile; tiles form a grid;
 *   - the candidate set is an explicit space: c x r tile grids with c <= Cmax, r <= Rmax,
 *     c r <= N <= Kmax c r, column/row boundaries within +-dt CTUs of the uniform position,
 *     k_t in [1, min(Kmax, h_t)] slices per tile with split offsets within +-dr of the uniform
 *     position inside the tile, sum of k_t = N.  dt = dr = -1 means unbounded (every CTU
 *     boundary).  When both are requested as "ladder", the first window pair of
 *     (inf,inf), (3,1), (2,1), (1,1), (1,0), (0,0) whose space has at most `budget`
 *     candidates is used, else (0,0);
 *   - areas are counted in luma samples and the balance test is strict;
 *   - Eq. 2 is evaluated exactly in integers: per region q = S2 - floor(S1^2 / n), i.e. the
 *     ceiling of the real-valued SSE; Q(P) is the sum over regions;
 *   - the Eq. 4 bound is non-strict and lambda = num / den is rational (num < 0: infinite);
 *   - ties in step 2 are broken by smaller T~(P), then by the candidate's rank in the
 *     canonical enumeration order (shape (c, r), then X, then Y lexicographically, then the
 *     per-tile choices with the first tile most significant, each ordered by k then by the
 *     split offsets lexicographically);
 *   - the "uniform" partition (Section 3.2) is the c_u x r_u grid, c_u r_u = N, most square
 *     with c_u >= r_u, boundaries floor(i W / c_u) and floor(j H / r_u), one RS per tile.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXN 64
#define ORC_MAXB 65

typedef struct {
    int64_t rank, t_min, t_sel, q_sel, n_enumerated, n_feasible, uniform_rank, t_unif, q_unif;
    int32_t status, tile_cols, tile_rows, n_rs, dtile_used, drs_used;
    int32_t col_bd[ORC_MAXB], row_bd[ORC_MAXB];
    int32_t rs[ORC_MAXN][4];
    int64_t rs_time[ORC_MAXN];
} orc_result;

typedef struct {
    int32_t n_threads, max_tile_cols, max_tile_rows, max_rs_per_tile, area_k;
    int32_t lambda_num, lambda_den, dtile, drs;
    int32_t prune;          /* bit 0: slice heights within 2x in a tile; bit 1: tile mean areas */
    int32_t min_rs;         /* RS counts n in [min_rs, N] (idle threads); 0 means N */
    int32_t span_tiles;     /* 1: an RS may be a block of complete tiles stacked in one tile column */
    int64_t space_budget;
} orc_params;

/* ------------------------------------------------------------------------------------- */
/* Features: direct loops over the luma plane.                                           */
/* ------------------------------------------------------------------------------------- */

int orc_features(int w, int h, int cs, const uint16_t *luma, int64_t stride,
                 uint32_t *s1, uint64_t *s2, uint32_t *grad, uint32_t *tex,
                 uint32_t *mean, uint32_t *var)
{
    if (w <= 0 || h <= 0 || cs <= 0 || stride < w) return -1;
    int W = (w + cs - 1) / cs, H = (h + cs - 1) / cs;
    uint64_t *a1 = calloc((size_t)W * H, sizeof(uint64_t));
    uint64_t *a2 = calloc((size_t)W * H, sizeof(uint64_t));
    uint64_t *ag = calloc((size_t)W * H, sizeof(uint64_t));
    if (!a1 || !a2 || !ag) { free(a1); free(a2); free(ag); return -1; }
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) {
            int c = (y / cs) * W + (x / cs);
            int64_t p = luma[(int64_t)y * stride + x];
            a1[c] += (uint64_t)p;
            a2[c] += (uint64_t)(p * p);
            if (x + 1 < w) {
                int64_t d = (int64_t)luma[(int64_t)y * stride + x + 1] - p;
                ag[c] += (uint64_t)(d < 0 ? -d : d);
            }
            if (y + 1 < h) {
                int64_t d = (int64_t)luma[(int64_t)(y + 1) * stride + x] - p;
                ag[c] += (uint64_t)(d < 0 ? -d : d);
            }
        }
    }
    for (int cy = 0; cy < H; cy++) {
        for (int cx = 0; cx < W; cx++) {
            int c = cy * W + cx;
            int cw = (cx + 1) * cs <= w ? cs : w - cx * cs;
            int ch = (cy + 1) * cs <= h ? cs : h - cy * cs;
            unsigned __int128 n = (unsigned __int128)(cw * ch);
            s1[c] = (uint32_t)a1[c];
            s2[c] = a2[c];
            grad[c] = (uint32_t)ag[c];
            tex[c] = (uint32_t)(ag[c] / n);
            mean[c] = (uint32_t)(a1[c] / n);
            unsigned __int128 num = n * a2[c] - (unsigned __int128)a1[c] * a1[c];
            var[c] = (uint32_t)(num / (n * n));
        }
    }
    free(a1); free(a2); free(ag);
    return 0;
}

/* ------------------------------------------------------------------------------------- */
/* Cost map: co-located previous time, optionally blended with a + b * texture.          */
/* Returns -2 when a value does not fit in 31 bits (it is then clamped to 2^31 - 1).      */
/* ------------------------------------------------------------------------------------- */

int orc_cost_map(int n_ctu, const uint32_t *tex, const uint32_t *prev,
                 uint32_t a, uint32_t b, uint32_t w_prev, uint32_t *cost)
{
    const __int128 lim = ((__int128)1 << 31) - 1;
    int rc = 0;
    if (w_prev > 256) return -1;
    for (int c = 0; c < n_ctu; c++) {
        __int128 model = (__int128)a + (__int128)b * tex[c];
        __int128 v;
        if (prev == NULL)
            v = model;
        else
            v = ((__int128)w_prev * prev[c] + (__int128)(256 - w_prev) * model + 128) / 256;
        if (v > lim) { v = lim; rc = -2; }
        cost[c] = (uint32_t)v;
    }
    return rc;
}

/* ------------------------------------------------------------------------------------- */
/* Candidate space: window predicate, counting (for the ladder rule) and enumeration.    */
/* ------------------------------------------------------------------------------------- */

/* Is b a legal position for the i-th of m-1 boundaries inside [0, L] under window d? */
static int in_window(int b, int i, int m, int L, int d)
{
    if (d < 0) return 1;
    int centre = (int)(((int64_t)i * L) / m);
    int diff = b - centre;
    if (diff < 0) diff = -diff;
    return diff <= d;
}

/* Number of strictly increasing (b_1..b_{m-1}) in [1, L-1] within the windows. */
static uint64_t sat_add(uint64_t x, uint64_t y) { uint64_t s = x + y; return s < x ? UINT64_MAX : s; }
static uint64_t sat_mul(uint64_t x, uint64_t y)
{
    if (x == 0 || y == 0) return 0;
    if (x > UINT64_MAX / y) return UINT64_MAX;
    return x * y;
}

static uint64_t count_vectors_rec(int i, int prev, int m, int L, int d)
{
    if (i == m) return 1;
    uint64_t total = 0;
    for (int b = prev + 1; b <= L - 1; b++)
        if (in_window(b, i, m, L, d)) total = sat_add(total, count_vectors_rec(i + 1, b, m, L, d));
    return total;
}

/* DP form of the same count (the recursion above is exponential for large windows). */
static uint64_t count_vectors(int m, int L, int d)
{
    if (m == 1) return 1;
    if (m > L) return 0;
    if (L <= 24 && m <= 6) return count_vectors_rec(1, 0, m, L, d);
    /* ways[b] = number of legal prefixes b_1..b_i ending at b */
    uint64_t *ways = calloc((size_t)L + 1, sizeof(uint64_t));
    uint64_t *nxt = calloc((size_t)L + 1, sizeof(uint64_t));
    for (int b = 1; b <= L - 1; b++) ways[b] = in_window(b, 1, m, L, d) ? 1 : 0;
    for (int i = 2; i <= m - 1; i++) {
        uint64_t run = 0;
        for (int b = 0; b <= L - 1; b++) {
            nxt[b] = (b >= 1 && in_window(b, i, m, L, d)) ? run : 0;
            run = sat_add(run, ways[b]);
        }
        memcpy(ways, nxt, sizeof(uint64_t) * ((size_t)L + 1));
    }
    uint64_t total = 0;
    for (int b = 1; b <= L - 1; b++) total = sat_add(total, ways[b]);
    free(ways); free(nxt);
    return total;
}

/* Enumerate all strictly increasing vectors in lexicographic order into a flat array. */
typedef struct { int *v; int64_t n, cap; int m; } vec_list;

static void gen_vectors_rec(vec_list *out, int *cur, int i, int prev, int m, int L, int d)
{
    if (i == m) {
        if (out->n == out->cap) {
            out->cap = out->cap ? out->cap * 2 : 64;
            out->v = realloc(out->v, sizeof(int) * (size_t)out->cap * (m + 1));
        }
        int *dst = out->v + out->n * (m + 1);
        dst[0] = 0;
        for (int q = 1; q < m; q++) dst[q] = cur[q];
        dst[m] = L;
        out->n++;
        return;
    }
    for (int b = prev + 1; b <= L - 1; b++) {
        if (!in_window(b, i, m, L, d)) continue;
        cur[i] = b;
        gen_vectors_rec(out, cur, i + 1, b, m, L, d);
    }
}

static vec_list gen_vectors(int m, int L, int d)
{
    vec_list out = {0};
    out.m = m;
    int cur[ORC_MAXB];
    if (m <= L) gen_vectors_rec(&out, cur, 1, 0, m, L, d);
    return out;
}

/* Smallest RS count of a candidate: min_rs, or N when it is 0. */
static int rs_lo(const orc_params *p)
{
    return p->min_rs > 0 ? p->min_rs : p->n_threads;
}

/* |C| for a window pair: sum over shapes of |X| * sum over Y of the coefficients of z^n,
 * n = min_rs .. N, of prod_j P_{h_j}(z)^c, where P_h(z) = sum_k z^k * (number of split
 * vectors of a height-h tile into k slices). */
static uint64_t space_size(int W, int H, const orc_params *p, int dt, int dr)
{
    int N = p->n_threads, Km = p->max_rs_per_tile, Nlo = rs_lo(p);
    uint64_t total = 0;
    uint64_t splits[257][ORC_MAXN + 1];
    for (int h = 1; h <= H; h++)
        for (int k = 0; k <= N; k++)
            splits[h][k] = (k >= 1 && k <= Km && k <= h) ? count_vectors(k, h, dr) : 0;
    for (int c = 1; c <= p->max_tile_cols; c++) {
        for (int r = 1; r <= p->max_tile_rows; r++) {
            if (!((int64_t)c * r <= N && (int64_t)Nlo <= (int64_t)Km * c * r)) continue;
            uint64_t nx = count_vectors(c, W, dt);
            if (nx == 0) continue;
            vec_list ys = gen_vectors(r, H, dt);
            uint64_t sum_m = 0;
            for (int64_t yi = 0; yi < ys.n; yi++) {
                const int *Y = ys.v + yi * (r + 1);
                uint64_t poly[ORC_MAXN + 1] = {0};
                poly[0] = 1;
                for (int j = 0; j < r; j++) {
                    int hj = Y[j + 1] - Y[j];
                    for (int rep = 0; rep < c; rep++) {
                        uint64_t q[ORC_MAXN + 1] = {0};
                        for (int s = 0; s <= N; s++) {
                            if (!poly[s]) continue;
                            for (int k = 1; s + k <= N; k++)
                                if (splits[hj][k])
                                    q[s + k] = sat_add(q[s + k], sat_mul(poly[s], splits[hj][k]));
                        }
                        memcpy(poly, q, sizeof(q));
                    }
                }
                for (int n = Nlo; n <= N; n++) sum_m = sat_add(sum_m, poly[n]);
            }
            free(ys.v);
            total = sat_add(total, sat_mul(nx, sum_m));
        }
    }
    return total;
}

static const int ladder[6][2] = { {-1, -1}, {3, 1}, {2, 1}, {1, 1}, {1, 0}, {0, 0} };

int orc_space_size(int W, int H, const orc_params *p, int64_t *n, int32_t *dt, int32_t *dr)
{
    if (W < 1 || H < 1 || W > 256 || H > 256) return -1;
    if (p->dtile == -2 && p->drs == -2) {
        uint64_t budget = p->space_budget > 0 ? (uint64_t)p->space_budget : ((uint64_t)1 << 24);
        int pick = 5;
        for (int i = 0; i < 6; i++) {
            if (space_size(W, H, p, ladder[i][0], ladder[i][1]) <= budget) { pick = i; break; }
        }
        *dt = ladder[pick][0];
        *dr = ladder[pick][1];
    } else if (p->dtile >= -1 && p->drs >= -1) {
        *dt = p->dtile;
        *dr = p->drs;
    } else {
        return -1;
    }
    uint64_t s = space_size(W, H, p, *dt, *dr);
    *n = s > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)s;
    return 0;
}

/* ------------------------------------------------------------------------------------- */
/* Exhaustive two-step search in canonical order.                                       */
/* ------------------------------------------------------------------------------------- */

typedef struct {
    /* geometry */
    int W, H, N, Nlo, Km, karea, cs, prune;
    int64_t *colpx, *rowpx;                /* pixel prefix: colpx[x] = width of CTU cols < x */
    int64_t *satT, *satS1, *satS2;         /* (H+1) x (W+1) inclusive prefix sums */
    int64_t lam_num, lam_den;
    /* current candidate */
    int c, r;
    const int *X, *Y;
    int k[ORC_MAXN];
    int Z[ORC_MAXN][ORC_MAXN + 1];
    int dr;
    /* uniform */
    int cu, ru;
    /* pass state */
    int pass;
    int64_t rank, tmin, n_feasible;
    int64_t best_q, best_t, best_rank;
    int64_t uniform_rank;
    orc_result *res;
} search_ctx;

static int64_t rect_sum(const int64_t *sat, int W, int x0, int y0, int x1, int y1)
{
    int S = W + 1;
    return sat[(int64_t)y1 * S + x1] - sat[(int64_t)y0 * S + x1]
         - sat[(int64_t)y1 * S + x0] + sat[(int64_t)y0 * S + x0];
}

/* RS rectangles of the current candidate, in tile raster order, top to bottom in a tile. */
static int current_regions(const search_ctx *s, int rs[][4])
{
    int n = 0;
    for (int j = 0; j < s->r; j++)
        for (int i = 0; i < s->c; i++) {
            int t = j * s->c + i;
            for (int q = 0; q < s->k[t]; q++) {
                rs[n][0] = s->X[i];
                rs[n][1] = s->Y[j] + s->Z[t][q];
                rs[n][2] = s->X[i + 1];
                rs[n][3] = s->Y[j] + s->Z[t][q + 1];
                n++;
            }
        }
    return n;
}

static int is_uniform(const search_ctx *s)
{
    if (s->c != s->cu || s->r != s->ru) return 0;
    for (int i = 0; i <= s->c; i++) if (s->X[i] != (int)(((int64_t)i * s->W) / s->c)) return 0;
    for (int j = 0; j <= s->r; j++) if (s->Y[j] != (int)(((int64_t)j * s->H) / s->r)) return 0;
    for (int t = 0; t < s->c * s->r; t++) if (s->k[t] != 1) return 0;
    return 1;
}

/* The authors' commented pruning notes, taken literally as geometric rules on the current
 * candidate (pixel units, as the area rule):
 *   heights: in every tile, the tallest slice is at most twice the shortest;
 *   means:   in every tile, mean slice area = tile area / k lies within [1/1.5, 1.5] times the
 *            mean slice area over the other tiles (other area / (n - k), n the candidate's RS
 *            count), when n > k.
 * Returns 1 when the candidate passes the rules selected by s->prune. */
static int coherent(const search_ctx *s)
{
    if (!s->prune) return 1;
    int64_t total = 0, tarea[ORC_MAXN], n = 0;
    for (int t = 0; t < s->c * s->r; t++) n += s->k[t];
    for (int j = 0; j < s->r; j++)
        for (int i = 0; i < s->c; i++) {
            const int t = j * s->c + i;
            const int64_t wpx = s->colpx[s->X[i + 1]] - s->colpx[s->X[i]];
            int64_t hmin = INT64_MAX, hmax = 0;
            for (int q = 0; q < s->k[t]; q++) {
                const int64_t h = s->rowpx[s->Y[j] + s->Z[t][q + 1]] - s->rowpx[s->Y[j] + s->Z[t][q]];
                if (h < hmin) hmin = h;
                if (h > hmax) hmax = h;
            }
            if ((s->prune & 1) && hmax > 2 * hmin) return 0;
            tarea[t] = wpx * (s->rowpx[s->Y[j + 1]] - s->rowpx[s->Y[j]]);
            total += tarea[t];
        }
    if (s->prune & 2)
        for (int t = 0; t < s->c * s->r; t++) {
            const int64_t k = s->k[t], rest = n - k;
            if (rest <= 0) continue;
            const int64_t a = tarea[t], o = total - tarea[t];
            /* a / k > 1.5 o / rest  or  a / k < o / (1.5 rest) */
            if (2 * a * rest > 3 * o * k || 3 * a * rest < 2 * o * k) return 0;
        }
    return 1;
}

static void evaluate(search_ctx *s)
{
    int rs[ORC_MAXN][4];
    int n = current_regions(s, rs);
    int64_t amin = INT64_MAX, amax = 0, tmax = 0;
    for (int q = 0; q < n; q++) {
        int64_t A = (s->colpx[rs[q][2]] - s->colpx[rs[q][0]]) * (s->rowpx[rs[q][3]] - s->rowpx[rs[q][1]]);
        if (A < amin) amin = A;
        if (A > amax) amax = A;
    }
    if (s->pass == 1 && is_uniform(s)) s->uniform_rank = s->rank;
    int feasible = ((s->karea == 0) || ((int64_t)s->karea * amin > amax)) && coherent(s);
    if (feasible) {
        for (int q = 0; q < n; q++) {
            int64_t T = rect_sum(s->satT, s->W, rs[q][0], rs[q][1], rs[q][2], rs[q][3]);
            if (T > tmax) tmax = T;
        }
        if (s->pass == 1) {
            s->n_feasible++;
            if (tmax < s->tmin) s->tmin = tmax;
        } else {
            int within = s->lam_num < 0 ||
                (__int128)tmax * s->lam_den <= (__int128)s->tmin * (s->lam_den + s->lam_num);
            if (within) {
                int64_t Q = 0;
                for (int q = 0; q < n; q++) {
                    int64_t A = (s->colpx[rs[q][2]] - s->colpx[rs[q][0]]) * (s->rowpx[rs[q][3]] - s->rowpx[rs[q][1]]);
                    int64_t S1 = rect_sum(s->satS1, s->W, rs[q][0], rs[q][1], rs[q][2], rs[q][3]);
                    int64_t S2 = rect_sum(s->satS2, s->W, rs[q][0], rs[q][1], rs[q][2], rs[q][3]);
                    __int128 sq = (__int128)S1 * S1;
                    Q += S2 - (int64_t)(sq / A);
                }
                if (s->best_rank < 0 || Q < s->best_q || (Q == s->best_q && tmax < s->best_t)) {
                    s->best_q = Q;
                    s->best_t = tmax;
                    s->best_rank = s->rank;
                    orc_result *o = s->res;
                    o->tile_cols = s->c;
                    o->tile_rows = s->r;
                    o->n_rs = n;
                    for (int i = 0; i <= s->c; i++) o->col_bd[i] = s->X[i];
                    for (int j = 0; j <= s->r; j++) o->row_bd[j] = s->Y[j];
                    for (int q = 0; q < n; q++) {
                        for (int e = 0; e < 4; e++) o->rs[q][e] = rs[q][e];
                        o->rs_time[q] = rect_sum(s->satT, s->W, rs[q][0], rs[q][1], rs[q][2], rs[q][3]);
                    }
                }
            }
        }
    }
    s->rank++;
}

static void enum_tiles(search_ctx *s, int t, int remaining);

/* Split offsets of tile t into k slices: 0 = z_0 < z_1 < ... < z_{k-1} < z_k = h. */
static void enum_splits(search_ctx *s, int t, int q, int remaining)
{
    int k = s->k[t];
    int h = s->Y[t / s->c + 1] - s->Y[t / s->c];
    if (q == k) {
        s->Z[t][k] = h;
        enum_tiles(s, t + 1, remaining - k);
        return;
    }
    for (int z = s->Z[t][q - 1] + 1; z <= h - 1; z++) {
        if (!in_window(z, q, k, h, s->dr)) continue;
        s->Z[t][q] = z;
        enum_splits(s, t, q + 1, remaining);
    }
}

static void enum_tiles(search_ctx *s, int t, int remaining)
{
    int T = s->c * s->r;
    if (t == T) {
        if (remaining <= s->N - s->Nlo) evaluate(s);     /* remaining threads stay idle */
        return;
    }
    int h = s->Y[t / s->c + 1] - s->Y[t / s->c];
    int later = T - t - 1;                    /* tiles after this one, each needs 1..Km */
    for (int k = 1; k <= s->Km && k <= h && k <= remaining; k++) {
        if (remaining - k < later) break;     /* no slice left for some later tile */
        if (remaining - k - later * s->Km > s->N - s->Nlo) continue;  /* too many idle threads */
        s->k[t] = k;
        s->Z[t][0] = 0;
        enum_splits(s, t, 1, remaining);
    }
}

static void run_pass(search_ctx *s, int dt, const orc_params *p)
{
    s->rank = 0;
    for (int c = 1; c <= p->max_tile_cols; c++) {
        for (int r = 1; r <= p->max_tile_rows; r++) {
            if (!((int64_t)c * r <= s->N && (int64_t)s->Nlo <= (int64_t)s->Km * c * r)) continue;
            vec_list xs = gen_vectors(c, s->W, dt);
            vec_list ys = gen_vectors(r, s->H, dt);
            s->c = c;
            s->r = r;
            for (int64_t xi = 0; xi < xs.n; xi++) {
                for (int64_t yi = 0; yi < ys.n; yi++) {
                    s->X = xs.v + xi * (c + 1);
                    s->Y = ys.v + yi * (r + 1);
                    enum_tiles(s, 0, s->N);
                }
            }
            free(xs.v);
            free(ys.v);
        }
    }
}

/* Inclusive 2D prefix sum over a per-CTU array (row-major W x H) into (H+1) x (W+1). */
static void build_sat(int W, int H, const int64_t *val, int64_t *sat)
{
    int S = W + 1;
    for (int x = 0; x <= W; x++) sat[x] = 0;
    for (int y = 1; y <= H; y++) {
        sat[(int64_t)y * S] = 0;
        for (int x = 1; x <= W; x++)
            sat[(int64_t)y * S + x] = val[(int64_t)(y - 1) * W + (x - 1)]
                + sat[(int64_t)(y - 1) * S + x] + sat[(int64_t)y * S + x - 1]
                - sat[(int64_t)(y - 1) * S + x - 1];
    }
}

/* Evaluate one explicit partition (used for the uniform partition and for tests). */
static void score_regions(const search_ctx *s, int n, int rs[][4], int64_t *t_out, int64_t *q_out)
{
    int64_t tmax = 0, Q = 0;
    for (int q = 0; q < n; q++) {
        int64_t A = (s->colpx[rs[q][2]] - s->colpx[rs[q][0]]) * (s->rowpx[rs[q][3]] - s->rowpx[rs[q][1]]);
        int64_t T = rect_sum(s->satT, s->W, rs[q][0], rs[q][1], rs[q][2], rs[q][3]);
        int64_t S1 = rect_sum(s->satS1, s->W, rs[q][0], rs[q][1], rs[q][2], rs[q][3]);
        int64_t S2 = rect_sum(s->satS2, s->W, rs[q][0], rs[q][1], rs[q][2], rs[q][3]);
        if (T > tmax) tmax = T;
        Q += S2 - (int64_t)(((__int128)S1 * S1) / A);
    }
    *t_out = tmax;
    *q_out = Q;
}

/*
 * Full search for one frame.  cost, s1, s2 are per-CTU arrays in raster order.
 * Returns 0 (a feasible partition was found), 1 (no feasible partition: the uniform
 * partition is returned), or a negative value for invalid arguments / empty space.
 */
int orc_search(int w, int h, int cs, const orc_params *p, const uint32_t *cost,
               const uint32_t *s1, const uint64_t *s2, orc_result *out)
{
    memset(out, 0, sizeof(*out));
    if (w <= 0 || h <= 0 || cs <= 0) return -1;
    int W = (w + cs - 1) / cs, H = (h + cs - 1) / cs;
    if (p->n_threads < 1 || p->n_threads > ORC_MAXN || p->max_tile_cols < 1 || p->max_tile_rows < 1 ||
        p->max_rs_per_tile < 1 || p->lambda_den < 1 || p->area_k < 0 || p->prune < 0 || p->prune > 3 ||
        p->min_rs < 0 || p->min_rs > p->n_threads)
        return -1;
    int64_t n_space; int32_t dt, dr;
    if (orc_space_size(W, H, p, &n_space, &dt, &dr) != 0) return -1;
    if (n_space <= 0 || n_space > ((int64_t)1 << 40)) return -3;

    search_ctx s;
    memset(&s, 0, sizeof(s));
    s.W = W; s.H = H; s.N = p->n_threads; s.Nlo = rs_lo(p); s.Km = p->max_rs_per_tile;
    s.karea = p->area_k; s.cs = cs;
    s.prune = p->prune;
    s.dr = dr;
    s.lam_num = p->lambda_num; s.lam_den = p->lambda_den;
    s.colpx = calloc((size_t)W + 1, sizeof(int64_t));
    s.rowpx = calloc((size_t)H + 1, sizeof(int64_t));
    for (int x = 1; x <= W; x++) s.colpx[x] = s.colpx[x - 1] + (x * cs <= w ? cs : w - (x - 1) * cs);
    for (int y = 1; y <= H; y++) s.rowpx[y] = s.rowpx[y - 1] + (y * cs <= h ? cs : h - (y - 1) * cs);
    int64_t *vt = malloc(sizeof(int64_t) * (size_t)W * H);
    int64_t *v1 = malloc(sizeof(int64_t) * (size_t)W * H);
    int64_t *v2 = malloc(sizeof(int64_t) * (size_t)W * H);
    for (int64_t c = 0; c < (int64_t)W * H; c++) { vt[c] = cost[c]; v1[c] = s1[c]; v2[c] = (int64_t)s2[c]; }
    size_t satn = (size_t)(W + 1) * (H + 1);
    s.satT = malloc(sizeof(int64_t) * satn);
    s.satS1 = malloc(sizeof(int64_t) * satn);
    s.satS2 = malloc(sizeof(int64_t) * satn);
    build_sat(W, H, vt, s.satT);
    build_sat(W, H, v1, s.satS1);
    build_sat(W, H, v2, s.satS2);
    free(vt); free(v1); free(v2);

    /* uniform grid: most square factorisation c_u * r_u = N with c_u >= r_u */
    s.ru = 1;
    for (int d = 1; (int64_t)d * d <= s.N; d++) if (s.N % d == 0) s.ru = d;
    s.cu = s.N / s.ru;
    s.uniform_rank = -1;
    s.res = out;

    /* step 1 (Eq. 3) */
    s.pass = 1;
    s.tmin = INT64_MAX;
    run_pass(&s, dt, p);
    out->n_enumerated = s.rank;
    out->n_feasible = s.n_feasible;
    out->dtile_used = dt;
    out->drs_used = dr;
    out->uniform_rank = s.uniform_rank;

    /* the uniform partition's own scores (reported, and the fallback) */
    int urs[ORC_MAXN][4];
    int un = 0;
    int64_t ut = -1, uq = -1;
    if (s.cu <= W && s.ru <= H) {
        for (int j = 0; j < s.ru; j++)
            for (int i = 0; i < s.cu; i++) {
                urs[un][0] = (int)(((int64_t)i * W) / s.cu);
                urs[un][1] = (int)(((int64_t)j * H) / s.ru);
                urs[un][2] = (int)(((int64_t)(i + 1) * W) / s.cu);
                urs[un][3] = (int)(((int64_t)(j + 1) * H) / s.ru);
                un++;
            }
        score_regions(&s, un, urs, &ut, &uq);
    }
    out->t_unif = ut;
    out->q_unif = uq;

    int rc;
    if (s.n_feasible == 0) {
        rc = 1;
        out->t_min = -1;
        out->rank = s.uniform_rank;
        out->t_sel = ut;
        out->q_sel = uq;
        if (un > 0) {
            out->tile_cols = s.cu;
            out->tile_rows = s.ru;
            out->n_rs = un;
            for (int i = 0; i <= s.cu; i++) out->col_bd[i] = (int)(((int64_t)i * W) / s.cu);
            for (int j = 0; j <= s.ru; j++) out->row_bd[j] = (int)(((int64_t)j * H) / s.ru);
            for (int q = 0; q < un; q++) {
                for (int e = 0; e < 4; e++) out->rs[q][e] = urs[q][e];
                out->rs_time[q] = rect_sum(s.satT, W, urs[q][0], urs[q][1], urs[q][2], urs[q][3]);
            }
        }
    } else {
        /* step 2 (Eq. 2 under Eq. 4) */
        out->t_min = s.tmin;
        s.pass = 2;
        s.best_rank = -1;
        run_pass(&s, dt, p);
        out->rank = s.best_rank;
        out->t_sel = s.best_t;
        out->q_sel = s.best_q;
        rc = 0;
    }
    out->status = rc;
    free(s.colpx); free(s.rowpx); free(s.satT); free(s.satS1); free(s.satS2);
    return rc;
}

/* ------------------------------------------------------------------------------------- */
/* Exact two-step search over the literal space, by decomposition.                      */
/* ------------------------------------------------------------------------------------- */
/*
 * The literal space lets every CTU boundary serve as a tile boundary and as a split row
 * (dt = dr = unbounded); otherwise as above: c <= Cmax, r <= Rmax, k_t in [1, min(Kmax, h_t)],
 * sum of k_t = N.  At 4K it holds 5.4e9 candidates, so instead of listing them the two steps
 * are solved exactly by splitting the problem:
 *
 *  - Area rule (Section 2.3): P passes iff every RS area lies in [a, k a) for a = A_min(P).
 *    So the feasible set is the union over a of the sets whose RS areas all lie in the window
 *    [a, k a), with a running over the distinct RS areas such that N a <= A_total < k N a
 *    (N areas in such a window could not add up to the frame otherwise).  With the window
 *    fixed, the rule is a condition on each RS alone.  k = 0 (rule off): one window, no bound.
 *  - Step 1 (Eq. 1, Eq. 3): with a window and the row boundaries Y fixed, the largest RS time
 *    is a maximum over tiles of a maximum over their slices.  Per tile rectangle and slice
 *    count k: the least possible largest slice time (a DP over the split rows).  Per column
 *    strip and RS count K: the least largest time of the strip's r tiles holding K slices in
 *    all (a DP over the tiles).  Then a DP over the column boundaries whose state is
 *    (tile columns used, RS used).  T~min is the least result over windows, r and Y.
 *  - Step 2 (Eq. 2 under Eq. 4): tau = floor(T~min (den + num) / den) bounds every RS time,
 *    a condition on each RS alone again, and Q is a sum over RS; the same three DPs then
 *    minimise (Q, T~(P)) lexicographically: sums and maxima both compose monotonically.
 * Ties: the first in the order (window ascending, r ascending, Y lexicographic, c ascending),
 * and inside the DPs the first minimising choice in ascending loop order.  The canonical rank
 * is not computed (-1) and n_feasible is not counted (-1).
 */

typedef struct { int64_t q, t; } lexv;          /* (Q, T~) of step 2; q = INT64_MAX: none */

static const int64_t LIT_INF = INT64_MAX;

typedef struct {
    int W, H, N, Cm, Rm, Km, span;
    int64_t *colpx, *rowpx, *satT, *satS1, *satS2;
    /* per rectangle (x0, x1, y0, y1): area, time, q = S2 - floor(S1^2 / n) */
    int64_t *A, *T, *Q;
    /* tile tables for the current window: [rect][k], k = 1..Km */
    int64_t *t1;
    lexv *t2;
    int64_t lo, hi;                 /* window [lo, hi); hi = LIT_INF when the rule is off */
    int64_t tau;                    /* step-2 bound on RS times */
} lit_ctx;

static size_t lit_rect(const lit_ctx *L, int x0, int x1, int y0, int y1)
{
    return (((size_t)x0 * (L->W + 1) + x1) * (L->H + 1) + y0) * (L->H + 1) + y1;
}

static int lit_ok(const lit_ctx *L, size_t r)
{
    return L->A[r] >= L->lo && L->A[r] < L->hi;
}

static lexv lex_join(lexv a, lexv b)       /* regions side by side: Q adds, T~ takes the max */
{
    lexv o;
    if (a.q == LIT_INF || b.q == LIT_INF) { o.q = LIT_INF; o.t = LIT_INF; return o; }
    o.q = a.q + b.q;
    o.t = a.t > b.t ? a.t : b.t;
    return o;
}

static int lex_less(lexv a, lexv b)
{
    return a.q < b.q || (a.q == b.q && a.t < b.t);
}

/* Tile tables for the current window (and, for step 2, tau): for every tile rectangle and k,
 * the best split of its rows into k slices, each slice an RS passing the per-RS conditions.
 * If choice is given (step 2 only, one rectangle), it receives the split rows of the best. */
static void lit_tile_dp(lit_ctx *L, int step, int x0, int x1, int y0,
                        int64_t f1[][ORC_MAXB], lexv f2[][ORC_MAXB], int arg[][ORC_MAXB])
{
    const int H = L->H, Km = L->Km;
    for (int q = 0; q <= Km; q++)
        for (int y = 0; y <= H; y++) {
            f1[q][y] = LIT_INF;
            f2[q][y].q = LIT_INF; f2[q][y].t = LIT_INF;
            arg[q][y] = -1;
        }
    f1[0][y0] = 0;
    f2[0][y0].q = 0; f2[0][y0].t = 0;
    for (int q = 1; q <= Km; q++)
        for (int y = y0 + q; y <= H; y++)
            for (int yp = y0 + q - 1; yp < y; yp++) {
                size_t r = lit_rect(L, x0, x1, yp, y);
                if (!lit_ok(L, r)) continue;
                if (step == 1) {
                    if (f1[q - 1][yp] == LIT_INF) continue;
                    int64_t v = f1[q - 1][yp] > L->T[r] ? f1[q - 1][yp] : L->T[r];
                    if (v < f1[q][y]) { f1[q][y] = v; arg[q][y] = yp; }
                } else {
                    if (L->T[r] > L->tau) continue;
                    lexv s = { L->Q[r], L->T[r] };
                    lexv v = lex_join(f2[q - 1][yp], s);
                    if (v.q != LIT_INF && lex_less(v, f2[q][y])) { f2[q][y] = v; arg[q][y] = yp; }
                }
            }
}

static void lit_tables(lit_ctx *L, int step)
{
    int64_t (*f1)[ORC_MAXB] = malloc(sizeof(int64_t) * ORC_MAXB * ORC_MAXB);
    lexv (*f2)[ORC_MAXB] = malloc(sizeof(lexv) * ORC_MAXB * ORC_MAXB);
    int (*arg)[ORC_MAXB] = malloc(sizeof(int) * ORC_MAXB * ORC_MAXB);
    for (int x0 = 0; x0 < L->W; x0++)
        for (int x1 = x0 + 1; x1 <= L->W; x1++)
            for (int y0 = 0; y0 < L->H; y0++) {
                lit_tile_dp(L, step, x0, x1, y0, f1, f2, arg);
                for (int y1 = y0 + 1; y1 <= L->H; y1++)
                    for (int k = 1; k <= L->Km; k++) {
                        size_t r = lit_rect(L, x0, x1, y0, y1) * (size_t)L->Km + (k - 1);
                        if (step == 1) L->t1[r] = f1[k][y1];
                        else L->t2[r] = f2[k][y1];
                    }
            }
    free(f1); free(f2); free(arg);
}

/* Best RS count split over the r tiles of column strip [x0, x1) with rows Y: out[K] for K
 * slices in the strip (K = 0..N).  Each tile takes k slices of its own, or (span_tiles) two or
 * more consecutive tiles form one RS; ch[b][K] records the choice that ends at tile row b: k > 0
 * for tile b - 1 cut into k slices, -(a + 1) for the block of tiles a .. b - 1.  Single tiles
 * are tried first (k ascending), then blocks (a ascending); the first minimum is kept.  kk
 * (optional) receives the choices of the best split with K = want, listed by ending row. */
static void lit_strip(const lit_ctx *L, int step, int x0, int x1, int r, const int *Y,
                      int64_t *o1, lexv *o2, int want, int *kk)
{
    const int N = L->N, Km = L->Km;
    int64_t u1[ORC_MAXB][ORC_MAXN + 1];
    lexv u2[ORC_MAXB][ORC_MAXN + 1];
    int ch[ORC_MAXB][ORC_MAXN + 1];
    for (int K = 0; K <= N; K++) { u1[0][K] = LIT_INF; u2[0][K].q = LIT_INF; u2[0][K].t = LIT_INF; }
    u1[0][0] = 0;
    u2[0][0].q = 0; u2[0][0].t = 0;
    for (int b = 1; b <= r; b++) {
        size_t base = lit_rect(L, x0, x1, Y[b - 1], Y[b]) * (size_t)Km;
        for (int K = 0; K <= N; K++) {
            u1[b][K] = LIT_INF;
            u2[b][K].q = LIT_INF; u2[b][K].t = LIT_INF;
            ch[b][K] = 0;
            for (int k = 1; k <= Km && k <= K; k++) {
                if (step == 1) {
                    int64_t a = u1[b - 1][K - k], c = L->t1[base + k - 1];
                    if (a == LIT_INF || c == LIT_INF) continue;
                    int64_t v = a > c ? a : c;
                    if (v < u1[b][K]) { u1[b][K] = v; ch[b][K] = k; }
                } else {
                    lexv v = lex_join(u2[b - 1][K - k], L->t2[base + k - 1]);
                    if (v.q != LIT_INF && lex_less(v, u2[b][K])) { u2[b][K] = v; ch[b][K] = k; }
                }
            }
            if (!L->span || K < 1) continue;
            for (int a = 0; a + 2 <= b; a++) {               /* block of tiles a .. b - 1: one RS */
                size_t rr = lit_rect(L, x0, x1, Y[a], Y[b]);
                if (!lit_ok(L, rr)) continue;
                if (step == 1) {
                    int64_t av = u1[a][K - 1];
                    if (av == LIT_INF) continue;
                    int64_t v = av > L->T[rr] ? av : L->T[rr];
                    if (v < u1[b][K]) { u1[b][K] = v; ch[b][K] = -(a + 1); }
                } else {
                    if (L->T[rr] > L->tau) continue;
                    lexv blk = { L->Q[rr], L->T[rr] };
                    lexv v = lex_join(u2[a][K - 1], blk);
                    if (v.q != LIT_INF && lex_less(v, u2[b][K])) { u2[b][K] = v; ch[b][K] = -(a + 1); }
                }
            }
        }
    }
    for (int K = 0; K <= N; K++) {
        if (o1) o1[K] = u1[r][K];
        if (o2) o2[K] = u2[r][K];
    }
    if (kk) {
        for (int b = 0; b <= r; b++) kk[b] = 0;
        for (int b = r, K = want; b > 0;) {
            const int c = ch[b][K];
            kk[b] = c;
            if (c > 0) { K -= c; b -= 1; }
            else { K -= 1; b = -c - 1; }
        }
    }
}

/* Column DP for fixed window and Y.  best1[c] / best2[c]: best over c tile columns (c = 1..Cm).
 * If cx / ck are given (step 2, target c = want_c), they receive the column boundaries and
 * per-strip RS counts of the best. */
static void lit_columns(const lit_ctx *L, int step, int r, const int *Y, int64_t *best1,
                        lexv *best2, int want_c, int *cx, int *ck)
{
    const int W = L->W, N = L->N, Cm = L->Cm;
    const size_t S = (size_t)(W + 1) * (W + 1) * (N + 1);
    int64_t *h1 = malloc(sizeof(int64_t) * S);
    lexv *h2 = malloc(sizeof(lexv) * S);
    for (int x0 = 0; x0 < W; x0++)
        for (int x1 = x0 + 1; x1 <= W; x1++) {
            size_t o = ((size_t)x0 * (W + 1) + x1) * (N + 1);
            lit_strip(L, step, x0, x1, r, Y, h1 + o, h2 + o, 0, NULL);
        }
    const size_t F = (size_t)(Cm + 1) * (W + 1) * (N + 1);
    int64_t *F1 = malloc(sizeof(int64_t) * F);
    lexv *F2 = malloc(sizeof(lexv) * F);
    int *AX = malloc(sizeof(int) * F), *AK = malloc(sizeof(int) * F);
#define FI(i, x, n) (((size_t)(i) * (W + 1) + (x)) * (N + 1) + (n))
    for (size_t e = 0; e < F; e++) { F1[e] = LIT_INF; F2[e].q = LIT_INF; F2[e].t = LIT_INF; AX[e] = AK[e] = -1; }
    F1[FI(0, 0, 0)] = 0;
    F2[FI(0, 0, 0)].q = 0; F2[FI(0, 0, 0)].t = 0;
    for (int i = 1; i <= Cm; i++)
        for (int x = i; x <= W; x++)
            for (int n = 1; n <= N; n++)
                for (int xp = i - 1; xp < x; xp++)
                    for (int K = 1; K <= n; K++) {
                        size_t hp = ((size_t)xp * (W + 1) + x) * (N + 1) + K, fp = FI(i - 1, xp, n - K);
                        if (step == 1) {
                            if (F1[fp] == LIT_INF || h1[hp] == LIT_INF) continue;
                            int64_t v = F1[fp] > h1[hp] ? F1[fp] : h1[hp];
                            if (v < F1[FI(i, x, n)]) { F1[FI(i, x, n)] = v; AX[FI(i, x, n)] = xp; AK[FI(i, x, n)] = K; }
                        } else {
                            lexv v = lex_join(F2[fp], h2[hp]);
                            if (v.q != LIT_INF && lex_less(v, F2[FI(i, x, n)])) {
                                F2[FI(i, x, n)] = v; AX[FI(i, x, n)] = xp; AK[FI(i, x, n)] = K;
                            }
                        }
                    }
    for (int c = 1; c <= Cm; c++) {
        if (best1) best1[c] = F1[FI(c, W, N)];
        if (best2) best2[c] = F2[FI(c, W, N)];
    }
    if (cx) {
        int x = W, n = N;
        cx[want_c] = W;
        for (int i = want_c; i > 0; i--) {
            int xp = AX[FI(i, x, n)], K = AK[FI(i, x, n)];
            cx[i - 1] = xp;
            ck[i - 1] = K;
            x = xp;
            n -= K;
        }
    }
#undef FI
    free(h1); free(h2); free(F1); free(F2); free(AX); free(AK);
}

/* Next increasing vector Y (Y[0] = 0, Y[r] = H) in lexicographic order; 0 when done. */
static int lit_next_y(int *Y, int r, int H)
{
    for (int j = r - 1; j >= 1; j--) {
        if (Y[j] < H - (r - j)) {
            Y[j]++;
            for (int q = j + 1; q < r; q++) Y[q] = Y[q - 1] + 1;
            return 1;
        }
    }
    return 0;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : x > y;
}

/* |C| of the literal space with spanning blocks: per shape, |X| times the sum over Y of the
 * coefficient of z^N in S_Y(z)^c, where S_Y(z) counts the ways to cover one tile column with
 * rows Y: tile rows one at a time (a tile of height h split into k slices: the number of split
 * vectors) or two or more consecutive tile rows as one RS (z).  Saturating. */
static int64_t span_space_size(int W, int H, const orc_params *p)
{
    const int N = p->n_threads, Km = p->max_rs_per_tile;
    uint64_t total = 0;
    for (int r = 1; r <= p->max_tile_rows && r <= H; r++) {
        vec_list ys = gen_vectors(r, H, -1);
        for (int64_t yi = 0; yi < ys.n; yi++) {
            const int *Y = ys.v + yi * (r + 1);
            uint64_t f[ORC_MAXB][ORC_MAXN + 1];
            memset(f, 0, sizeof(f));
            f[0][0] = 1;
            for (int b = 1; b <= r; b++) {
                const int hb = Y[b] - Y[b - 1];
                for (int n = 0; n <= N; n++) {
                    uint64_t acc = 0;
                    for (int k = 1; k <= Km && k <= hb && k <= n; k++)
                        acc = sat_add(acc, sat_mul(f[b - 1][n - k], count_vectors(k, hb, -1)));
                    for (int a = 0; a + 2 <= b && n >= 1; a++) acc = sat_add(acc, f[a][n - 1]);
                    f[b][n] = acc;
                }
            }
            uint64_t poly[ORC_MAXN + 1] = {0};
            poly[0] = 1;
            for (int c = 1; c <= p->max_tile_cols && c <= W; c++) {
                uint64_t q[ORC_MAXN + 1] = {0};
                for (int a = 0; a <= N; a++) {
                    if (!poly[a]) continue;
                    for (int b2 = 0; a + b2 <= N; b2++)
                        if (f[r][b2]) q[a + b2] = sat_add(q[a + b2], sat_mul(poly[a], f[r][b2]));
                }
                memcpy(poly, q, sizeof(q));
                total = sat_add(total, sat_mul(count_vectors(c, W, -1), poly[N]));
            }
        }
        free(ys.v);
    }
    return total > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)total;
}

int orc_literal_search(int w, int h, int cs, const orc_params *p, const uint32_t *cost,
                       const uint32_t *s1, const uint64_t *s2, orc_result *out)
{
    memset(out, 0, sizeof(*out));
    if (w <= 0 || h <= 0 || cs <= 0 || !p) return -1;
    const int W = (w + cs - 1) / cs, H = (h + cs - 1) / cs;
    if (W > 64 || H > 64 || p->n_threads < 1 || p->n_threads > ORC_MAXN || p->max_tile_cols < 1 ||
        p->max_tile_rows < 1 || p->max_rs_per_tile < 1 || p->lambda_den < 1 || p->area_k < 0 ||
        p->prune != 0 || (p->min_rs != 0 && p->min_rs != p->n_threads) || p->span_tiles < 0 ||
        p->span_tiles > 1)
        return -1;
    lit_ctx L;
    memset(&L, 0, sizeof(L));
    L.W = W; L.H = H; L.N = p->n_threads; L.span = p->span_tiles;
    L.Cm = p->max_tile_cols < W ? p->max_tile_cols : W;
    L.Rm = p->max_tile_rows < H ? p->max_tile_rows : H;
    L.Km = p->max_rs_per_tile < H ? p->max_rs_per_tile : H;
    L.colpx = calloc((size_t)W + 1, sizeof(int64_t));
    L.rowpx = calloc((size_t)H + 1, sizeof(int64_t));
    for (int x = 1; x <= W; x++) L.colpx[x] = L.colpx[x - 1] + (x * cs <= w ? cs : w - (x - 1) * cs);
    for (int y = 1; y <= H; y++) L.rowpx[y] = L.rowpx[y - 1] + (y * cs <= h ? cs : h - (y - 1) * cs);
    int64_t *vt = malloc(sizeof(int64_t) * (size_t)W * H);
    int64_t *v1 = malloc(sizeof(int64_t) * (size_t)W * H);
    int64_t *v2 = malloc(sizeof(int64_t) * (size_t)W * H);
    for (int64_t c = 0; c < (int64_t)W * H; c++) { vt[c] = cost[c]; v1[c] = s1[c]; v2[c] = (int64_t)s2[c]; }
    size_t satn = (size_t)(W + 1) * (H + 1);
    L.satT = malloc(sizeof(int64_t) * satn);
    L.satS1 = malloc(sizeof(int64_t) * satn);
    L.satS2 = malloc(sizeof(int64_t) * satn);
    build_sat(W, H, vt, L.satT);
    build_sat(W, H, v1, L.satS1);
    build_sat(W, H, v2, L.satS2);
    free(vt); free(v1); free(v2);

    /* every rectangle: area, time, q */
    const size_t nrect = (size_t)(W + 1) * (W + 1) * (H + 1) * (H + 1);
    L.A = calloc(nrect, sizeof(int64_t));
    L.T = calloc(nrect, sizeof(int64_t));
    L.Q = calloc(nrect, sizeof(int64_t));
    int64_t *areas = malloc(sizeof(int64_t) * nrect);
    size_t n_areas = 0;
    for (int x0 = 0; x0 < W; x0++)
        for (int x1 = x0 + 1; x1 <= W; x1++)
            for (int y0 = 0; y0 < H; y0++)
                for (int y1 = y0 + 1; y1 <= H; y1++) {
                    size_t r = lit_rect(&L, x0, x1, y0, y1);
                    int64_t A = (L.colpx[x1] - L.colpx[x0]) * (L.rowpx[y1] - L.rowpx[y0]);
                    int64_t S1 = rect_sum(L.satS1, W, x0, y0, x1, y1);
                    int64_t S2 = rect_sum(L.satS2, W, x0, y0, x1, y1);
                    L.A[r] = A;
                    L.T[r] = rect_sum(L.satT, W, x0, y0, x1, y1);
                    L.Q[r] = S2 - (int64_t)(((__int128)S1 * S1) / A);
                    areas[n_areas++] = A;
                }
    /* windows */
    const int64_t Atot = L.colpx[W] * L.rowpx[H], N = L.N, k = p->area_k;
    int64_t *win = malloc(sizeof(int64_t) * (n_areas + 1));
    size_t n_win = 0;
    if (k == 0) {
        win[n_win++] = 0;
    } else {
        qsort(areas, n_areas, sizeof(int64_t), cmp_i64);
        for (size_t i = 0; i < n_areas; i++) {
            if (i > 0 && areas[i] == areas[i - 1]) continue;
            if (N * areas[i] <= Atot && (__int128)k * N * areas[i] > Atot) win[n_win++] = areas[i];
        }
    }
    free(areas);
    L.t1 = malloc(sizeof(int64_t) * nrect * L.Km);
    L.t2 = malloc(sizeof(lexv) * nrect * L.Km);

    int64_t cnt;
    int32_t dtu, dru;
    orc_params lp = *p;
    lp.dtile = -1; lp.drs = -1;
    orc_space_size(W, H, &lp, &cnt, &dtu, &dru);
    if (p->span_tiles) cnt = span_space_size(W, H, p);
    out->n_enumerated = cnt;
    out->n_feasible = -1;
    out->rank = -1;
    out->uniform_rank = -1;
    out->dtile_used = -1;
    out->drs_used = -1;

    /* step 1 */
    int64_t tmin = LIT_INF, best1[ORC_MAXB];
    int Y[ORC_MAXB];
    for (size_t wi = 0; wi < n_win; wi++) {
        L.lo = win[wi];
        L.hi = k == 0 ? LIT_INF : k * win[wi];
        lit_tables(&L, 1);
        for (int r = 1; r <= L.Rm; r++) {
            for (int j = 0; j < r; j++) Y[j] = j;
            Y[r] = H;
            do {
                lit_columns(&L, 1, r, Y, best1, NULL, 0, NULL, NULL);
                for (int c = 1; c <= L.Cm; c++) if (best1[c] < tmin) tmin = best1[c];
            } while (lit_next_y(Y, r, H));
        }
    }
    /* the uniform grid (Section 3.2), reported and returned when nothing is feasible */
    int cu, ru = 1;
    for (int d = 1; (int64_t)d * d <= N; d++) if (N % d == 0) ru = d;
    cu = (int)N / ru;
    int64_t ut = -1, uq = -1;
    if (cu <= W && ru <= H) {
        ut = 0; uq = 0;
        for (int j = 0; j < ru; j++)
            for (int i = 0; i < cu; i++) {
                size_t rr = lit_rect(&L, (int)((int64_t)i * W / cu), (int)((int64_t)(i + 1) * W / cu),
                                     (int)((int64_t)j * H / ru), (int)((int64_t)(j + 1) * H / ru));
                if (L.T[rr] > ut) ut = L.T[rr];
                uq += L.Q[rr];
            }
    }
    out->t_unif = ut;
    out->q_unif = uq;
    int rc = 0;
    if (tmin == LIT_INF) {
        out->status = 1;
        out->t_min = -1;
        out->t_sel = ut;
        out->q_sel = uq;
        if (ut >= 0) {
            int n = 0;
            out->tile_cols = cu;
            out->tile_rows = ru;
            for (int i = 0; i <= cu; i++) out->col_bd[i] = (int)((int64_t)i * W / cu);
            for (int j = 0; j <= ru; j++) out->row_bd[j] = (int)((int64_t)j * H / ru);
            for (int j = 0; j < ru; j++)
                for (int i = 0; i < cu; i++, n++) {
                    out->rs[n][0] = out->col_bd[i]; out->rs[n][1] = out->row_bd[j];
                    out->rs[n][2] = out->col_bd[i + 1]; out->rs[n][3] = out->row_bd[j + 1];
                    out->rs_time[n] = L.T[lit_rect(&L, out->rs[n][0], out->rs[n][2], out->rs[n][1], out->rs[n][3])];
                }
            out->n_rs = n;
        }
        rc = 1;
    } else {
        /* step 2 */
        L.tau = p->lambda_num < 0 ? LIT_INF
              : (int64_t)(((__int128)tmin * (p->lambda_den + p->lambda_num)) / p->lambda_den);
        lexv best = { LIT_INF, LIT_INF }, b2[ORC_MAXB];
        size_t bw = 0;
        int br = 0, bc = 0, bY[ORC_MAXB] = {0};
        for (size_t wi = 0; wi < n_win; wi++) {
            L.lo = win[wi];
            L.hi = k == 0 ? LIT_INF : k * win[wi];
            lit_tables(&L, 2);
            for (int r = 1; r <= L.Rm; r++) {
                for (int j = 0; j < r; j++) Y[j] = j;
                Y[r] = H;
                do {
                    lit_columns(&L, 2, r, Y, NULL, b2, 0, NULL, NULL);
                    for (int c = 1; c <= L.Cm; c++)
                        if (b2[c].q != LIT_INF && lex_less(b2[c], best)) {
                            best = b2[c]; bw = wi; br = r; bc = c;
                            memcpy(bY, Y, sizeof(int) * (r + 1));
                        }
                } while (lit_next_y(Y, r, H));
            }
        }
        /* rebuild the winner: column boundaries, per-strip counts, per-tile counts, splits */
        L.lo = win[bw];
        L.hi = k == 0 ? LIT_INF : k * win[bw];
        lit_tables(&L, 2);
        int cx[ORC_MAXB], ck[ORC_MAXB];
        lit_columns(&L, 2, br, bY, NULL, b2, bc, cx, ck);
        /* per tile: its slice count, or -(b + 1) on the top tile of a block ending at row b,
           or 0 inside a block */
        int tk[ORC_MAXB][ORC_MAXB];
        for (int i = 0; i < bc; i++) {
            int kk[ORC_MAXB + 1];
            lit_strip(&L, 2, cx[i], cx[i + 1], br, bY, NULL, NULL, ck[i], kk);
            for (int j = 0; j < br; j++) tk[i][j] = 0;
            for (int b = 1; b <= br; b++) {
                if (kk[b] > 0) tk[i][b - 1] = kk[b];
                else if (kk[b] < 0) tk[i][-kk[b] - 1] = -(b + 1);
            }
        }
        int64_t (*f1)[ORC_MAXB] = malloc(sizeof(int64_t) * ORC_MAXB * ORC_MAXB);
        lexv (*f2)[ORC_MAXB] = malloc(sizeof(lexv) * ORC_MAXB * ORC_MAXB);
        int (*arg)[ORC_MAXB] = malloc(sizeof(int) * ORC_MAXB * ORC_MAXB);
        int n = 0;
        int64_t tsel = 0, qsel = 0;
        for (int j = 0; j < br; j++)
            for (int i = 0; i < bc; i++) {
                if (tk[i][j] < 0) {                   /* a block of tiles j .. b - 1 as one RS */
                    const int b = -tk[i][j] - 1;
                    size_t rr = lit_rect(&L, cx[i], cx[i + 1], bY[j], bY[b]);
                    out->rs[n][0] = cx[i]; out->rs[n][1] = bY[j];
                    out->rs[n][2] = cx[i + 1]; out->rs[n][3] = bY[b];
                    out->rs_time[n] = L.T[rr];
                    if (L.T[rr] > tsel) tsel = L.T[rr];
                    qsel += L.Q[rr];
                    n++;
                    continue;
                }
                if (tk[i][j] == 0) continue;          /* inside a block */
                lit_tile_dp(&L, 2, cx[i], cx[i + 1], bY[j], f1, f2, arg);
                int rows[ORC_MAXB], kq = tk[i][j];
                rows[kq] = bY[j + 1];
                for (int q = kq, y = bY[j + 1]; q > 0; q--) { y = arg[q][y]; rows[q - 1] = y; }
                for (int q = 0; q < kq; q++) {
                    size_t rr = lit_rect(&L, cx[i], cx[i + 1], rows[q], rows[q + 1]);
                    out->rs[n][0] = cx[i]; out->rs[n][1] = rows[q];
                    out->rs[n][2] = cx[i + 1]; out->rs[n][3] = rows[q + 1];
                    out->rs_time[n] = L.T[rr];
                    if (L.T[rr] > tsel) tsel = L.T[rr];
                    qsel += L.Q[rr];
                    n++;
                }
            }
        free(f1); free(f2); free(arg);
        out->n_rs = n;
        out->tile_cols = bc;
        out->tile_rows = br;
        for (int i = 0; i <= bc; i++) out->col_bd[i] = cx[i];
        for (int j = 0; j <= br; j++) out->row_bd[j] = bY[j];
        out->t_min = tmin;
        out->t_sel = tsel;
        out->q_sel = qsel;
        out->status = 0;
        /* the rebuilt partition must score what the DP promised */
        if (tsel != best.t || qsel != best.q) rc = -2;
    }
    free(win);
    free(L.colpx); free(L.rowpx); free(L.satT); free(L.satS1); free(L.satS2);
    free(L.A); free(L.T); free(L.Q); free(L.t1); free(L.t2);
    return rc;
}
