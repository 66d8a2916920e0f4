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
