// Host construction of the candidate-space plan (see space.hpp).
#include "space.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <utility>

namespace trs {
namespace {

using u64 = uint64_t;

u64 sadd(u64 a, u64 b) { u64 s = a + b; return s < a ? UINT64_MAX : s; }
u64 smul(u64 a, u64 b)
{
    if (!a || !b) return 0;
    unsigned __int128 p = (unsigned __int128)a * b;
    return p > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (u64)p;
}

// Boundary b may be the i-th of m - 1 interior boundaries of [0, L] under window d.
inline bool legal(int b, int i, int m, int L, int d)
{
    if (d < 0) return true;
    int centre = (int)(((int64_t)i * L) / m);
    return std::abs(b - centre) <= d;
}

// Number of legal strictly increasing (b_1 .. b_{m-1}) in [1, L - 1].
u64 count_vectors(int m, int L, int d)
{
    if (m < 1 || m > L) return 0;
    if (m == 1) return 1;
    std::vector<u64> cur(L + 1, 0), nxt(L + 1, 0);
    for (int b = 1; b < L; b++) cur[b] = legal(b, 1, m, L, d) ? 1 : 0;
    for (int i = 2; i < m; i++) {
        u64 below = 0;                       // sum of cur[b'] over b' < b
        for (int b = 0; b < L; b++) {
            nxt[b] = (b >= 1 && legal(b, i, m, L, d)) ? below : 0;
            below = sadd(below, cur[b]);
        }
        std::swap(cur, nxt);
    }
    u64 total = 0;
    for (int b = 1; b < L; b++) total = sadd(total, cur[b]);
    return total;
}

// Lexicographic list of the vectors above, each stored as m + 1 values 0, b_1 .. b_{m-1}, L.
bool list_vectors(int m, int L, int d, int64_t cap, std::vector<uint16_t> &out, int64_t &n)
{
    n = 0;
    if (m < 1 || m > L) return true;
    std::vector<int> cur(m + 1, 0);
    cur[0] = 0;
    cur[m] = L;
    // iterative depth-first walk: position i in [1, m-1]
    if (m == 1) {
        out.push_back(0);
        out.push_back((uint16_t)L);
        n = 1;
        return true;
    }
    int i = 1;
    cur[1] = 0;
    while (i >= 1) {
        int b = cur[i] + 1;
        // remaining boundaries after i need room: b <= L - 1 - (m - 1 - i)
        int hi = L - 1 - (m - 1 - i);
        while (b <= hi && !legal(b, i, m, L, d)) b++;
        if (b > hi) {                         // exhausted this level: backtrack
            i--;
            continue;
        }
        cur[i] = b;
        if (i == m - 1) {
            if (n >= cap) return false;
            for (int q = 0; q <= m; q++) out.push_back((uint16_t)cur[q]);
            n++;
        } else {
            i++;
            cur[i] = cur[i - 1];
        }
    }
    return true;
}

// P_h(z) truncated at degree N: coefficient k = number of split vectors of a height-h tile
// into k slices (k <= Kmax).
void tile_poly(int h, int N, int Km, int dr, std::vector<u64> &P)
{
    P.assign(N + 1, 0);
    for (int k = 1; k <= std::min(std::min(Km, h), N); k++) P[k] = count_vectors(k, h, dr);
}

void poly_mul(const std::vector<u64> &a, const std::vector<u64> &b, std::vector<u64> &out, int N)
{
    out.assign(N + 1, 0);
    for (int i = 0; i <= N; i++) {
        if (!a[i]) continue;
        for (int j = 0; i + j <= N; j++)
            if (b[j]) out[i + j] = sadd(out[i + j], smul(a[i], b[j]));
    }
}

// Smallest RS count of a candidate (trs_search_params.min_rs; 0 means N).
int rs_floor(const trs_search_params *p)
{
    return p->min_rs > 0 ? p->min_rs : p->n_threads;
}

// |C| for one window pair, by a DP over tile-row boundaries (no enumeration of Y).
u64 space_count(int W, int H, const trs_search_params *p, int dt, int dr)
{
    const int N = p->n_threads, Km = p->max_rs_per_tile, Nlo = rs_floor(p);
    std::vector<std::vector<u64>> P(H + 1);
    for (int h = 1; h <= H; h++) tile_poly(h, N, Km, dr, P[h]);
    u64 total = 0;
    for (int c = 1; c <= p->max_tile_cols; c++) {
        u64 nx = count_vectors(c, W, dt);
        if (!nx) continue;
        // P_h^c for every h
        std::vector<std::vector<u64>> Pc(H + 1);
        for (int h = 1; h <= H; h++) {
            std::vector<u64> acc(N + 1, 0), tmp;
            acc[0] = 1;
            for (int rep = 0; rep < c; rep++) { poly_mul(acc, P[h], tmp, N); acc.swap(tmp); }
            Pc[h] = acc;
        }
        for (int r = 1; r <= p->max_tile_rows; r++) {
            if (!((int64_t)c * r <= N && (int64_t)Nlo <= (int64_t)Km * c * r)) continue;
            if (r > H) continue;
            // F[y] = polynomial over ways to place the first j row boundaries ending at y
            std::vector<std::vector<u64>> F(H + 1, std::vector<u64>(N + 1, 0)), G;
            F[0][0] = 1;
            for (int j = 1; j <= r; j++) {
                G.assign(H + 1, std::vector<u64>(N + 1, 0));
                for (int y = 1; y <= H; y++) {
                    if (j < r && (y == H || !legal(y, j, r, H, dt))) continue;
                    if (j == r && y != H) continue;
                    for (int yp = 0; yp < y; yp++) {
                        bool any = false;
                        for (int q = 0; q <= N && !any; q++) any = F[yp][q] != 0;
                        if (!any) continue;
                        std::vector<u64> prod;
                        poly_mul(F[yp], Pc[y - yp], prod, N);
                        for (int q = 0; q <= N; q++) G[y][q] = sadd(G[y][q], prod[q]);
                    }
                }
                F.swap(G);
            }
            for (int q = Nlo; q <= N; q++) total = sadd(total, smul(nx, F[H][q]));
        }
    }
    return total;
}

const int kLadder[6][2] = {{-1, -1}, {3, 1}, {2, 1}, {1, 1}, {1, 0}, {0, 0}};

}  // namespace

trs_status check_space_args(const trs_frame *f, const trs_search_params *p)
{
    if (!f || !p) return TRS_EINVAL;
    if (f->width < 1 || f->height < 1 || f->width > 8192 || f->height > 8192) return TRS_EINVAL;
    if (f->ctu_size != 32 && f->ctu_size != 64 && f->ctu_size != 128) return TRS_EINVAL;
    if (f->bit_depth < 8 || f->bit_depth > 12) return TRS_EINVAL;
    if (p->n_threads < 1 || p->n_threads > kMaxRS) return TRS_EINVAL;
    if (p->max_tile_cols < 1 || p->max_tile_rows < 1 || p->max_rs_per_tile < 1) return TRS_EINVAL;
    if (p->max_tile_cols > kMaxRS || p->max_tile_rows > kMaxRS) return TRS_EINVAL;
    if (p->area_k < 0 || p->area_k > 1000000) return TRS_EINVAL;
    if (p->prune < 0 || p->prune > 3) return TRS_EINVAL;
    if (p->min_rs < 0 || p->min_rs > p->n_threads) return TRS_EINVAL;
    if (p->span_tiles < 0 || p->span_tiles > 1) return TRS_EINVAL;
    if (p->lambda_den < 1 || p->lambda_den > 65535 || p->lambda_num > 65535) return TRS_EINVAL;
    bool ladder = p->dtile == -2 && p->drs == -2;
    if (!ladder && (p->dtile < -1 || p->drs < -1)) return TRS_EINVAL;
    if (p->sched_block != 0 && p->sched_block != 64 && p->sched_block != 128 &&
        p->sched_block != 256 && p->sched_block != 512) return TRS_EINVAL;
    if (p->sched_item < 0) return TRS_EINVAL;
    return TRS_OK;
}

trs_status space_size(int W, int H, const trs_search_params *p, int64_t *n, int32_t *dt, int32_t *dr)
{
    if (W < 1 || H < 1 || W > kMaxGrid || H > kMaxGrid) return TRS_EINVAL;
    if (p->span_tiles) return TRS_ENOTIMPL;          // only the literal-space search covers blocks
    int a, b;
    if (p->dtile == -2 && p->drs == -2) {
        u64 budget = p->space_budget > 0 ? (u64)p->space_budget : (u64(1) << 24);
        int pick = 5;
        for (int i = 0; i < 6; i++)
            if (space_count(W, H, p, kLadder[i][0], kLadder[i][1]) <= budget) { pick = i; break; }
        a = kLadder[pick][0];
        b = kLadder[pick][1];
    } else {
        a = p->dtile;
        b = p->drs;
    }
    u64 s = space_count(W, H, p, a, b);
    *n = s > (u64)INT64_MAX ? INT64_MAX : (int64_t)s;
    *dt = a;
    *dr = b;
    return TRS_OK;
}

// The optional pruning rules (trs_search_params.prune) for candidate m of one (shape, Y, X):
// bit 0, every tile's tallest slice is at most twice its shortest (pixel heights); bit 1,
// every tile's mean slice area lies within [1/1.5, 1.5] times the mean slice area of the
// other tiles.  Geometry only, like the area rule.
static bool coherent_tiles(int prune, int T, int M, int m, const uint16_t *cmb,
                           const std::vector<int> &rowoff, const std::vector<int> &trow,
                           const std::vector<int> &tcol, const std::vector<uint64_t> &wpx,
                           const std::vector<uint64_t> &tile_hpx, const std::vector<uint64_t> &hmn,
                           const std::vector<uint64_t> &hmx, const std::vector<int32_t> &optk,
                           uint64_t frame_px)
{
    int64_t n = 0;
    for (int t = 0; t < T; t++) n += optk[rowoff[trow[t]] + cmb[(size_t)t * M + m]];
    for (int t = 0; t < T; t++) {
        const int ro = rowoff[trow[t]] + cmb[(size_t)t * M + m];
        if ((prune & 1) && hmx[ro] > 2 * hmn[ro]) return false;
        if (prune & 2) {
            const int64_t k = optk[ro], rest = n - k;
            if (rest <= 0) continue;
            const int64_t a = (int64_t)(wpx[tcol[t]] * tile_hpx[trow[t]]), o = (int64_t)frame_px - a;
            if (2 * a * rest > 3 * o * k || 3 * a * rest < 2 * o * k) return false;
        }
    }
    return true;
}

trs_status build_plan(const trs_frame *f, const trs_search_params *p, Plan &pl)
{
    trs_status st = check_space_args(f, p);
    if (st != TRS_OK) return st;
    const int cs = f->ctu_size;
    const int W = (f->width + cs - 1) / cs, H = (f->height + cs - 1) / cs;
    const int N = p->n_threads, Km = p->max_rs_per_tile, Nlo = rs_floor(p);
    pl.width = f->width;
    pl.height = f->height;
    pl.cs = cs;
    pl.N = N;
    pl.Cm = p->max_tile_cols;
    pl.Rm = p->max_tile_rows;
    pl.Km = Km;
    pl.dtile_req = p->dtile;
    pl.drs_req = p->drs;
    pl.item_target = p->sched_item;
    pl.budget = p->space_budget;
    pl.W = W;
    pl.H = H;
    st = space_size(W, H, p, &pl.total, &pl.dt, &pl.dr);
    if (st != TRS_OK) return st;
    if (pl.total <= 0 || pl.total > kSpaceCap) return TRS_ENOSPACE;
    const int dt = pl.dt, dr = pl.dr;

    pl.colpx.assign(W + 1, 0);
    pl.rowpx.assign(H + 1, 0);
    for (int x = 0; x < W; x++) pl.colpx[x + 1] = pl.colpx[x] + std::min(cs, f->width - x * cs);
    for (int y = 0; y < H; y++) pl.rowpx[y + 1] = pl.rowpx[y] + std::min(cs, f->height - y * cs);

    // Shapes with their X and Y lists.
    struct ShapeHost { int c, r; std::vector<uint16_t> X, Y; int64_t nX, nY; };
    std::vector<ShapeHost> sh;
    std::vector<char> height_used(H + 1, 0);
    const int64_t vec_cap = int64_t(1) << 24;
    for (int c = 1; c <= p->max_tile_cols; c++) {
        for (int r = 1; r <= p->max_tile_rows; r++) {
            if (!((int64_t)c * r <= N && (int64_t)Nlo <= (int64_t)Km * c * r)) continue;
            ShapeHost s{c, r, {}, {}, 0, 0};
            if (!list_vectors(c, W, dt, vec_cap, s.X, s.nX)) return TRS_ENOSPACE;
            if (!list_vectors(r, H, dt, vec_cap, s.Y, s.nY)) return TRS_ENOSPACE;
            if (!s.nX || !s.nY) continue;
            for (int64_t yi = 0; yi < s.nY; yi++)
                for (int j = 0; j < r; j++)
                    height_used[s.Y[yi * (r + 1) + j + 1] - s.Y[yi * (r + 1) + j]] = 1;
            sh.push_back(std::move(s));
        }
    }

    // Options per used height: k ascending, Z lexicographic; opt_z rows of Km + 1 entries.
    pl.opt_base.assign(H + 2, 0);
    pl.opt_kcnt.assign((size_t)(H + 1) * (Km + 1), 0);
    for (int h = 1; h <= H; h++) {
        pl.opt_base[h] = (int32_t)pl.opt_k.size();
        int cnt = 0;
        if (height_used[h]) {
            for (int k = 1; k <= std::min(std::min(Km, h), N); k++) {
                std::vector<uint16_t> zs;
                int64_t nz = 0;
                if (!list_vectors(k, h, dr, 65536, zs, nz)) return TRS_ENOSPACE;
                for (int64_t q = 0; q < nz; q++) {
                    pl.opt_k.push_back((uint8_t)k);
                    for (int e = 0; e <= Km; e++)
                        pl.opt_z.push_back(e <= k ? zs[q * (k + 1) + e] : (uint16_t)h);
                }
                cnt += (int)nz;
                if (cnt > 65535) return TRS_ENOSPACE;
                pl.opt_kcnt[(size_t)h * (Km + 1) + k] = cnt;
            }
        }
        for (int k = 1; k <= Km; k++) {
            size_t i = (size_t)h * (Km + 1) + k;
            if (pl.opt_kcnt[i] < pl.opt_kcnt[i - 1]) pl.opt_kcnt[i] = pl.opt_kcnt[i - 1];
        }
    }
    pl.opt_base[H + 1] = (int32_t)pl.opt_k.size();
    auto kcnt = [&](int h, int kk) { return pl.opt_kcnt[(size_t)h * (Km + 1) + std::min(kk, Km)]; };

    // Combination tables per (shape, Y), in canonical order.
    int64_t rank_base = 0;
    const int64_t target = p->sched_item > 0 ? p->sched_item : 512;
    for (auto &s : sh) {
        const int c = s.c, r = s.r, T = c * r;
        const int kcap = std::min(Km, N - (T - 1));
        ShapeDev sd{};
        sd.c = c; sd.r = r; sd.T = T; sd.kcap = kcap;
        sd.nX = s.nX; sd.nY = s.nY;
        sd.x_off = (int64_t)pl.xtab.size();
        sd.y_off = (int64_t)pl.ytab.size();
        sd.yinfo_off = (int64_t)pl.y_M.size();
        int64_t SM = 0;
        std::vector<int> heights(T);
        for (int64_t yi = 0; yi < s.nY; yi++) {
            const uint16_t *Y = &s.Y[yi * (r + 1)];
            for (int t = 0; t < T; t++) heights[t] = Y[t / c + 1] - Y[t / c];
            // comp[t][n]: ways for tiles t..T-1 to take slices from n free threads, leaving
            // at most N - Nlo of them idle (saturating)
            std::vector<u64> comp((size_t)(T + 1) * (N + 1), 0);
            for (int n = 0; n <= N - Nlo; n++) comp[(size_t)T * (N + 1) + n] = 1;
            for (int t = T - 1; t >= 0; t--) {
                int h = heights[t];
                for (int n = 0; n <= N; n++) {
                    u64 acc = 0;
                    for (int k = 1; k <= std::min(kcap, std::min(h, n)); k++) {
                        u64 ways = (u64)(kcnt(h, k) - kcnt(h, k - 1));
                        acc = sadd(acc, smul(ways, comp[(size_t)(t + 1) * (N + 1) + n - k]));
                    }
                    comp[(size_t)t * (N + 1) + n] = acc;
                }
            }
            u64 M = comp[N];
            if (M > (u64)INT32_MAX) return TRS_ENOSPACE;
            pl.y_prefM.push_back(SM);
            pl.y_M.push_back((int32_t)M);
            pl.y_combo.push_back((int64_t)pl.combos.size());
            if ((int64_t)pl.combos.size() + (int64_t)M * T > kComboCap) return TRS_ENOSPACE;
            if (M) {
                size_t off = pl.combos.size();
                pl.combos.resize(off + (size_t)M * T);
                // depth-first walk in canonical order; cur[t] = local option index
                std::vector<int> cur(T, 0), kk(T, 0), left(T + 1, 0);
                int64_t m = 0;
                // explicit stack: for each tile, iterate over options with usable k
                std::vector<int> opt_end(T, 0);
                int t = 0;
                left[0] = N;
                bool descend = true;
                while (t >= 0) {
                    int h = (t < T) ? heights[t] : 0;
                    if (t == T) {
                        for (int q = 0; q < T; q++) pl.combos[off + (size_t)q * M + m] = (uint16_t)cur[q];
                        m++;
                        t--;
                        descend = false;
                        continue;
                    }
                    int o;
                    if (descend) {
                        o = 0;
                    } else {
                        o = cur[t] + 1;
                    }
                    // advance o to the next option whose k leaves a completable remainder
                    int n = left[t];
                    int last = kcnt(h, std::min(kcap, n));
                    while (o < last) {
                        int k = pl.opt_k[pl.opt_base[h] + o];
                        if (comp[(size_t)(t + 1) * (N + 1) + n - k]) break;
                        o = kcnt(h, k);                      // skip every option with this k
                    }
                    if (o >= last) {
                        t--;
                        descend = false;
                        continue;
                    }
                    cur[t] = o;
                    left[t + 1] = n - pl.opt_k[pl.opt_base[h] + o];
                    t++;
                    descend = true;
                }
                if (m != (int64_t)M) return TRS_EINVAL;      // internal consistency
            }
            SM += (int64_t)M;
        }
        if (SM == 0) {
            pl.y_prefM.resize(sd.yinfo_off);
            pl.y_M.resize(sd.yinfo_off);
            pl.y_combo.resize(sd.yinfo_off);
            continue;
        }
        sd.SM = SM;
        sd.rank_base = rank_base;
        pl.xtab.insert(pl.xtab.end(), s.X.begin(), s.X.end());
        pl.ytab.insert(pl.ytab.end(), s.Y.begin(), s.Y.end());
        const int32_t shape_idx = (int32_t)pl.shapes.size();

        // Work items.  Every candidate of (shape, Y) is tested against the area rule here,
        // once per geometry; the feasible ones are grouped into items of about `target`
        // candidates, each with the tile-option records its candidates reference.
        for (int64_t yi = 0; yi < s.nY; yi++) {
            const int32_t M = pl.y_M[sd.yinfo_off + yi];
            if (!M) continue;
            const uint16_t *Y = &s.Y[yi * (r + 1)];
            const uint16_t *cmb = &pl.combos[pl.y_combo[sd.yinfo_off + yi]];
            std::vector<int> rowoff(r + 1, 0);
            for (int j = 0; j < r; j++) {
                int h = Y[j + 1] - Y[j];
                rowoff[j + 1] = rowoff[j] + kcnt(h, std::min(kcap, h));
            }
            const int rrow = rowoff[r];
            // pixel heights of the smallest / largest slice of each (tile row, option)
            std::vector<uint64_t> hmn(rrow), hmx(rrow);
            std::vector<int32_t> optg(rrow), optk(rrow);
            for (int j = 0; j < r; j++) {
                int h = Y[j + 1] - Y[j];
                for (int o = 0; o < rowoff[j + 1] - rowoff[j]; o++) {
                    int opt = pl.opt_base[h] + o;
                    int k = pl.opt_k[opt];
                    const uint16_t *z = &pl.opt_z[(size_t)opt * (Km + 1)];
                    uint64_t lo = UINT64_MAX, hi = 0;
                    for (int q = 0; q < k; q++) {
                        uint64_t px = (uint64_t)(pl.rowpx[Y[j] + z[q + 1]] - pl.rowpx[Y[j] + z[q]]);
                        lo = std::min(lo, px);
                        hi = std::max(hi, px);
                    }
                    hmn[rowoff[j] + o] = lo;
                    hmx[rowoff[j] + o] = hi;
                    optg[rowoff[j] + o] = opt;
                    optk[rowoff[j] + o] = k;
                }
            }
            // open item
            std::vector<uint32_t> cur_f;
            std::vector<uint16_t> cur_rid;             // entry-major while building
            std::vector<uint32_t> cur_desc;
            std::vector<std::pair<int, int>> cur_spans;
            std::vector<int32_t> remap;               // span * rrow + rowoff[j] + o -> record
            int64_t cur_xa = -1;
            int64_t cur_slices = 0;
            auto close_item = [&]() {
                if (cur_f.empty()) return;
                const int n = (int)cur_f.size();
                ItemDev it{};
                it.rank0 = rank_base + cur_xa * SM + pl.y_prefM[sd.yinfo_off + yi];
                it.combo_off = pl.y_combo[sd.yinfo_off + yi];
                it.SM = SM;
                it.y_row = sd.y_off + yi * (r + 1);
                it.ent_off = (int64_t)pl.ent_f.size();
                it.rid_off = (int64_t)pl.ent_rid.size();
                it.rec_off = (int64_t)(pl.rdesc.size() / 2);
                it.shape = shape_idx;
                it.yi = (int32_t)yi;
                it.xa = (int32_t)cur_xa;
                it.M = M;
                it.n_ent = n;
                it.n_rec = (int32_t)(cur_desc.size() / 2);
                it.c = c;
                it.r = r;
                it.T = T;
                pl.ent_f.insert(pl.ent_f.end(), cur_f.begin(), cur_f.end());
                const size_t base = pl.ent_rid.size();
                pl.ent_rid.resize(base + (size_t)n * T);
                for (int e = 0; e < n; e++)
                    for (int t = 0; t < T; t++) pl.ent_rid[base + (size_t)t * n + e] = cur_rid[(size_t)e * T + t];
                // every item's array starts on 16 bytes and may be read in 16-byte pieces
                pl.ent_rid.resize((pl.ent_rid.size() + 7) & ~size_t(7), 0);
                pl.rid_max = std::max(pl.rid_max, (int32_t)(((int64_t)n * T + 7) & ~int64_t(7)));
                pl.rdesc.insert(pl.rdesc.end(), cur_desc.begin(), cur_desc.end());
                pl.items.push_back(it);
                pl.rec_max = std::max(pl.rec_max, it.n_rec);
                pl.records += it.n_rec;
                pl.record_slices += cur_slices;
                pl.tile_lookups += (int64_t)n * T;
                pl.n_feasible += n;
                cur_f.clear();
                cur_rid.clear();
                cur_desc.clear();
                cur_spans.clear();
                remap.clear();
                cur_xa = -1;
                cur_slices = 0;
            };
            std::vector<uint64_t> wpx(c), tile_hpx(r);
            for (int j = 0; j < r; j++) tile_hpx[j] = (uint64_t)(pl.rowpx[Y[j + 1]] - pl.rowpx[Y[j]]);
            const uint64_t frame_px = (uint64_t)pl.colpx[W] * (uint64_t)pl.rowpx[H];
            std::vector<int> sidx(c), tcol(T), trow(T);
            for (int t = 0; t < T; t++) { tcol[t] = t % c; trow[t] = t / c; }
            for (int64_t xi = 0; xi < s.nX; xi++) {
                const uint16_t *X = &s.X[xi * (c + 1)];
                for (int i = 0; i < c; i++) wpx[i] = (uint64_t)(pl.colpx[X[i + 1]] - pl.colpx[X[i]]);
                bool have_sidx = false;
                for (int32_t m = 0; m < M; m++) {
                    uint64_t amin = UINT64_MAX, amax = 0;
                    for (int t = 0; t < T; t++) {
                        const int ro = rowoff[trow[t]] + cmb[(size_t)t * M + m];
                        amin = std::min(amin, wpx[tcol[t]] * hmn[ro]);
                        amax = std::max(amax, wpx[tcol[t]] * hmx[ro]);
                    }
                    if (p->area_k != 0 && !((uint64_t)p->area_k * amin > amax)) continue;
                    if (p->prune && !coherent_tiles(p->prune, T, M, m, cmb, rowoff, trow, tcol, wpx,
                                                    tile_hpx, hmn, hmx, optk, frame_px))
                        continue;
                    if (!cur_f.empty() && ((int64_t)cur_desc.size() / 2 + T > kRecCap ||
                                           (int)cur_spans.size() + c > kSpanCap ||
                                           (xi - cur_xa + 1) * (int64_t)M > INT32_MAX)) {
                        close_item();
                        have_sidx = false;
                    }
                    if (cur_f.empty()) {
                        cur_xa = xi;
                        have_sidx = false;
                    }
                    if (!have_sidx) {
                        for (int i = 0; i < c; i++) {
                            std::pair<int, int> key(X[i], X[i + 1]);
                            int idx = -1;
                            for (size_t q = 0; q < cur_spans.size(); q++)
                                if (cur_spans[q] == key) { idx = (int)q; break; }
                            if (idx < 0) {
                                idx = (int)cur_spans.size();
                                cur_spans.push_back(key);
                                remap.resize(cur_spans.size() * (size_t)rrow, -1);
                            }
                            sidx[i] = idx;
                        }
                        have_sidx = true;
                    }
                    for (int t = 0; t < T; t++) {
                        const int ro = rowoff[trow[t]] + cmb[(size_t)t * M + m];
                        const size_t dense = (size_t)sidx[tcol[t]] * rrow + ro;
                        if (remap[dense] < 0) {
                            remap[dense] = (int32_t)(cur_desc.size() / 2);
                            const int i = tcol[t];
                            cur_desc.push_back((uint32_t)X[i] | ((uint32_t)X[i + 1] << 9) |
                                               ((uint32_t)Y[trow[t]] << 18));
                            cur_desc.push_back((uint32_t)optg[ro]);
                            cur_slices += optk[ro];
                        }
                        cur_rid.push_back((uint16_t)remap[dense]);
                    }
                    cur_f.push_back((uint32_t)((xi - cur_xa) * M + m));
                    if ((int64_t)cur_f.size() >= target) {
                        close_item();
                        have_sidx = false;
                    }
                }
            }
            close_item();
        }
        if (pl.items.size() > (size_t)1 << 26) return TRS_ENOSPACE;
        rank_base += s.nX * SM;
        pl.shapes.push_back(sd);
    }
    if (rank_base != pl.total) return TRS_EINVAL;            // two counts must agree

    // Compact record descriptors: the option's split rows inline, so a record is one load.
    {
        const size_t nrec = pl.rdesc.size() / 2;
        bool ok = true;
        std::vector<uint32_t> d4(nrec * 4, 0);
        for (size_t q = 0; q < nrec && ok; q++) {
            const int opt = (int)pl.rdesc[2 * q + 1];
            const int k = pl.opt_k[opt];
            const uint16_t *z = &pl.opt_z[(size_t)opt * (Km + 1)];
            if (k > 11 || z[k] > 255) { ok = false; break; }
            uint8_t bytes[12] = {0};
            bytes[0] = (uint8_t)k;
            for (int i = 1; i <= k; i++) bytes[i] = (uint8_t)z[i];
            d4[4 * q] = pl.rdesc[2 * q];
            for (int w = 0; w < 3; w++)
                d4[4 * q + 1 + w] = (uint32_t)bytes[4 * w] | ((uint32_t)bytes[4 * w + 1] << 8) |
                                    ((uint32_t)bytes[4 * w + 2] << 16) | ((uint32_t)bytes[4 * w + 3] << 24);
        }
        pl.compact = ok ? 1 : 0;
        if (ok) pl.rdesc4.swap(d4);
        else pl.rdesc4.clear();
    }

    // The uniform grid (Section 3.2): c_u r_u = N, most square, c_u >= r_u, one RS per tile.
    pl.ru = 1;
    for (int d = 1; d * d <= N; d++) if (N % d == 0) pl.ru = d;
    pl.cu = N / pl.ru;
    pl.n_unif = 0;
    pl.unif_rs.clear();
    pl.uniform_rank = -1;
    if (pl.cu <= W && pl.ru <= H) {
        for (int j = 0; j < pl.ru; j++)
            for (int i = 0; i < pl.cu; i++) {
                pl.unif_rs.push_back((int32_t)((int64_t)i * W / pl.cu));
                pl.unif_rs.push_back((int32_t)((int64_t)j * H / pl.ru));
                pl.unif_rs.push_back((int32_t)((int64_t)(i + 1) * W / pl.cu));
                pl.unif_rs.push_back((int32_t)((int64_t)(j + 1) * H / pl.ru));
                pl.n_unif++;
            }
        for (const auto &sd : pl.shapes) {
            if (sd.c != pl.cu || sd.r != pl.ru) continue;
            int64_t xi = -1, yi = -1;
            for (int64_t q = 0; q < sd.nX && xi < 0; q++) {
                bool eq = true;
                for (int i = 0; i <= sd.c && eq; i++)
                    eq = pl.xtab[sd.x_off + q * (sd.c + 1) + i] == (int64_t)i * W / sd.c;
                if (eq) xi = q;
            }
            for (int64_t q = 0; q < sd.nY && yi < 0; q++) {
                bool eq = true;
                for (int j = 0; j <= sd.r && eq; j++)
                    eq = pl.ytab[sd.y_off + q * (sd.r + 1) + j] == (int64_t)j * H / sd.r;
                if (eq) yi = q;
            }
            if (xi >= 0 && yi >= 0 && pl.y_M[sd.yinfo_off + yi] > 0)
                pl.uniform_rank = sd.rank_base + xi * sd.SM + pl.y_prefM[sd.yinfo_off + yi];
        }
    }
    return TRS_OK;
}

trs_status decode_rank(const Plan &pl, int64_t rank, trs_result *o)
{
    if (rank < 0 || rank >= pl.total) return TRS_EINVAL;
    size_t s = 0;
    while (s + 1 < pl.shapes.size() && pl.shapes[s + 1].rank_base <= rank) s++;
    const ShapeDev &sd = pl.shapes[s];
    int64_t rem = rank - sd.rank_base;
    int64_t xi = rem / sd.SM, r2 = rem % sd.SM;
    const int64_t *pref = &pl.y_prefM[sd.yinfo_off];
    int64_t yi = std::upper_bound(pref, pref + sd.nY, r2) - pref - 1;
    while (yi > 0 && pl.y_M[sd.yinfo_off + yi] == 0) yi--;
    int64_t m = r2 - pref[yi];
    const int32_t M = pl.y_M[sd.yinfo_off + yi];
    const int64_t coff = pl.y_combo[sd.yinfo_off + yi];
    const uint16_t *X = &pl.xtab[sd.x_off + xi * (sd.c + 1)];
    const uint16_t *Y = &pl.ytab[sd.y_off + yi * (sd.r + 1)];
    o->rank = rank;
    o->tile_cols = sd.c;
    o->tile_rows = sd.r;
    for (int i = 0; i <= sd.c; i++) o->col_bd[i] = X[i];
    for (int j = 0; j <= sd.r; j++) o->row_bd[j] = Y[j];
    int n = 0;
    const int Km = pl.Km;
    for (int t = 0; t < sd.T; t++) {
        int i = t % sd.c, j = t / sd.c;
        int h = Y[j + 1] - Y[j];
        int opt = pl.opt_base[h] + pl.combos[coff + (int64_t)t * M + m];
        int k = pl.opt_k[opt];
        const uint16_t *z = &pl.opt_z[(size_t)opt * (Km + 1)];
        for (int q = 0; q < k; q++) {
            o->rs[n][0] = X[i];
            o->rs[n][1] = Y[j] + z[q];
            o->rs[n][2] = X[i + 1];
            o->rs[n][3] = Y[j] + z[q + 1];
            n++;
        }
    }
    o->n_rs = n;
    o->dtile_used = pl.dt;
    o->drs_used = pl.dr;
    o->n_enumerated = pl.total;
    return TRS_OK;
}

}  // namespace trs
