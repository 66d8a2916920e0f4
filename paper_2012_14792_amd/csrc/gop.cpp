// Random-access GOP bookkeeping for the time estimator's reference frame (Section 2.1).
//
// In a dyadic hierarchical GOP of size G, frame p (display order) sits in temporal layer 0
// when G divides p, else in layer log2(G) - ctz(p).  Each GOP codes its last frame first, then
// the midpoint of every open interval before the two halves (depth first, left half first).
// The co-TL reference of a frame is the frame coded most recently before it in the same
// temporal layer; the closest reference is the already coded frame nearest in display order.
#include <cstdint>
#include <vector>

#include "trs.h"

namespace {

int log2_exact(int g)
{
    int l = 0;
    while ((1 << l) < g) l++;
    return (1 << l) == g ? l : -1;
}

}  // namespace

extern "C" trs_status trs_ra_schedule(int32_t gop_size, int32_t n_frames, int32_t *coding_order,
                                      int32_t *layer, int32_t *cotl_ref, int32_t *closest_ref)
{
    const int lg = log2_exact(gop_size);
    if (gop_size < 1 || gop_size > 256 || lg < 0 || n_frames < 1 || n_frames > (1 << 24))
        return TRS_EINVAL;
    if (!coding_order || !layer || !cotl_ref || !closest_ref) return TRS_EINVAL;

    for (int32_t p = 0; p < n_frames; p++)
        layer[p] = (p % gop_size == 0) ? 0 : lg - __builtin_ctz((unsigned)p);

    // Coding order: frame 0, then per GOP its key frame and the bisection points.
    int32_t n = 0;
    coding_order[n++] = 0;
    struct Span { int32_t lo, hi; };
    std::vector<Span> stack;
    for (int32_t base = 0; base + 1 < n_frames; base += gop_size) {
        const int32_t key = base + gop_size;
        if (key < n_frames) coding_order[n++] = key;
        stack.assign(1, Span{base, key});
        while (!stack.empty()) {
            const Span s = stack.back();
            stack.pop_back();
            if (s.hi - s.lo < 2) continue;
            const int32_t mid = s.lo + (s.hi - s.lo) / 2;
            if (mid < n_frames) coding_order[n++] = mid;
            stack.push_back(Span{mid, s.hi});           // right half after the left one
            stack.push_back(Span{s.lo, mid});
        }
    }
    if (n != n_frames) return TRS_EINVAL;                // every frame coded exactly once

    // References, walking the coding order once.
    std::vector<int32_t> last(lg + 1, -1);
    std::vector<char> coded(n_frames, 0);
    for (int32_t i = 0; i < n_frames; i++) {
        const int32_t p = coding_order[i];
        cotl_ref[p] = last[layer[p]];
        last[layer[p]] = p;
        int32_t best = -1;
        for (int32_t d = 1; d < n_frames && best < 0; d++) {
            if (p - d >= 0 && coded[p - d]) best = p - d;                 // ties: earlier frame
            else if (p + d < n_frames && coded[p + d]) best = p + d;
        }
        closest_ref[p] = best;
        coded[p] = 1;
    }
    return TRS_OK;
}
