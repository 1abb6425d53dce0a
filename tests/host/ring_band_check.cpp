// Host check of the block-ring enumeration used by the colour sweeps: for every block of every
// image up to 23 x 23 and block sides 2..16 (powers of two and 2^j - 1), the candidates listed by
// ring_band / band_at lie inside the image, are distinct, number at most 8b, and include every ring
// pixel, i.e. every pixel whose nine clamped taps lie partly inside and partly outside the block
// (brute force).  For every candidate's clamped taps, tap_block (the coarse levels' lookup of a
// tap's pending correction) equals the block index by division.  The b = 2 split of a colour's
// blocks into border and interior ones (split2) is checked against its definition, and the
// sign-bit side tests (side_of, inside_of) against comparisons.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <set>
#include <utility>

#include "../../paper_2204_07921_amd/csrc/mgc_sweep.h"

static int clampi_h(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static bool is_ring(int H, int W, int i, int j, int r0, int r1, int c0, int c1)
{
    if (i < 0 || i >= H || j < 0 || j >= W) return false;
    int n = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int ci = clampi_h(i + dy, 0, H - 1), cj = clampi_h(j + dx, 0, W - 1);
            n += (ci >= r0 && ci < r1 && cj >= c0 && cj < c1) ? 1 : 0;
        }
    return n > 0 && n < 9;
}

int main()
{
    long cases = 0, bad = 0;
    for (int H = 1; H <= 23; ++H)
        for (int W = 1; W <= 23; ++W)
            for (int b : {2, 3, 4, 7, 8, 15, 16})
                for (int r0 = 0; r0 < H; r0 += b)
                    for (int c0 = 0; c0 < W; c0 += b) {
                        const int r1 = r0 + b < H ? r0 + b : H, c1 = c0 + b < W ? c0 + b : W;
                        const int nj = (W + b - 1) / b, pq = (r0 / b) * nj + c0 / b;
                        const mgc::RingBand B = mgc::ring_band(H, W, r0, r1, c0, c1);
                        std::set<std::pair<int, int>> got;
                        bool dup = false, outside = false, index = true;
                        for (int k = 0; k < B.n; ++k) {
                            int i, j;
                            mgc::band_at(B, k, i, j);
                            outside = outside || i < 0 || i >= H || j < 0 || j >= W;
                            dup = dup || !got.insert({i, j}).second;
                            for (int dy = -1; dy <= 1; ++dy)
                                for (int dx = -1; dx <= 1; ++dx) {
                                    const int ci = clampi_h(i + dy, 0, H - 1), cj = clampi_h(j + dx, 0, W - 1);
                                    if (mgc::tap_block(pq, nj, ci, cj, r0, r1, c0, c1) != (ci / b) * nj + cj / b)
                                        index = false;
                                }
                        }
                        bool cover = true;
                        for (int i = r0 - 2; i <= r1 + 1; ++i)
                            for (int j = c0 - 2; j <= c1 + 1; ++j)
                                if (is_ring(H, W, i, j, r0, r1, c0, c1) && !got.count({i, j})) cover = false;
                        ++cases;
                        if (dup || outside || !cover || !index || B.n > 8 * b) {
                            if (bad < 5)
                                std::printf("H %d W %d b %d block (%d, %d): n %d dup %d outside %d cover %d index %d\n",
                                            H, W, b, r0, c0, B.n, dup, outside, cover, index);
                            ++bad;
                        }
                    }
    // b = 2 colour split: every block of the colour exactly once, border blocks (p or q on the
    // first or last block row or column) numbered before the interior ones
    for (int mj = 1; mj <= 13; ++mj)
        for (int nj = 1; nj <= 13; ++nj)
            for (int pr = 0; pr < 2; ++pr)
                for (int pc = 0; pc < 2; ++pc) {
                    const mgc::Split2 S = mgc::split2(mj, nj, pr, pc);
                    std::set<std::pair<int, int>> seen;
                    bool ok = S.nbr == (mj - pr + 1) / 2 && S.nbc == (nj - pc + 1) / 2;
                    for (int k = 0; k < S.nbr * S.nbc; ++k) {
                        int bi, bj;
                        const bool interior = mgc::split2_at(S, k, bi, bj);
                        const int p = 2 * bi + pr, q = 2 * bj + pc;
                        ok = ok && bi >= 0 && bi < S.nbr && bj >= 0 && bj < S.nbc && seen.insert({bi, bj}).second;
                        ok = ok && interior == (p >= 1 && p <= mj - 2 && q >= 1 && q <= nj - 2);
                        ok = ok && interior == (k >= S.nborder);
                    }
                    ok = ok && (int)seen.size() == S.nbr * S.nbc;
                    ++cases;
                    if (!ok) {
                        if (bad < 5) std::printf("split2 mj %d nj %d pr %d pc %d\n", mj, nj, pr, pc);
                        ++bad;
                    }
                }
    // the sign-bit side tests behind tap_block and the in-block tap mask, against comparisons
    // (every v near and across the interval, intervals from width 1 up to wide image spans)
    for (int lo = -3; lo <= 40; ++lo)
        for (int hi : {lo + 1, lo + 2, lo + 3, lo + 7, lo + 64, lo + 1000, 1 << 30})
            for (int v = -70; v <= 1100; ++v) {
                const int side = v < lo ? -1 : (v >= hi ? 1 : 0);
                const int in = (v >= lo && v < hi) ? 1 : 0;
                ++cases;
                if (mgc::side_of(v, lo, hi) != side || mgc::inside_of(v, lo, hi) != in) {
                    if (bad < 5) std::printf("side_of/inside_of v %d lo %d hi %d\n", v, lo, hi);
                    ++bad;
                }
            }
    std::printf("cases %ld bad %ld\n", cases, bad);
    return bad == 0 ? 0 : 1;
}
