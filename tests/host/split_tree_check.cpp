// Host check of the split coarse solve's bookkeeping (the device code's own headers, built for
// the host):
//  * the bisection tree: for random brackets and G = 0..64 bisection steps, rounds of d = 1..8
//    steps whose node signs are taken at tree_node_mid (as the workgroups of a split launch take
//    them) and walked with tree_walk end on the bitwise same bracket as G sequential steps, and
//    every midpoint the walk visits equals its node's tree_node_mid.  Two kinds of sign: a
//    monotone V' (one root) and an arbitrary function of the midpoint's bits (many sign changes,
//    so any midpoint formed differently would be caught);
//  * split_depth: the largest depth whose workgroups fit the CUs (and, for streamed sides, whose
//    record copies fit the budget), zero below the minimum depth or for sides under 256, and
//    split_slot_words / split_record_doubles large enough for the launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2204_07921_amd/csrc/mgc_split.hip"

static uint64_t bits_of(double x)
{
    uint64_t b;
    std::memcpy(&b, &x, sizeof b);
    return b;
}

// an arbitrary sign: a hash of the midpoint's bits
static bool hashed_sign(double mid, uint64_t salt)
{
    uint64_t z = bits_of(mid) ^ salt;
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdull;
    z ^= z >> 33;
    z *= 0xc4ceb9fe1a85ec53ull;
    z ^= z >> 33;
    return (z & 1u) != 0;
}

int main()
{
    long cases = 0, bad = 0;
    std::mt19937_64 rng(20220415);
    std::uniform_real_distribution<double> U(-3.0, 3.0);
    for (int trial = 0; trial < 400; ++trial) {
        double lo0 = U(rng), hi0 = U(rng);
        if (hi0 < lo0) std::swap(lo0, hi0);
        if (hi0 == lo0) hi0 += 1.0;
        const double root = lo0 + (hi0 - lo0) * std::uniform_real_distribution<double>(0.0, 1.0)(rng);
        const uint64_t salt = rng();
        for (int kind = 0; kind < 2; ++kind) {
            auto vpos = [&](double mid) { return kind == 0 ? mid > root : hashed_sign(mid, salt); };
            for (int G : {0, 1, 2, 3, 5, 7, 8, 13, 31, 32, 33, 64}) {
                double slo = lo0, shi = hi0;   // sequential steps
                for (int g = 0; g < G; ++g) {
                    const double mid = 0.5 * (slo + shi);
                    if (vpos(mid)) shi = mid; else slo = mid;
                }
                for (int d = 1; d <= 8; ++d) {
                    double lo = lo0, hi = hi0;
                    bool ok = true;
                    for (int g0 = 0; g0 < G; g0 += d) {
                        const int dd = G - g0 < d ? G - g0 : d;
                        const int nn = (1 << dd) - 1;
                        std::vector<double> mids(nn + 1);
                        std::vector<char> pos(nn + 1);
                        for (int node = 1; node <= nn; ++node) {   // one workgroup per node
                            mids[node] = mgc::tree_node_mid(node, lo, hi);
                            pos[node] = vpos(mids[node]);
                        }
                        mgc::tree_walk(dd, lo, hi, [&](int node, double mid) {
                            ok = ok && node >= 1 && node <= nn && bits_of(mid) == bits_of(mids[node]);
                            return pos[node] != 0;
                        });
                    }
                    ok = ok && bits_of(lo) == bits_of(slo) && bits_of(hi) == bits_of(shi);
                    ++cases;
                    if (!ok) {
                        if (bad < 5) std::printf("tree trial %d kind %d G %d d %d\n", trial, kind, G, d);
                        ++bad;
                    }
                }
            }
        }
    }
    for (int cus : {32, 80, 256, 304})
        for (int nblocks = 0; nblocks <= 300; ++nblocks)
            for (int G : {0, 1, 2, 3, 5, 32, 64})
                for (int b : {63, 64, 127, 128, 255, 256, 511, 512, 1023, 1024, 2047, 2048, 4096, 8191}) {
                    const int d = mgc::split_depth(nblocks, cus, G, b);
                    const int s = mgc::shape_side(b);
                    const bool streamed = s >= mgc::STREAMED_B;
                    const double copy = 7.0 * 8.0 * 8.0 * b;
                    auto fits = [&](int dd) {
                        const double wg = (double)nblocks * ((1 << dd) - 1);
                        return dd <= (streamed ? 6 : 8) && dd <= G && wg <= cus &&
                               (!streamed || wg * copy <= mgc::SPLIT_STREAM_BYTES);
                    };
                    bool ok = true;
                    if (s < 256 || nblocks == 0 || G == 0) {
                        ok = d == 0;
                    } else {
                        int best = 0;
                        while (best < 8 && fits(best + 1)) ++best;
                        const int dmin = streamed ? 2 : 4;
                        ok = d == (best >= dmin ? best : 0);
                    }
                    if (d > 0) {
                        const size_t words = mgc::split_slot_words(16, G, d);
                        ok = ok && words >= 2 * 16 + (size_t)((G + d - 1) / d) * ((1u << d) - 1u);
                        const size_t recs = mgc::split_record_doubles(nblocks, cus, G, b);
                        ok = ok && (streamed ? recs >= (size_t)nblocks * ((1u << d) - 1u) * 7 * (size_t)(8 * b)
                                             : recs == 0);
                    }
                    ++cases;
                    if (!ok) {
                        if (bad < 10) std::printf("depth cus %d nblocks %d G %d b %d: d %d\n", cus, nblocks, G, b, d);
                        ++bad;
                    }
                }
    std::printf("cases %ld bad %ld\n", cases, bad);
    return bad == 0 ? 0 : 1;
}
