// Internal interface between the host runtime and the kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace mgc {

struct LaunchCtx {
    hipStream_t stream;
    int H, W;
    double alpha;
    int kind;   // 0 mean, 1 Gaussian
    bool f64;   // state dtype
    int M, G;   // samples, bisection steps
};

// Scratch of the coarse (lazily applied) levels.
struct CoarseScratch {
    double* partials;   // per block and row chunk: partial sums of f - u
    int nchunk;         // set by launch_level_begin
    double* cpend;      // pending corrections of the level being swept, m_j x n_j
    double* cpend_alt;  // the previous coarse level's, while they are applied by the next level's sums pass
    double* rec;        // expanded ring records of the streamed levels (shape side >= STREAMED_B)
    size_t rec_cap;     // doubles in rec
    // split solve (one block on several workgroups, see mgc_split.hip); split_cus = 0: off
    unsigned long long* xslots;   // xblocks regions of xstride exchange words
    int xstride, xblocks;
    unsigned xepoch;              // tag of the last split launch (0 is never a tag)
    int split_cus;                // workgroups one launch may keep resident (the CU count)
    int split_polls;              // bound on the polls of one exchange wait
};

// Exchange slots of one split launch: block k of the launch uses slots[k * stride ..];
// P = 2^d - 1 workgroups per block; tag marks the words this launch writes.
struct SplitArgs {
    unsigned long long* slots;
    int P, d;
    int stride;
    unsigned tag;
    int polls;    // bound on the polls of one wait; a value not seen by then is computed locally
};

// Block side at level j (1-based): 2^(j-1) (schedule 0, nested blocks) or 2^j - 1
// (schedule 1, the patch side of Section 2.2).  Level 1 is the pixel level in both.
inline int block_side(int level, int schedule)
{
    // unsigned: level 31 (2^31 - 1) is in range for a 2^29-pixel-wide image
    return schedule == 1 ? (int)((1u << level) - 1u) : (int)(1u << (level - 1));
}
// Smallest power of two >= b: the lane-group shape of a level is that of this side
// (a 2^j - 1 ring has 8 fewer pixels than the 2^j one, so the same slots hold it).
inline int shape_side(int b)
{
    int s = 1;
    while (s < b) s <<= 1;
    return s;
}
// Shape side from which the ring no longer fits in registers (one workgroup per block,
// records rebuilt from memory or read from the record scratch at every evaluation).
constexpr int STREAMED_B = 1024;
// Doubles of record scratch the streamed levels of an H x W image with J levels need.
size_t record_scratch_doubles(int H, int W, int J, int schedule);

// b = 1: colour sweep from uin into uout (every pixel of uout is written).
hipError_t launch_sweep_pixels(const LaunchCtx& L, const void* uin, void* uout, const void* f, int colour, int ncolours);
// Tree depth d of the split solve for a launch of nblocks blocks of side b (0: not split):
// the largest d <= min(8, G) with nblocks (2^d - 1) <= cus (and, for streamed sides, the
// workgroups' record copies within a cache-sized budget), for sides >= 256; 0 below depth 4
// (register-resident rings) or 2 (streamed rings).
int split_depth(int nblocks, int cus, int G, int b);
// Record-scratch doubles a split launch of a streamed side needs (one region per workgroup).
size_t split_record_doubles(int nblocks, int cus, int G, int b);
// Polls of one exchange wait by default (some milliseconds).
constexpr int SPLIT_POLLS = 1 << 14;
// Exchange words one block of a split launch needs: 2 M sample words and ceil(G / d) rounds of 2^d - 1.
size_t split_slot_words(int M, int G, int d);
// Coarse colour sweep of nbr x nbc blocks (colour (pr, pc)) by the split solve, P workgroups per block.
struct CoarseArgs;
hipError_t launch_sweep_split(const LaunchCtx& L, void* u, const void* f, int b, int pr, int pc, int nbr, int nbc,
                              const CoarseArgs& ca, const SplitArgs& sa);
// b >= 2: colour sweep (in place on fine levels, into cs.cpend on coarse levels).
hipError_t launch_sweep_blocks(const LaunchCtx& L, void* u, const void* f, int b, int colour, CoarseScratch& cs);
// Coarse levels (level_is_lazy(b)): block sums and zeroed corrections before the
// colours, the correction pass after them.
bool level_is_lazy(int b);
void coarse_geometry(int H, int W, int b, int* nblocks, int* nchunk, int* rows_per);
// prev_b > 0: the coarse level of side prev_b left its corrections in cs.cpend
// unapplied; this level's sums pass applies them to u (the same rounding as the
// correction pass) before summing, so that level needs no correction pass of its own.
hipError_t launch_level_begin(const LaunchCtx& L, void* u, const void* f, int b, CoarseScratch& cs, int prev_b = 0);
hipError_t launch_level_end(const LaunchCtx& L, void* u, int b, const CoarseScratch& cs);
// out[0] = ||u - prev||^2, out[1] = ||u||^2 (device, FP64, fixed order), using
// partials (2 x energy_partials_count doubles).
hipError_t launch_diff_norms(const LaunchCtx& L, const void* u, const void* prev, double* partials, double* out);
// F(u) into out[0] (device), using partials (energy_partials_count doubles).
hipError_t launch_energy(const LaunchCtx& L, const void* u, const void* f, double* partials, double* out);
int energy_partials_count(int H, int W);

}  // namespace mgc
