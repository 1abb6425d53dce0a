// Coarse levels with one block solved by several workgroups (gfx950).
//
// On the coarse levels of an image the size of the 1024 x 1024 workload a
// colour holds few blocks (one at b = 512, four at b = 256; larger images
// reach such colours at larger sides), so the one-
// workgroup-per-block sweep keeps a handful of the 256 CUs busy while each
// block's 51 ring evaluations (K(0) and K(f*), M samples, G bisection steps,
// the final K) run one after another on its CU.  Here one block is solved by
// P = 2^d - 1 workgroups (one launch of at most one workgroup per CU):
//
//   * every workgroup builds the whole ring in registers and takes K(0) and
//     K(f*) itself (bitwise the same sums everywhere, so no exchange);
//   * the M samples are dealt out round-robin and exchanged once;
//   * the bisection takes d steps per exchange.  The midpoints that d
//     successive steps can visit form a binary tree; node n's interval follows
//     from the round's bracket alone (left child: the upper end becomes the
//     parent's midpoint, right child: the lower end), and each midpoint is
//     formed from its own interval ends exactly as the sequential step forms
//     it.  Workgroup w takes the sign of V' at node w + 1; after the exchange
//     every workgroup walks the tree along the signs, which moves the bracket
//     exactly as d sequential steps would.
//
// Rings too large for the registers (sides from 1023 on) are streamed: each
// workgroup expands the whole ring once into its own region of the record
// scratch and reads it back at every evaluation, so no record written by one
// CU has to be seen by another.
//
// Every evaluation is the same group sum over the same records as in the
// one-workgroup kernel (sweep_blocks_kernel with LAZY), and the decisions are
// taken in the same order on the same values, so a block's c is bitwise that
// kernel's.  Only the arg min of Algorithm 3 (Section 2.2) is being computed.
//
// Exchange.  Lane 0 of a workgroup publishes a value as 64-bit words whose
// upper half is a tag (a double as two words, one per half, a sign as one
// word); words are written and read whole with relaxed agent-scope atomics,
// so a tag and its payload always arrive together and no fence is needed.
// Wave 0 of every workgroup polls the words it needs (each lane all of its
// words at once) until they carry the launch's tag, then hands the values to
// the other waves through LDS.  The tag is a per-context launch counter
// passed by the host, so words left by earlier launches never match.  A wait
// is bounded; a value whose word has not arrived by then (a workgroup of the
// launch not yet resident, say) is computed by the waiting workgroup itself,
// with the same records and the same group sum, so the results never depend
// on residency or timing, only the speed does.
#include "mgc_internal.h"
#include "mgc_sweep.h"

namespace mgc {

namespace {

constexpr int SPLIT_MAX_SAMPLES = 256;   // the largest M the parameters allow
constexpr double SPLIT_STREAM_BYTES = 128.0 * 1024 * 1024;

__device__ __forceinline__ unsigned long long xload(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void xstore(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long tagged(unsigned tag, unsigned payload)
{
    return ((unsigned long long)tag << 32) | payload;
}

// Wave 0 (lanes 0..63): wait until words [0, n) of `base` carry `tag` (n <= 512; lane t
// owns words t, t + 64, ...), polling all of a lane's words at once, at most `polls` times.
// payload[k] receives word k's low half and ok[k] whether it arrived within the wait.
__device__ __forceinline__ void gather_words(const unsigned long long* base, int n, unsigned tag, int polls,
                                             unsigned* payload, unsigned char* ok)
{
    constexpr int PER = 8;
    const int lane = threadIdx.x;
    unsigned need = 0, done = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if (lane + 64 * k < n) need |= 1u << k;
    for (int it = 0; it < polls && done != need; ++it) {
        unsigned long long v[PER];
        const unsigned open = need & ~done;
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if ((open >> k) & 1u) v[k] = xload(base + lane + 64 * k);
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (((open >> k) & 1u) && (unsigned)(v[k] >> 32) == tag) {
                payload[lane + 64 * k] = (unsigned)v[k];
                done |= 1u << k;
            }
        if (done != need) __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k)
        if ((need >> k) & 1u) ok[lane + 64 * k] = (unsigned char)((done >> k) & 1u);
}

}  // namespace

template <typename T, int KIND, int GROUP, int RPL>
__global__ __launch_bounds__(GROUP) void sweep_split_kernel(T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                                            int b, int pr, int pc, int nbc, double alpha, int M, int G,
                                                            CoarseArgs ca, SplitArgs sa)
{
    static_assert(GROUP % 64 == 0, "whole wavefronts");
    __shared__ double lds[2 * (GROUP / 64) * BlockSum<GROUP>::NMAX];
    __shared__ unsigned xpay[2 * SPLIT_MAX_SAMPLES];
    __shared__ unsigned char xok[2 * SPLIT_MAX_SAMPLES];
    __shared__ double ksamp[SPLIT_MAX_SAMPLES];
    __shared__ int xall;

    const int P = sa.P, d = sa.d;
    const unsigned tag = sa.tag;
    const int blk = (int)blockIdx.x / P, w = (int)blockIdx.x - blk * P;
    const int bi = blk / nbc, bj = blk - bi * nbc;
    const int p = 2 * bi + pr, q = 2 * bj + pc;
    const int r0 = p * b, c0 = q * b;
    const int r1 = min(r0 + b, H), c1 = min(c0 + b, W);
    const int lane = threadIdx.x;
    unsigned long long* slots = sa.slots + (size_t)blk * sa.stride;

    // the block's sum of f - u and its ring, as the one-workgroup kernel takes them
    double rsum = 0.0;
    const double* part = ca.partials + ((size_t)p * ca.nj + q) * ca.nchunk;
    for (int k = lane; k < ca.nchunk; k += GROUP) rsum += part[k];
    const double s = (double)(r1 - r0) * (double)(c1 - c0);
    const int pq = p * ca.nj + q;
    const RingBand band = ring_band(H, W, r0, r1, c0, c1);
    const int ncand = band.n;
    // the ring: RPL records per lane in registers, or (RPL = 0, rings larger than the registers
    // hold) expanded once into this workgroup's own region of the record scratch and read back
    // by the lane that wrote them, in the order of the one-workgroup kernel's streamed form
    PolyRing<KIND> rg[RPL > 0 ? RPL : 1];
    double* rec = nullptr;
    if constexpr (RPL > 0) {
        ring_to_regs<T, KIND, GROUP, RPL, true>(u, H, W, band, lane, ca.cpend, ca.nj, pq, rg);
    } else {
        rec = ca.rec + (size_t)blockIdx.x * PolyRing<KIND>::NCOEF * ca.rec_stride;
        ring_to_region<T, KIND, GROUP, true>(u, H, W, band, lane, ca.cpend, ca.nj, pq, rec, ca.rec_stride);
    }
    BlockSum<GROUP> gs{lds, 0};
    const double fs = gs(rsum) / s;
    auto Kpart = [&](const auto& cs, auto& out) {
        constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
        for (int k = 0; k < N; ++k) out[k] = 0.0;
        if constexpr (RPL > 0) {
#pragma unroll
            for (int t = 0; t < RPL; ++t)
                if (lane + t * GROUP < ncand) {
#pragma unroll
                    for (int k = 0; k < N; ++k) out[k] += abs_poly<KIND>(rg[t], cs[k]);
                }
        } else {
            for_region_records<KIND, GROUP>(rec, ca.rec_stride, ncand, lane, [&](const PolyRing<KIND>& pr) {
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] += abs_poly<KIND>(pr, cs[k]);
            });
        }
    };
    auto Dpart = [&](double c) {
        double acc = 0.0;
        if constexpr (RPL > 0) {
#pragma unroll
            for (int t = 0; t < RPL; ++t)
                if (lane + t * GROUP < ncand) acc += dabs_poly<KIND>(rg[t], c);
        } else {
            for_region_records<KIND, GROUP>(rec, ca.rec_stride, ncand, lane,
                                            [&](const PolyRing<KIND>& pr) { acc += dabs_poly<KIND>(pr, c); });
        }
        return acc;
    };
    auto Ksum = [&](double c) {
        const double cs1[1] = {c};
        double k1[1];
        Kpart(cs1, k1);
        gs.template sum_n<1>(k1);
        return k1[0];
    };
    const double as = alpha * s;

    // local_solve's steps, in its order and arithmetic
    double k2[2];
    {
        const double c2[2] = {0.0, fs};
        Kpart(c2, k2);
        gs.template sum_n<2>(k2);
    }
    const double K0 = k2[0];
    const double Kf = k2[1];
    const double rho = sqrt(2.0 * Kf / as);
    const double V0 = K0 + 0.5 * as * fs * fs;
    const double eta = 1e-12 * (1.0 + V0);
    double ct, Kt;
    if (rho == 0.0) {   // the same on every workgroup: nothing to exchange
        if (w != 0) return;
        ct = fs;
        Kt = Kf;
    } else {
        // the sample offsets (2i - M) / M: for M a power of two the product with the exact
        // 1/M, otherwise the quotient, as the one-workgroup kernel forms them
        const bool p2 = (M & (M - 1)) == 0;
        const double invm = 1.0 / (double)M;
        auto frac = [&](int i) {
            const double n = (double)(2 * i - M);
            return p2 ? n * invm : n / (double)M;
        };
        auto sample_index = [&](int t) { return t < M / 2 ? t : t + 1; };   // i = M/2 is f*
        for (int t = w; t < M; t += P) {
            const double kv = Ksum(fs + rho * frac(sample_index(t)));
            if (lane == 0) {
                const unsigned long long bits = (unsigned long long)__double_as_longlong(kv);
                xstore(slots + 2 * t, tagged(tag, (unsigned)(bits >> 32)));
                xstore(slots + 2 * t + 1, tagged(tag, (unsigned)bits));
            }
        }
        if (lane < 64) {
            gather_words(slots, 2 * M, tag, sa.polls, xpay, xok);
            bool all = true;
            for (int t = lane; t < M; t += 64) {
                ksamp[t] = __longlong_as_double((long long)(((unsigned long long)xpay[2 * t] << 32) | xpay[2 * t + 1]));
                all = all && xok[2 * t] && xok[2 * t + 1];
            }
            all = __all(all);
            if (lane == 0) xall = all;
        }
        __syncthreads();
        if (!xall) {   // samples whose words did not arrive in time are evaluated here
            for (int t = 0; t < M; ++t) {
                const bool got = xok[2 * t] && xok[2 * t + 1];
                __syncthreads();
                if (!got) {
                    const double kv = Ksum(fs + rho * frac(sample_index(t)));
                    if (lane == 0) ksamp[t] = kv;
                }
            }
            __syncthreads();
        }
        // scan in increasing i, f* (i = M/2) in its place; ties keep the first index
        double vbest = 0.0, kbest = 0.0;
        int istar = -1;
        auto consider = [&](int i, double ci, double ki) {
            const double vi = ki + 0.5 * as * (ci - fs) * (ci - fs);
            if (istar < 0 || vi < vbest) { vbest = vi; kbest = ki; istar = i; }
        };
        for (int t = 0; t < M; ++t) {
            const int i = sample_index(t);
            if (i == M / 2 + 1) consider(M / 2, fs, Kf);
            consider(i, fs + rho * frac(i), ksamp[t]);
        }
        __syncthreads();   // xpay and xok are reused by the bisection rounds
        const double cbest = fs + rho * frac(istar);
        const int ilo = istar > 0 ? istar - 1 : 0;
        const int ihi = istar < M ? istar + 1 : M;
        double lo = fs + rho * frac(ilo);
        double hi = fs + rho * frac(ihi);
        auto sign_at = [&](double mid) { return gs(Dpart(mid)) + as * (mid - fs) > 0.0; };
        unsigned long long* rs = slots + 2 * M;
        for (int g0 = 0; g0 < G; g0 += d, rs += P) {
            const int dd = min(d, G - g0);
            const int nn = (1 << dd) - 1;
            if (w < nn) {
                const bool sg = sign_at(tree_node_mid(w + 1, lo, hi));
                if (lane == 0) xstore(rs + w, tagged(tag, sg ? 1u : 0u));
            }
            if (lane < 64) gather_words(rs, nn, tag, sa.polls, xpay, xok);
            __syncthreads();
            tree_walk(dd, lo, hi, [&](int node, double mid) {
                return xok[node - 1] ? xpay[node - 1] != 0u : sign_at(mid);
            });
            __syncthreads();   // every wave has read this round's words before the next round's
        }
        if (w != 0) return;
        const double cbis = 0.5 * (lo + hi);
        const double kbis = Ksum(cbis);
        const double vbis = kbis + 0.5 * as * (cbis - fs) * (cbis - fs);
        if (vbest < vbis - eta) { ct = cbest; Kt = kbest; }
        else { ct = cbis; Kt = kbis; }
    }
    if (lane == 0) {
        const double delta = (Kt - K0) + 0.5 * as * ct * (ct - 2.0 * fs);
        ca.cpend[(size_t)p * ca.nj + q] = delta < -eta ? ct : 0.0;
    }
}

namespace {

template <typename T, int KIND, int GROUP, int RPL>
hipError_t launch_split_cfg(const LaunchCtx& L, void* u, const void* f, int b, int pr, int pc, int nbr, int nbc,
                            const CoarseArgs& ca, const SplitArgs& sa)
{
    hipLaunchKernelGGL((sweep_split_kernel<T, KIND, GROUP, RPL>), dim3((unsigned)(nbr * nbc * sa.P)), dim3(GROUP), 0,
                       L.stream, (T*)u, (const T*)f, L.H, L.W, b, pr, pc, nbc, L.alpha, L.M, L.G, ca, sa);
    return hipGetLastError();
}

template <typename T, int KIND>
hipError_t launch_split_t(const LaunchCtx& L, void* u, const void* f, int b, int pr, int pc, int nbr, int nbc,
                          const CoarseArgs& ca, const SplitArgs& sa)
{
    // the lane shapes of the one-workgroup kernel at these sides (the records per lane
    // decide the summation order, so they must match for bitwise equal results)
    switch (shape_side(b)) {
    case 256: return launch_split_cfg<T, KIND, 512, 4>(L, u, f, b, pr, pc, nbr, nbc, ca, sa);
    case 512: return launch_split_cfg<T, KIND, 512, 8>(L, u, f, b, pr, pc, nbr, nbc, ca, sa);
    default:   // streamed sides; the caller has checked that ca.rec holds a region per workgroup
        if (shape_side(b) < STREAMED_B || !ca.rec) return hipErrorInvalidValue;
        return launch_split_cfg<T, KIND, 1024, 0>(L, u, f, b, pr, pc, nbr, nbc, ca, sa);
    }
}

}  // namespace

int split_depth(int nblocks, int cus, int G, int b)
{
    const int s = shape_side(b);
    if (s < 256 || nblocks <= 0 || G <= 0) return 0;   // smaller rings: cheaper kept on one CU
    const bool streamed = s >= STREAMED_B;
    // streamed rings: every workgroup keeps its own copy of the block's records (7 doubles per
    // ring pixel) and streams it at each evaluation; the copies of one launch stay within
    // SPLIT_STREAM_BYTES and at most 63 workgroups share a block, beyond which the copies'
    // traffic costs more than the exchanges saved (measured at 2048^2 to 8192^2)
    const double copy = 7.0 * 8.0 * 8.0 * (double)b;
    const int dmax = streamed ? 6 : 8;
    int d = 0;
    while (d < dmax && d < G) {
        const size_t wg = (size_t)nblocks * ((2u << d) - 1u);
        if (wg > (size_t)cus || (streamed && (double)wg * copy > SPLIT_STREAM_BYTES)) break;
        ++d;
    }
    // a register-resident ring evaluates in about a microsecond, an exchange costs 1-3: the split
    // pays from 4 steps per exchange on; a streamed evaluation takes several microseconds
    return d >= (streamed ? 2 : 4) ? d : 0;
}

size_t split_record_doubles(int nblocks, int cus, int G, int b)
{
    const int d = shape_side(b) >= STREAMED_B ? split_depth(nblocks, cus, G, b) : 0;
    return d > 0 ? (size_t)nblocks * ((1u << d) - 1u) * 7 * (size_t)(8 * b) : 0;
}

size_t split_slot_words(int M, int G, int d) { return d > 0 ? 2 * (size_t)M + (size_t)((G + d - 1) / d) * ((1u << d) - 1u) : 0; }

hipError_t launch_sweep_split(const LaunchCtx& L, void* u, const void* f, int b, int pr, int pc, int nbr, int nbc,
                              const CoarseArgs& ca, const SplitArgs& sa)
{
    if (L.f64) return L.kind ? launch_split_t<double, 1>(L, u, f, b, pr, pc, nbr, nbc, ca, sa)
                             : launch_split_t<double, 0>(L, u, f, b, pr, pc, nbr, nbc, ca, sa);
    return L.kind ? launch_split_t<float, 1>(L, u, f, b, pr, pc, nbr, nbc, ca, sa)
                  : launch_split_t<float, 0>(L, u, f, b, pr, pc, nbr, nbc, ca, sa);
}

}  // namespace mgc
