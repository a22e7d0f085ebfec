// Branch-and-bound driver (Algorithm 1, Section 6) for one or many pose
// problems, with device-resident queues and device-side control, so that a
// whole iteration is a fixed sequence of kernel launches (captured once in a
// HIP graph and replayed).
//
// Queue of each problem: a small "hot" part holding every queued cube whose
// priority key is below a threshold theta, and a large append-only "cold"
// part holding the rest.  Each iteration only the hot part is scanned:
//   select   3 radix passes (11 + 11 + 10 bits) over the ordered 32-bit key of
//            the priority find the k-th lowest key; compaction moves the k
//            lowest into the parent list and keeps the rest (cubes whose lower
//            bound is no longer below d* are dropped)
//   branch   8 children per parent, split in rotation or translation by the
//            flag the bound kernel computed for the parent (Section 5.1); a
//            rotation split shares one translation cell among its 8 children
//   bound    S11 per translation cell, S12 and both bounds per child; the
//            upper bounds update d* with an atomic minimum (bound.hip)
//   push     children whose lower bound (raised to the parent's, minus the
//            rounding margin) is below d* are queued: hot if their key is
//            below theta, cold otherwise; the child holding d* records the pose
//   control  stop test d* - (lowest lower bound in the queue) <= eps, caps,
//            and the decision to re-partition: when the hot part runs low or
//            fills up, the next iteration first redistributes hot and cold
//            around a new theta (one pass over the whole queue).
// With the best-first order (priority = lower bound) every hot cube has a
// lower key than every cold cube, so the k cubes taken are the k lowest of
// the whole queue, as in Algorithm 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "cube_core.h"
#include "gosma_impl.h"
#include "sma_core.h"

namespace gosma {

namespace {

constexpr int kHistBins = 4096;
constexpr int kBlock = 256;
constexpr int kGridX = 2048;            // blocks per grid-stride kernel (divided among problems)
constexpr int kMaxLevel = 19;
constexpr uint32_t kNoChildren = 0xffffffffu;   // pchild of a parent that cannot be split
// Rounding margin of the FP32 bounds, relative to the magnitude S11 + 2 S12 of
// each bound: over 3x the largest relative error measured against the FP64
// oracle on every parity set (1.2e-6).
constexpr double kMarginGamma = 4e-6;

enum Done : uint32_t { RUNNING = 0, EPS_OPTIMAL = 1, EXHAUSTED = 2, CAPPED = 3, OVERFLOW = 4 };

struct PState {
    unsigned long long dstar;      // ordered bits of d*, the best upper bound
    unsigned long long minH;       // ordered bits: lowest lower bound in the hot part
    unsigned long long minC;       // ordered bits: lowest lower bound in the cold part
    unsigned long long floor_lb;   // ordered bits: lowest bound of cubes that cannot be split
    unsigned long long best_rkey, best_tkey;
    unsigned long long bounded;    // cubes bounded
    double eps_f;                  // eps * S22
    uint32_t nH[2], nC[2];
    uint32_t hcur, ccur;
    uint32_t theta;                // hot iff key32(priority) < theta (0xffffffff: all hot)
    uint32_t nsel, rebuild, done, overflow, iters, max_iters;
    uint32_t nskip;                // selected cubes that cannot be split (no children)
    uint32_t take_all, prefix, need, eq_quota, eq_taken;   // radix select
    // a range holding the keys of each hot buffer (indexed like nH; empty: kmin > kmax)
    uint32_t kmin[2], kmax[2];
    uint32_t tshift;               // the selection compares (key - kmin) >> tshift with prefix
    uint32_t rb_target;            // hot entries wanted after a re-partition
    // SMA (Section 6): the pose of d* when SMA set it, and the d* it last started from
    double pose[6];
    unsigned long long sma_from;   // ordered bits of d* at the last SMA start
    uint32_t pose_sma;             // 1: d* was found by SMA at `pose` (else: the centre of the best keys)
    uint32_t sma_runs, sma_gain, pad_sma;
};

struct GState {
    uint32_t nchild, running;
    uint32_t ntrec;    // translation records reserved by this iteration's new cells
    uint32_t nrows;    // learned order: children queued this iteration (rows of the network input)
    // per size bucket: children and distinct translation cells of the iteration
    uint32_t nchild_b[kBuckets], ntcell_b[kBuckets];
};

struct Queue {
    uint64_t *rkey, *tkey;
    double *lb;
    float *prio;
    uint8_t *flags;
    float *ubn, *t8;   // record logging only: normalised upper bound and top-8 pair terms
};

__device__ __forceinline__ unsigned long long ord64(double x)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __host__ __forceinline__ double unord64(unsigned long long u)
{
    unsigned long long v = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    double d;
    memcpy(&d, &v, sizeof d);
    return d;
}
__device__ __forceinline__ uint32_t key32(float x)
{
    uint32_t u = __float_as_uint(x);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}
// A NaN bound is never pruned: it orders like -inf.
__device__ __forceinline__ double sane_lb(double x) { return x != x ? -INFINITY : x; }

// Block-aggregated reservation of cnt consecutive slots per thread: an
// inclusive scan within each wave (shuffles), wave totals combined in LDS, one
// atomic per block.
__device__ __forceinline__ uint32_t block_reserve(uint32_t *counter, uint32_t cnt, uint32_t *block_total = nullptr)
{
    __shared__ uint32_t wtot[kBlock / 64];
    __shared__ uint32_t base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            const uint32_t c = wtot[w];
            wtot[w] = s;
            s += c;
        }
        base = s ? atomicAdd(counter, s) : 0u;
        if (block_total && s) atomicAdd(block_total, s);
    }
    __syncthreads();
    const uint32_t r = base + wtot[wave] + incl - cnt;
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_min(double v)
{
    __shared__ double w[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = w[0];
    for (int k = 1; k < kBlock / 64; ++k) m = fmin(m, w[k]);
    __syncthreads();
    return m;
}

// Block-wide lowest and highest key (every thread gets them).
__device__ __forceinline__ void block_key_range(uint32_t &lo, uint32_t &hi)
{
    __shared__ uint32_t wl[kBlock / 64], wh[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor(lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        wl[threadIdx.x >> 6] = lo;
        wh[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    lo = wl[0];
    hi = wh[0];
    for (int k = 1; k < kBlock / 64; ++k) {
        lo = min(lo, wl[k]);
        hi = max(hi, wh[k]);
    }
    __syncthreads();
}

// Widen the key range of hot buffer `buf` to [lo, hi] (nothing when lo > hi).
// The atomics are skipped when the range already covers the keys, as it
// does for most callers once a few have widened it.
__device__ __forceinline__ void widen_key_range(PState &s, uint32_t buf, uint32_t lo, uint32_t hi)
{
    if (lo > hi) return;
    if (lo < __atomic_load_n(&s.kmin[buf], __ATOMIC_RELAXED)) atomicMin(&s.kmin[buf], lo);
    if (hi > __atomic_load_n(&s.kmax[buf], __ATOMIC_RELAXED)) atomicMax(&s.kmax[buf], hi);
}

// Key range of the next hot buffer at the start of an iteration: the cubes
// that stay hot keep their keys, which lie in the current buffer's range;
// children's keys are at least their parent's (their bound is at least the
// parent's); and no hot key exceeds theta (keys below it go hot, and a
// re-partition's ties equal it).  So the pushes widen the range only for
// priorities that do not follow the bound, or while theta is open.
__device__ __forceinline__ void start_key_range(PState &s)
{
    s.kmin[s.hcur ^ 1] = s.kmin[s.hcur];
    s.kmax[s.hcur ^ 1] = s.theta != 0xffffffffu ? s.theta : s.kmax[s.hcur];
}

__device__ __forceinline__ int key_level(uint64_t k) { return (int)((k >> 57) & 63); }
__device__ __forceinline__ uint64_t child_key(uint64_t k, int c)
{
    const uint64_t m = (1ull << 19) - 1;
    uint64_t L = (uint64_t)key_level(k) + 1;
    uint64_t ix = 2 * ((k >> 38) & m) + ((c >> 2) & 1);
    uint64_t iy = 2 * ((k >> 19) & m) + ((c >> 1) & 1);
    uint64_t iz = 2 * (k & m) + (c & 1);
    return (L << 57) | (ix << 38) | (iy << 19) | iz;
}

// Buffers of all problems: queue part b of problem p occupies
// [p * cap, (p + 1) * cap) of array b.
struct Bufs {
    Queue H[2], C[2];
    uint32_t hcap, ccap;
    Queue par;                    // parents, problem p at [p * k, (p + 1) * k)
    uint32_t k;
    // children: size bucket b owns indices [kbase[b], kbase[b] + kcap[b]) and
    // fills them from the start (g->nchild_b[b]); its distinct translation
    // cells use the same range of the cell list
    uint32_t kbase[kBuckets], kcap[kBuckets];
    uint64_t *crk, *ctk;
    uint32_t *cpid, *cpar;        // problem and parent slot of each child
    int64_t *ctidx;
    // translation cells of the iteration's children: a hash table of
    // 2^tbits slots per problem (key or kEmptyCell), one slot per distinct
    // cell, so parents that share a translation cell share its S11 sums
    uint64_t *tcells;
    uint32_t *tpid;               // problem of each slot (fixed)
    uint32_t tbits;
    // the distinct cells of the iteration, per bucket from kbase[b]
    // (g->ntcell_b[b] of them): key, problem and table slot (where their S11
    // sums are stored)
    uint64_t *ckey;
    uint32_t *cpid2;
    int64_t *cslot;
    double *cub, *clb, *clbs;
    uint8_t *cflags;
    double *s11ub, *s11lo;
    CubeSetup *csetup;            // per-child set-up of the pair kernel
    // translation records of the iteration's cells for the pair kernel (M
    // per cell, reserved by the claiming thread; kNoTRec when the capacity is
    // used up) and each cell's offset and sums, indexed by table slot
    TransRec *trec;
    uint32_t *toff;
    CellSums *csum;
    uint32_t tcap;
    uint32_t *hist;               // kHistBins per problem
    PState *st;
    GState *g;
    // learned order / record logging
    float *ctop8;                 // children: 8 largest S12 pair terms
    float *cfeat, *cpred, *cprio; // network rows: features, output; children: priority
    uint32_t *crow;               // network row -> child
    uint32_t *pchild;             // first child of each parent slot
    const ProbDesc *prob;
    float *rec;                   // record sink
    unsigned long long *rec_count;
    uint64_t rec_cap;
};

// The t-th child of the iteration (t < g->nchild), bucket after bucket, from
// the per-bucket counts n[] read once by the caller.
__device__ __forceinline__ uint32_t child_at(const Bufs &b, const uint32_t (&n)[kBuckets], uint32_t t)
{
#pragma unroll
    for (int k = 0; k < kBuckets; ++k) {
        if (t < n[k]) return b.kbase[k] + t;
        t -= n[k];
    }
    return 0u;   // not reached for t < g->nchild
}
__device__ __forceinline__ void child_counts(const Bufs &b, uint32_t (&n)[kBuckets])
{
#pragma unroll
    for (int k = 0; k < kBuckets; ++k) n[k] = b.g->nchild_b[k];
}

__device__ __forceinline__ Queue qoff(Queue q, size_t off)
{
    return Queue{q.rkey + off, q.tkey + off, q.lb + off, q.prio + off, q.flags + off,
                 q.ubn ? q.ubn + off : nullptr, q.t8 ? q.t8 + 8 * off : nullptr};
}
__device__ __forceinline__ void copy_payload(const Queue &dst, uint32_t d, const Queue &src, uint32_t i)
{
    if (dst.ubn) {
        dst.ubn[d] = src.ubn[i];
        for (int k = 0; k < 8; ++k) dst.t8[8 * d + k] = src.t8[8 * i + k];
    }
}

// Tiled two-way partition of the index range [0, n): classify(i) returns 0
// (drop), 1 (output A) or 2 (output B); writeA(i, slot) / writeB(i, slot)
// store the element.  Each block handles tiles of kBlock * kPer elements with
// one atomic per output per tile; element e of a tile is i = base + e * kBlock
// + thread, so reads and writes stay coalesced.  All threads must call it.
constexpr int kPer = 4;

template <class Classify, class WriteA, class WriteB>
__device__ __forceinline__ void partition_tiles(uint32_t n, uint32_t *cntA, uint32_t *cntB, Classify classify,
                                                WriteA writeA, WriteB writeB)
{
    __shared__ uint32_t wa[kBlock / 64], wb[kBlock / 64], tileA, tileB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t base = blockIdx.x * kBlock * kPer; base < n; base += gridDim.x * kBlock * kPer) {
        uint32_t ma = 0, mb = 0;
        for (int e = 0; e < kPer; ++e) {
            const uint32_t i = base + e * kBlock + threadIdx.x;
            const int c = i < n ? classify(i) : 0;
            if (c == 1) ma |= 1u << e;
            if (c == 2) mb |= 1u << e;
        }
        // tile totals -> one atomic per output
        uint32_t ca = (uint32_t)__popc(ma), cb = (uint32_t)__popc(mb);
        for (int off = 32; off > 0; off >>= 1) {
            ca += __shfl_xor(ca, off, 64);
            cb += __shfl_xor(cb, off, 64);
        }
        if (lane == 0) {
            wa[wave] = ca;
            wb[wave] = cb;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t ta = 0, tb = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                ta += wa[w];
                tb += wb[w];
            }
            tileA = ta ? atomicAdd(cntA, ta) : 0u;
            tileB = tb ? atomicAdd(cntB, tb) : 0u;
        }
        __syncthreads();
        uint32_t ra = tileA, rb = tileB;
        for (int e = 0; e < kPer; ++e) {
            const bool fa = (ma >> e) & 1u, fb = (mb >> e) & 1u;
            const unsigned long long ba = __ballot(fa), bb = __ballot(fb);
            if (lane == 0) {
                wa[wave] = (uint32_t)__popcll(ba);
                wb[wave] = (uint32_t)__popcll(bb);
            }
            __syncthreads();
            uint32_t pa = ra, pb = rb, sa = 0, sb = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                if (w < wave) {
                    pa += wa[w];
                    pb += wb[w];
                }
                sa += wa[w];
                sb += wb[w];
            }
            const uint32_t i = base + e * kBlock + threadIdx.x;
            const unsigned long long lt = (1ull << lane) - 1ull;
            if (fa) writeA(i, pa + (uint32_t)__popcll(ba & lt));
            if (fb) writeB(i, pb + (uint32_t)__popcll(bb & lt));
            ra += sa;
            rb += sb;
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------

// rb_slot: this iteration runs the re-partition kernels (the problems that
// asked for one re-partition now).
__global__ __launch_bounds__(kBlock) void k_iter_begin(Bufs b, int P, int rb_slot)
{
    const int p = blockIdx.x;
    PState &s = b.st[p];
    if (p == 0 && threadIdx.x == 0) {
        b.g->nchild = 0;
        b.g->running = 0;
        b.g->ntrec = 0;
        b.g->nrows = 0;
        for (int k = 0; k < kBuckets; ++k) b.g->nchild_b[k] = b.g->ntcell_b[k] = 0;
    }
    if (s.done) {              // finished problems keep their final state
        if (threadIdx.x == 0) s.nsel = 0;
        return;
    }
    uint32_t *h = b.hist + (size_t)p * kHistBins;
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) h[i] = 0;
    if (threadIdx.x == 0) {
        s.nsel = 0;
        s.nskip = 0;
        s.take_all = 0;
        s.prefix = 0;
        s.need = 0;
        s.eq_quota = 0;
        s.eq_taken = 0;
        s.tshift = 0;
        s.nH[s.hcur ^ 1] = 0;
        start_key_range(s);
        s.minH = ord64(INFINITY);
        if (rb_slot && s.rebuild) {
            s.nC[s.ccur ^ 1] = 0;
            s.minC = ord64(INFINITY);
        }
    }
}

// Radix select over the ordered 32-bit key of the priority: the k-th lowest
// key is found exactly, and cubes whose key equals it are taken in arbitrary
// order up to the quota.  (Stopping at a coarser bucket is not enough:
// children inherit their parent's lower bound, so a bucket that straddles
// d* - eps keeps refilling itself with cubes that best-first order would
// never split.)  A re-partition (hot and cold parts) takes three passes over
// the whole key, of 11, 11 and 10 bits.
constexpr int kRadixPasses = 3;
constexpr uint32_t kHistPer = 16;   // keys per thread of a histogram pass (at least)

// The selection takes two passes of 12 bits over the hot part, on the key's
// offset from kmin.  The keys lie in [kmin, kmax]: a re-partition sets the
// range from its histogram and threshold, each iteration starts the next
// buffer's range from the current one, and pushes widen it where needed.  So
// the offsets have D = bit length of kmax - kmin bits, and the passes resolve
// offset bits D-1 .. D-24: every bit when kmax - kmin < 2^24 (priorities of
// one sign within a factor of four of each other); otherwise the lowest
// D - 24 bits are left out, and keys whose offsets agree above them (values
// at most 2^(D-24) - 1 units in the last place apart) rank as ties of the
// threshold.
constexpr int kSelPasses = 2;
constexpr int kSelBits = 12;
struct SelDigits {
    int s0, s1;   // lowest offset bit of the first and of the second digit
};
__device__ __forceinline__ SelDigits sel_digits(const PState &s)
{
    const uint32_t lo = s.kmin[s.hcur], hi = s.kmax[s.hcur];
    const uint32_t w = hi >= lo ? hi - lo : 0xffffffffu;
    const int D = w ? 32 - __clz((int)w) : 0;
    const int s0 = max(D - kSelBits, 0);
    return {s0, max(s0 - kSelBits, 0)};
}

// One radix pass over a problem's hot part (selection) or hot + cold parts
// (re-partition): histogram of the next digit below the prefix fixed so far.
__global__ __launch_bounds__(kBlock) void k_hist(Bufs b, int rebuild_pass, int pass)
{
    __shared__ uint32_t h[kHistBins];
    const int p = blockIdx.y;
    const PState &s = b.st[p];
    if (s.done || s.take_all || (rebuild_pass && !s.rebuild)) return;
    const int nparts = rebuild_pass ? 2 : 1;
    // only as many blocks as give each thread about kHistPer keys take part:
    // every block pays for clearing and flushing its histogram
    const uint32_t total = s.nH[s.hcur] + (rebuild_pass ? s.nC[s.ccur] : 0u);
    const uint32_t nb = min(gridDim.x, max(1u, (total + kBlock * kHistPer - 1) / (kBlock * kHistPer)));
    if (blockIdx.x >= nb) return;
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    // digit of this pass: ((key - kbase) >> shift) & mask; a key takes part in
    // a later pass when (((key - kbase) >> pshift) & pmask) equals the prefix
    int shift, pshift;
    uint32_t mask, pmask, kbase = 0u;
    if (rebuild_pass) {
        shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
        mask = pass == 2 ? 0x3ffu : 0x7ffu;
        pshift = pass == 1 ? 21 : 10;
        pmask = 0xffffffffu;
    } else {
        const SelDigits d = sel_digits(s);
        shift = pass == 0 ? d.s0 : d.s1;
        mask = pass == 0 ? (1u << kSelBits) - 1u : (1u << (d.s0 - d.s1)) - 1u;
        pshift = d.s0;
        pmask = (1u << kSelBits) - 1u;
        kbase = s.kmin[s.hcur];
    }
    const uint32_t prefix = s.prefix;
    const int lane = threadIdx.x & 63;
    for (int part = 0; part < nparts; ++part) {
        const Queue q = part == 0 ? qoff(b.H[s.hcur], (size_t)p * b.hcap) : qoff(b.C[s.ccur], (size_t)p * b.ccap);
        const uint32_t n = part == 0 ? s.nH[s.hcur] : s.nC[s.ccur];
        for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += nb * blockDim.x) {
            const uint32_t i = base + threadIdx.x;
            uint32_t bin = 0;
            bool m = false;
            if (i < n) {
                const uint32_t key = key32(q.prio[i]) - kbase;
                m = pass == 0 || ((key >> pshift) & pmask) == prefix;
                bin = (key >> shift) & mask;
            }
            // keys cluster: when every counted lane of the wave hits one bin,
            // add the count once instead of serialising 64 LDS atomics
            const unsigned long long all = __ballot(m);
            if (!all) continue;
            const int leader = __ffsll((long long)all) - 1;
            const uint32_t lb = __shfl(bin, leader, 64);
            if (__ballot(m && bin == lb) == all) {
                if (lane == leader) atomicAdd(&h[lb], (uint32_t)__popcll(all));
            } else if (m) {
                atomicAdd(&h[bin], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *gh = b.hist + (size_t)p * kHistBins;
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x)
        if (h[i]) atomicAdd(&gh[i], h[i]);
}

// Radix pass: the digit holding the need-th lowest key.  One block per problem.
__global__ __launch_bounds__(kBlock) void k_scan(Bufs b, int rebuild_pass, int pass)
{
    __shared__ uint32_t wtot[kBlock / 64];
    __shared__ uint32_t found, left;
    const int p = blockIdx.x;
    PState &s = b.st[p];
    if (s.done || s.take_all || (rebuild_pass && !s.rebuild)) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t want = rebuild_pass ? s.rb_target : b.k;
    const uint32_t total = rebuild_pass ? s.nH[s.hcur] + s.nC[s.ccur] : s.nH[s.hcur];
    const bool all_in = pass == 0 && total <= want;   // every key is taken
    const uint32_t need = pass == 0 ? want : s.need;
    constexpr int per = kHistBins / kBlock;
    uint32_t *gh = b.hist + (size_t)p * kHistBins;
    uint32_t loc[per], sum = 0;
    for (int j = 0; j < per; ++j) {
        loc[j] = gh[t * per + j];
        sum += loc[j];
    }
    if (rebuild_pass && pass == 0) {
        // key range of the new hot part: from the start of the lowest
        // non-empty bin of the first digit (key >> 21) to the threshold (set
        // by the last pass), or to the end of the highest non-empty bin when
        // every key goes hot; an empty histogram leaves an empty range
        uint32_t lo = 0xffffffffu, hi = 0u;
        for (int j = 0; j < per; ++j)
            if (loc[j]) {
                lo = min(lo, (uint32_t)(t * per + j));
                hi = max(hi, (uint32_t)(t * per + j));
            }
        block_key_range(lo, hi);
        if (t == 0) {
            s.kmin[s.hcur ^ 1] = lo << 21;
            if (all_in) s.kmax[s.hcur ^ 1] = (hi << 21) | 0x1fffffu;
        }
    }
    if (all_in) {
        __syncthreads();
        for (int j = 0; j < per; ++j) gh[t * per + j] = 0;   // the next select starts from zero
        if (t == 0) {
            s.take_all = 1;
            s.prefix = 0xffffffffu;
        }
        return;
    }
    // exclusive prefix of the per-thread sums: wave scan, then wave totals
    uint32_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wtot[wave] = incl;
    if (t == 0) {
        found = 0;
        left = need;
    }
    __syncthreads();
    uint32_t cum = incl - sum;
    for (int w = 0; w < wave; ++w) cum += wtot[w];
    for (int j = 0; j < per; ++j) {
        if (cum < need && need <= cum + loc[j]) {   // exactly one bin qualifies
            found = (uint32_t)(t * per + j);
            left = need - cum;
        }
        cum += loc[j];
    }
    __syncthreads();
    for (int j = 0; j < per; ++j) gh[t * per + j] = 0;
    if (t == 0) {
        if (rebuild_pass) {
            s.prefix = (pass == 0 ? 0u : s.prefix << (pass == 2 ? 10 : 11)) | found;
            if (pass == kRadixPasses - 1) s.kmax[s.hcur ^ 1] = s.prefix;
        } else if (pass == 0) {
            s.prefix = found;
        } else {
            // the threshold on (key - kmin) >> s1: both digits
            const SelDigits d = sel_digits(s);
            s.prefix = (s.prefix << (d.s0 - d.s1)) | found;
            s.tshift = (uint32_t)d.s1;
        }
        s.need = left;
        if (pass == (rebuild_pass ? kRadixPasses : kSelPasses) - 1) s.eq_quota = left;
    }
}

// Class of a queued cube in a selection or re-partition: 0 (no longer below
// d*, dropped), 1 (taken: key below the threshold T, or equal to it within
// the quota of equal keys) or 2 (kept).  Cubes whose key equals T are ranked
// with one atomic per wave (children inherit their parent's bound, so many
// keys can be equal); called by all active lanes of a wave together.
__device__ __forceinline__ int classify_key(PState &s, double lb, double dstar, uint32_t key, uint32_t T, bool all)
{
    const bool live = lb < dstar;
    const bool tie = live && !all && key == T;
    int c = !live ? 0 : ((all || key < T) ? 1 : 2);
    const unsigned long long tm = __ballot(tie);
    if (tm) {
        const int lane = threadIdx.x & 63, leader = __ffsll((long long)tm) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&s.eq_taken, (uint32_t)__popcll(tm));
        base = __shfl(base, leader, 64);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(tm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)tm, base));
        if (tie && rank < s.eq_quota) c = 1;
    }
    return c;
}

// Re-partition: hot + cold -> new hot (key below the threshold, ties up to the
// quota) and new cold, dropping cubes no longer below d*.
__global__ __launch_bounds__(kBlock) void k_rebuild_compact(Bufs b)
{
    const int p = blockIdx.y;
    PState &s = b.st[p];
    if (s.done || !s.rebuild) return;
    if ((uint32_t)blockIdx.x * kBlock * kPer >= max(s.nH[s.hcur], s.nC[s.ccur])) return;   // no tile for this block
    const double dstar = unord64(s.dstar);
    const uint32_t T = s.prefix;
    const bool all = s.take_all;
    const Queue Hout = qoff(b.H[s.hcur ^ 1], (size_t)p * b.hcap);
    const Queue Cout = qoff(b.C[s.ccur ^ 1], (size_t)p * b.ccap);
    const uint32_t hcap = b.hcap, ccap = b.ccap;
    double mh = INFINITY, mc = INFINITY;
    for (int part = 0; part < 2; ++part) {
        const Queue q = part == 0 ? qoff(b.H[s.hcur], (size_t)p * b.hcap) : qoff(b.C[s.ccur], (size_t)p * b.ccap);
        const uint32_t n = part == 0 ? s.nH[s.hcur] : s.nC[s.ccur];
        auto classify = [&](uint32_t i) -> int {
            return classify_key(s, sane_lb(q.lb[i]), dstar, key32(q.prio[i]), T, all);
        };
        auto move = [&](const Queue &o, uint32_t cap, uint32_t i, uint32_t slot, double &mn) {
            const double lb = sane_lb(q.lb[i]);
            mn = fmin(mn, lb);
            if (slot >= cap) {
                s.overflow = 1;
                return;
            }
            o.rkey[slot] = q.rkey[i];
            o.tkey[slot] = q.tkey[i];
            o.lb[slot] = lb;
            o.prio[slot] = q.prio[i];
            o.flags[slot] = q.flags[i];
            copy_payload(o, slot, q, i);
        };
        partition_tiles(n, &s.nH[s.hcur ^ 1], &s.nC[s.ccur ^ 1], classify,
                        [&](uint32_t i, uint32_t slot) { move(Hout, hcap, i, slot, mh); },
                        [&](uint32_t i, uint32_t slot) { move(Cout, ccap, i, slot, mc); });
    }
    mh = block_min(mh);
    mc = block_min(mc);
    if (threadIdx.x == 0) {
        if (mh < INFINITY) atomicMin(&s.minH, ord64(mh));
        if (mc < INFINITY) atomicMin(&s.minC, ord64(mc));
    }
}

// After a re-partition: switch both parts, set the new threshold, reset the
// radix state for the selection.
__global__ void k_rebuild_finish(Bufs b, int P)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    PState &s = b.st[p];
    if (s.done || !s.rebuild) return;
    if (s.overflow) {          // counts may exceed the capacity: stop before anything reads them
        s.done = OVERFLOW;
        return;
    }
    s.theta = s.take_all ? 0xffffffffu : s.prefix;   // hot iff the key is below the threshold
    s.minH = ord64(INFINITY);  // recomputed by the selection and the pushes
    s.hcur ^= 1;
    s.ccur ^= 1;
    s.rebuild = 0;
    s.take_all = 0;
    s.prefix = 0;
    s.need = 0;
    s.eq_quota = 0;
    s.eq_taken = 0;
    s.tshift = 0;
    s.nH[s.hcur ^ 1] = 0;
    s.nC[s.ccur ^ 1] = 0;
    start_key_range(s);
}

// Selection: the k lowest keys of the hot part -> parents; the rest stays hot.
__global__ __launch_bounds__(kBlock) void k_select_compact(Bufs b)
{
    const int p = blockIdx.y;
    PState &s = b.st[p];
    if (s.done) return;
    const double dstar = unord64(s.dstar);
    const uint32_t T = s.prefix;
    const bool all = s.take_all;
    if ((uint32_t)blockIdx.x * kBlock * kPer >= s.nH[s.hcur]) return;   // no tile for this block
    const Queue q = qoff(b.H[s.hcur], (size_t)p * b.hcap);
    const Queue Hout = qoff(b.H[s.hcur ^ 1], (size_t)p * b.hcap);
    const Queue par = qoff(b.par, (size_t)p * b.k);
    const uint32_t kb = s.kmin[s.hcur], ts = s.tshift;   // the threshold is on (key - kb) >> ts
    double mh = INFINITY;
    auto classify = [&](uint32_t i) -> int {
        return classify_key(s, sane_lb(q.lb[i]), dstar, (key32(q.prio[i]) - kb) >> ts, T, all);
    };
    partition_tiles(
        s.nH[s.hcur], &s.nsel, &s.nH[s.hcur ^ 1], classify,
        [&](uint32_t i, uint32_t slot) {
            if (slot >= b.k) {   // the threshold admits at most k keys; stop loudly if not
                s.overflow = 1;
                return;
            }
            par.rkey[slot] = q.rkey[i];
            par.tkey[slot] = q.tkey[i];
            par.lb[slot] = sane_lb(q.lb[i]);
            par.flags[slot] = q.flags[i];
            copy_payload(par, slot, q, i);
        },
        [&](uint32_t i, uint32_t slot) {
            const double lb = sane_lb(q.lb[i]);
            Hout.rkey[slot] = q.rkey[i];
            Hout.tkey[slot] = q.tkey[i];
            Hout.lb[slot] = lb;
            Hout.prio[slot] = q.prio[i];
            Hout.flags[slot] = q.flags[i];
            copy_payload(Hout, slot, q, i);
            mh = fmin(mh, lb);
        });
    mh = block_min(mh);
    if (threadIdx.x == 0 && mh < INFINITY) atomicMin(&s.minH, ord64(mh));
}

// Every slot of the cell table empty, and its problem index (once per solve).
__global__ void k_cells_init(Bufs b, int P)
{
    const size_t n = (size_t)P << b.tbits;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        b.tcells[i] = kEmptyCell;
        b.tpid[i] = (uint32_t)(i >> b.tbits);
    }
}

// Branching and the children's set-up in one pass, one thread per child:
// the eight consecutive threads of a parent split it (in rotation or
// translation by the flag its bound evaluation set, Section 5.1), the first
// of them reserves eight consecutive child slots (reservations aggregated
// per block), and each thread writes its child's keys, the GMM-vMF kernel's
// set-up record and the slot of its translation cell in the cell table (a
// rotation split shares its parent's cell among the eight children); the
// thread that claims a new cell lists it for the GMM-GMM kernel.  Children of
// all problems are appended to one list.  A parent at
// the finest level in both groups has no children (its lower bound stays in
// the queue minimum through floor_lb).
__global__ __launch_bounds__(kBlock) void k_branch_setup(Bufs b)
{
    const int p = blockIdx.y;
    PState &s = b.st[p];
    const uint32_t n = s.done ? 0u : min(s.nsel, b.k);   // more than k only on overflow
    const Queue par = qoff(b.par, (size_t)p * b.k);
    const int lane = threadIdx.x & 63;
    const int bk = b.prob[p].bucket;
    for (uint32_t base = blockIdx.x * blockDim.x; base < 8u * n; base += gridDim.x * blockDim.x) {
        const uint32_t t = base + threadIdx.x;
        const uint32_t i = t >> 3;
        const int c = (int)(t & 7u);
        const bool valid = t < 8u * n;
        bool rot = false, skip = false;
        uint64_t rk = 0, tk = 0;
        if (valid) {
            rk = par.rkey[i];
            tk = par.tkey[i];
            rot = (par.flags[i] & GOSMA_FLAG_SPLIT_ROT) != 0;
            const bool rmax = key_level(rk) >= kMaxLevel, tmax = key_level(tk) >= kMaxLevel;
            if (rot && rmax) rot = false;
            if (!rot && tmax) rot = !rmax;
            skip = rmax && tmax;
            if (skip && c == 0) {
                atomicMin(&s.floor_lb, ord64(par.lb[i]));
                atomicAdd(&s.nskip, 1u);
            }
        }
        // blockDim is a multiple of 8, so lanes 8q .. 8q + 7 hold one parent;
        // children go to the problem's size bucket
        uint32_t c0 = b.kbase[bk] + block_reserve(&b.g->nchild_b[bk], (valid && !skip && c == 0) ? 8u : 0u,
                                                   &b.g->nchild);
        c0 = __shfl(c0, lane & ~7, 64);
        if (valid && c == 0) b.pchild[(size_t)p * b.k + i] = skip ? kNoChildren : c0;
        bool claimed = false;
        int64_t at = 0;
        uint64_t ctk = 0;
        if (valid && !skip) {
            const uint32_t ci = c0 + (uint32_t)c;
            const uint64_t crk = rot ? child_key(rk, c) : rk;
            ctk = rot ? tk : child_key(tk, c);
            b.crk[ci] = crk;
            b.ctk[ci] = ctk;
            b.cpid[ci] = (uint32_t)p;
            b.cpar[ci] = (uint32_t)p * b.k + i;
            b.csetup[ci] = make_cube_setup(b.prob[p], crk, ctk);
            unsigned long long *tab = (unsigned long long *)(b.tcells + ((size_t)p << b.tbits));
            at = (int64_t)(((size_t)p << b.tbits) + cell_slot(tab, b.tbits, ctk, claimed));
            b.ctidx[ci] = at;
        }
        // the claiming threads list their cells (one atomic per wave)
        const unsigned long long m = __ballot(claimed);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t first = 0;
            if (lane == leader) first = b.kbase[bk] + atomicAdd(&b.g->ntcell_b[bk], (uint32_t)__popcll(m));
            first = __shfl(first, leader, 64);
            // and reserve the cells' translation records (M of them per cell)
            const uint32_t M = (uint32_t)b.prob[p].M;
            uint32_t r0 = 0;
            if (lane == leader) r0 = atomicAdd(&b.g->ntrec, M * (uint32_t)__popcll(m));
            r0 = __shfl(r0, leader, 64);
            if (claimed) {
                const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                const uint32_t j = first + rank;
                b.ckey[j] = ctk;
                b.cpid2[j] = (uint32_t)p;
                b.cslot[j] = at;
                const uint64_t roff = (uint64_t)r0 + (uint64_t)M * rank;
                b.toff[at] = roff + M <= (uint64_t)b.tcap ? (uint32_t)roff : kNoTRec;
            }
        }
    }
}

// Queue the children whose raised, margined lower bound is below d*.  Slots
// are reserved per wavefront and target (problem, hot or cold): one atomic
// per distinct target in the wave instead of one per child.
// The cell table is emptied here for the next iteration (its S11 sums have
// been read by the bound kernels).
__device__ __forceinline__ void clear_cells(const Bufs &b, int P)
{
    const size_t n = (size_t)P << b.tbits;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b.tcells[i] = kEmptyCell;
}

__global__ __launch_bounds__(kBlock) void k_push(Bufs b, const float *prio_override, int P)
{
    clear_cells(b, P);
    const uint32_t n = b.g->nchild;
    uint32_t nb[kBuckets];
    child_counts(b, nb);
    const int lane = threadIdx.x & 63;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t t = base + threadIdx.x;
        const uint32_t i = t < n ? child_at(b, nb, t) : 0u;
        bool push = false, hot = false;
        uint32_t p = 0;
        double lbs = 0.0;
        float pr = 0.0f;
        uint8_t fl = 0;
        if (t < n) {
            p = b.cpid[i];
            PState &s = b.st[p];
            fl = b.cflags[i];
            if (!(fl & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS))) {
                const unsigned long long draw = s.dstar;
                if (b.cub[i] < INFINITY && ord64(b.cub[i]) == draw) {
                    s.best_rkey = b.crk[i];
                    s.best_tkey = b.ctk[i];
                    s.pose_sma = 0;
                }
                lbs = fmax(sane_lb(b.clbs[i]), b.par.lb[b.cpar[i]]);
                if (lbs < unord64(draw)) {
                    push = true;
                    pr = prio_override ? prio_override[i] : (float)lbs;
                    hot = s.theta == 0xffffffffu || key32(pr) < s.theta;
                }
            }
        }
        // group the pushing lanes of this wave by target
        const uint32_t tgt = 2u * p + (hot ? 1u : 0u);
        unsigned long long todo = __ballot(push);
        uint32_t slot = 0;
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const uint32_t lt = __shfl(tgt, leader, 64);
            const unsigned long long grp = __ballot(push && tgt == lt) & todo;
            const uint32_t rank = (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
            const bool in = push && tgt == lt;
            double m = in ? lbs : INFINITY;
            uint32_t klo = in ? key32(pr) : 0xffffffffu, khi = in ? key32(pr) : 0u;
            for (int off = 32; off > 0; off >>= 1) {
                m = fmin(m, __shfl_xor(m, off, 64));
                klo = min(klo, (uint32_t)__shfl_xor(klo, off, 64));
                khi = max(khi, (uint32_t)__shfl_xor(khi, off, 64));
            }
            uint32_t first = 0;
            if (lane == leader) {
                PState &s = b.st[lt >> 1];
                const bool h = lt & 1u;
                uint32_t *cnt = h ? &s.nH[s.hcur ^ 1] : &s.nC[s.ccur];
                first = atomicAdd(cnt, (uint32_t)__popcll(grp));
                unsigned long long *mn = h ? &s.minH : &s.minC;
                const unsigned long long om = ord64(m);
                if (om < __atomic_load_n(mn, __ATOMIC_RELAXED)) atomicMin(mn, om);
                if (h) widen_key_range(s, s.hcur ^ 1, klo, khi);
            }
            first = __shfl(first, leader, 64);
            if (push && tgt == lt) slot = first + rank;
            todo &= ~grp;
        }
        if (!push) continue;
        PState &s = b.st[p];
        const Queue q = hot ? qoff(b.H[s.hcur ^ 1], (size_t)p * b.hcap) : qoff(b.C[s.ccur], (size_t)p * b.ccap);
        if (slot >= (hot ? b.hcap : b.ccap)) {
            s.overflow = 1;
            continue;
        }
        q.rkey[slot] = b.crk[i];
        q.tkey[slot] = b.ctk[i];
        q.lb[slot] = lbs;
        q.prio[slot] = pr;
        q.flags[slot] = fl & GOSMA_FLAG_SPLIT_ROT;
        if (q.ubn) {
            const double S22 = b.prob[p].S22;
            q.ubn[slot] = (float)fmin(fmax((b.cub[i] + S22) / S22, -10.0), 10.0);
            for (int k = 0; k < 8; ++k) q.t8[8 * slot + k] = b.ctop8[8 * (size_t)i + k];
        }
    }
}

// The same pushes with the slots reserved per block: each child takes its
// place among the block's children of the same target (problem, hot or cold)
// with an LDS atomic, and one global atomic per target and block reserves
// the block's run.  For up to kPushAggProblems problems.
constexpr int kPushAggProblems = 256;
__global__ __launch_bounds__(kBlock) void k_push_agg(Bufs b, const float *prio_override, int P)
{
    __shared__ uint32_t cnt[2 * kPushAggProblems], base[2 * kPushAggProblems];
    __shared__ unsigned long long mn[2 * kPushAggProblems];
    __shared__ uint32_t kmn[kPushAggProblems], kmx[kPushAggProblems];   // hot keys per problem
    clear_cells(b, P);
    const uint32_t n = b.g->nchild;
    uint32_t nb[kBuckets];
    child_counts(b, nb);
    const int T = 2 * P;
    for (uint32_t start = blockIdx.x * blockDim.x; start < n; start += gridDim.x * blockDim.x) {
        for (int t = threadIdx.x; t < T; t += blockDim.x) {
            cnt[t] = 0;
            mn[t] = ord64(INFINITY);
        }
        for (int t = threadIdx.x; t < P; t += blockDim.x) {
            kmn[t] = 0xffffffffu;
            kmx[t] = 0u;
        }
        __syncthreads();
        const uint32_t ti = start + threadIdx.x;
        const uint32_t i = ti < n ? child_at(b, nb, ti) : 0u;
        bool push = false, hot = false;
        uint32_t p = 0, local = 0;
        double lbs = 0.0;
        float pr = 0.0f;
        uint8_t fl = 0;
        if (ti < n) {
            p = b.cpid[i];
            PState &s = b.st[p];
            fl = b.cflags[i];
            if (!(fl & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS))) {
                const unsigned long long draw = s.dstar;
                if (b.cub[i] < INFINITY && ord64(b.cub[i]) == draw) {
                    s.best_rkey = b.crk[i];
                    s.best_tkey = b.ctk[i];
                    s.pose_sma = 0;
                }
                lbs = fmax(sane_lb(b.clbs[i]), b.par.lb[b.cpar[i]]);
                if (lbs < unord64(draw)) {
                    push = true;
                    pr = prio_override ? prio_override[i] : (float)lbs;
                    hot = s.theta == 0xffffffffu || key32(pr) < s.theta;
                }
            }
        }
        const uint32_t tgt = 2u * p + (hot ? 1u : 0u);
        if (push) {
            local = atomicAdd(&cnt[tgt], 1u);
            atomicMin(&mn[tgt], ord64(lbs));
        }
        // key range of the hot pushes: reduced over the wave when all of its
        // hot lanes push to one problem (the usual case), else per lane
        {
            const bool hp = push && hot;
            const unsigned long long hm = __ballot(hp);
            if (hm) {
                const int leader = __ffsll((long long)hm) - 1;
                const uint32_t lp = __shfl(p, leader, 64);
                uint32_t klo = hp ? key32(pr) : 0xffffffffu, khi = hp ? key32(pr) : 0u;
                if (__ballot(hp && p == lp) == hm) {
                    for (int off = 32; off > 0; off >>= 1) {
                        klo = min(klo, (uint32_t)__shfl_xor(klo, off, 64));
                        khi = max(khi, (uint32_t)__shfl_xor(khi, off, 64));
                    }
                    if ((int)(threadIdx.x & 63) == leader) {
                        atomicMin(&kmn[lp], klo);
                        atomicMax(&kmx[lp], khi);
                    }
                } else if (hp) {
                    atomicMin(&kmn[p], klo);
                    atomicMax(&kmx[p], khi);
                }
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < T; t += blockDim.x) {
            if (!cnt[t]) continue;
            PState &s = b.st[t >> 1];
            const bool h = t & 1;
            base[t] = atomicAdd(h ? &s.nH[s.hcur ^ 1] : &s.nC[s.ccur], cnt[t]);
            unsigned long long *m = h ? &s.minH : &s.minC;
            if (mn[t] < __atomic_load_n(m, __ATOMIC_RELAXED)) atomicMin(m, mn[t]);
            if (h) widen_key_range(s, s.hcur ^ 1, kmn[t >> 1], kmx[t >> 1]);
        }
        __syncthreads();
        if (push) {
            PState &s = b.st[p];
            const uint32_t slot = base[tgt] + local;
            const Queue q = hot ? qoff(b.H[s.hcur ^ 1], (size_t)p * b.hcap) : qoff(b.C[s.ccur], (size_t)p * b.ccap);
            if (slot >= (hot ? b.hcap : b.ccap)) {
                s.overflow = 1;
            } else {
                q.rkey[slot] = b.crk[i];
                q.tkey[slot] = b.ctk[i];
                q.lb[slot] = lbs;
                q.prio[slot] = pr;
                q.flags[slot] = fl & GOSMA_FLAG_SPLIT_ROT;
                if (q.ubn) {
                    const double S22 = b.prob[p].S22;
                    q.ubn[slot] = (float)fmin(fmax((b.cub[i] + S22) / S22, -10.0), 10.0);
                    for (int k = 0; k < 8; ++k) q.t8[8 * slot + k] = b.ctop8[8 * (size_t)i + k];
                }
            }
        }
        __syncthreads();
    }
}

// Features of a cube for the queue-ordering network (layout documented in
// include/gosma.h): geometry from the keys, normalised bounds, top-8 terms.
__device__ void cube_features(const ProbDesc &P, uint64_t rk, uint64_t tk, double ubn, double lbn,
                              const float *t8, float *f)
{
    const uint64_t m = (1ull << 19) - 1;
    const int Lr = key_level(rk), Lt = key_level(tk);
    const uint64_t ir[3] = {(rk >> 38) & m, (rk >> 19) & m, rk & m};
    const uint64_t it[3] = {(tk >> 38) & m, (tk >> 19) & m, tk & m};
    double hr2 = 0.0, ht2 = 0.0, hd2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double hr = ldexp(P.r_w[a], -(Lr + 1)), ht = ldexp(P.t_w[a], -(Lt + 1));
        const double rc = P.r_lo[a] + (2.0 * (double)ir[a] + 1.0) * hr;
        const double tc = P.t_lo[a] + (2.0 * (double)it[a] + 1.0) * ht;
        f[a] = (float)(rc / 3.14159265358979323846);
        f[3 + a] = (float)(2.0 * (tc - P.t_lo[a]) / P.t_w[a] - 1.0);
        hr2 += hr * hr;
        ht2 += ht * ht;
        hd2 += 0.25 * P.t_w[a] * P.t_w[a];
    }
    f[6] = (float)Lr / 19.0f;
    f[7] = (float)Lt / 19.0f;
    f[8] = (float)(sqrt(hr2) / 3.14159265358979323846);
    f[9] = (float)sqrt(ht2 / hd2);
    f[10] = (float)fmin(fmax(ubn, -10.0), 10.0);
    f[11] = (float)fmin(fmax(lbn, -10.0), 10.0);
    for (int k = 0; k < 8; ++k) f[12 + k] = (float)(t8[k] / P.S22);
}

// Features of the children that the push will queue (input of the learned
// priority): those not dropped whose raised lower bound is below d*, the test
// the push applies (d* does not change in between).  The others need no
// priority.  Their rows are packed, one atomic per wave; crow maps each row
// to its child.
__global__ __launch_bounds__(kBlock) void k_child_features(Bufs b)
{
    const uint32_t n = b.g->nchild;
    uint32_t nb[kBuckets];
    child_counts(b, nb);
    const int lane = threadIdx.x & 63;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const uint32_t i = child_at(b, nb, t);
        const uint32_t p = b.cpid[i];
        const double lbs = fmax(sane_lb(b.clbs[i]), b.par.lb[b.cpar[i]]);
        const bool keep = !(b.cflags[i] & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS)) &&
                          lbs < unord64(b.st[p].dstar);
        const unsigned long long m = __ballot(keep);
        if (!m) continue;
        const int leader = __ffsll((long long)m) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&b.g->nrows, (uint32_t)__popcll(m));
        base = __shfl(base, leader, 64);
        if (!keep) continue;
        const uint32_t row = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        b.crow[row] = i;
        const ProbDesc &P = b.prob[p];
        cube_features(P, b.crk[i], b.ctk[i], (b.cub[i] + P.S22) / P.S22, (lbs + P.S22) / P.S22,
                      b.ctop8 + 8 * (size_t)i, b.cfeat + (size_t)GOSMA_MLP_FEATURES * row);
    }
}

// Learned priority: the cube's normalised lower bound plus the predicted rise
// of its children's (at most 10, the range of the features); the plain order
// where the prediction is not finite.  A cube whose lower bound is already
// within eps of d* never has to be split before the stop test holds (d* only
// decreases), so it is ordered after every cube that has to be, by its lower
// bound; the network only reorders the cubes that every order must split.
constexpr float kMaxRise = 10.0f, kDeferred = 16.0f;
__global__ __launch_bounds__(kBlock) void k_learned_prio(Bufs b, float window)
{
    const uint32_t n = b.g->nrows;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const uint32_t i = b.crow[t];
        const uint32_t p = b.cpid[i];
        const double S22 = b.prob[p].S22;
        const double dstar_n = (unord64(b.st[p].dstar) + S22) / S22, eps_n = b.st[p].eps_f / S22;
        const float lbn = b.cfeat[(size_t)GOSMA_MLP_FEATURES * t + 11];
        const float y = b.cpred[t];
        const float rise = fminf(fmaxf(y, 0.0f), window > 0.0f ? window : kMaxRise);
        float pr = isfinite(y) ? lbn + rise : lbn;
        if ((double)lbn >= dstar_n - eps_n) pr = lbn + kDeferred;
        b.cprio[i] = pr;
    }
}

// Training records: for each parent split this iteration, its features (as
// queued) and the lowest normalised lower bound of its children minus its own.
__global__ __launch_bounds__(kBlock) void k_log_records(Bufs b, int P)
{
    const int p = blockIdx.y;
    if (p >= P) return;
    const PState &s = b.st[p];
    const uint32_t n = s.done ? 0u : min(s.nsel, b.k);   // more than k only on overflow
    const ProbDesc &D = b.prob[p];
    const Queue par = qoff(b.par, (size_t)p * b.k);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t c0 = b.pchild[(size_t)p * b.k + i];
        if (c0 == kNoChildren) continue;
        double best = INFINITY;
        for (int c = 0; c < 8; ++c) {
            const uint32_t ci = c0 + c;
            if (b.cflags[ci] & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS)) continue;
            best = fmin(best, fmax(sane_lb(b.clbs[ci]), par.lb[i]));
        }
        if (!(best < INFINITY)) continue;
        const unsigned long long slot = atomicAdd(b.rec_count, 1ull);
        if (slot >= b.rec_cap) continue;
        float *r = b.rec + slot * GOSMA_MLP_RECORD;
        const double lbn = (par.lb[i] + D.S22) / D.S22;
        cube_features(D, par.rkey[i], par.tkey[i], par.ubn[i], lbn, par.t8 + 8 * (size_t)i, r);
        r[GOSMA_MLP_FEATURES] = (float)fmin((best + D.S22) / D.S22 - (double)r[11], 10.0);
    }
}

// Per-problem control at the end of an iteration.  Re-partitions run once
// every rb_every iterations, so one is asked for when the hot part would run
// low or fill up within that many iterations.
__device__ void iter_end_problem(Bufs &b, int p, int rb_every)
{
    PState &s = b.st[p];
    if (s.done) return;
    s.bounded += 8ull * (s.nsel - s.nskip);
    s.hcur ^= 1;
    s.iters += 1;
    const uint32_t nh = s.nH[s.hcur], nc = s.nC[s.ccur];
    const double lbq = fmin(fmin(unord64(s.minH), unord64(s.minC)), unord64(s.floor_lb));
    const double dstar = unord64(s.dstar);
    if (s.overflow)
        s.done = OVERFLOW;
    else if (nh + nc == 0)
        s.done = EXHAUSTED;
    else if (dstar - lbq <= s.eps_f)
        s.done = EPS_OPTIMAL;
    else if (s.max_iters && s.iters >= s.max_iters)
        s.done = CAPPED;
    if (s.done) return;
    atomicAdd(&b.g->running, 1u);
    // re-partition when the hot part runs low (and cold cubes exist) or fills
    // up.  The target is a sixteenth of the queue, between 16 k and half the
    // capacity; the hot part may grow to twice the target (at least 64 k), so
    // that it stays as small as selections want while the queue is small and
    // grows, with the target, once re-partitions of a large queue dominate
    const uint32_t span = b.k * (uint32_t)rb_every;
    const uint32_t total = nh + nc;
    const uint32_t target = min(max(total / 16u, 16u * b.k), b.hcap / 2u);
    const uint32_t cap = min(b.hcap, max(64u * b.k, 2u * target));
    if ((nh < span && nc > 0) || nh + 8u * span > cap) {
        s.rebuild = 1;
        s.rb_target = target;
    }
}

__global__ void k_iter_end(Bufs b, int P, int rb_every)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) iter_end_problem(b, p, rb_every);
}

// Queue the root cube of each problem (after its bounds were evaluated).
__global__ void k_seed(Bufs b, int P)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    PState &s = b.st[p];
    s.bounded = 1;
    const uint8_t fl = b.cflags[p];
    if (b.cub[p] < INFINITY && ord64(b.cub[p]) == s.dstar) {
        s.best_rkey = b.crk[p];
        s.best_tkey = b.ctk[p];
        s.pose_sma = 0;
    }
    if (fl & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS)) {
        s.done = EXHAUSTED;
        return;
    }
    const double lbs = sane_lb(b.clbs[p]);
    if (!(lbs < unord64(s.dstar))) {
        s.done = EXHAUSTED;
        return;
    }
    const Queue q = qoff(b.H[s.hcur], (size_t)p * b.hcap);
    q.rkey[0] = b.crk[p];
    q.tkey[0] = b.ctk[p];
    q.lb[0] = lbs;
    q.prio[0] = (float)lbs;
    q.flags[0] = fl & GOSMA_FLAG_SPLIT_ROT;
    if (q.ubn) {
        const double S22 = b.prob[p].S22;
        q.ubn[0] = (float)fmin(fmax((b.cub[p] + S22) / S22, -10.0), 10.0);
        for (int k = 0; k < 8; ++k) q.t8[k] = b.ctop8[8 * (size_t)p + k];
    }
    s.nH[s.hcur] = 1;
    s.minH = ord64(lbs);
    s.kmin[s.hcur] = s.kmax[s.hcur] = key32((float)lbs);
}

// Algorithm 1's SMA step: when a bounded cube has lowered d* since SMA last
// ran, refine from the centre of that cube (the child holding d*, recorded by
// the push) and keep the result if it lowers d* further.  One block per
// problem; a problem whose d* did not move since the last start, or whose d*
// came from SMA, returns at once.
__global__ __launch_bounds__(sma::kSmaThreads) void k_sma_search(Bufs b, DevMix mx, int P, int max_iters)
{
    extern __shared__ float4 lds[];
    __shared__ sma::SmaShared sh;
    __shared__ sma::SmaState sst;
    const int tid = threadIdx.x;
    for (int p = blockIdx.x; p < P; p += gridDim.x) {
        PState &s = b.st[p];
        const unsigned long long dbits = s.dstar;
        const bool run = !s.done && !s.pose_sma && dbits != s.sma_from && unord64(dbits) < INFINITY;
        __syncthreads();
        if (!run) continue;
        const ProbDesc D = mx.prob[p];
        if (tid == 0) {
            const uint64_t m = (1ull << 19) - 1;
            const uint64_t rk = s.best_rkey, tk = s.best_tkey;
            const int Lr = key_level(rk), Lt = key_level(tk);
            const uint64_t ir[3] = {(rk >> 38) & m, (rk >> 19) & m, rk & m};
            const uint64_t it[3] = {(tk >> 38) & m, (tk >> 19) & m, tk & m};
            for (int a = 0; a < 3; ++a) {
                sh.x[a] = D.r_lo[a] + (2.0 * (double)ir[a] + 1.0) * ldexp(D.r_w[a], -(Lr + 1));
                sh.x[3 + a] = D.t_lo[a] + (2.0 * (double)it[a] + 1.0) * ldexp(D.t_w[a], -(Lt + 1));
            }
        }
        __syncthreads();
        double x[6], f, g[6];
        float4 *base = mx.grec ? mx.grec + (int64_t)blockIdx.x * mx.grec_stride : lds;
        const int it = sma::sma_run(mx, D, sh, sst, sma::sma_lds(base, D.M, D.N), max_iters, kSmaMemory, kSmaGtol,
                                    kSmaFtol, x, f, g);
        if (tid == 0) {
            s.sma_from = dbits;
            s.sma_runs += 1;
            if (it >= 0 && f < unord64(dbits)) {
                s.dstar = ord64(f);
                for (int a = 0; a < 6; ++a) s.pose[a] = x[a];
                s.pose_sma = 1;
                s.sma_from = s.dstar;
                s.sma_gain += 1;
            }
        }
    }
}

}  // namespace

// Device buffers of a solve, owned by the context and reused while large enough.
struct Solver {
    int P = 0;
    size_t k = 0, hcap = 0, ccap = 0;
    Bufs b{};
    PState *h_st = nullptr;   // pinned host copies
    GState *h_g = nullptr;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;         // `check` iterations, re-partitions in the first
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_nr = nullptr;      // the same iterations without the re-partition launches
    hipGraphExec_t exec_nr = nullptr;
    int graph_maxM = 0;
    bool payload = false;     // logging payload buffers present
    int maxM = 0;             // largest M the Lemma 3 record buffer is sized for
    int bucket_nprob[kBuckets] = {};   // problems per size bucket (the children's ranges)
    int graph_mode = -1;      // captured mode: learned | logging
    float graph_window = 0.0f;
    int graph_iters = 0;      // iterations per captured graph
    int graph_sma = 0;        // SMA iterations of the captured graph
};

}  // namespace gosma

namespace {

using gosma::Bufs;
using gosma::GState;
using gosma::PState;
using gosma::Queue;
using gosma::Solver;

template <class T>
hipError_t dalloc(T *&p, size_t n)
{
    return hipMalloc((void **)&p, sizeof(T) * std::max<size_t>(n, 1));
}
template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}
void free_queue(Queue &q)
{
    dfree(q.rkey);
    dfree(q.tkey);
    dfree(q.lb);
    dfree(q.prio);
    dfree(q.flags);
    dfree(q.ubn);
    dfree(q.t8);
}
hipError_t alloc_queue(Queue &q, size_t n, bool payload)
{
    hipError_t e;
    if ((e = dalloc(q.rkey, n)) || (e = dalloc(q.tkey, n)) || (e = dalloc(q.lb, n)) || (e = dalloc(q.prio, n)) ||
        (e = dalloc(q.flags, n)))
        return e;
    if (payload && ((e = dalloc(q.ubn, n)) || (e = dalloc(q.t8, 8 * n)))) return e;
    return hipSuccess;
}

void drop_graph(Solver *s)
{
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->exec_nr) (void)hipGraphExecDestroy(s->exec_nr);
    if (s->graph_nr) (void)hipGraphDestroy(s->graph_nr);
    s->exec = s->exec_nr = nullptr;
    s->graph = s->graph_nr = nullptr;
}

void free_solver(Solver *s)
{
    drop_graph(s);
    Bufs &b = s->b;
    for (int i = 0; i < 2; ++i) {
        free_queue(b.H[i]);
        free_queue(b.C[i]);
    }
    free_queue(b.par);
    dfree(b.crk);
    dfree(b.ctk);
    dfree(b.cpid);
    dfree(b.cpar);
    dfree(b.ctidx);
    dfree(b.tcells);
    dfree(b.tpid);
    dfree(b.ckey);
    dfree(b.cpid2);
    dfree(b.cslot);
    dfree(b.cub);
    dfree(b.clb);
    dfree(b.clbs);
    dfree(b.cflags);
    dfree(b.s11ub);
    dfree(b.s11lo);
    dfree(b.csetup);
    dfree(b.trec);
    dfree(b.toff);
    dfree(b.csum);
    dfree(b.hist);
    dfree(b.st);
    dfree(b.g);
    dfree(b.ctop8);
    dfree(b.cfeat);
    dfree(b.cpred);
    dfree(b.cprio);
    dfree(b.crow);
    dfree(b.pchild);
    if (s->h_st) (void)hipHostFree(s->h_st);
    if (s->h_g) (void)hipHostFree(s->h_g);
    s->h_st = nullptr;
    s->h_g = nullptr;
    if (s->stream) (void)hipStreamDestroy(s->stream);
    s->stream = nullptr;
    s->P = 0;
    s->k = s->hcap = s->ccap = 0;
}

hipError_t ensure_solver(Solver *s, int P, size_t k, size_t hcap, size_t ccap, bool payload, int maxM,
                         const int (&bucket_nprob)[gosma::kBuckets])
{
    if (s->P == P && s->k == k && s->hcap == hcap && s->ccap == ccap && s->b.st && s->payload == payload &&
        s->maxM == maxM && std::equal(bucket_nprob, bucket_nprob + gosma::kBuckets, s->bucket_nprob))
        return hipSuccess;
    free_solver(s);
    Bufs &b = s->b;
    b = Bufs{};
    hipError_t e = hipSuccess;
    const size_t nc = 8 * k * (size_t)P + (size_t)P;   // children (+ one root per problem)
    for (int i = 0; i < 2 && !e; ++i) {
        e = alloc_queue(b.H[i], hcap * P, payload);
        if (!e) e = alloc_queue(b.C[i], ccap * P, payload);
    }
    if (!e) e = alloc_queue(b.par, k * P, payload);
    if (!e) e = dalloc(b.ctop8, 8 * nc);
    if (!e) e = dalloc(b.cfeat, (size_t)GOSMA_MLP_FEATURES * nc);
    if (!e) e = dalloc(b.cpred, nc);
    if (!e) e = dalloc(b.cprio, nc);
    if (!e) e = dalloc(b.crow, nc);
    if (!e) e = dalloc(b.pchild, k * P);
    if (!e) e = dalloc(b.crk, nc);
    if (!e) e = dalloc(b.ctk, nc);
    if (!e) e = dalloc(b.cpid, nc);
    if (!e) e = dalloc(b.cpar, nc);
    if (!e) e = dalloc(b.ctidx, nc);
    // cell table: 2^tbits >= 16 k slots per problem (at most 8 k used)
    uint32_t tbits = 4;
    while (((size_t)1 << tbits) < 16 * k) ++tbits;
    const size_t nt = (size_t)P << tbits;
    if (!e) e = dalloc(b.tcells, nt);
    if (!e) e = dalloc(b.tpid, nt);
    if (!e) e = dalloc(b.ckey, nc);
    if (!e) e = dalloc(b.cpid2, nc);
    if (!e) e = dalloc(b.cslot, nc);
    if (!e) e = dalloc(b.cub, nc);
    if (!e) e = dalloc(b.clb, nc);
    if (!e) e = dalloc(b.clbs, nc);
    if (!e) e = dalloc(b.cflags, nc);
    if (!e) e = dalloc(b.s11ub, std::max(nt, nc));
    if (!e) e = dalloc(b.s11lo, std::max(nt, nc));
    if (!e) e = dalloc(b.csetup, nc);
    // translation records: one per GMM component of every new cell of an
    // iteration, up to 1 GB; cells beyond compute them in the pair kernel
    const size_t tcap = std::min<size_t>(nc * (size_t)std::max(maxM, 1), ((size_t)1 << 30) / sizeof(gosma::TransRec));
    if (!e) e = dalloc(b.trec, tcap);
    if (!e) e = dalloc(b.toff, nt);
    if (!e) e = dalloc(b.csum, nt);
    if (!e) e = dalloc(b.hist, (size_t)gosma::kHistBins * P);
    if (!e) e = dalloc(b.st, (size_t)P);
    if (!e) e = dalloc(b.g, 1);
    if (!e) e = hipHostMalloc((void **)&s->h_st, sizeof(PState) * P, hipHostMallocDefault);
    if (!e) e = hipHostMalloc((void **)&s->h_g, sizeof(GState), hipHostMallocDefault);
    if (!e) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e) {
        free_solver(s);
        return e;
    }
    b.hcap = (uint32_t)hcap;
    b.ccap = (uint32_t)ccap;
    b.k = (uint32_t)k;
    b.tbits = tbits;
    b.tcap = (uint32_t)tcap;
    // children (and cells) of size bucket j: 8 k per problem of the bucket
    {
        uint32_t at = 0;
        for (int j = 0; j < gosma::kBuckets; ++j) {
            b.kbase[j] = at;
            b.kcap[j] = (uint32_t)(8 * k * (size_t)bucket_nprob[j]);
            at += b.kcap[j];
            s->bucket_nprob[j] = bucket_nprob[j];
        }
    }
    s->payload = payload;
    s->maxM = maxM;
    s->P = P;
    s->k = k;
    s->hcap = hcap;
    s->ccap = ccap;
    return hipSuccess;
}

unsigned long long ordh(double x)
{
    unsigned long long u;
    std::memcpy(&u, &x, sizeof u);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Launch one iteration (all problems).  Every launch has a fixed shape and
// reads its work counts from device memory, so the sequence can be captured.
hipError_t launch_iteration(gosma_ctx *ctx, Solver &S, hipStream_t st, bool timed, bool learned, bool logging,
                            float window, bool rb_slot, int rb_every, int sma_iters)
{
    using namespace gosma;
    Bufs &b = S.b;
    const int P = S.P;
    const int gx = std::max(1, kGridX / P);
    const DevMix mx = ctx->mix();
    auto T0 = [&](int kind) { return timed ? ctx->time_begin(kind, st) : -1; };
    auto T1 = [&](int idx) {
        if (timed) ctx->time_end(idx, st);
    };
    int ti = T0(GOSMA_KERNEL_SELECT);
    hipLaunchKernelGGL(k_iter_begin, dim3(P), dim3(kBlock), 0, st, b, P, (int)rb_slot);
    // re-partition of the problems that asked for it
    if (rb_slot) {
        for (int pass = 0; pass < kRadixPasses; ++pass) {
            hipLaunchKernelGGL(k_hist, dim3(gx, P), dim3(kBlock), 0, st, b, 1, pass);
            hipLaunchKernelGGL(k_scan, dim3(P), dim3(kBlock), 0, st, b, 1, pass);
        }
        hipLaunchKernelGGL(k_rebuild_compact, dim3(gx, P), dim3(kBlock), 0, st, b);
        hipLaunchKernelGGL(k_rebuild_finish, dim3((P + 63) / 64), dim3(64), 0, st, b, P);
    }
    // selection of the k lowest hot cubes
    // the hot part holds at most hcap keys: blocks for kHistPer keys per thread
    const int gh = std::max(1, std::min<int>(gx, (int)((b.hcap + kBlock * kHistPer - 1) / (kBlock * kHistPer))));
    for (int pass = 0; pass < kSelPasses; ++pass) {
        hipLaunchKernelGGL(k_hist, dim3(gh, P), dim3(kBlock), 0, st, b, 0, pass);
        hipLaunchKernelGGL(k_scan, dim3(P), dim3(kBlock), 0, st, b, 0, pass);
    }
    hipLaunchKernelGGL(k_select_compact, dim3(gx, P), dim3(kBlock), 0, st, b);
    T1(ti);
    ti = T0(GOSMA_KERNEL_BRANCH);
    // children, their set-up records and their translation cells (table slots,
    // and the list of distinct cells that k_s11 evaluates): one thread per child
    {
        const int per = (int)((8 * S.k + kBlock - 1) / kBlock);
        const int gb = std::max(1, std::min(per, std::max(1, 8 * kGridX / P)));
        hipLaunchKernelGGL(k_branch_setup, dim3(gb, P), dim3(kBlock), 0, st, b);
    }
    const int64_t maxc = 8 * (int64_t)S.k * P;
    T1(ti);
    // the bound kernels, one launch per non-empty size bucket over its range
    // of children and cells, in the bucket's launch shape
    hipError_t e = hipSuccess;
    ti = T0(GOSMA_KERNEL_S11);
    for (int k = 0; k < kBuckets && !e; ++k) {
        if (!b.kcap[k]) continue;
        const size_t o = b.kbase[k];
        e = launch_s11(mx, b.ckey + o, b.cpid2 + o, b.kcap[k], &b.g->ntcell_b[k],
                       S11Out{b.s11ub, b.s11lo, timed ? ctx->d_counts : nullptr, b.trec, b.toff, b.csum,
                              &b.g->nchild_b[k]},
                       ctx->bucket_maxM[k],
                       ctx->btile11[k], st, b.cslot + o);
    }
    T1(ti);
    if (e) return e;
    ti = T0(GOSMA_KERNEL_S12);
    const bool top8 = learned || logging;
    for (int k = 0; k < kBuckets && !e; ++k) {
        if (!b.kcap[k]) continue;
        const size_t o = b.kbase[k];
        BoundOut bo{b.cub + o, b.clb + o, b.clbs + o, nullptr, b.cflags + o, top8 ? b.ctop8 + 8 * o : nullptr, nullptr,
                    &b.st->dstar, (int)(sizeof(PState) / sizeof(unsigned long long)), timed ? ctx->d_counts : nullptr};
        e = launch_s12(mx, b.crk + o, b.ctk + o, b.cpid + o, b.ctidx + o, b.s11ub, b.s11lo, b.kcap[k],
                       &b.g->nchild_b[k], 1, bo, kMarginGamma, ctx->bucket_maxM[k], ctx->bucket_maxN[k], top8,
                       ctx->btile12[k], b.csetup + o, st, true, TransRecs{b.trec, b.toff, b.csum}, ctx->kpieces);
    }
    T1(ti);
    if (e) return e;
    if (logging) hipLaunchKernelGGL(k_log_records, dim3(std::max(1, gx / 8), P), dim3(kBlock), 0, st, b, P);
    if (learned) {
        ti = T0(GOSMA_KERNEL_MLP);
        hipLaunchKernelGGL(k_child_features, dim3(kGridX / 2), dim3(kBlock), 0, st, b);
        e = mlp_predict(*ctx->mlp, b.cfeat, maxc, &b.g->nrows, b.cpred, 0, st);
        if (e) return e;
        hipLaunchKernelGGL(k_learned_prio, dim3(kGridX / 2), dim3(kBlock), 0, st, b, window);
        T1(ti);
    }
    ti = T0(GOSMA_KERNEL_PUSH);
    {
        const float *po = learned ? (const float *)b.cprio : nullptr;
        // blocks for the children of all problems (8 k per problem at most)
        const int gp = std::max(1, std::min<int>(kGridX, (int)((8 * (size_t)b.k * P + kBlock - 1) / kBlock)));
        if (P <= kPushAggProblems)
            hipLaunchKernelGGL(k_push_agg, dim3(gp), dim3(kBlock), 0, st, b, po, P);
        else
            hipLaunchKernelGGL(k_push, dim3(kGridX), dim3(kBlock), 0, st, b, po, P);
    }
    T1(ti);
    if (sma_iters > 0) {
        ti = T0(GOSMA_KERNEL_SMA);
        hipLaunchKernelGGL(k_sma_search, dim3(std::min(P, mx.grec ? mx.grec_blocks : 1024)), dim3(sma::kSmaThreads),
                           mx.grec ? 0 : sma_lds_bytes(ctx->maxM, ctx->maxN), st, b, mx, P, sma_iters);
        T1(ti);
    }
    hipLaunchKernelGGL(k_iter_end, dim3((P + 63) / 64), dim3(64), 0, st, b, P, rb_every);
    return hipGetLastError();
}

// Search-state snapshot (gosma_snapshot / gosma_resume), host bytes: a
// SnapHead, one SnapProb per problem, then per problem its n queued cubes as
// n rkeys (u64), n tkeys (u64), n margined lower bounds (f64) and n flag
// bytes, padded to a multiple of 8 bytes.  The problem's sizes, S22 and
// domain are stored to reject a snapshot of another problem.
struct SnapHead {
    char magic[8];
    uint32_t version, n_problems;
    uint64_t bytes;
};
struct SnapProb {
    int32_t M, N;
    double S22, zeta, r_lo[3], r_w[3], t_lo[3], t_w[3];
    double dstar, floor_lb;
    uint64_t best_rkey, best_tkey, bounded, n;
    uint32_t iters, pose_sma;
    double pose[6];            // the pose of d* when SMA found it (pose_sma = 1)
};
constexpr char kSnapMagic[8] = {'G', 'O', 'S', 'M', 'A', 'Q', 'S', '1'};
constexpr uint32_t kSnapVersion = 2;

size_t snap_cube_bytes(uint64_t n) { return 24 * (size_t)n + (size_t)((n + 7) & ~7ull); }

void snap_fingerprint(const gosma::ProbDesc &D, SnapProb &q)
{
    q.M = D.M;
    q.N = D.N;
    q.S22 = D.S22;
    q.zeta = D.zeta;
    for (int a = 0; a < 3; ++a) {
        q.r_lo[a] = D.r_lo[a];
        q.r_w[a] = D.r_w[a];
        q.t_lo[a] = D.t_lo[a];
        q.t_w[a] = D.t_w[a];
    }
}

// Check a snapshot against the context's problems; fills the per-problem
// records and the offset of each problem's cube arrays.
int snap_parse(gosma_ctx *ctx, const uint8_t *buf, size_t bytes, std::vector<SnapProb> &pr, std::vector<size_t> &off)
{
    auto bad = [&](const char *what) {
        ctx->err = std::string("snapshot: ") + what;
        return GOSMA_E_INVAL;
    };
    SnapHead h;
    if (bytes < sizeof h) return bad("shorter than its header");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, kSnapMagic, 8) != 0 || h.version != kSnapVersion) return bad("not a snapshot of this format");
    if (h.bytes != bytes) return bad("size differs from the size it records");
    if ((int)h.n_problems != ctx->n_problems) return bad("problem count differs from the current problems");
    size_t at = sizeof h + sizeof(SnapProb) * (size_t)h.n_problems;
    if (at > bytes) return bad("truncated");
    pr.resize(h.n_problems);
    off.resize(h.n_problems);
    for (uint32_t p = 0; p < h.n_problems; ++p) {
        std::memcpy(&pr[p], buf + sizeof h + sizeof(SnapProb) * p, sizeof(SnapProb));
        SnapProb want{};
        snap_fingerprint(ctx->h_prob[p], want);
        const SnapProb &q = pr[p];
        if (q.M != want.M || q.N != want.N || std::memcmp(&q.S22, &want.S22, sizeof(double) * 14) != 0)
            return bad("recorded for different mixtures or a different domain");
        if (q.n > ((uint64_t)1 << 34) || snap_cube_bytes(q.n) > bytes - at) return bad("truncated");
        off[p] = at;
        at += snap_cube_bytes(q.n);
    }
    if (at != bytes) return bad("size does not match its contents");
    return GOSMA_OK;
}

int solve_problems(gosma_ctx *ctx, const gosma_opts *opts, gosma_result *res, int P)
{
    using namespace gosma;
    const auto t_start = std::chrono::steady_clock::now();
    auto fail = [&](int code, const char *what, hipError_t e = hipSuccess) {
        ctx->err = std::string(what) + (e ? std::string(": ") + hipGetErrorString(e) : std::string());
        return code;
    };
    if (!opts || !res) return fail(GOSMA_E_INVAL, "opts and result must not be NULL");
    if (ctx->n_problems < 1 || !ctx->has_domain) return fail(GOSMA_E_STATE, "no problem set");
    if (!(opts->eps >= 0) || opts->batch_parents < 1 || opts->batch_parents > (1 << 20) || opts->max_queue < 16 ||
        opts->max_queue > ((int64_t)1 << 31) || (uint64_t)opts->max_queue * P > ((uint64_t)1 << 34))
        return fail(GOSMA_E_INVAL, "invalid options (eps >= 0, 1 <= batch_parents <= 2^20, 16 <= max_queue <= 2^31)");
    const bool learned = opts->order == 1, logging = opts->log_records != 0;
    if (opts->order != 0 && opts->order != 1) return fail(GOSMA_E_INVAL, "order must be 0 (best-first) or 1 (learned)");
    if (learned && !ctx->mlp_ready()) return fail(GOSMA_E_STATE, "learned order needs a network (gosma_mlp_init/set_params)");
    if (ctx->kpieces > 1 && (learned || logging || ctx->d_grec))
        return fail(GOSMA_E_INVAL, "kappa pieces > 1 need the plain order, no record logging and mixtures whose "
                                   "records fit LDS");
    if (opts->sma_iters < 0 || opts->sma_iters > 10000) return fail(GOSMA_E_INVAL, "sma_iters must be in [0, 10000]");
    const int sma_iters = opts->sma_iters;
    if (logging && !ctx->rec_sink) return fail(GOSMA_E_STATE, "record logging needs gosma_set_record_sink");
    // a pending gosma_resume: the problems may have changed since, so check again
    const bool resuming = !ctx->resume.empty();
    std::vector<SnapProb> sp;
    std::vector<size_t> soff;
    if (resuming) {
        if (logging) return fail(GOSMA_E_STATE, "record logging cannot start from a snapshot (its cubes carry no records)");
        const int rc = snap_parse(ctx, ctx->resume.data(), ctx->resume.size(), sp, soff);
        if (rc) return rc;
        for (int p = 0; p < P; ++p)
            if (sp[p].n > (uint64_t)opts->max_queue)
                return fail(GOSMA_E_INVAL, "the snapshot holds more cubes of a problem than max_queue");
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e) return fail(GOSMA_E_HIP, "hipSetDevice", e);
    ctx->snap_ready = false;   // the solver's buffers are about to change
    ctx->trace.clear();
    for (int p = 0; p < P; ++p) std::memset(res + p, 0, sizeof *res);
    if (!ctx->solver) ctx->solver = new Solver;
    Solver &S = *ctx->solver;
    const size_t k = (size_t)opts->batch_parents;
    const size_t ccap = (size_t)opts->max_queue;
    // hot part: room for a re-partition's target (at most half of it) plus the
    // children of the iterations until the next re-partition (7 k net each).
    // Every selection passes over the hot part, and every re-partition over the
    // whole queue; the target grows with the queue (a sixteenth of it) up to
    // half this capacity, so a long search with a queue of 10^8 cubes and more
    // re-partitions every ~128 iterations (with 64 entries per parent: every
    // ~32, and 64x64 searches of 10^4 iterations took 14-18% longer).  While
    // the queue is small the hot part is held to 64 entries per parent (see
    // iter_end_problem).
    const size_t hcap = 256 * k + 16;
    const float window = (float)opts->learned_window;
    const int mode = (learned ? 1 : 0) | (logging ? 2 : 0) | (sma_iters > 0 ? 4 : 0);
    const bool timed = ctx->timing;
    const bool tracing = opts->trace_every > 0 && P == 1;
    const int check = (timed || tracing) ? 1 : 4;   // iterations between status reads
    if (S.graph_maxM != ctx->maxM || S.graph_mode != mode || S.graph_window != window || S.graph_iters != check ||
        S.graph_sma != sma_iters)
        drop_graph(&S);   // the captured launches depend on these
    if (sma_iters > 0 && !ctx->d_grec) {
        e = hipFuncSetAttribute((const void *)k_sma_search, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)sma_lds_bytes(ctx->maxM, ctx->maxN));
        if (e) return fail(GOSMA_E_HIP, "SMA kernel set-up", e);
    }
    if ((e = ensure_solver(&S, P, k, hcap, ccap, logging, ctx->maxM, ctx->bucket_nprob)))
        return fail(GOSMA_E_NOMEM, "allocating solver buffers", e);
    Bufs &b = S.b;
    b.prob = ctx->d_prob;
    {
        // an empty cell table (the pushes of every iteration empty it again)
        const size_t nt = (size_t)P << b.tbits;
        hipLaunchKernelGGL(k_cells_init, dim3((unsigned)std::min<size_t>((nt + kBlock - 1) / kBlock, 4096)),
                           dim3(kBlock), 0, S.stream, b, P);
        if ((e = hipGetLastError())) return fail(GOSMA_E_HIP, "cell table", e);
    }
    b.rec = ctx->rec_sink;
    b.rec_count = ctx->rec_count;
    b.rec_cap = (uint64_t)ctx->rec_cap;
    hipStream_t st = S.stream;

    // initial state and the root cube of each problem
    std::vector<PState> init(P);
    for (int p = 0; p < P; ++p) {
        PState &s = init[p];
        std::memset(&s, 0, sizeof s);
        s.dstar = s.minH = s.minC = s.floor_lb = s.sma_from = ordh(INFINITY);
        s.eps_f = opts->eps * ctx->h_prob[p].S22;
        s.theta = 0xffffffffu;
        s.kmin[0] = s.kmin[1] = 0xffffffffu;   // both hot buffers empty
        s.max_iters = (uint32_t)std::min<int64_t>(opts->max_iters, 0xffffffffll);
    }
    if (resuming) {
        // the snapshot's cubes go to the cold part; the first iteration
        // re-partitions them (hot part: the lowest keys) before it selects
        for (int p = 0; p < P; ++p) {
            PState &s = init[p];
            const SnapProb &q = sp[p];
            const uint8_t *base = ctx->resume.data() + soff[p];
            const size_t n = (size_t)q.n;
            std::vector<double> lbv(n);
            std::vector<float> prio(n);
            std::memcpy(lbv.data(), base + 16 * n, 8 * n);
            double mn = INFINITY;
            for (size_t i = 0; i < n; ++i) {
                prio[i] = (float)lbv[i];
                mn = std::min(mn, lbv[i]);
            }
            s.dstar = ordh(q.dstar);
            s.floor_lb = ordh(q.floor_lb);
            s.minC = ordh(mn);
            s.best_rkey = q.best_rkey;
            s.best_tkey = q.best_tkey;
            s.pose_sma = q.pose_sma != 0;
            for (int a = 0; a < 6; ++a) s.pose[a] = q.pose[a];
            s.sma_from = s.dstar;   // SMA restarts only once d* moves again
            s.bounded = q.bounded;
            s.iters = q.iters;
            if (opts->max_iters > 0)
                s.max_iters = (uint32_t)std::min<int64_t>((int64_t)q.iters + opts->max_iters, 0xffffffffll);
            s.nC[0] = (uint32_t)n;
            s.rebuild = n > 0;
            s.rb_target = (uint32_t)std::min<size_t>(std::max<size_t>(n / 16, 16 * k), hcap / 2);
            s.done = n > 0 ? RUNNING : EXHAUSTED;
            const Queue C = b.C[0];
            const size_t at = (size_t)p * ccap;
            if ((e = hipMemcpyAsync(C.rkey + at, base, 8 * n, hipMemcpyHostToDevice, st)) ||
                (e = hipMemcpyAsync(C.tkey + at, base + 8 * n, 8 * n, hipMemcpyHostToDevice, st)) ||
                (e = hipMemcpyAsync(C.lb + at, base + 16 * n, 8 * n, hipMemcpyHostToDevice, st)) ||
                (e = hipMemcpyAsync(C.flags + at, base + 24 * n, n, hipMemcpyHostToDevice, st)) ||
                (e = hipMemcpyAsync(C.prio + at, prio.data(), 4 * n, hipMemcpyHostToDevice, st)) ||
                (e = hipStreamSynchronize(st)))
                return fail(GOSMA_E_HIP, "restoring the snapshot", e);
        }
        if ((e = hipMemcpyAsync(b.st, init.data(), sizeof(PState) * P, hipMemcpyHostToDevice, st)) ||
            (e = hipStreamSynchronize(st)))
            return fail(GOSMA_E_HIP, "solver initialisation", e);
        ctx->resume.clear();   // one solve starts from it
    }
    if (!resuming) {
        std::vector<uint64_t> zeros(P, 0);
        std::vector<uint32_t> pids(P);
        for (int p = 0; p < P; ++p) pids[p] = (uint32_t)p;
        if ((e = hipMemcpyAsync(b.st, init.data(), sizeof(PState) * P, hipMemcpyHostToDevice, st)) ||
            (e = hipMemcpyAsync(b.crk, zeros.data(), 8 * P, hipMemcpyHostToDevice, st)) ||
            (e = hipMemcpyAsync(b.ctk, zeros.data(), 8 * P, hipMemcpyHostToDevice, st)) ||
            (e = hipMemcpyAsync(b.cpid, pids.data(), 4 * P, hipMemcpyHostToDevice, st)) ||
            (e = hipStreamSynchronize(st)))
            return fail(GOSMA_E_HIP, "solver initialisation", e);
        const DevMix mx = ctx->mix();
        BoundOut bo{b.cub, b.clb, b.clbs, nullptr, b.cflags, b.ctop8, nullptr, &b.st->dstar,
                    (int)(sizeof(PState) / sizeof(unsigned long long))};
        e = launch_s11(mx, b.ctk, b.cpid, P, nullptr, S11Out{b.s11ub, b.s11lo}, ctx->maxM, ctx->tile11, st);
        if (!e)
            e = launch_s12(mx, b.crk, b.ctk, b.cpid, nullptr, b.s11ub, b.s11lo, P, nullptr, 1, bo, kMarginGamma,
                           ctx->maxM, ctx->maxN, learned || logging, ctx->tile12, b.csetup, st, false, TransRecs{},
                           ctx->kpieces);
        if (!e) {
            hipLaunchKernelGGL(k_seed, dim3((P + 63) / 64), dim3(64), 0, st, b, P);
            e = hipGetLastError();
        }
        if (e) return fail(GOSMA_E_HIP, "root cubes", e);
    }

    // iterations: replay a captured graph of `check` iterations, reading the
    // status after each replay (every iteration when tracing or timing)
    bool use_graph = !timed && !opts->no_graph;
    // Re-partitions run in the first iteration of a replay.  Two graphs: with
    // the re-partition launches, for replays that start while a problem has
    // asked for one (the status read before the replay says so), and without
    // them (their eight launches cost about 4 us each even when no problem
    // re-partitions).
    if (use_graph && !S.exec) {
        for (int g = 0; g < 2 && !e; ++g) {
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e) break;
            hipError_t le = hipSuccess;
            for (int r = 0; r < check && !le; ++r)
                le = launch_iteration(ctx, S, st, false, learned, logging, window, g == 0 && r == 0, check, sma_iters);
            e = hipStreamEndCapture(st, g == 0 ? &S.graph : &S.graph_nr);
            if (!e) e = le;
            if (!e) e = hipGraphInstantiate(g == 0 ? &S.exec : &S.exec_nr, g == 0 ? S.graph : S.graph_nr, nullptr,
                                            nullptr, 0);
        }
        if (e) {
            drop_graph(&S);
            (void)hipGetLastError();
            use_graph = false;
        } else {
            S.graph_maxM = ctx->maxM;
            S.graph_mode = mode;
            S.graph_window = window;
            S.graph_iters = check;
            S.graph_sma = sma_iters;
        }
    }
    int rc = GOSMA_OK;
    int64_t launched = 0;
    for (;;) {
        if ((e = hipMemcpyAsync(S.h_st, b.st, sizeof(PState) * P, hipMemcpyDeviceToHost, st)) ||
            (e = hipStreamSynchronize(st))) {
            rc = fail(GOSMA_E_HIP, "branch-and-bound iteration", e);
            break;
        }
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        int running = 0;
        for (int p = 0; p < P; ++p) running += S.h_st[p].done == RUNNING;
        if (tracing && (launched / check) % opts->trace_every == 0) {
            const PState &h = S.h_st[0];
            const double lbq = std::min({unord64(h.minH), unord64(h.minC), unord64(h.floor_lb)});
            const double row[6] = {(double)h.iters, el, (double)h.bounded, (double)(h.nH[h.hcur] + h.nC[h.ccur]),
                                   unord64(h.dstar), lbq};
            ctx->trace.insert(ctx->trace.end(), row, row + 6);
        }
        if (running == 0) break;
        if (opts->time_limit_s > 0 && el > opts->time_limit_s) break;
        bool rebuild = false;   // a running problem asked for a re-partition
        for (int p = 0; p < P; ++p) rebuild |= S.h_st[p].rebuild && S.h_st[p].done == RUNNING;
        if (use_graph)
            e = hipGraphLaunch(rebuild ? S.exec : S.exec_nr, st);
        else
            for (int r = 0; r < check && !e; ++r)
                e = launch_iteration(ctx, S, st, timed, learned, logging, window, rebuild && r == 0, check, sma_iters);
        if (e) {
            rc = fail(GOSMA_E_HIP, "branch-and-bound iteration", e);
            break;
        }
        launched += check;
    }
    const double seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int p = 0; p < P; ++p) {
        const PState &h = S.h_st[p];
        gosma_result &r = res[p];
        const double S22 = ctx->h_prob[p].S22;
        const double lbq = std::min({unord64(h.minH), unord64(h.minC), unord64(h.floor_lb)});
        r.f_best = unord64(h.dstar);
        r.lb_global = h.done == EXHAUSTED ? std::min(r.f_best, unord64(h.floor_lb)) : std::min(lbq, r.f_best);
        r.f_norm_best = (r.f_best + S22) / S22;
        r.lb_norm = (r.lb_global + S22) / S22;
        r.iters = h.iters;
        r.cubes = (int64_t)h.bounded;
        r.max_queue_used = (int64_t)h.nH[h.hcur] + h.nC[h.ccur];
        r.seconds = seconds;
        r.status = h.done == EPS_OPTIMAL ? 0 : (h.done == EXHAUSTED ? 1 : (h.done == OVERFLOW ? 3 : 2));
        const ProbDesc &D = ctx->h_prob[p];
        auto centre = [](uint64_t key, const double *lo, const double *w, double *c) {
            const uint64_t m = (1ull << 19) - 1;
            int L = (int)((key >> 57) & 63);
            uint64_t idx[3] = {(key >> 38) & m, (key >> 19) & m, key & m};
            for (int a = 0; a < 3; ++a) c[a] = lo[a] + (2.0 * (double)idx[a] + 1.0) * std::ldexp(w[a], -(L + 1));
        };
        if (h.pose_sma) {
            for (int a = 0; a < 3; ++a) {
                r.r[a] = h.pose[a];
                r.t[a] = h.pose[3 + a];
            }
        } else {
            centre(h.best_rkey, D.r_lo, D.r_w, r.r);
            centre(h.best_tkey, D.t_lo, D.t_w, r.t);
        }
        r.sma_runs = h.sma_runs;
        r.sma_improved = h.sma_gain;
        if (h.done == OVERFLOW && rc == GOSMA_OK)
            rc = fail(GOSMA_E_QUEUE_OVERFLOW, "branch-and-bound queue capacity exceeded");
    }
    ctx->snap_ready = rc == GOSMA_OK || rc == GOSMA_E_QUEUE_OVERFLOW;
    return rc;
}

}  // namespace

extern "C" {

void gosma_drop_graph(gosma_ctx *ctx)
{
    if (ctx && ctx->solver) drop_graph(ctx->solver);
}

void gosma_release_solver(gosma_ctx *ctx)
{
    if (!ctx || !ctx->solver) return;
    ctx->snap_ready = false;
    free_solver(ctx->solver);
    delete ctx->solver;
    ctx->solver = nullptr;
}

int gosma_solve(gosma_ctx *ctx, const gosma_opts *opts, gosma_result *res)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (ctx->n_problems != 1) {
        ctx->err = "gosma_solve needs exactly one problem (use gosma_solve_batch)";
        return GOSMA_E_STATE;
    }
    return solve_problems(ctx, opts, res, 1);
}

int gosma_solve_batch(gosma_ctx *ctx, const gosma_opts *opts, gosma_result *res)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    return solve_problems(ctx, opts, res, ctx->n_problems);
}

int gosma_snapshot(gosma_ctx *ctx, void *buf, size_t *bytes)
{
    using namespace gosma;
    if (!ctx || !bytes) return GOSMA_E_INVAL;
    ctx->err.clear();
    Solver *S = ctx->solver;
    if (!ctx->snap_ready || !S || S->P != ctx->n_problems) {
        ctx->err = "no finished search of the current problems to snapshot";
        return GOSMA_E_STATE;
    }
    const int P = S->P;
    hipError_t e = hipSetDevice(ctx->device);
    std::vector<PState> st(P);
    if (!e) e = hipMemcpyAsync(st.data(), S->b.st, sizeof(PState) * P, hipMemcpyDeviceToHost, S->stream);
    if (!e) e = hipStreamSynchronize(S->stream);
    if (e) {
        ctx->err = std::string("snapshot: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    size_t total = sizeof(SnapHead) + sizeof(SnapProb) * (size_t)P;
    std::vector<SnapProb> pr(P);
    for (int p = 0; p < P; ++p) {
        const PState &h = st[p];
        if (h.done == OVERFLOW) {
            ctx->err = "snapshot: a problem overflowed its queue, so its queued cubes are incomplete";
            return GOSMA_E_STATE;
        }
        if (h.nH[h.hcur] > S->hcap || h.nC[h.ccur] > S->ccap) {
            ctx->err = "snapshot: queue counts exceed the queue's capacity";
            return GOSMA_E_STATE;
        }
        SnapProb &q = pr[p];
        std::memset(&q, 0, sizeof q);
        snap_fingerprint(ctx->h_prob[p], q);
        q.dstar = unord64(h.dstar);
        q.floor_lb = unord64(h.floor_lb);
        q.best_rkey = h.best_rkey;
        q.best_tkey = h.best_tkey;
        q.pose_sma = h.pose_sma;
        for (int a = 0; a < 6; ++a) q.pose[a] = h.pose[a];
        q.bounded = h.bounded;
        q.iters = h.iters;
        q.n = (uint64_t)h.nH[h.hcur] + h.nC[h.ccur];
        total += snap_cube_bytes(q.n);
    }
    if (!buf) {
        *bytes = total;
        return GOSMA_OK;
    }
    if (*bytes < total) {
        ctx->err = "snapshot: buffer of " + std::to_string(*bytes) + " bytes, " + std::to_string(total) + " needed";
        *bytes = total;
        return GOSMA_E_INVAL;
    }
    uint8_t *out = static_cast<uint8_t *>(buf);
    SnapHead hd;
    std::memcpy(hd.magic, kSnapMagic, 8);
    hd.version = kSnapVersion;
    hd.n_problems = (uint32_t)P;
    hd.bytes = total;
    std::memcpy(out, &hd, sizeof hd);
    std::memcpy(out + sizeof hd, pr.data(), sizeof(SnapProb) * (size_t)P);
    size_t at = sizeof hd + sizeof(SnapProb) * (size_t)P;
    for (int p = 0; p < P && !e; ++p) {
        const PState &h = st[p];
        const size_t n = (size_t)pr[p].n, nh = h.nH[h.hcur], nc = h.nC[h.ccur];
        uint8_t *rk = out + at, *tk = rk + 8 * n, *lb = tk + 8 * n, *fl = lb + 8 * n;
        // the hot part's cubes, then the cold part's
        auto copy_part = [&](const Queue &q, size_t o, size_t cnt, size_t dst) {
            if (!cnt || e) return;
            if ((e = hipMemcpyAsync(rk + 8 * dst, q.rkey + o, 8 * cnt, hipMemcpyDeviceToHost, S->stream)) ||
                (e = hipMemcpyAsync(tk + 8 * dst, q.tkey + o, 8 * cnt, hipMemcpyDeviceToHost, S->stream)) ||
                (e = hipMemcpyAsync(lb + 8 * dst, q.lb + o, 8 * cnt, hipMemcpyDeviceToHost, S->stream)))
                return;
            e = hipMemcpyAsync(fl + dst, q.flags + o, cnt, hipMemcpyDeviceToHost, S->stream);
        };
        copy_part(S->b.H[h.hcur], (size_t)p * S->hcap, nh, 0);
        copy_part(S->b.C[h.ccur], (size_t)p * S->ccap, nc, nh);
        std::memset(fl + n, 0, snap_cube_bytes(n) - 25 * n);   // padding
        at += snap_cube_bytes(n);
    }
    if (!e) e = hipStreamSynchronize(S->stream);
    if (e) {
        ctx->err = std::string("snapshot: ") + hipGetErrorString(e);
        return GOSMA_E_HIP;
    }
    *bytes = total;
    return GOSMA_OK;
}

int gosma_resume(gosma_ctx *ctx, const void *buf, size_t bytes)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!buf) {
        if (bytes) {
            ctx->err = "resume: NULL buffer with a non-zero size";
            return GOSMA_E_INVAL;
        }
        ctx->resume.clear();
        return GOSMA_OK;
    }
    if (ctx->n_problems < 1 || !ctx->has_domain) {
        ctx->err = "resume: no problem set";
        return GOSMA_E_STATE;
    }
    std::vector<SnapProb> pr;
    std::vector<size_t> off;
    const uint8_t *b = static_cast<const uint8_t *>(buf);
    const int rc = snap_parse(ctx, b, bytes, pr, off);
    if (rc) return rc;
    ctx->resume.assign(b, b + bytes);
    return GOSMA_OK;
}

int gosma_get_trace(gosma_ctx *ctx, double *buf, int64_t cap, int64_t *n)
{
    if (!ctx || !n || (cap > 0 && !buf)) return GOSMA_E_INVAL;
    const int64_t rows = (int64_t)(ctx->trace.size() / 6);
    *n = rows;
    const int64_t w = std::min(rows, cap);
    if (w > 0) std::memcpy(buf, ctx->trace.data(), sizeof(double) * 6 * (size_t)w);
    return GOSMA_OK;
}

}  // extern "C"
