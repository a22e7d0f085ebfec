// Branch-and-bound driver (Algorithm 1, Section 6) with a device-resident queue.
//
// One iteration, all on the device (the host reads a 100-byte status block):
//   begin     reset the per-iteration counters
//   select    3 radix passes (11 + 11 + 10 bits) over the 32-bit ordered key of
//             each queued cube's priority find the key of the k-th lowest;
//             compaction then moves the k lowest into the parent list, keeps
//             the rest in the other queue buffer and drops cubes whose lower
//             bound is no longer below d*
//   branch    8 children per parent, split in rotation or translation by the
//             flag the bound kernel computed for the parent; a rotation split
//             shares one translation cell among its 8 children
//   bound     S11 per translation cell, S12 and both bounds per child (bound.hip);
//             the upper bounds update d* with an atomic minimum
//   push      children whose lower bound (raised to the parent's, minus the
//             rounding margin) is below d* join the queue; the child holding d*
//             records the incumbent pose
// The stop test d* - min LB <= eps uses the minimum lower bound over the queue
// after the push, i.e. the "lowest lower bound in Q" at the start of the next
// iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "gosma_impl.h"

namespace gosma {

namespace {

constexpr int kHistBins = 2048;
constexpr int kBlock = 256;
constexpr int kGridCap = 2048;           // blocks for grid-stride kernels
constexpr int kBoundGrid = 8192;         // blocks (one wavefront each) for the bound kernels
constexpr int kMaxLevel = 19;
// Rounding margin of the FP32 bounds relative to the magnitude S11 + 2 S12 of
// each bound: about 8x the largest relative error measured against the FP64
// oracle.
constexpr double kMarginGamma = 4e-6;

struct BBState {
    unsigned long long dstar;     // ordered bits of d*, the best upper bound
    unsigned long long lbmin;     // ordered bits of the lowest lower bound in the queue
    unsigned long long floor_lb;  // ordered bits: lowest bound of cubes that cannot be split
    unsigned long long best_rkey, best_tkey;
    unsigned long long bounded;   // cubes bounded so far
    uint32_t qcount[2];
    uint32_t nsel, tcount, overflow, take_all;
    uint32_t prefix, need, eq_quota, eq_taken;
    uint32_t kept;                // queue entries kept by the compaction
    uint32_t pad;
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

// Wavefront-aggregated append: one atomic per wave.  Every lane of the wave
// must call it (pred false for lanes with nothing to append).
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred)
{
    unsigned long long mask = __ballot(pred);
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (mask) {
        int leader = __ffsll((long long)mask) - 1;
        if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
        base = __shfl(base, leader, 64);
    }
    return base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

struct Queue {
    uint64_t *rkey, *tkey;
    double *lb;
    float *prio;
    uint8_t *flags;
};

__global__ void k_begin(BBState *st, int out, uint32_t *hist)
{
    int t = threadIdx.x;
    if (t == 0) {
        st->qcount[out] = 0;
        st->nsel = 0;
        st->tcount = 0;
        st->take_all = 0;
        st->prefix = 0;
        st->need = 0;
        st->eq_quota = 0;
        st->eq_taken = 0;
        st->kept = 0;
        st->lbmin = ord64(INFINITY);
    }
    for (int b = t; b < kHistBins; b += blockDim.x) hist[b] = 0;
}

// Radix pass: histogram of the digit below the prefix fixed by earlier passes.
__global__ __launch_bounds__(kBlock) void k_hist(Queue q, const BBState *st, int in, int pass, uint32_t *hist)
{
    __shared__ uint32_t h[kHistBins];
    if (st->take_all) return;
    for (int b = threadIdx.x; b < kHistBins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const uint32_t n = st->qcount[in];
    const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
    const uint32_t mask = pass == 2 ? 0x3ffu : 0x7ffu;
    const int pshift = pass == 0 ? 32 : (pass == 1 ? 21 : 10);
    const uint32_t prefix = st->prefix;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint32_t k = key32(q.prio[i]);
        if (pass == 0 || (k >> pshift) == prefix) atomicAdd(&h[(k >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kHistBins; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Radix pass: pick the digit holding the k-th lowest key.  One block.
__global__ __launch_bounds__(kBlock) void k_scan(BBState *st, int in, int pass, uint32_t k, uint32_t *hist)
{
    __shared__ uint32_t part[kBlock];
    __shared__ uint32_t found, left;
    if (st->take_all) return;
    const int t = threadIdx.x;
    if (pass == 0 && st->qcount[in] <= k) {
        if (t == 0) st->take_all = 1;
        return;
    }
    const uint32_t need = pass == 0 ? k : st->need;
    constexpr int per = kHistBins / kBlock;   // 8 bins per thread
    uint32_t loc[per], sum = 0;
    for (int j = 0; j < per; ++j) {
        loc[j] = hist[t * per + j];
        sum += loc[j];
    }
    part[t] = sum;
    if (t == 0) {
        found = 0;
        left = need;
    }
    __syncthreads();
    uint32_t cum = 0;
    for (int u = 0; u < t; ++u) cum += part[u];
    for (int j = 0; j < per; ++j) {
        if (cum < need && need <= cum + loc[j]) {     // exactly one bin qualifies
            found = (uint32_t)(t * per + j);
            left = need - cum;
        }
        cum += loc[j];
    }
    __syncthreads();
    for (int j = 0; j < per; ++j) hist[t * per + j] = 0;
    if (t == 0) {
        const int bits = pass == 2 ? 10 : 11;
        st->prefix = (st->prefix << bits) | found;
        st->need = left;
        if (pass == 2) st->eq_quota = left;
    }
}

// Compaction: k lowest -> parents; the rest (still below d*) -> the other buffer.
__global__ __launch_bounds__(kBlock) void k_compact(Queue qin, Queue qout, BBState *st, int in, int out,
                                                    Queue par, uint32_t capacity)
{
    const uint32_t n = st->qcount[in];
    const bool all = st->take_all != 0;
    const uint32_t T = st->prefix;
    const double dstar = unord64(st->dstar);
    const uint32_t stride = gridDim.x * blockDim.x;
    double local_min = INFINITY;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < n;
        bool sel = false, keep = false;
        double lb = 0.0;
        if (valid) {
            lb = sane_lb(qin.lb[i]);
            if (lb < dstar) {
                uint32_t key = key32(qin.prio[i]);
                if (all || key < T)
                    sel = true;
                else if (key == T)
                    sel = atomicAdd(&st->eq_taken, 1u) < st->eq_quota;
                keep = !sel;
                if (keep) local_min = fmin(local_min, lb);
            }
        }
        uint32_t ps = wave_append(&st->nsel, sel);
        if (sel) {
            par.rkey[ps] = qin.rkey[i];
            par.tkey[ps] = qin.tkey[i];
            par.lb[ps] = lb;
            par.flags[ps] = qin.flags[i];
        }
        uint32_t qs = wave_append(&st->qcount[out], keep);
        if (keep) {
            if (qs < capacity) {
                qout.rkey[qs] = qin.rkey[i];
                qout.tkey[qs] = qin.tkey[i];
                qout.lb[qs] = lb;
                qout.prio[qs] = qin.prio[i];
                qout.flags[qs] = qin.flags[i];
            } else {
                st->overflow = 1;
            }
        }
    }
    // lowest bound of the cubes that stay; k_push merges the children in
    for (int off = 32; off > 0; off >>= 1) local_min = fmin(local_min, __shfl_xor(local_min, off, 64));
    if ((threadIdx.x & 63) == 0 && local_min < INFINITY) atomicMin(&st->lbmin, ord64(local_min));
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

// Wavefront-aggregated reservation of cnt consecutive slots per lane.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t *counter, uint32_t cnt)
{
    const int lane = threadIdx.x & 63;
    uint32_t x = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    const uint32_t total = __shfl(x, 63, 64);
    uint32_t base = 0;
    if (lane == 0 && total) base = atomicAdd(counter, total);
    base = __shfl(base, 0, 64);
    return base + x - cnt;
}

// 8 children per parent.  A rotation split shares its parent's translation
// cell among the 8 children (one cell); a translation split has 8 cells.
__global__ __launch_bounds__(kBlock) void k_branch(Queue par, BBState *st, uint64_t *crk, uint64_t *ctk,
                                                   int64_t *ctidx, uint8_t *cskip, uint64_t *tcells)
{
    const uint32_t n = st->nsel;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t p = base + threadIdx.x;
        const bool valid = p < n;
        bool rot = false, skip = false;
        uint64_t rk = 0, tk = 0;
        if (valid) {
            rk = par.rkey[p];
            tk = par.tkey[p];
            rot = (par.flags[p] & GOSMA_FLAG_SPLIT_ROT) != 0;
            const bool rmax = key_level(rk) >= kMaxLevel, tmax = key_level(tk) >= kMaxLevel;
            if (rot && rmax) rot = false;
            if (!rot && tmax) rot = !rmax;
            skip = rmax && tmax;
            if (skip) atomicMin(&st->floor_lb, ord64(par.lb[p]));
        }
        const bool one = rot || skip;
        const uint32_t tb = wave_reserve(&st->tcount, valid ? (one ? 1u : 8u) : 0u);
        if (!valid) continue;
        for (int c = 0; c < 8; ++c) {
            const uint32_t ci = 8 * p + c;
            const uint64_t ck = one ? tk : child_key(tk, c);
            crk[ci] = one ? child_key(rk, c) : rk;
            ctk[ci] = ck;
            cskip[ci] = skip;
            ctidx[ci] = one ? tb : tb + c;
            if (!one) tcells[tb + c] = ck;
        }
        if (one) tcells[tb] = tk;
    }
}

struct ChildOut {
    double *ub, *lb, *lb_safe, *aux;
    uint8_t *flags;
};

__global__ __launch_bounds__(kBlock) void k_push(Queue par, const uint64_t *crk, const uint64_t *ctk,
                                                 const uint8_t *cskip, ChildOut co, BBState *st, int out,
                                                 Queue qout, uint32_t capacity)
{
    const uint32_t n = 8 * st->nsel;
    const unsigned long long draw = st->dstar;
    const double dstar = unord64(draw);
    const uint32_t stride = gridDim.x * blockDim.x;
    double local_min = INFINITY;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < n;
        bool push = false;
        double lbs = 0.0;
        uint8_t fl = 0;
        if (valid) {
            fl = co.flags[i];
            const bool dropped = (fl & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS)) || cskip[i];
            if (!dropped) {
                lbs = fmax(sane_lb(co.lb_safe[i]), par.lb[i >> 3]);
                push = lbs < dstar;
                if (co.ub[i] < INFINITY && ord64(co.ub[i]) == draw) {
                    st->best_rkey = crk[i];
                    st->best_tkey = ctk[i];
                }
            }
        }
        uint32_t qs = wave_append(&st->qcount[out], push);
        if (push) {
            if (qs < capacity) {
                qout.rkey[qs] = crk[i];
                qout.tkey[qs] = ctk[i];
                qout.lb[qs] = lbs;
                qout.prio[qs] = (float)lbs;
                qout.flags[qs] = fl & GOSMA_FLAG_SPLIT_ROT;
            } else {
                st->overflow = 1;
            }
            local_min = fmin(local_min, lbs);
        }
    }
    for (int off = 32; off > 0; off >>= 1) local_min = fmin(local_min, __shfl_xor(local_min, off, 64));
    if ((threadIdx.x & 63) == 0 && local_min < INFINITY) atomicMin(&st->lbmin, ord64(local_min));
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&st->bounded, (unsigned long long)n);
}

__global__ void k_seed(Queue q, BBState *st, const uint64_t *rk, const uint64_t *tk, ChildOut co, int out,
                       uint32_t capacity)
{
    // root cube: push it unless dropped (lower bound raised to -inf parent)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->bounded += 1;
    uint8_t fl = co.flags[0];
    if (fl & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS)) return;
    double lbs = sane_lb(co.lb_safe[0]);
    if (co.ub[0] < INFINITY && ord64(co.ub[0]) == st->dstar) {
        st->best_rkey = rk[0];
        st->best_tkey = tk[0];
    }
    if (!(lbs < unord64(st->dstar))) return;
    uint32_t qs = st->qcount[out]++;
    if (qs >= capacity) {
        st->overflow = 1;
        return;
    }
    q.rkey[qs] = rk[0];
    q.tkey[qs] = tk[0];
    q.lb[qs] = lbs;
    q.prio[qs] = (float)lbs;
    q.flags[qs] = fl & GOSMA_FLAG_SPLIT_ROT;
    st->lbmin = ord64(lbs);
}

}  // namespace

// Device buffers of one solve (owned by the context, grown on demand).
struct Solver {
    size_t cap = 0, kcap = 0;
    Queue q[2] = {};
    Queue par = {};
    uint64_t *crk = nullptr, *ctk = nullptr, *tcells = nullptr;
    int64_t *ctidx = nullptr;
    uint8_t *cskip = nullptr;
    double *cub = nullptr, *clb = nullptr, *clbs = nullptr, *s11ub = nullptr, *s11lo = nullptr;
    uint8_t *cflags = nullptr;
    uint32_t *hist = nullptr;
    BBState *st = nullptr;
    BBState *h_st = nullptr;   // pinned host copy
};

}  // namespace gosma

namespace {

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

void free_queue(gosma::Queue &q)
{
    dfree(q.rkey);
    dfree(q.tkey);
    dfree(q.lb);
    dfree(q.prio);
    dfree(q.flags);
}

hipError_t alloc_queue(gosma::Queue &q, size_t n)
{
    hipError_t e;
    if ((e = dalloc(q.rkey, n)) || (e = dalloc(q.tkey, n)) || (e = dalloc(q.lb, n)) || (e = dalloc(q.prio, n)) ||
        (e = dalloc(q.flags, n)))
        return e;
    return hipSuccess;
}

void free_solver(gosma::Solver *s)
{
    if (!s) return;
    free_queue(s->q[0]);
    free_queue(s->q[1]);
    free_queue(s->par);
    dfree(s->crk);
    dfree(s->ctk);
    dfree(s->tcells);
    dfree(s->ctidx);
    dfree(s->cskip);
    dfree(s->cub);
    dfree(s->clb);
    dfree(s->clbs);
    dfree(s->s11ub);
    dfree(s->s11lo);
    dfree(s->cflags);
    dfree(s->hist);
    dfree(s->st);
    if (s->h_st) (void)hipHostFree(s->h_st);
    s->h_st = nullptr;
    s->cap = s->kcap = 0;
}

hipError_t ensure_solver(gosma::Solver *s, size_t cap, size_t k)
{
    if (s->cap >= cap && s->kcap >= k && s->st) return hipSuccess;
    free_solver(s);
    hipError_t e;
    const size_t c8 = 8 * k;
    if ((e = alloc_queue(s->q[0], cap)) || (e = alloc_queue(s->q[1], cap)) || (e = alloc_queue(s->par, k)) ||
        (e = dalloc(s->crk, c8)) || (e = dalloc(s->ctk, c8)) || (e = dalloc(s->tcells, c8)) ||
        (e = dalloc(s->ctidx, c8)) || (e = dalloc(s->cskip, c8)) || (e = dalloc(s->cub, c8)) ||
        (e = dalloc(s->clb, c8)) || (e = dalloc(s->clbs, c8)) || (e = dalloc(s->s11ub, c8)) ||
        (e = dalloc(s->s11lo, c8)) || (e = dalloc(s->cflags, c8)) || (e = dalloc(s->hist, gosma::kHistBins)) ||
        (e = dalloc(s->st, 1)))
        return e;
    if ((e = hipHostMalloc((void **)&s->h_st, sizeof(gosma::BBState), hipHostMallocDefault))) return e;
    s->cap = cap;
    s->kcap = k;
    return hipSuccess;
}

}  // namespace

extern "C" {

void gosma_release_solver(gosma_ctx *ctx)
{
    if (!ctx || !ctx->solver) return;
    free_solver(ctx->solver);
    delete ctx->solver;
    ctx->solver = nullptr;
}

int gosma_solve(gosma_ctx *ctx, const gosma_opts *opts, gosma_result *res)
{
    using namespace gosma;
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!opts || !res) {
        ctx->err = "opts and result must not be NULL";
        return GOSMA_E_INVAL;
    }
    if (ctx->n_problems != 1 || !ctx->has_domain) {
        ctx->err = "gosma_solve needs exactly one problem with a domain";
        return GOSMA_E_STATE;
    }
    if (!(opts->eps >= 0) || opts->batch_parents < 1 || opts->batch_parents > (1 << 20) || opts->max_queue < 16 ||
        opts->max_queue > ((int64_t)1 << 31)) {
        ctx->err = "invalid options (eps >= 0, 1 <= batch_parents <= 2^20, 16 <= max_queue <= 2^31)";
        return GOSMA_E_INVAL;
    }
    if (opts->order != 0) {
        ctx->err = "learned order needs a loaded network";
        return GOSMA_E_STATE;
    }
    const auto t_start = std::chrono::steady_clock::now();
    std::memset(res, 0, sizeof *res);
    auto hipcheck = [&](hipError_t e, const char *what) {
        if (e != hipSuccess) ctx->err = std::string(what) + ": " + hipGetErrorString(e);
        return e != hipSuccess;
    };
    if (hipcheck(hipSetDevice(ctx->device), "hipSetDevice")) return GOSMA_E_HIP;
    if (!ctx->solver) ctx->solver = new Solver;
    Solver &S = *ctx->solver;
    const size_t k = (size_t)opts->batch_parents;
    const uint32_t cap = (uint32_t)opts->max_queue;
    if (hipcheck(ensure_solver(&S, cap, k), "allocating solver buffers")) {
        free_solver(&S);
        return GOSMA_E_NOMEM;
    }
    hipStream_t s = nullptr;
    const double S22 = ctx->h_prob[0].S22;
    const double eps_f = opts->eps * S22;
    const DevMix mx = ctx->mix();
    const int maxM = ctx->maxM;

    // initial state
    BBState init;
    std::memset(&init, 0, sizeof init);
    auto ordh = [](double x) {
        unsigned long long u;
        std::memcpy(&u, &x, sizeof u);
        return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
    };
    init.dstar = ordh(INFINITY);
    init.lbmin = ordh(INFINITY);
    init.floor_lb = ordh(INFINITY);
    if (hipcheck(hipMemcpy(S.st, &init, sizeof init, hipMemcpyHostToDevice), "state init")) return GOSMA_E_HIP;

    ChildOut co{S.cub, S.clb, S.clbs, nullptr, S.cflags};
    // d*: the S12 epilogue takes the atomic minimum of the FP32 upper bounds.
    // The rounding margin is carried by the lower bounds (lb_safe), so the
    // certificate is d* - min lb_safe <= eps up to the margin.
    BoundOut bo{S.cub, S.clb, S.clbs, nullptr, S.cflags, nullptr, nullptr, &S.st->dstar};

    // root cube
    {
        uint64_t zero64 = 0;
        hipError_t e = hipMemcpy(S.crk, &zero64, 8, hipMemcpyHostToDevice);
        if (!e) e = hipMemcpy(S.ctk, &zero64, 8, hipMemcpyHostToDevice);
        if (!e) {
            hipLaunchKernelGGL(k_begin, dim3(1), dim3(kBlock), 0, s, S.st, 0, S.hist);
            e = launch_s11(mx, S.ctk, nullptr, 1, nullptr, S11Out{S.s11ub, S.s11lo}, maxM, 0, s);
        }
        if (!e)
            e = launch_s12(mx, S.crk, S.ctk, nullptr, nullptr, S.s11ub, S.s11lo, 1, nullptr, 1, bo, kMarginGamma, maxM,
                           false, 0, s);
        if (!e) {
            hipLaunchKernelGGL(k_seed, dim3(1), dim3(64), 0, s, S.q[0], S.st, S.crk, S.ctk, co, 0, cap);
            e = hipGetLastError();
        }
        if (hipcheck(e, "root cube")) return GOSMA_E_HIP;
    }
    int cur = 0;
    int status = 1;
    int rc = GOSMA_OK;
    int64_t iters = 0;
    const int gsel = kGridCap;
    for (;;) {
        // status of the queue after the last push
        if (hipcheck(hipMemcpyAsync(S.h_st, S.st, sizeof(BBState), hipMemcpyDeviceToHost, s), "status copy") ||
            hipcheck(hipStreamSynchronize(s), "iteration")) {
            rc = GOSMA_E_HIP;
            break;
        }
        const BBState &h = *S.h_st;
        const double dstar = unord64(h.dstar);
        const double lbq = std::min(unord64(h.lbmin), unord64(h.floor_lb));
        res->max_queue_used = std::max<int64_t>(res->max_queue_used, h.qcount[cur]);
        if (h.overflow) {
            rc = GOSMA_E_QUEUE_OVERFLOW;
            ctx->err = "branch-and-bound queue capacity exceeded";
            status = 2;
            res->lb_global = lbq;
            break;
        }
        if (h.qcount[cur] == 0) {
            status = 1;
            res->lb_global = std::min(dstar, unord64(h.floor_lb));
            break;
        }
        res->lb_global = lbq;
        if (dstar - lbq <= eps_f) {
            status = 0;
            break;
        }
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if ((opts->max_iters > 0 && iters >= opts->max_iters) || (opts->time_limit_s > 0 && el > opts->time_limit_s)) {
            status = 2;
            break;
        }
        const int out = cur ^ 1;
        // select
        int ti = ctx->time_begin(GOSMA_KERNEL_SELECT, s);
        hipLaunchKernelGGL(k_begin, dim3(1), dim3(kBlock), 0, s, S.st, out, S.hist);
        for (int pass = 0; pass < 3; ++pass) {
            hipLaunchKernelGGL(k_hist, dim3(gsel), dim3(kBlock), 0, s, S.q[cur], S.st, cur, pass, S.hist);
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(kBlock), 0, s, S.st, cur, pass, (uint32_t)k, S.hist);
        }
        hipLaunchKernelGGL(k_compact, dim3(gsel), dim3(kBlock), 0, s, S.q[cur], S.q[out], S.st, cur, out, S.par,
                           cap);
        ctx->time_end(ti, s);
        // branch
        ti = ctx->time_begin(GOSMA_KERNEL_BRANCH, s);
        hipLaunchKernelGGL(k_branch, dim3(64), dim3(kBlock), 0, s, S.par, S.st, S.crk, S.ctk, S.ctidx, S.cskip,
                           S.tcells);
        ctx->time_end(ti, s);
        // bound
        ti = ctx->time_begin(GOSMA_KERNEL_S11, s);
        hipError_t e = launch_s11(mx, S.tcells, nullptr, 8 * (int64_t)k, &S.st->tcount, S11Out{S.s11ub, S.s11lo},
                                  maxM, kBoundGrid, s);
        ctx->time_end(ti, s);
        ti = ctx->time_begin(GOSMA_KERNEL_S12, s);
        if (!e)
            e = launch_s12(mx, S.crk, S.ctk, nullptr, S.ctidx, S.s11ub, S.s11lo, 8 * (int64_t)k, &S.st->nsel, 8, bo,
                           kMarginGamma, maxM, false, kBoundGrid, s);
        ctx->time_end(ti, s);
        if (hipcheck(e, "bound kernels")) {
            rc = GOSMA_E_HIP;
            break;
        }
        // push
        ti = ctx->time_begin(GOSMA_KERNEL_PUSH, s);
        hipLaunchKernelGGL(k_push, dim3(gsel), dim3(kBlock), 0, s, S.par, S.crk, S.ctk, S.cskip, co, S.st, out,
                           S.q[out], cap);
        ctx->time_end(ti, s);
        if (hipcheck(hipGetLastError(), "kernel launch")) {
            rc = GOSMA_E_HIP;
            break;
        }
        cur = out;
        ++iters;
    }
    // final state
    if (hipcheck(hipMemcpy(S.h_st, S.st, sizeof(BBState), hipMemcpyDeviceToHost), "final status")) return GOSMA_E_HIP;
    const BBState &h = *S.h_st;
    res->f_best = unord64(h.dstar);
    res->iters = iters;
    res->cubes = (int64_t)h.bounded;
    res->status = status;
    res->f_norm_best = (res->f_best + S22) / S22;
    res->lb_norm = (res->lb_global + S22) / S22;
    // pose of d*: cube centre
    const ProbDesc &P = ctx->h_prob[0];
    auto centre = [](uint64_t key, const double *lo, const double *w, double *c) {
        const uint64_t m = (1ull << 19) - 1;
        int L = (int)((key >> 57) & 63);
        uint64_t idx[3] = {(key >> 38) & m, (key >> 19) & m, key & m};
        for (int a = 0; a < 3; ++a) c[a] = lo[a] + (2.0 * (double)idx[a] + 1.0) * std::ldexp(w[a], -(L + 1));
    };
    centre(h.best_rkey, P.r_lo, P.r_w, res->r);
    centre(h.best_tkey, P.t_lo, P.t_w, res->t);
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return rc;
}

int gosma_solve_batch(gosma_ctx *ctx, const gosma_opts *, gosma_result *)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err = "gosma_solve_batch: not built yet";
    return GOSMA_E_STATE;
}

}  // extern "C"
