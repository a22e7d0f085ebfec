// Mixture generation (Section 7): DP-means on the 3D point set and
// DP-vMF-means on the bearing vectors, then maximum-likelihood components
// (isotropic Gaussian sigma; vMF concentration) for the clusters.
//
// Each clustering pass has the meaning of the serial batch algorithm (points
// in index order; a point joins the best cluster that exists when it is
// visited -- the clusters of the previous pass and those opened earlier in
// this pass -- or opens a new one at itself when even the best is beyond the
// threshold; ties go to the cluster created first), computed in parallel:
//   k_score_old    every point's best cluster of the previous pass (centres in
//                  LDS) and whether it is beyond the threshold (a candidate);
//   k_open         one block walks the candidates in index order, chunk by
//                  chunk: the chunk's candidates are first checked in
//                  parallel against the clusters opened so far, then the ones
//                  still beyond the threshold are settled in order against the
//                  clusters opened earlier in the chunk;
//   k_assign       every point's label: its opener's cluster, else the best of
//                  its previous-pass cluster and the clusters opened at lower
//                  indices (in opening order);
//   k_sums         per-cluster sums and counts (FP64 atomics; the inputs lie on
//                  a grid on which these sums are exact, so the order of the
//                  additions does not matter);
//   k_centres      new centres, empty clusters removed in order (one block);
//   k_relabel      labels renumbered, changes counted.
// Scores are FP64 expressions evaluated left to right with no fused
// multiply-adds (this file is compiled with -ffp-contract=off), so each
// decision is the one a serial FP64 evaluation of the same expression takes.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gosma_impl.h"

namespace gosma {
namespace {

constexpr int kMgBlock = 256;
constexpr int kOpenBlock = 1024;
constexpr int kMaxLds = 2048;   // centres staged in LDS per pass (3 doubles each)
constexpr int kMaxOpen = 2048;  // clusters one pass can open (LDS of k_open); max_clusters <= this

struct MgBufs {
    const double *x;
    int64_t n;
    int spherical;
    double lambda;
    int max_clusters;
    int32_t *z, *prev;
    double *best;            // per point: best score over the previous pass's clusters
    int32_t *bestc;          // and that cluster
    uint8_t *cand;           // 1: beyond the threshold of every previous-pass cluster
    double *mu;              // centres of the previous pass, then of this pass (max_clusters x 3)
    double *sum;             // per-cluster sums (max_clusters x 3)
    unsigned long long *cnt; // per-cluster counts
    int32_t *opener;         // point index that opened each new cluster of this pass, in order
    int *state;              // {K_old, K_new, overflow, changed, K_after}
};

__device__ __forceinline__ double score(const double *x, const double *m, int spherical)
{
    if (spherical) return x[0] * m[0] + x[1] * m[1] + x[2] * m[2];
    const double a = x[0] - m[0], b = x[1] - m[1], c = x[2] - m[2];
    return a * a + b * b + c * c;
}
__device__ __forceinline__ bool better(double s, double b, int spherical) { return spherical ? s > b : s < b; }
__device__ __forceinline__ bool beyond(double s, double lam, int spherical) { return spherical ? s < lam : s > lam; }

// Sum of all points and the count (the starting cluster).
__global__ __launch_bounds__(kMgBlock) void k_total(MgBufs B)
{
    double s[3] = {0, 0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B.n; i += (int64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 3; ++a) s[a] += B.x[3 * i + a];
    for (int a = 0; a < 3; ++a) {
        double v = s[a];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(&B.sum[a], v);
    }
}

__global__ void k_start(MgBufs B)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double sx = B.sum[0], sy = B.sum[1], sz = B.sum[2];
    if (B.spherical) {
        const double nr = sqrt(sx * sx + sy * sy + sz * sz);
        B.mu[0] = nr > 0.0 ? sx / nr : 0.0;
        B.mu[1] = nr > 0.0 ? sy / nr : 0.0;
        B.mu[2] = nr > 0.0 ? sz / nr : 1.0;
    } else {
        B.mu[0] = sx / (double)B.n;
        B.mu[1] = sy / (double)B.n;
        B.mu[2] = sz / (double)B.n;
    }
    B.state[0] = 1;
}

// Best previous-pass cluster of every point; candidates flagged.
__global__ __launch_bounds__(kMgBlock) void k_score_old(MgBufs B)
{
    __shared__ double m[3 * kMaxLds];
    const int K = B.state[0];
    const int Kl = K < kMaxLds ? K : kMaxLds;
    for (int t = threadIdx.x; t < 3 * Kl; t += blockDim.x) m[t] = B.mu[t];
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double xi[3] = {B.x[3 * i], B.x[3 * i + 1], B.x[3 * i + 2]};
        double bs = score(xi, m, B.spherical);
        int bc = 0;
        for (int c = 1; c < K; ++c) {
            const double s = score(xi, c < kMaxLds ? m + 3 * c : B.mu + 3 * c, B.spherical);
            if (better(s, bs, B.spherical)) {
                bs = s;
                bc = c;
            }
        }
        B.best[i] = bs;
        B.bestc[i] = bc;
        B.cand[i] = beyond(bs, B.lambda, B.spherical) ? 1 : 0;
    }
}

// The clusters opened in this pass, in index order (one block).
__global__ __launch_bounds__(kOpenBlock) void k_open(MgBufs B)
{
    __shared__ int32_t list[kOpenBlock];
    __shared__ double opened[3 * kMaxOpen];   // centres opened in this pass (LDS: read back at once)
    __shared__ int nlist, nopen_sh, overflow_sh;
    const int tid = threadIdx.x;
    const int K_old = B.state[0];
    if (tid == 0) {
        nopen_sh = 0;
        overflow_sh = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < B.n; base += kOpenBlock) {
        const int64_t i = base + tid;
        const int nopen0 = nopen_sh;
        // parallel: still beyond the threshold of every cluster opened so far?
        bool c = i < B.n && B.cand[i];
        if (c) {
            const double xi[3] = {B.x[3 * i], B.x[3 * i + 1], B.x[3 * i + 2]};
            for (int k = 0; k < nopen0; ++k) {
                if (!beyond(score(xi, opened + 3 * k, B.spherical), B.lambda, B.spherical)) {
                    c = false;
                    break;
                }
            }
        }
        // ordered list of the chunk's remaining candidates
        if (tid == 0) nlist = 0;
        __syncthreads();
        const unsigned long long bal = __ballot(c);
        __shared__ int wcount[kOpenBlock / 64];
        if ((tid & 63) == 0) wcount[tid >> 6] = __popcll(bal);
        __syncthreads();
        if (c) {
            int off = 0;
            for (int w = 0; w < (tid >> 6); ++w) off += wcount[w];
            off += __popcll(bal & ((1ull << (tid & 63)) - 1ull));
            list[off] = (int32_t)i;
        }
        if (tid == 0) {
            int t = 0;
            for (int w = 0; w < kOpenBlock / 64; ++w) t += wcount[w];
            nlist = t;
        }
        __syncthreads();
        // serial: each remaining candidate against the clusters opened in this chunk
        if (tid == 0) {
            int nopen = nopen0;
            for (int q = 0; q < nlist; ++q) {
                const int32_t j = list[q];
                const double xj[3] = {B.x[3 * j], B.x[3 * j + 1], B.x[3 * j + 2]};
                bool opens = true;
                for (int k = nopen0; k < nopen && opens; ++k)
                    if (!beyond(score(xj, opened + 3 * k, B.spherical), B.lambda, B.spherical)) opens = false;
                if (!opens) continue;
                if (K_old + nopen >= B.max_clusters) {
                    overflow_sh = 1;
                    continue;
                }
                for (int a = 0; a < 3; ++a) opened[3 * nopen + a] = xj[a];
                B.opener[nopen] = j;
                ++nopen;
            }
            nopen_sh = nopen;
        }
        __syncthreads();
    }
    for (int t = tid; t < 3 * nopen_sh; t += blockDim.x) B.mu[3 * K_old + t] = opened[t];
    if (tid == 0) {
        B.state[1] = nopen_sh;
        B.state[2] |= overflow_sh;
    }
}

// Label of every point: its own new cluster if it opened one, else the best
// of its previous-pass cluster and the clusters opened at lower indices.
__global__ __launch_bounds__(kMgBlock) void k_assign(MgBufs B)
{
    const int K_old = B.state[0], nopen = B.state[1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double xi[3] = {B.x[3 * i], B.x[3 * i + 1], B.x[3 * i + 2]};
        double bs = B.best[i];
        int bc = B.bestc[i];
        int lab = -1;
        for (int k = 0; k < nopen; ++k) {
            const int32_t o = B.opener[k];
            if (o > i) break;
            if (o == i) {
                lab = K_old + k;
                break;
            }
            const double s = score(xi, B.mu + 3 * (K_old + k), B.spherical);
            if (better(s, bs, B.spherical)) {
                bs = s;
                bc = K_old + k;
            }
        }
        B.z[i] = lab >= 0 ? lab : bc;
    }
}

__global__ __launch_bounds__(kMgBlock) void k_sums(MgBufs B)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = B.z[i];
        atomicAdd(&B.cnt[c], 1ull);
        for (int a = 0; a < 3; ++a) atomicAdd(&B.sum[3 * c + a], B.x[3 * i + a]);
    }
}

// New centres from the sums, empty clusters removed in order; the old-to-new
// numbering goes to `opener` (reused: this pass's openers are no longer read).
__global__ void k_centres(MgBufs B)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int K = B.state[0] + B.state[1];
    int k2 = 0;
    for (int c = 0; c < K; ++c) {
        const unsigned long long n = B.cnt[c];
        if (n == 0) {
            B.opener[c] = -1;
            continue;
        }
        B.opener[c] = k2;
        const double sx = B.sum[3 * c], sy = B.sum[3 * c + 1], sz = B.sum[3 * c + 2];
        if (B.spherical) {
            const double nr = sqrt(sx * sx + sy * sy + sz * sz);
            B.mu[3 * k2] = sx / nr;
            B.mu[3 * k2 + 1] = sy / nr;
            B.mu[3 * k2 + 2] = sz / nr;
        } else {
            B.mu[3 * k2] = sx / (double)n;
            B.mu[3 * k2 + 1] = sy / (double)n;
            B.mu[3 * k2 + 2] = sz / (double)n;
        }
        B.cnt[k2] = n;
        B.sum[3 * k2] = sx;
        B.sum[3 * k2 + 1] = sy;
        B.sum[3 * k2 + 2] = sz;
        ++k2;
    }
    B.state[4] = k2;
}

__global__ __launch_bounds__(kMgBlock) void k_relabel(MgBufs B)
{
    int changed = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t z = B.opener[B.z[i]];
        B.z[i] = z;
        changed |= z != B.prev[i];
        B.prev[i] = z;
    }
    if (__ballot(changed) && (threadIdx.x & 63) == 0) atomicOr(&B.state[3], 1);
}

// Spread of each final cluster: sum of squared distances to its centre.
__global__ __launch_bounds__(kMgBlock) void k_spread(MgBufs B, double *acc)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = B.z[i];
        const double xi[3] = {B.x[3 * i], B.x[3 * i + 1], B.x[3 * i + 2]};
        const double a = xi[0] - B.mu[3 * c], b = xi[1] - B.mu[3 * c + 1], d = xi[2] - B.mu[3 * c + 2];
        atomicAdd(&acc[c], a * a + b * b + d * d);
    }
}

__device__ double a3(double k) { return k < 1e-6 ? k / 3.0 : 1.0 / tanh(k) - 1.0 / k; }

// Maximum-likelihood concentration of a vMF on S^2: the root of
// A3(k) = coth k - 1/k = rbar (A3 increases from 0 to 1), by bisection on
// [0, 2/(1 - rbar) + 1] (A3(k) >= 1 - 1/k there exceeds rbar) to a relative
// width of 1e-15; rbar >= 1 (one direction) gives +inf.
__device__ double vmf_kappa_ml(double rbar)
{
    if (!(rbar > 0.0)) return 0.0;
    if (rbar >= 1.0) return INFINITY;
    double lo = 0.0, hi = 2.0 / (1.0 - rbar) + 1.0;
    while (hi - lo > 1e-15 * hi) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (a3(mid) < rbar)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

// The fitted spread of each cluster: isotropic Gaussian sigma =
// sqrt(sum |x - mu|^2 / (3 n)); vMF concentration from rbar = |sum x| / n.
// clamp: sigma at least `clamp` (GMM), kappa at most `clamp` (vMF), so that
// single-point clusters give valid components.
__global__ void k_fit(MgBufs B, const double *acc, int K, double clamp, double *spread)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < K; c += gridDim.x * blockDim.x) {
        const double n = (double)B.cnt[c];
        if (B.spherical) {
            const double sx = B.sum[3 * c], sy = B.sum[3 * c + 1], sz = B.sum[3 * c + 2];
            spread[c] = fmin(vmf_kappa_ml(sqrt(sx * sx + sy * sy + sz * sz) / n), clamp);
        } else {
            spread[c] = fmax(sqrt(acc[c] / (3.0 * n)), clamp);
        }
    }
}

}  // namespace

// Run one clustering on device points x (n x 3) into device labels z.
// Host outputs: centres (K x 3), counts (K), spread (GMM: sigma, vMF:
// concentration), K, passes (negated when a pass wanted more than
// max_clusters clusters).
hipError_t dp_cluster(const double *x, int64_t n, double lambda, int spherical, int max_clusters, int max_passes,
                      double clamp, int32_t *z, std::vector<double> &centres, std::vector<int64_t> &counts,
                      std::vector<double> &spread, int &K_out, int &passes_out, hipStream_t st)
{
    const size_t mc = (size_t)max_clusters + 1;
    MgBufs B{};
    B.x = x;
    B.n = n;
    B.spherical = spherical;
    B.lambda = lambda;
    B.max_clusters = max_clusters;
    B.z = z;
    if (max_clusters < 1 || max_clusters > kMaxOpen || n < 1) return hipErrorInvalidValue;
    uint8_t *mem = nullptr;
    auto rnd = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bytes = rnd(4 * n) * 2 + rnd(8 * n) + rnd(n) + rnd(24 * mc) * 2 + rnd(8 * mc) * 3 + rnd(4 * mc) +
                         rnd(32);
    hipError_t e = hipMalloc((void **)&mem, bytes);
    if (e) return e;
    size_t at = 0;
    auto take = [&](size_t b) {
        uint8_t *p = mem + at;
        at += rnd(b);
        return p;
    };
    B.prev = (int32_t *)take(sizeof(int32_t) * n);
    B.best = (double *)take(sizeof(double) * n);
    B.bestc = (int32_t *)take(sizeof(int32_t) * n);
    B.cand = take(n);
    B.mu = (double *)take(sizeof(double) * 3 * mc);
    B.sum = (double *)take(sizeof(double) * 3 * mc);
    B.cnt = (unsigned long long *)take(sizeof(unsigned long long) * mc);
    B.opener = (int32_t *)take(sizeof(int32_t) * mc);
    B.state = (int *)take(sizeof(int) * 8);
    double *acc = (double *)take(sizeof(double) * mc);
    double *d_spread = (double *)take(sizeof(double) * mc);
    const int grid = (int)std::min<int64_t>((n + kMgBlock - 1) / kMgBlock, 4096);
    int st_h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int passes = 0, K = 1, overflow = 0;
    if (!e) e = hipMemsetAsync(B.sum, 0, sizeof(double) * 3, st);
    if (!e) e = hipMemsetAsync(B.state, 0, sizeof(int) * 8, st);
    if (!e) e = hipMemsetAsync(B.prev, 0xff, sizeof(int32_t) * n, st);
    if (!e) {
        hipLaunchKernelGGL(k_total, dim3(grid), dim3(kMgBlock), 0, st, B);
        hipLaunchKernelGGL(k_start, dim3(1), dim3(64), 0, st, B);
        e = hipGetLastError();
    }
    for (; !e && passes < max_passes;) {
        if ((e = hipMemsetAsync(B.sum, 0, sizeof(double) * 3 * mc, st)) ||
            (e = hipMemsetAsync(B.cnt, 0, sizeof(unsigned long long) * mc, st)) ||
            (e = hipMemsetAsync(B.state + 1, 0, sizeof(int) * 4, st)))
            break;
        hipLaunchKernelGGL(k_score_old, dim3(grid), dim3(kMgBlock), 0, st, B);
        hipLaunchKernelGGL(k_open, dim3(1), dim3(kOpenBlock), 0, st, B);
        hipLaunchKernelGGL(k_assign, dim3(grid), dim3(kMgBlock), 0, st, B);
        hipLaunchKernelGGL(k_sums, dim3(grid), dim3(kMgBlock), 0, st, B);
        hipLaunchKernelGGL(k_centres, dim3(1), dim3(64), 0, st, B);
        hipLaunchKernelGGL(k_relabel, dim3(grid), dim3(kMgBlock), 0, st, B);
        if ((e = hipGetLastError()) || (e = hipMemcpyAsync(st_h, B.state, sizeof st_h, hipMemcpyDeviceToHost, st)) ||
            (e = hipStreamSynchronize(st)))
            break;
        ++passes;
        K = st_h[4];
        overflow |= st_h[2];
        if ((e = hipMemcpyAsync(B.state, &K, sizeof(int), hipMemcpyHostToDevice, st))) break;
        if (!st_h[3]) break;
    }
    if (!e) e = hipMemsetAsync(acc, 0, sizeof(double) * mc, st);
    if (!e) {
        if (!spherical) hipLaunchKernelGGL(k_spread, dim3(grid), dim3(kMgBlock), 0, st, B, acc);
        hipLaunchKernelGGL(k_fit, dim3((K + 255) / 256), dim3(256), 0, st, B, acc, K, clamp, d_spread);
        e = hipGetLastError();
    }
    std::vector<unsigned long long> h_cnt(K);
    centres.assign(3 * (size_t)K, 0.0);
    spread.assign(K, 0.0);
    if (!e) e = hipMemcpyAsync(centres.data(), B.mu, sizeof(double) * 3 * K, hipMemcpyDeviceToHost, st);
    if (!e) e = hipMemcpyAsync(h_cnt.data(), B.cnt, sizeof(unsigned long long) * K, hipMemcpyDeviceToHost, st);
    if (!e) e = hipMemcpyAsync(spread.data(), d_spread, sizeof(double) * K, hipMemcpyDeviceToHost, st);
    if (!e) e = hipStreamSynchronize(st);
    (void)hipFree(mem);
    if (e) return e;
    counts.assign(h_cnt.begin(), h_cnt.end());
    K_out = K;
    passes_out = overflow ? -passes : passes;
    return hipSuccess;
}

}  // namespace gosma

namespace {

int mg_fail(gosma_ctx *ctx, int code, const char *msg)
{
    ctx->err = msg;
    return code;
}

bool on_device(const gosma_ctx *ctx, const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == ctx->device;
}

int mg_run(gosma_ctx *ctx, const double *x, int64_t n, double lambda, int spherical, int max_clusters, int max_passes,
           double clamp, int32_t *labels, double *centres, int64_t *counts, double *spread, int *K, int *passes,
           void *stream)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (!x || !labels || !centres || !counts || !spread || !K || !passes)
        return mg_fail(ctx, GOSMA_E_INVAL, "a required pointer is NULL");
    if (n < 1 || n > ((int64_t)1 << 30)) return mg_fail(ctx, GOSMA_E_INVAL, "n must be in [1, 2^30]");
    if (max_clusters < 1 || max_clusters > GOSMA_MAX_CLUSTERS)
        return mg_fail(ctx, GOSMA_E_INVAL, "max_clusters must be in [1, GOSMA_MAX_CLUSTERS]");
    if (max_passes < 1) return mg_fail(ctx, GOSMA_E_INVAL, "max_passes must be >= 1");
    if (!std::isfinite(lambda) || !(clamp > 0)) return mg_fail(ctx, GOSMA_E_INVAL, "lambda must be finite, the clamp > 0");
    hipError_t e = hipSetDevice(ctx->device);
    if (e) return mg_fail(ctx, GOSMA_E_HIP, hipGetErrorString(e));
    if (!on_device(ctx, x) || !on_device(ctx, labels))
        return mg_fail(ctx, GOSMA_E_INVAL, "points and labels must be device memory of the context's device");
    std::vector<double> mu, sp;
    std::vector<int64_t> cnt;
    int k = 0, p = 0;
    e = gosma::dp_cluster(x, n, lambda, spherical, max_clusters, max_passes, clamp, labels, mu, cnt, sp, k, p,
                          (hipStream_t)stream);
    if (e) return mg_fail(ctx, GOSMA_E_HIP, hipGetErrorString(e));
    std::copy(mu.begin(), mu.end(), centres);
    std::copy(cnt.begin(), cnt.end(), counts);
    std::copy(sp.begin(), sp.end(), spread);
    *K = k;
    *passes = p;
    return GOSMA_OK;
}

}  // namespace

extern "C" int gosma_dpmeans(gosma_ctx *ctx, const double *points, int64_t n, double lambda, int max_clusters,
                             int max_passes, double sigma_min, int32_t *labels, double *centres, int64_t *counts,
                             double *sigma, int *K, int *passes, void *stream)
{
    return mg_run(ctx, points, n, lambda, 0, max_clusters, max_passes, sigma_min, labels, centres, counts, sigma, K,
                  passes, stream);
}

extern "C" int gosma_dpvmf_means(gosma_ctx *ctx, const double *dirs, int64_t n, double cos_lambda, int max_clusters,
                                 int max_passes, double kappa_max, int32_t *labels, double *centres, int64_t *counts,
                                 double *kappa, int *K, int *passes, void *stream)
{
    return mg_run(ctx, dirs, n, cos_lambda, 1, max_clusters, max_passes, kappa_max, labels, centres, counts, kappa, K,
                  passes, stream);
}
