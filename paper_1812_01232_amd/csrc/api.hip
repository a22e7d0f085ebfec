// C-ABI entry points of libgosma: context, problem upload, bound evaluation.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "gosma_impl.h"

using gosma::ClassRange;
using gosma::ProbDesc;

namespace {

int fail(gosma_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

int hip_fail(gosma_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, GOSMA_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, call)                                 \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

// Launch shape used until gosma_set_tiles or gosma_autotune: more waves per
// cell for larger pair counts, and about 8,192 waves in the grid.
gosma::Tile default_tile(int64_t pairs)
{
    const int w = pairs <= 64 * 64 ? 1 : (pairs <= 128 * 128 ? 2 : 4);
    return gosma::Tile{w, 8192 / w};
}
// The search's GMM-GMM kernel runs over the iteration's distinct translation
// cells: from a few dozen (rotation splits share their parent's cell) to
// several thousand.  Blocks of at least two waves: while there are fewer
// cells than blocks, the waves of a block share a cell (its latency decides:
// on the 64x64 search 28 -> 22 us per launch over the first 25 iterations),
// and with more cells every wave takes a cell of its own.
gosma::Tile default_search_tile11(int64_t pairs)
{
    const gosma::Tile t = default_tile(pairs);
    return t.waves >= 2 ? t : gosma::Tile{2, 4096};
}

template <class T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void free_problems(gosma_ctx *ctx)
{
    dfree(ctx->d_mu);
    dfree(ctx->d_isig2);
    dfree(ctx->d_w1);
    dfree(ctx->d_pbar);
    dfree(ctx->d_vmf);
    dfree(ctx->d_cls);
    dfree(ctx->d_prob);
    dfree(ctx->d_grec);
    ctx->grec_stride = 0;
    ctx->n_problems = 0;
    ctx->h_prob.clear();
    ctx->gmm_order.clear();
    ctx->has_domain = false;
    ctx->snap_ready = false;
    ctx->resume.clear();
}

double log_Z(double x) { return x <= 0 ? std::log(2.0) : x + std::log(-std::expm1(-2.0 * x)) - std::log(x); }

template <class T>
hipError_t upload(T *&dst, const std::vector<T> &src)
{
    hipError_t e = hipMalloc((void **)&dst, sizeof(T) * std::max<size_t>(src.size(), 1));
    if (e != hipSuccess) return e;
    return hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

int check_domain(gosma_ctx *ctx, const gosma_domain *d)
{
    if (!d) return fail(ctx, GOSMA_E_INVAL, "domain is NULL");
    for (int k = 0; k < 3; ++k) {
        if (!(d->r_hi[k] > d->r_lo[k]) || !std::isfinite(d->r_lo[k]) || !std::isfinite(d->r_hi[k]))
            return fail(ctx, GOSMA_E_INVAL, "rotation box axis %d is empty or not finite", k);
        if (!(d->t_hi[k] > d->t_lo[k]) || !std::isfinite(d->t_lo[k]) || !std::isfinite(d->t_hi[k]))
            return fail(ctx, GOSMA_E_INVAL, "translation box axis %d is empty or not finite", k);
    }
    if (!(d->zeta >= 0) || !std::isfinite(d->zeta)) return fail(ctx, GOSMA_E_INVAL, "zeta must be >= 0");
    return GOSMA_OK;
}

void set_domain_desc(ProbDesc &P, const gosma_domain &d)
{
    for (int k = 0; k < 3; ++k) {
        P.r_lo[k] = d.r_lo[k];
        P.r_w[k] = d.r_hi[k] - d.r_lo[k];
        P.t_lo[k] = d.t_lo[k];
        P.t_w[k] = d.t_hi[k] - d.t_lo[k];
    }
    P.zeta = d.zeta;
}

// Scratch of gosma_eval_bounds_noalloc: a fixed device array holding, for
// up to GOSMA_NOALLOC_MAX_CUBES cubes, the S11 sums of each cube's
// translation cell and the pair kernel's per-cube set-up record.  Host code
// never uses the symbol itself as an address: gosma_create looks up the
// array's device address once per device (hipGetSymbolAddress) and every
// launch takes that pointer.
constexpr size_t kScratchAlign = 256;
constexpr size_t scratch_part(size_t bytes) { return (bytes + kScratchAlign - 1) / kScratchAlign * kScratchAlign; }
constexpr size_t kScratchBytes = 2 * scratch_part(sizeof(double) * GOSMA_NOALLOC_MAX_CUBES) +
                                 scratch_part(sizeof(gosma::CubeSetup) * GOSMA_NOALLOC_MAX_CUBES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchLayout {
    double *s11ub, *s11lo;
    gosma::CubeSetup *setup;
};
ScratchLayout scratch_layout(unsigned char *base, int64_t n)
{
    (void)n;   // the parts are laid out for the maximum, so a call's view does not depend on n
    const size_t part = scratch_part(sizeof(double) * GOSMA_NOALLOC_MAX_CUBES);
    return ScratchLayout{(double *)base, (double *)(base + part), (gosma::CubeSetup *)(base + 2 * part)};
}

// Device address of `scratch` per device, looked up once per device with
// that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int device, unsigned char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" {

int gosma_create(int device, gosma_ctx **out)
{
    if (!out) return GOSMA_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GOSMA_E_INVAL;
    gosma_ctx *ctx = new (std::nothrow) gosma_ctx;
    if (!ctx) return GOSMA_E_NOMEM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return GOSMA_E_HIP;
    }
    if (scratch_address(device, &ctx->d_scratch) != hipSuccess) {
        delete ctx;
        return GOSMA_E_HIP;
    }
    *out = ctx;
    return GOSMA_OK;
}

void gosma_release_solver(gosma_ctx *ctx);   // bb.hip
void gosma_drop_graph(gosma_ctx *ctx);       // bb.hip
void gosma_release_mlp(gosma_ctx *ctx);      // mlp.hip

void gosma_destroy(gosma_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    free_problems(ctx);
    dfree(ctx->d_s11ub);
    dfree(ctx->d_s11lo);
    dfree(ctx->d_setup);
    dfree(ctx->d_counts);
    dfree(ctx->d_stage);
    gosma_release_solver(ctx);
    gosma_release_mlp(ctx);
    delete ctx;
}

const char *gosma_last_error(const gosma_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int gosma_set_problems(gosma_ctx *ctx, int n_problems, const int64_t *gmm_off, const int64_t *vmf_off,
                       const double *mu, const double *sigma, const double *phi1, const int32_t *label1,
                       const double *dir2, const double *kappa2, const double *phi2, const int32_t *label2,
                       int n_labels, const gosma_domain *domains)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (n_problems < 1) return fail(ctx, GOSMA_E_INVAL, "n_problems must be >= 1");
    if (!gmm_off || !vmf_off || !mu || !sigma || !phi1 || !dir2 || !kappa2 || !phi2 || !domains)
        return fail(ctx, GOSMA_E_INVAL, "a required array is NULL");
    if ((label1 == nullptr) != (label2 == nullptr))
        return fail(ctx, GOSMA_E_INVAL, "label1 and label2 must both be NULL or both be set");
    const bool labelled = label1 != nullptr;
    if (labelled && (n_labels < 1 || n_labels > GOSMA_MAX_LABELS))
        return fail(ctx, GOSMA_E_INVAL, "n_labels must be in [1, %d]", GOSMA_MAX_LABELS);
    const int L = labelled ? n_labels : 1;
    if (gmm_off[0] != 0 || vmf_off[0] != 0) return fail(ctx, GOSMA_E_INVAL, "offsets must start at 0");
    for (int p = 0; p < n_problems; ++p) {
        int64_t M = gmm_off[p + 1] - gmm_off[p], N = vmf_off[p + 1] - vmf_off[p];
        if (M < 1 || M > GOSMA_MAX_COMPONENTS || N < 1 || N > GOSMA_MAX_COMPONENTS)
            return fail(ctx, GOSMA_E_INVAL, "problem %d: M=%lld N=%lld outside [1, %d]", p, (long long)M,
                        (long long)N, GOSMA_MAX_COMPONENTS);
        int rc = check_domain(ctx, domains + p);
        if (rc) return rc;
    }
    const int64_t TM = gmm_off[n_problems], TN = vmf_off[n_problems];
    for (int64_t i = 0; i < TM; ++i) {
        if (!std::isfinite(mu[3 * i]) || !std::isfinite(mu[3 * i + 1]) || !std::isfinite(mu[3 * i + 2]))
            return fail(ctx, GOSMA_E_INVAL, "GMM mean %lld is not finite", (long long)i);
        if (!(sigma[i] > 0) || !std::isfinite(sigma[i]))
            return fail(ctx, GOSMA_E_INVAL, "sigma[%lld] must be > 0", (long long)i);
        if (!(phi1[i] >= 0) || !std::isfinite(phi1[i]))
            return fail(ctx, GOSMA_E_INVAL, "phi1[%lld] must be >= 0", (long long)i);
        if (labelled && (label1[i] < 0 || label1[i] >= n_labels))
            return fail(ctx, GOSMA_E_INVAL, "label1[%lld] outside [0, n_labels)", (long long)i);
    }
    for (int64_t j = 0; j < TN; ++j) {
        double n2 = dir2[3 * j] * dir2[3 * j] + dir2[3 * j + 1] * dir2[3 * j + 1] + dir2[3 * j + 2] * dir2[3 * j + 2];
        if (!(std::fabs(std::sqrt(n2) - 1.0) <= 1e-6))
            return fail(ctx, GOSMA_E_INVAL, "dir2[%lld] is not a unit vector", (long long)j);
        if (!(kappa2[j] > 0) || !std::isfinite(kappa2[j]))
            return fail(ctx, GOSMA_E_INVAL, "kappa2[%lld] must be > 0", (long long)j);
        if (!(phi2[j] >= 0) || !std::isfinite(phi2[j]))
            return fail(ctx, GOSMA_E_INVAL, "phi2[%lld] must be >= 0", (long long)j);
        if (labelled && (label2[j] < 0 || label2[j] >= n_labels))
            return fail(ctx, GOSMA_E_INVAL, "label2[%lld] outside [0, n_labels)", (long long)j);
    }

    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // Every cell of a bound kernel (and every SMA start) stages its problem's
    // components in LDS while they fit; larger mixtures stage them in a global
    // buffer of kGrecBlocks per-block slices instead.
    bool use_grec = false;
    {
        int needM = 0, needN = 0, lds_max = 0;
        for (int p = 0; p < n_problems; ++p) {
            needM = std::max(needM, (int)(gmm_off[p + 1] - gmm_off[p]));
            needN = std::max(needN, (int)(vmf_off[p + 1] - vmf_off[p]));
        }
        HIP_TRY(ctx, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
        const size_t need = std::max({gosma::s11_lds_bytes(needM, gosma::kMaxWaves),
                                      gosma::s12_lds_bytes(needM, needN, gosma::kMaxWaves, n_problems > 1),
                                      gosma::sma_lds_bytes(needM, needN)}) + 2048;
        use_grec = need > (size_t)lds_max;
    }
    gosma_drop_graph(ctx);   // a captured iteration holds the old mixture pointers
    free_problems(ctx);
    std::vector<double> h_mu(3 * TM), h_isig2(TM);
    std::vector<float> h_w1(TM), h_pbar(TM);
    std::vector<float4> h_vmf(2 * TN);
    std::vector<ClassRange> h_cls;
    std::vector<ProbDesc> h_prob(n_problems);
    ctx->gmm_order.assign(n_problems, {});
    int maxM = 0, maxN = 0;
    const double phil_sqrt = std::sqrt(1.0 / L);
    for (int p = 0; p < n_problems; ++p) {
        const int64_t g0 = gmm_off[p], v0 = vmf_off[p];
        const int M = (int)(gmm_off[p + 1] - g0), N = (int)(vmf_off[p + 1] - v0);
        maxM = std::max(maxM, M);
        maxN = std::max(maxN, N);
        // sort rows by class (stable)
        std::vector<int32_t> og(M), ov(N);
        for (int i = 0; i < M; ++i) og[i] = i;
        for (int j = 0; j < N; ++j) ov[j] = j;
        if (labelled) {
            std::stable_sort(og.begin(), og.end(), [&](int a, int b) { return label1[g0 + a] < label1[g0 + b]; });
            std::stable_sort(ov.begin(), ov.end(), [&](int a, int b) { return label2[v0 + a] < label2[v0 + b]; });
        }
        std::vector<double> s1(L, 0.0), s2(L, 0.0);
        double ssum = 0.0;
        for (int i = 0; i < M; ++i) {
            s1[labelled ? label1[g0 + i] : 0] += phi1[g0 + i];
            ssum += phi1[g0 + i];
        }
        for (int j = 0; j < N; ++j) s2[labelled ? label2[v0 + j] : 0] += phi2[v0 + j];
        if (!(ssum > 0)) return fail(ctx, GOSMA_E_INVAL, "problem %d: GMM weights sum to 0", p);
        ProbDesc &P = h_prob[p];
        std::memset(&P, 0, sizeof P);
        P.gmm_off = (int32_t)g0;
        P.M = M;
        P.vmf_off = (int32_t)v0;
        P.N = N;
        P.cls_off = (int32_t)h_cls.size();
        P.n_cls = L;
        P.bucket = gosma::size_bucket(M, N);
        set_domain_desc(P, domains[p]);
        // class table
        {
            int gi = 0, vj = 0;
            for (int l = 0; l < L; ++l) {
                ClassRange cr;
                cr.g0 = (int32_t)(g0 + gi);
                while (gi < M && (labelled ? label1[g0 + og[gi]] : 0) == l) ++gi;
                cr.g1 = (int32_t)(g0 + gi);
                cr.v0 = (int32_t)(v0 + vj);
                while (vj < N && (labelled ? label2[v0 + ov[vj]] : 0) == l) ++vj;
                cr.v1 = (int32_t)(v0 + vj);
                h_cls.push_back(cr);
            }
        }
        for (int i = 0; i < M; ++i) {
            int src = og[i];
            int lab = labelled ? label1[g0 + src] : 0;
            int64_t dst = g0 + i;
            for (int k = 0; k < 3; ++k) h_mu[3 * dst + k] = mu[3 * (g0 + src) + k];
            h_isig2[dst] = 1.0 / (sigma[g0 + src] * sigma[g0 + src]);
            h_w1[dst] = s1[lab] > 0 ? (float)(phil_sqrt * phi1[g0 + src] / s1[lab]) : 0.0f;
            h_pbar[dst] = (float)(phi1[g0 + src] / ssum);
        }
        std::vector<double> w2(N), ks(N), dx(3 * N);
        std::vector<int> lab2(N);
        for (int j = 0; j < N; ++j) {
            int src = ov[j];
            int lab = labelled ? label2[v0 + src] : 0;
            int64_t dst = v0 + j;
            double k = kappa2[v0 + src];
            double nrm = std::sqrt(dir2[3 * (v0 + src)] * dir2[3 * (v0 + src)] +
                                   dir2[3 * (v0 + src) + 1] * dir2[3 * (v0 + src) + 1] +
                                   dir2[3 * (v0 + src) + 2] * dir2[3 * (v0 + src) + 2]);
            for (int a = 0; a < 3; ++a) dx[3 * j + a] = dir2[3 * (v0 + src) + a] / nrm;
            w2[j] = s2[lab] > 0 ? phil_sqrt * phi2[v0 + src] / s2[lab] : 0.0;
            ks[j] = k;
            lab2[j] = lab;
            double G = k / (-std::expm1(-2.0 * k));
            double coth = 1.0 + 2.0 / std::expm1(2.0 * k);
            h_vmf[2 * dst] = make_float4((float)dx[3 * j], (float)dx[3 * j + 1], (float)dx[3 * j + 2], (float)k);
            // ln(2 kappa) / 2 enters the far-apart cap of the upper term
            h_vmf[2 * dst + 1] = make_float4((float)w2[j], (float)G, (float)coth, (float)(0.5 * std::log(2.0 * k)));
        }

        // S22 (FP64, host): sum over same-class vMF pairs of w w' Z(K)/(Z Z)
        double S22 = 0.0;
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) {
                if (lab2[j] != lab2[k]) continue;
                double v[3];
                for (int a = 0; a < 3; ++a) v[a] = ks[j] * dx[3 * j + a] + ks[k] * dx[3 * k + a];
                double K = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                S22 += w2[j] * w2[k] * std::exp(log_Z(K) - log_Z(ks[j]) - log_Z(ks[k]));
            }
        P.S22 = S22;
        ctx->gmm_order[p] = og;
    }
    hipError_t e;
    if (!use_grec && (e = gosma::prepare_bound_kernels(maxM, maxN)) != hipSuccess)
        return hip_fail(ctx, e, "bound kernel LDS limit");
    if (use_grec) {
        const int64_t stride = gosma::grec_stride(maxM, maxN);
        if ((e = hipMalloc((void **)&ctx->d_grec, sizeof(float4) * stride * gosma::kGrecBlocks)) != hipSuccess) {
            ctx->d_grec = nullptr;
            free_problems(ctx);
            return fail(ctx, GOSMA_E_NOMEM, "global component records (%lld bytes): %s",
                        (long long)(sizeof(float4) * stride * gosma::kGrecBlocks), hipGetErrorString(e));
        }
        ctx->grec_stride = stride;
    }
    if ((e = upload(ctx->d_mu, h_mu)) != hipSuccess || (e = upload(ctx->d_isig2, h_isig2)) != hipSuccess ||
        (e = upload(ctx->d_w1, h_w1)) != hipSuccess || (e = upload(ctx->d_pbar, h_pbar)) != hipSuccess ||
        (e = upload(ctx->d_vmf, h_vmf)) != hipSuccess ||
        (e = upload(ctx->d_cls, h_cls)) != hipSuccess ||
        (e = upload(ctx->d_prob, h_prob)) != hipSuccess) {
        free_problems(ctx);
        return hip_fail(ctx, e, "uploading mixtures");
    }
    ctx->h_prob = h_prob;
    ctx->n_problems = n_problems;
    ctx->maxM = maxM;
    ctx->maxN = maxN;
    ctx->has_domain = true;
    ctx->tile11 = default_tile((int64_t)maxM * maxM / 2);
    ctx->tile12 = default_tile((int64_t)maxM * maxN);
    for (int b = 0; b < gosma::kBuckets; ++b) ctx->bucket_nprob[b] = ctx->bucket_maxM[b] = ctx->bucket_maxN[b] = 0;
    for (const ProbDesc &P : h_prob) {
        ++ctx->bucket_nprob[P.bucket];
        ctx->bucket_maxM[P.bucket] = std::max(ctx->bucket_maxM[P.bucket], (int)P.M);
        ctx->bucket_maxN[P.bucket] = std::max(ctx->bucket_maxN[P.bucket], (int)P.N);
    }
    for (int b = 0; b < gosma::kBuckets; ++b) {
        const int64_t m = ctx->bucket_maxM[b], n = ctx->bucket_maxN[b];
        ctx->btile11[b] = default_search_tile11(m * m / 2);
        ctx->btile12[b] = default_tile(m * n);
    }
    return GOSMA_OK;
}

int gosma_set_mixtures(gosma_ctx *ctx, int M, const double *mu, const double *sigma, const double *phi1,
                       const int32_t *label1, int N, const double *dir2, const double *kappa2, const double *phi2,
                       const int32_t *label2, int n_labels)
{
    if (!ctx) return GOSMA_E_INVAL;
    int64_t go[2] = {0, M}, vo[2] = {0, N};
    gosma_domain d;
    bool had = ctx->has_domain && ctx->n_problems == 1;
    if (had) {
        const ProbDesc &P = ctx->h_prob[0];
        for (int k = 0; k < 3; ++k) {
            d.r_lo[k] = P.r_lo[k];
            d.r_hi[k] = P.r_lo[k] + P.r_w[k];
            d.t_lo[k] = P.t_lo[k];
            d.t_hi[k] = P.t_lo[k] + P.t_w[k];
        }
        d.zeta = P.zeta;
    } else {
        // placeholder domain until gosma_set_domain is called
        for (int k = 0; k < 3; ++k) {
            d.r_lo[k] = -M_PI;
            d.r_hi[k] = M_PI;
            d.t_lo[k] = -1.0;
            d.t_hi[k] = 1.0;
        }
        d.zeta = 0.0;
    }
    int rc = gosma_set_problems(ctx, 1, go, vo, mu, sigma, phi1, label1, dir2, kappa2, phi2, label2, n_labels, &d);
    if (rc == GOSMA_OK) ctx->has_domain = had;
    return rc;
}

int gosma_set_domain(gosma_ctx *ctx, const gosma_domain *domain)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (ctx->n_problems != 1) return fail(ctx, GOSMA_E_STATE, "gosma_set_domain needs exactly one problem set");
    int rc = check_domain(ctx, domain);
    if (rc) return rc;
    set_domain_desc(ctx->h_prob[0], *domain);
    ctx->snap_ready = false;   // the solver's queue belongs to the old domain
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemcpy(ctx->d_prob, ctx->h_prob.data(), sizeof(ProbDesc), hipMemcpyHostToDevice));
    ctx->has_domain = true;
    return GOSMA_OK;
}

int gosma_get_S22(gosma_ctx *ctx, int problem, double *S22)
{
    if (!ctx || !S22) return GOSMA_E_INVAL;
    if (problem < 0 || problem >= ctx->n_problems) return fail(ctx, GOSMA_E_INVAL, "no problem %d", problem);
    *S22 = ctx->h_prob[problem].S22;
    return GOSMA_OK;
}

// Where an argument of gosma_eval_bounds lives: memory of the context's
// device (used in place), host memory of any kind (staged), or memory of
// another device (rejected).
enum class Where { device, host, other };
static Where where_is(const gosma_ctx *ctx, const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();   // not known to HIP: plain host memory
        return Where::host;
    }
    if (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged)
        return a.device == ctx->device ? Where::device : Where::other;
    return Where::host;
}

int gosma_eval_bounds(gosma_ctx *ctx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *problem,
                      int64_t n, double *ub, double *lb, uint8_t *flags, double *aux, float *top8, void *stream)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (ctx->n_problems < 1 || !ctx->has_domain)
        return fail(ctx, GOSMA_E_STATE, "set mixtures and a domain before evaluating bounds");
    if (n < 0) return fail(ctx, GOSMA_E_INVAL, "n must be >= 0");
    if (n == 0) return GOSMA_OK;
    if (!rkeys || !tkeys || !ub || !lb || !flags) return fail(ctx, GOSMA_E_INVAL, "a required pointer is NULL");
    if (n > (int64_t)0x7fffffff) return fail(ctx, GOSMA_E_INVAL, "n exceeds the launch limit");
    if (!problem && ctx->n_problems != 1)
        return fail(ctx, GOSMA_E_INVAL, "problem indices are required when several problems are set");
    if (ctx->kpieces > 1 && (top8 || ctx->d_grec))
        return fail(ctx, GOSMA_E_INVAL, "kappa pieces > 1 need top8 == NULL and mixtures whose records fit LDS");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;

    // host arrays go through device copies: inputs before the launches,
    // outputs after them, then the call waits for the copies
    struct Arg {
        void *user;
        size_t bytes;
        bool in;
        void *dev;
    } args[8] = {{(void *)rkeys, 8, true, nullptr},  {(void *)tkeys, 8, true, nullptr},
                 {(void *)problem, 4, true, nullptr}, {(void *)ub, 8, false, nullptr},
                 {(void *)lb, 8, false, nullptr},     {(void *)flags, 1, false, nullptr},
                 {(void *)aux, 32, false, nullptr},   {(void *)top8, 32, false, nullptr}};
    size_t stage = 0;
    for (Arg &a : args) {
        a.bytes *= (size_t)n;
        if (!a.user) continue;
        const Where w = where_is(ctx, a.user);
        if (w == Where::other) return fail(ctx, GOSMA_E_INVAL, "an array is device memory of another device");
        if (w == Where::host) stage += (a.bytes + 255) & ~(size_t)255;
    }
    if (stage > ctx->stage_cap) {
        dfree(ctx->d_stage);
        ctx->stage_cap = 0;
        HIP_TRY(ctx, hipMalloc((void **)&ctx->d_stage, stage));
        ctx->stage_cap = stage;
    }
    {
        size_t at = 0;
        for (Arg &a : args) {
            if (!a.user) continue;
            if (where_is(ctx, a.user) != Where::host) {
                a.dev = a.user;
                continue;
            }
            a.dev = ctx->d_stage + at;
            at += (a.bytes + 255) & ~(size_t)255;
            if (a.in) HIP_TRY(ctx, hipMemcpyAsync(a.dev, a.user, a.bytes, hipMemcpyHostToDevice, s));
        }
    }
    rkeys = (const uint64_t *)args[0].dev;
    tkeys = (const uint64_t *)args[1].dev;
    problem = (const uint32_t *)args[2].dev;
    ub = (double *)args[3].dev;
    lb = (double *)args[4].dev;
    flags = (uint8_t *)args[5].dev;
    aux = (double *)args[6].dev;
    top8 = (float *)args[7].dev;

    if (ctx->s11_cap < n) {
        dfree(ctx->d_s11ub);
        dfree(ctx->d_s11lo);
        dfree(ctx->d_setup);
        ctx->s11_cap = 0;
        HIP_TRY(ctx, hipMalloc((void **)&ctx->d_s11ub, sizeof(double) * n));
        HIP_TRY(ctx, hipMalloc((void **)&ctx->d_s11lo, sizeof(double) * n));
        HIP_TRY(ctx, hipMalloc((void **)&ctx->d_setup, sizeof(gosma::CubeSetup) * n));
        ctx->s11_cap = n;
    }
    gosma::DevMix mx = ctx->mix();
    int ti = ctx->time_begin(GOSMA_KERNEL_S11, s);
    gosma::S11Out o11{ctx->d_s11ub, ctx->d_s11lo, ctx->timing ? ctx->d_counts : nullptr};
    HIP_TRY(ctx, gosma::launch_s11(mx, tkeys, problem, n, nullptr, o11, ctx->maxM, ctx->tile11, s));
    ctx->time_end(ti, s);
    gosma::BoundOut out{ub, lb, nullptr, aux, flags, top8, nullptr, nullptr, 0, nullptr};
    if (ctx->timing) out.counts = ctx->d_counts;
    ti = ctx->time_begin(GOSMA_KERNEL_S12, s);
    HIP_TRY(ctx, gosma::launch_s12(mx, rkeys, tkeys, problem, nullptr, ctx->d_s11ub, ctx->d_s11lo, n, nullptr, 1, out,
                                   0.0, ctx->maxM, ctx->maxN, top8 != nullptr, ctx->tile12, ctx->d_setup, s, false,
                                   gosma::TransRecs{}, ctx->kpieces));
    ctx->time_end(ti, s);
    if (stage) {
        for (const Arg &a : args)
            if (a.user && !a.in && a.dev != a.user)
                HIP_TRY(ctx, hipMemcpyAsync(a.user, a.dev, a.bytes, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
    }
    return GOSMA_OK;
}

int gosma_eval_bounds_noalloc(gosma_ctx *ctx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *problem,
                              int64_t n, double *ub, double *lb, uint8_t *flags, double *aux, float *top8,
                              void *stream)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (ctx->n_problems < 1 || !ctx->has_domain)
        return fail(ctx, GOSMA_E_STATE, "set mixtures and a domain before evaluating bounds");
    if (n < 0) return fail(ctx, GOSMA_E_INVAL, "n must be >= 0");
    if (n > GOSMA_NOALLOC_MAX_CUBES)
        return fail(ctx, GOSMA_E_INVAL, "n = %lld exceeds GOSMA_NOALLOC_MAX_CUBES (%d), the capacity of the "
                    "library's fixed scratch array", (long long)n, GOSMA_NOALLOC_MAX_CUBES);
    if (n == 0) return GOSMA_OK;
    if (!rkeys || !tkeys || !ub || !lb || !flags) return fail(ctx, GOSMA_E_INVAL, "a required pointer is NULL");
    if (!problem && ctx->n_problems != 1)
        return fail(ctx, GOSMA_E_INVAL, "problem indices are required when several problems are set");
    if (!ctx->d_scratch) return fail(ctx, GOSMA_E_STATE, "the scratch array of this device is not available");
    if (ctx->kpieces > 1 && (top8 || ctx->d_grec))
        return fail(ctx, GOSMA_E_INVAL, "kappa pieces > 1 need top8 == NULL and mixtures whose records fit LDS");
    const void *ptrs[8] = {rkeys, tkeys, problem, ub, lb, flags, aux, top8};
    for (const void *q : ptrs)
        if (q && where_is(ctx, q) != Where::device)
            return fail(ctx, GOSMA_E_INVAL, "every array must be device memory of the context's device");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // the scratch array's address on this device (from hipGetSymbolAddress at
    // gosma_create), carved into the per-cube S11 sums and set-up records;
    // every element used is written by this call's kernels before it is read
    const ScratchLayout L = scratch_layout(ctx->d_scratch, n);
    gosma::DevMix mx = ctx->mix();
    gosma::S11Out o11{L.s11ub, L.s11lo, nullptr};
    HIP_TRY(ctx, gosma::launch_s11(mx, tkeys, problem, n, nullptr, o11, ctx->maxM, ctx->tile11, s));
    gosma::BoundOut out{ub, lb, nullptr, aux, flags, top8, nullptr, nullptr, 0, nullptr};
    HIP_TRY(ctx, gosma::launch_s12(mx, rkeys, tkeys, problem, nullptr, L.s11ub, L.s11lo, n, nullptr, 1, out, 0.0,
                                   ctx->maxM, ctx->maxN, top8 != nullptr, ctx->tile12, L.setup, s, false,
                                   gosma::TransRecs{}, ctx->kpieces));
    return GOSMA_OK;
}

int gosma_set_kappa_pieces(gosma_ctx *ctx, int m)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (m != 1 && m != 2 && m != 4) return fail(ctx, GOSMA_E_INVAL, "kappa pieces must be 1, 2 or 4 (got %d)", m);
    ctx->kpieces = m;
    gosma_drop_graph(ctx);   // a captured search iteration holds the old kernels
    return GOSMA_OK;
}

int gosma_get_kappa_pieces(const gosma_ctx *ctx)
{
    return ctx ? ctx->kpieces : GOSMA_E_INVAL;
}

int gosma_refine(gosma_ctx *ctx, int64_t n, const uint32_t *problem, const double *r0, const double *t0,
                 int max_iters, double *r_out, double *t_out, double *f_out, double *grad_out, int32_t *iters_out)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (ctx->n_problems < 1 || !ctx->has_domain)
        return fail(ctx, GOSMA_E_STATE, "set mixtures and a domain before refining poses");
    if (n < 0 || max_iters < 0) return fail(ctx, GOSMA_E_INVAL, "n and max_iters must be >= 0");
    if (n == 0) return GOSMA_OK;
    if (!r0 || !t0 || !r_out || !t_out || !f_out || !iters_out)
        return fail(ctx, GOSMA_E_INVAL, "a required pointer is NULL");
    if (!problem && ctx->n_problems != 1)
        return fail(ctx, GOSMA_E_INVAL, "problem indices are required when several problems are set");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    std::vector<double> x0(6 * (size_t)n);
    for (int64_t s = 0; s < n; ++s)
        for (int a = 0; a < 3; ++a) {
            x0[6 * s + a] = r0[3 * s + a];
            x0[6 * s + 3 + a] = t0[3 * s + a];
        }
    // one device block: starts, problem indices, poses, values, gradients, iterations
    const size_t b_x = sizeof(double) * 6 * n, b_p = (sizeof(uint32_t) * n + 255) & ~(size_t)255;
    const size_t b_f = (sizeof(double) * n + 255) & ~(size_t)255, b_i = sizeof(int32_t) * n;
    const size_t bytes = 3 * ((b_x + 255) & ~(size_t)255) + b_p + b_f + b_i;
    uint8_t *buf = nullptr;
    HIP_TRY(ctx, hipMalloc((void **)&buf, bytes));
    double *d_x0 = (double *)buf, *d_x = (double *)(buf + ((b_x + 255) & ~(size_t)255));
    double *d_g = (double *)(buf + 2 * ((b_x + 255) & ~(size_t)255));
    uint32_t *d_p = (uint32_t *)(buf + 3 * ((b_x + 255) & ~(size_t)255));
    double *d_f = (double *)((uint8_t *)d_p + b_p);
    int32_t *d_it = (int32_t *)((uint8_t *)d_f + b_f);
    hipError_t e = hipMemcpy(d_x0, x0.data(), b_x, hipMemcpyHostToDevice);
    if (e == hipSuccess && problem) e = hipMemcpy(d_p, problem, sizeof(uint32_t) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = gosma::launch_sma(ctx->mix(), ctx->maxM, ctx->maxN, n, problem ? d_p : nullptr, d_x0, max_iters,
                              gosma::kSmaMemory, gosma::kSmaGtol, gosma::kSmaFtol, d_x, d_f, d_g, d_it, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<double> hx(6 * (size_t)n), hg(grad_out ? 6 * (size_t)n : 0);
    if (e == hipSuccess) e = hipMemcpy(hx.data(), d_x, b_x, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(f_out, d_f, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(iters_out, d_it, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && grad_out) e = hipMemcpy(grad_out, d_g, b_x, hipMemcpyDeviceToHost);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(ctx, e, "gosma_refine");
    for (int64_t s = 0; s < n; ++s)
        for (int a = 0; a < 3; ++a) {
            r_out[3 * s + a] = hx[6 * s + a];
            t_out[3 * s + a] = hx[6 * s + 3 + a];
        }
    return GOSMA_OK;
}

int gosma_set_record_sink(gosma_ctx *ctx, float *records, int64_t capacity, unsigned long long *count)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (capacity < 0 || (capacity > 0 && !records) || (records && !count)) {
        ctx->err = "record sink: records and count must both be set, capacity >= 0";
        return GOSMA_E_INVAL;
    }
    gosma_drop_graph(ctx);    // a captured iteration holds the old sink
    ctx->rec_sink = records;
    ctx->rec_cap = capacity;
    ctx->rec_count = count;
    return GOSMA_OK;
}

int gosma_set_timing(gosma_ctx *ctx, int enable)
{
    if (!ctx) return GOSMA_E_INVAL;
    ctx->err.clear();
    if (enable && !ctx->d_counts) {
        const size_t bytes = (size_t)gosma::kCountSlots * gosma::kCounters * sizeof(unsigned long long);
        HIP_TRY(ctx, hipSetDevice(ctx->device));
        HIP_TRY(ctx, hipMalloc((void **)&ctx->d_counts, bytes));
        HIP_TRY(ctx, hipMemset(ctx->d_counts, 0, bytes));
    }
    ctx->timing = enable != 0;
    return GOSMA_OK;
}

int gosma_get_work_counts(gosma_ctx *ctx, int64_t *counts)
{
    if (!ctx || !counts) return GOSMA_E_INVAL;
    ctx->err.clear();
    for (int c = 0; c < GOSMA_N_COUNTS; ++c) counts[c] = 0;
    if (!ctx->d_counts) return GOSMA_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    unsigned long long h[gosma::kCountSlots * gosma::kCounters];
    HIP_TRY(ctx, hipMemcpy(h, ctx->d_counts, sizeof h, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemset(ctx->d_counts, 0, sizeof h));
    for (int k = 0; k < gosma::kCountSlots; ++k)
        for (int c = 0; c < GOSMA_N_COUNTS; ++c) counts[c] += (int64_t)h[gosma::kCounters * k + c];
    return GOSMA_OK;
}

int gosma_get_timing(gosma_ctx *ctx, double *ms, int64_t *launches)
{
    if (!ctx || !ms || !launches) return GOSMA_E_INVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    for (int k = 0; k < GOSMA_N_KERNELS; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    int rc = GOSMA_OK;
    for (auto &e : ctx->tev) {
        float t = 0.0f;
        hipError_t err = hipEventSynchronize(e.second.second);
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e.second.first, e.second.second);
        if (err != hipSuccess && rc == GOSMA_OK) rc = hip_fail(ctx, err, "reading kernel timing events");
        ms[e.first] += t;
        launches[e.first] += 1;
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    ctx->tev.clear();
    return rc;
}

}  // extern "C"

int gosma_ctx::time_begin(int kind, hipStream_t s)
{
    if (!timing) return -1;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1;
    }
    (void)hipEventRecord(a, s);
    tev.push_back({kind, {a, b}});
    return (int)tev.size() - 1;
}

void gosma_ctx::time_end(int idx, hipStream_t s)
{
    if (idx >= 0) (void)hipEventRecord(tev[idx].second.second, s);
}
