// Bound evaluation kernels for GOSMA sub-cubes on CDNA4 (gfx950).
//
// For a rotation x translation sub-cube C_r x C_t the bounds of Theorem 1
// (Section 5.2) are sums over component pairs:
//   upper bound (eq. 20):  S11(t0) - 2 S12(R_r0, t0), the objective of Lemma 1
//                          (eqs. 10-13) at the cube centre;
//   lower bound (eq. 21):  sum over GMM pairs of a lower bound on each summand
//                          over the cube, minus 2 x the sum over GMM-vMF pairs
//                          of an upper bound on each summand, with the angles
//                          A (eq. 24) and B (eq. 25) built from the uncertainty
//                          angles of Lemmas 2-3.
// S11 depends on the translation cell only, so it is evaluated once per
// translation cell (k_s11) and shared by every rotation cell paired with it;
// k_s12 evaluates the GMM-vMF sums and combines.
//
// Work mapping: one block of 64 x W threads per cell (W = 1, 2 or 4, the
// launch shape chosen by the autotuner; k_s11 lets each wave take a cell of
// its own once there are more cells than blocks).  The per-component
// quantities of the cell (kappa, its interval over the cell, uncertainty
// half-angles, rotated directions, normaliser factors) are computed in FP64,
// one component per thread (in the search, k_s12 reads the translation part
// from records that k_s11 writes once per distinct translation cell), and
// staged in LDS as one FP32 record per component (four float4,
// padded to 80 bytes so that neighbouring records fall on distinct banks),
// read back with 16-byte loads.  The pair sums then run over the (i, j) rectangle
// of each class: when the class's vMF count divides the block or is a
// multiple of it, each thread keeps one vMF row in registers and walks the
// GMM rows (the same row for the whole wave when the count is a multiple, so
// the LDS reads are broadcasts); otherwise the rectangle is flattened with
// 64 x W consecutive pairs per step.  Terms are FP32 in log space, summed in
// FP32 over runs of 8 per thread and the runs in FP64; waves combine in LDS.
//
// Summand algebra.  With G(y) = y / (1 - e^{-2y}) and h(K) = (1 - e^{-2K})/K,
//   Z(K) / (Z(a) Z(b)) = e^{K - a - b} h(K) G(a) G(b)            (eq. 2)
// and K - a - b = -a b q / (K + a + b) for the squared chord q = |u - v|^2 of
// the two directions (K^2 = (a + b)^2 - a b q), which avoids the cancellation
// of K - a - b for concentrations in the thousands.
#include <algorithm>
#include <cmath>

#include "cube_core.h"
#include "gosma_impl.h"

namespace gosma {

namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

// sin and cos of x in [0, pi/2] in FP32: Maclaurin series through x^13 and
// x^14 in nested form (truncation below 1e-9).
__device__ __forceinline__ void sincos_half(float x, float *s, float *c)
{
    const float x2 = x * x;
    float ts = 1.0f, tc = 1.0f;
#pragma unroll
    for (int k = 7; k >= 1; --k) {
        ts = fmaf(-x2 * (1.0f / ((2.0f * k) * (2.0f * k + 1.0f))), ts, 1.0f);
        tc = fmaf(-x2 * (1.0f / ((2.0f * k - 1.0f) * (2.0f * k))), tc, 1.0f);
    }
    *s = x * ts;
    *c = tc;
}

// Order-preserving map of a double onto unsigned 64-bit integers.
__device__ __forceinline__ unsigned long long ordered_bits(double x)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ float wave_sumf(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
// Orders this wave's LDS accesses before and after the call (LDS operations
// of one wave complete in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_or(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v;
}

// Per-component translation quantities for one translation cell, FP64.
struct TransPrep {
    double u[3];          // (mu - t0)/|mu - t0|
    double kap;           // kappa_1i(t0), eq. 13
    double klo, ac, ha;   // kappa interval over the feasible cell: [klo, klo + 2 ha], centre ac
    double cps, sps;      // cos, sin of psi_t / 2 (Lemma 3, guarded)
    float psi;            // psi_t itself (for the branching rule)
    bool drop, ub_inf;    // cell inside the zeta ball of this mean; centre inside it
};

// Lemma 3's half-angle record of a component for a translation cell:
// {cos, sin of psi_t / 2, psi_t, 0}, computed by lemma3_record.  The search
// computes it once per distinct translation cell (k_s11) and the pair kernel
// reads it instead of recomputing it per cube.
__device__ float4 lemma3_record(const double c[3], double rho2, const double tau[3], bool inside);

// The interval part of trans_prep (everything but Lemma 3); *inside: mu lies
// in the cell (then psi_t = pi).
__device__ TransPrep trans_interval(const double *mu, double isig2, const double t0[3], const double tau[3],
                                    double zeta, double c_out[3], double *rho2_out, bool *inside_out)
{
    TransPrep o;
    double c[3] = {mu[0] - t0[0], mu[1] - t0[1], mu[2] - t0[2]};
    double rho2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    double rho = sqrt(rho2);
    const double irho = 1.0 / rho;
    for (int k = 0; k < 3; ++k) o.u[k] = c[k] * irho;
    o.kap = rho2 * isig2 + 1.0;
    // distance interval from mu to the cell: [max(zeta, dist to box), farthest vertex]
    double dmin2 = 0.0, dmax2 = 0.0, width = 0.0;
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
        double a = fabs(c[k]);
        double e = a - tau[k];
        double f = a + tau[k];
        dmax2 += f * f;
        if (e > 0.0) {
            dmin2 += e * e;
            width += 4.0 * a * tau[k];      // f^2 - e^2 without cancellation
            inside = false;
        } else {
            width += f * f;
        }
    }
    double z2 = zeta * zeta;
    o.drop = dmax2 < z2;
    o.ub_inf = rho2 < z2;
    if (dmin2 < z2) {
        dmin2 = z2;
        width = dmax2 - z2;
    }
    o.klo = dmin2 * isig2 + 1.0;
    o.ha = 0.5 * width * isig2;
    o.ac = o.klo + o.ha;

    for (int k = 0; k < 3; ++k) c_out[k] = c[k];
    *rho2_out = rho2;
    *inside_out = inside;
    return o;
}

__device__ float4 lemma3_record(const double c[3], double rho2, const double tau[3], bool inside)
{
    // psi_t: largest vertex angle between mu - v and mu - t0 (Lemma 3); pi if
    // mu is in the cell or any vertex angle exceeds pi/2.  For angles below
    // pi/2 the largest angle has the largest sine, |c x (s tau)|^2 / (|a|^2 |c|^2)
    // with a = c - s tau, computed without cancellation.  FP32 (the angle
    // enters the bound through FP32 records): the sines are compared as
    // fractions by cross-multiplication, and only the largest is divided out.
    bool guard = inside;
    const float cf[3] = {(float)c[0], (float)c[1], (float)c[2]};
    const float tf[3] = {(float)tau[0], (float)tau[1], (float)tau[2]};
    const float rho2f = (float)rho2;
    float bn = -1.0f, bd = 1.0f, bdot = 1.0f;   // largest sine^2 = bn / bd, its cosine's numerator
#pragma unroll 1   // sequential: keeps the set-up's register footprint small
    for (int v = 0; v < 8; ++v) {
        const float st[3] = {(v & 4) ? tf[0] : -tf[0], (v & 2) ? tf[1] : -tf[1], (v & 1) ? tf[2] : -tf[2]};
        const float a[3] = {cf[0] - st[0], cf[1] - st[1], cf[2] - st[2]};
        const float a2 = fmaf(a[0], a[0], fmaf(a[1], a[1], a[2] * a[2]));
        const float dot = rho2f - fmaf(st[0], cf[0], fmaf(st[1], cf[1], st[2] * cf[2]));
        const float cr[3] = {cf[1] * st[2] - cf[2] * st[1], cf[2] * st[0] - cf[0] * st[2], cf[0] * st[1] - cf[1] * st[0]};
        const float num = fmaf(cr[0], cr[0], fmaf(cr[1], cr[1], cr[2] * cr[2]));
        const float den = a2 * rho2f;
        if (dot < 0.0f) guard = true;
        if (num * bd > bn * den) {
            bn = num;
            bd = den;
            bdot = dot;
        }
    }
    if (guard) return make_float4(0.0f, 1.0f, (float)kPi, 0.0f);
    // sine and cosine of the angle from |c x s tau|^2 and (a . c)^2 over the same denominator
    const float nrm = frcp(fsqrt(bn + bdot * bdot));
    const float sp = fsqrt(bn) * nrm, cp = fabsf(bdot) * nrm;
    const float cps = fsqrt(0.5f * (1.0f + cp));
    return make_float4(cps, sp * frcp(2.0f * cps), atan2f(sp, cp), 0.0f);
}

__device__ __forceinline__ void apply_lemma3(TransPrep &o, const float4 r)
{
    o.cps = r.x;
    o.sps = r.y;
    o.psi = r.z;
}

// Functions of one concentration y >= 1 (every kappa here is at least 1),
// in FP32 because they are stored in FP32: with e = e^{-2y} and d = 1 - e
// (d >= 0.86, so no cancellation), G(y) = y / d, coth y = (1 + e) / d and
// nu(y) = 1 - L(y) = 1 + 1/y - coth y = 1/y - 2 e / d, where L is the
// derivative of log Z.
struct YFun {
    float G, coth, nu;
};

__device__ __forceinline__ YFun yfun(double y64)
{
    const float y = (float)y64;
    const float e = fexp2(-2.0f * kLog2e * y);
    const float id = frcp(1.0f - e);
    YFun o;
    o.G = y * id;
    o.coth = (1.0f + e) * id;
    o.nu = frcp(y) - 2.0f * e * id;
    return o;
}

// The record of a component for a translation cell (see TransRec), from its
// interval set-up tp, its weight w and the functions of kappa and klo; the
// values are the ones the pair kernel computes from the same inputs.
__device__ __forceinline__ TransRec trans_record(const TransPrep &tp, float w, const YFun &fk, const YFun &fl)
{
    TransRec r;
    r.u[0] = tp.u[0];
    r.u[1] = tp.u[1];
    r.u[2] = tp.u[2];
    const double ahi = tp.klo + 2.0 * tp.ha;
    const YFun fh = yfun(ahi);
    r.kap = (float)tp.kap;
    r.klo = (float)tp.klo;
    r.ahi = (float)ahi;
    r.ha = (float)tp.ha;
    r.cps = (float)tp.cps;
    r.sps = (float)tp.sps;
    r.psi = tp.psi;
    r.Gk = fk.G;
    r.cothl = fl.coth;
    r.Gl = fl.G;
    r.Gh = fh.G;
    r.nul = fl.nu;
    r.nuh = fh.nu;
    r.hla = 0.5f * kLn2 * __builtin_amdgcn_logf((float)tp.klo);
    r.lam = fmaxf(__builtin_amdgcn_logf(w * fh.G) * kLn2 - r.hla, -100.0f);
    r.ia = frcp((float)tp.klo);
    r.pad = 0.0f;
    return r;
}

// yfun for an FP32 concentration (interior points of a kappa interval).
__device__ __forceinline__ void yfun_f(float y, float *G, float *nu)
{
    const float e = fexp2(-2.0f * kLog2e * y);
    const float id = frcp(1.0f - e);
    *G = y * id;
    *nu = frcp(y) - 2.0f * e * id;
}

// Pair kernel pieces for concentrations a, b and squared chord q.
struct PairK {
    float ks;     // K^2
    float x;      // K - a - b
    float K, r;   // K and 1 / (K (K + a + b))
    float invK;   // 1 / K
    float hK;     // (1 - e^{-2K}) / K
    float nuK;    // 1 + 1/K - coth K
};

// min(a, b) as the median of a, b and -infinity (v_med3_f32), with the
// infinity passed in a kernel argument so that the compiler keeps the median:
// the same value as fminf(a, b) for operands that are not NaN, in one
// instruction where fminf spends up to two more quieting operands it cannot
// prove canonical (values read from memory, or merged across branches).
__device__ __forceinline__ float fmin_med3(float a, float b, float inf)
{
    return __builtin_amdgcn_fmed3f(a, b, -inf);
}

// Below this K, e^{-2K} is not negligible next to 1 in FP32.
constexpr float kSmallK = 9.0f;

// The PairK terms that hold for K >= kSmallK (h(K) / K and nu(K) taken as 1 / K).
__device__ __forceinline__ PairK pair_k_large(float a, float b, float q)
{
    PairK o;
    const float s = a + b;
    const float t = a * b * q;
    // K^2 = (a + b)^2 - a b q, kept off zero for the reciprocal square root
    o.ks = fmaxf(fmaf(s, s, -t), 1e-36f);
    const float iK = __builtin_amdgcn_rsqf(o.ks);   // 1 / K
    const float K = o.ks * iK;
    const float rd = frcp(K + s);                   // 1 / (K + a + b)
    o.K = K;
    o.r = iK * rd;
    o.x = -t * rd;                                  // K - a - b without cancellation
    o.invK = iK;
    o.hK = iK;
    o.nuK = iK;
    return o;
}

// The terms with e^{-2K} for K < kSmallK.
__device__ __forceinline__ void pair_k_small(PairK &o)
{
    const float K = o.K;
    if (__builtin_expect(K < kSmallK, 0)) {
        float e = fexp2(-2.0f * kLog2e * K);
        if (K < 0.05f)
            o.hK = 2.0f + K * (-2.0f + K * (4.0f / 3.0f + K * (-2.0f / 3.0f + K * (4.0f / 15.0f))));
        else
            o.hK = (1.0f - e) * o.invK;
        if (K < 0.25f) {
            float K2b = K * K;
            o.nuK = 1.0f + K * (-1.0f / 3.0f + K2b * (1.0f / 45.0f - K2b * (2.0f / 945.0f)));
        } else {
            o.nuK = o.invK - 2.0f * e * frcp(1.0f - e);
        }
    }
}

__device__ __forceinline__ PairK pair_k(float a, float b, float q)
{
    PairK o = pair_k_large(a, b, q);
    pair_k_small(o);
    return o;
}

// Block-level shared state of the bound kernels (up to kMaxWaves waves).
struct BlockShared {
    double s0[kMaxWaves], s1[kMaxWaves];
    int drop[kMaxWaves], ubinf[kMaxWaves];
    float psum[kMaxWaves], prsum[kMaxWaves];
    float top[kMaxWaves][8];
    double dk[kMaxWaves];   // per wave: sum of w_i^2 klo_i / 2 (the pair screen's scale)
};

// The pair screens drop a pair when its summand is provably below
// kCullRel D / (number of pairs), D = sum_i w_i^2 klo_i / 2 over the cell's
// components: D is at most each diagonal summand sum w_i^2 k coth(k) / 2 of
// S11 (k >= klo), hence a lower bound of the scale S11 + 2 S12 of both bounds,
// and all dropped pairs together move a bound by at most kCullRel of it.
constexpr double kCullRel = 1e-8;

// Pairs that pass the screen are evaluated kBatch per lane at a time; each
// wave collects them in a list of kList entries (a full batch plus one step
// of 64 offers).  One pair per lane measured fastest: five waves per SIMD
// already keep enough independent work in flight, and a short list flushes
// with fewer idle lanes.
constexpr int kBatch = 1, kList = 64 * kBatch + 64;

// Pairs are summed in FP32 over runs of at most this many steps per lane and
// the runs are accumulated in FP64.
constexpr int kRun = 8;

// LDS record stride in float4: an S11 GMM record holds five float4 (a stride
// of 20 dwords, so 16-byte reads of consecutive records by consecutive lanes
// hit distinct banks).  The pair kernel's GMM record holds four (its pair
// list is read by row, mostly the same row across a wave) and a separate
// two-float4 screen record per component is read from one address.  The vMF rows (two float4 per component) are read from the
// global table when one problem is set (every block reads the same few KB,
// which stay in L1/L2); with several problems a block's successive cubes
// belong to different problems, so their rows are staged in LDS per cube.
constexpr int kG = 5, kG12 = 4;

// ---------------------------------------------------------------------------
// S11 over translation cells
// ---------------------------------------------------------------------------
//
// Component record in LDS, four float4 (64 bytes, padded to 80):
//   [0] u (unit vector mu - t0), weight      [1] kappa(t0), G(kappa), cos, sin of psi_t / 2
//   [2] kappa interval centre ac, half-width ha, G(ac), nu(ac)
//   [3] min(1/3, 1/klo^2) (curvature bound), Lam (pair screen), 2 / kappa(t0), -
//
// Pair screen.  The summand of a pair at the centre is at most
// G(k) G(k') exp(-min(q, 2) k k' / (2 (k + k'))) / sqrt(2 k k') (h(K) <= 1/K,
// K <= k + k', K^2 >= 2 k k' up to a right angle, and the summand decreases
// with the angle), and the lower term over the cell is at most the centre
// value (the centre lies in the box of concentrations and A >= theta).  A
// pair whose weighted bound is below thr11 is dropped: the lower sum loses at
// most thr11 (and stays a lower bound) and the centre sum is charged thr11
// (and stays an upper bound).  With min(q, 2) in place of q, the
// test is  q k k' >= 2 (Lam_i + Lam_i' - ln thr11)(k + k'),  Lam_i =
// ln(w_i G(k_i) / sqrt(k_i)) + ln(2) / 4, with thr11 = kCullRel D / (M (M - 1) / 2);
// the kernel divides it by k k' and takes q from the dot product of the
// two unit vectors.

__device__ __forceinline__ void s11_terms(const float4 &A0, const float4 &A1, const float4 &A2, const float4 &A3,
                                          const float4 &B0, const float4 &B1, const float4 &B2, const float4 &B3,
                                          float &sub, float &slo)
{
    const float dx = A0.x - B0.x, dy = A0.y - B0.y, dz = A0.z - B0.z;
    const float q = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float px = A0.x + B0.x, py = A0.y + B0.y, pz = A0.z + B0.z;
    const float pp = fmaf(px, px, fmaf(py, py, pz * pz));
    const float w2 = 2.0f * A0.w * B0.w;
    // lower bound summand: angle A = min(pi, theta + psi_i + psi_i') (eq. 24)
    // via half angles: A/2 = theta/2 + (psi_i + psi_i')/2, clamped at pi/2;
    // half-angle sine and cosine from the two chords |u - v|, |u + v|
    const float st = 0.5f * fsqrt(q), ct = 0.5f * fsqrt(pp);
    const float ca = A1.z * B1.z - A1.w * B1.w, sa = A1.w * B1.z + A1.z * B1.w;
    const float cA = ct * ca - st * sa;
    float sA = st * ca + ct * sa;
    sA = cA <= 0.0f ? 1.0f : sA;
    const float qA = 4.0f * sA * sA;
    const float a = A2.x, b = B2.x, ha = A2.y, hb = B2.y;
    auto terms = [&](const PairK &k0, const PairK &k) __attribute__((always_inline)) {
        // upper bound summand at the centre
        sub += w2 * (fexp2(k0.x * kLog2e) * k0.hK * A1.y * B1.y);
        // gradient of g = log Z(K) - log Z(a) - log Z(b) at the box centre:
        // g_a = (K_a - 1) + nu(a) - nu(K) K_a with
        // K_a - 1 = b qA (a - b - K) / (2 K (K + a + b)).
        const float ka1 = 0.5f * b * qA * (a - b - k.K) * k.r;
        const float kb1 = 0.5f * a * qA * (b - a - k.K) * k.r;
        const float ga = ka1 + A2.w - k.nuK * (1.0f + ka1);
        const float gb = kb1 + B2.w - k.nuK * (1.0f + kb1);
        // curvature remainder per axis: the Hessian of g is at least
        // diag(-L'(a), -L'(b)) (log Z(K) is convex in (a, b)); slot 3.x holds
        // min(1/3, 1/klo^2) >= L' over the component's interval
        const float corr = -fabsf(ga) * ha - fabsf(gb) * hb - 0.5f * fmaf(A3.x * ha, ha, B3.x * hb * hb);
        slo += w2 * (fexp2((k.x + corr) * kLog2e) * k.hK * A2.z * B2.z);
    };
    // the small-K corrections of both K in one rarely taken branch (the wave
    // runs both copies of the terms only when one of its lanes has a small K)
    PairK k0 = pair_k_large(A1.x, B1.x, q), k = pair_k_large(a, b, qA);
    if (__builtin_expect(fminf(k0.K, k.K) < kSmallK, 0)) {
        pair_k_small(k0);
        pair_k_small(k);
        terms(k0, k);
        asm volatile("");   // the two copies of terms stay apart
    } else {
        terms(k0, k);
    }
}

__device__ __forceinline__ void s11_pair(const float4 *__restrict__ rec, int a_, int b_, float &sub, float &slo)
{
    s11_terms(rec[kG * a_], rec[kG * a_ + 1], rec[kG * a_ + 2], rec[kG * a_ + 3], rec[kG * b_], rec[kG * b_ + 1],
              rec[kG * b_ + 2], rec[kG * b_ + 3], sub, slo);
}

template <bool GREC>
__global__ __launch_bounds__(64 * kMaxWaves) void k_s11(DevMix mx, const uint64_t *__restrict__ tkeys,
                                                         const uint32_t *__restrict__ pids, int64_t nt_host,
                                                         const uint32_t *__restrict__ nt_dev, S11Out out, int maxM,
                                                         const int64_t *__restrict__ out_idx, int split_ok)
{
    extern __shared__ float4 lds4[];
    __shared__ BlockShared sh;
    const int W = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nt = nt_dev ? (int64_t)nt_dev[0] : nt_host;
    // A cell is evaluated by a team: the whole block while there are fewer
    // cells than blocks (the cell's latency decides), or each wave on its own
    // once every wave can have a cell (with split_ok: LDS for one record set
    // per wave).  The choice is uniform over the block.
    const bool split = split_ok && W > 1 && nt > (int64_t)gridDim.x;
    const int tid = split ? lane : (int)threadIdx.x, T = split ? 64 : (int)blockDim.x;
    auto team_sync = [&]() __attribute__((always_inline)) {
        if (split)
            wave_lds_sync();
        else
            __syncthreads();
    };
    // component records: LDS (one set per team), or the block's slice of the
    // global records
    float4 *rec = GREC ? mx.grec + (int64_t)blockIdx.x * mx.grec_stride : lds4 + (split ? wv * kG * maxM : 0);
    // per wave: pairs that passed the screen
    uint32_t *plist = reinterpret_cast<uint32_t *>(GREC ? lds4 : lds4 + kG * maxM * (split_ok ? W : 1));
    unsigned ncells = 0, noff_all = 0, nkeep_all = 0;   // per wave, over the block's cells (for out.counts)
    const bool recs = out.trec && (!out.ncubes || (int64_t)out.ncubes[0] >= (int64_t)kTRecMinCubes * nt);
    const int64_t c_first = split ? (int64_t)blockIdx.x * W + wv : (int64_t)blockIdx.x;
    const int64_t c_step = split ? (int64_t)gridDim.x * W : (int64_t)gridDim.x;
    for (int64_t cell = c_first; cell < nt; cell += c_step) {
        team_sync();
        const int64_t o = out_idx ? out_idx[cell] : cell;   // where the cell's sums go
        const uint32_t pid = pids ? pids[cell] : 0u;
        if (pid >= (uint32_t)mx.n_prob) {     // invalid problem index: no bound
            if (tid == 0) {
                out.ub[o] = NAN;
                out.lo[o] = NAN;
            }
            continue;
        }
        const ProbDesc P = mx.prob[pid];
        double t0[3], tau[3];
        decode_key(tkeys[cell], P.t_lo, P.t_w, t0, tau);
        // where this cell's records for the pair kernel go (none without a
        // record buffer or when the buffer is used up); with too few cubes
        // per cell to pay for the full records, Lemma 3's records only
        const uint32_t toff = out.trec ? out.toff[o] : kNoTRec;
        // (another wave of the team may already have flagged the offset)
        const uint32_t tbase = toff == kNoTRec ? kNoTRec : toff & ~kTRecLemma3;
        float4 *l3rec = nullptr;
        if (tbase != kNoTRec && !recs) {
            l3rec = reinterpret_cast<float4 *>(out.trec + tbase);
            if (tid == 0) out.toff[o] = tbase | kTRecLemma3;
        }

        // per-component prep; the diagonal (i = i') summands are added here:
        // Z(2k)/Z(k)^2 = k coth(k) / 2 at the centre, and at the low end of the
        // kappa interval for the lower bound (the angle is exactly 0 and the
        // summand increases with kappa).
        double dub = 0.0, dlo = 0.0, dk = 0.0;
        float psum = 0.0f;
        int drop = 0, ubinf = 0;
        for (int i = tid; i < P.M; i += T) {
            const int g = P.gmm_off + i;
            double cd[3], rho2;
            bool inside;
            TransPrep tp = trans_interval(mx.mu + 3 * g, mx.isig2[g], t0, tau, P.zeta, cd, &rho2, &inside);
            const float4 l3 = lemma3_record(cd, rho2, tau, inside);
            apply_lemma3(tp, l3);
            drop |= tp.drop;
            ubinf |= tp.ub_inf;
            psum += mx.pbar[g] * tp.psi;
            const double w = mx.w1[g];
            const YFun fk = yfun(tp.kap), fa = yfun(tp.ac), fl = yfun(tp.klo);
            if (l3rec)
                l3rec[i] = l3;
            else if (tbase != kNoTRec)
                out.trec[(size_t)tbase + i] = trans_record(tp, (float)w, fk, fl);
            dub += w * w * 0.5 * tp.kap * (double)fk.coth;
            dlo += w * w * 0.5 * tp.klo * (double)fl.coth;
            rec[kG * i] = make_float4((float)tp.u[0], (float)tp.u[1], (float)tp.u[2], (float)w);
            rec[kG * i + 1] = make_float4((float)tp.kap, (float)fk.G, (float)tp.cps, (float)tp.sps);
            rec[kG * i + 2] = make_float4((float)tp.ac, (float)tp.ha, (float)fa.G, (float)fa.nu);
            const float lam = fminf(fmaxf(__builtin_amdgcn_logf((float)w * fk.G * __builtin_amdgcn_rsqf((float)tp.kap)) *
                                                  kLn2 + 0.25f * kLn2, -1e30f), 1e30f);
            dk += 0.5 * w * w * tp.klo;
            rec[kG * i + 3] = make_float4((float)fmin(1.0 / 3.0, 1.0 / (tp.klo * tp.klo)), lam, (float)(2.0 / tp.kap), 0.0f);
        }
        drop = wave_or(drop);
        ubinf = wave_or(ubinf);
        dk = wave_sum(dk);
        psum = wave_sumf(psum);
        if (!split) {
            if (lane == 0) {
                sh.drop[wv] = drop;
                sh.ubinf[wv] = ubinf;
                sh.dk[wv] = dk;
                sh.psum[wv] = psum;
            }
            __syncthreads();
            drop = 0;
            ubinf = 0;
            dk = 0.0;
            psum = 0.0f;
            for (int w = 0; w < W; ++w) {
                drop |= sh.drop[w];
                ubinf |= sh.ubinf[w];
                dk += sh.dk[w];
                psum += sh.psum[w];
            }
        } else {
            wave_lds_sync();   // the team's records are written
        }
        if (out.csum && tid == 0)
            out.csum[o] = CellSums{dk, psum, (drop ? kCellDrop : 0u) | (ubinf ? kCellUbInf : 0u)};
        if (drop) {
            if (tid == 0) {
                out.ub[o] = INFINITY;
                out.lo[o] = INFINITY;
            }
            continue;
        }
        ncells += 1;
        // threshold of the pair screen, per unordered GMM pair
        const double thr11 = P.M > 1 ? kCullRel * dk / (0.5 * (double)P.M * (double)(P.M - 1)) : 0.0;
        const float lthr11 = thr11 > 0.0 ? __builtin_amdgcn_logf((float)thr11) * kLn2 : -INFINITY;

        double acc_ub = dub, acc_lo = dlo;
        // Candidate pairs are offered by every lane of a wave in lockstep; the
        // pairs not screened out are listed per wave and evaluated kBatch per lane.
        uint32_t *pl = plist + kList * wv;
        int pc = 0, run = 0, ncull = 0;
        float sub = 0.0f, slo = 0.0f;
        auto evaluate = [&](int base_, int cnt) __attribute__((always_inline)) {
            uint32_t e[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int x = 64 * k + lane;
                e[k] = x < cnt ? pl[base_ + x] : 0xffffffffu;
            }
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                if (e[k] != 0xffffffffu) s11_pair(rec, (int)(e[k] >> 16), (int)(e[k] & 0xffffu), sub, slo);
            run += kBatch;
            if (run >= kRun) {
                acc_ub += (double)sub;
                acc_lo += (double)slo;
                sub = slo = 0.0f;
                run = 0;
            }
        };
        auto offer = [&](const float4 &A0, const float4 &A3, int a_, int b_, bool valid) __attribute__((always_inline)) {
            if (out.counts) noff_all += (unsigned)__popcll(__ballot(valid));
            bool keep = false;
            if (valid) {
                const float4 B0 = rec[kG * b_], B3 = rec[kG * b_ + 3];
                // q = |u - u'|^2 = 2 - 2 u.u', the test divided by k k' (slot 3 holds 2 / k)
                const float dot = fmaf(A0.x, B0.x, fmaf(A0.y, B0.y, A0.z * B0.z));
                const float q = fminf(fmaf(-2.0f, dot, 2.0f), 2.0f);
                keep = q < (A3.y + B3.y - lthr11) * (A3.z + B3.z);
                ncull += keep ? 0 : 1;
            }
            const unsigned long long m = __ballot(keep);
            if (keep) {
                // slot = pc + kept lanes below this one (mbcnt adds to pc)
                const uint32_t slot = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)pc));
                pl[slot] = ((uint32_t)a_ << 16) | (uint32_t)b_;
            }
            nkeep_all += (unsigned)__popcll(m);
            pc += __popcll(m);
            if (pc >= 64 * kBatch) {
                pc -= 64 * kBatch;
                wave_lds_sync();
                evaluate(pc, 64 * kBatch);
            }
        };
        for (int c = 0; c < P.n_cls; ++c) {
            const ClassRange cr = mx.cls[P.cls_off + c];
            const int n = cr.g1 - cr.g0;
            if (n < 2) continue;
            const int base = cr.g0 - P.gmm_off;
            // Circulant walk: a thread keeps component f's record in registers and
            // visits f + d (mod n) for d = 1 .. n/2, so each unordered pair is met
            // once (d = n/2 only from f < n/2 when n is even); with n < T, g = T/n
            // threads share f and take every g-th distance.  Used when it keeps at
            // least 90% of the threads busy.
            const int gq = n < T ? T / n : 1;
            const int fstep = n < T ? n : T;
            const int passes = (n + T - 1) / T;
            if (n < T ? 10 * gq * n >= 9 * T : 10 * n >= 9 * T * passes) {
                const int q = n < T ? tid / n : 0;
                const int f0 = n < T ? tid % n : tid;
                const int smax = (n / 2 + gq - 1) / gq;   // steps of the longest walk
                for (int pass = 0; pass < passes; ++pass) {
                    const int f = f0 + pass * fstep;
                    const bool on = q < gq && f < n;
                    const int fa = on ? f : 0;
                    const int a_ = base + fa;
                    const float4 A0 = rec[kG * a_], A3 = rec[kG * a_ + 3];
                    const int dmax = (n & 1) ? (n - 1) / 2 : (fa < n / 2 ? n / 2 : n / 2 - 1);
                    for (int st = 0; st < smax; ++st) {
                        const int d = 1 + q + st * gq;
                        const bool valid = on && d <= dmax;
                        int o = fa + (valid ? d : 0);
                        o -= o >= n ? n : 0;
                        offer(A0, A3, a_, base + o, valid);
                    }
                }
                continue;
            }
            // The upper triangle (i <= i') of the class, folded into a rectangle of
            // n2/2 rows and n2 + 1 columns (n2 = n rounded up to even): folded row
            // r holds triangle rows r and n2 - 1 - r.  T consecutive cells per step.
            const int n2 = n + (n & 1);
            const int R = n2 >> 1, C = n2 + 1;
            int r = tid / C, col = tid % C;
            const int dr = T / C, dc = T % C;
            const int steps = (R * C + T - 1) / T;
            for (int st = 0; st < steps; ++st) {
                int i = 0, i2 = 0;
                if (r < R) {
                    if (col < n2 - r) {
                        i = r;
                        i2 = r + col;
                    } else {
                        i = n2 - 1 - r;
                        i2 = i + col - (n2 - r);
                    }
                }
                const bool valid = r < R && i2 < n && i != i2;
                const int a_ = base + (valid ? i : 0), b_ = base + (valid ? i2 : 0);
                const float4 A0 = rec[kG * a_], A3 = rec[kG * a_ + 3];
                offer(A0, A3, a_, b_, valid);
                col += dc;
                r += dr;
                if (col >= C) {
                    col -= C;
                    r += 1;
                }
            }
        }
        // the rest of the list; dropped pairs are charged to the centre sum
        wave_lds_sync();
        if (pc > 0) evaluate(0, pc);
        acc_ub += (double)sub + (double)ncull * thr11;
        acc_lo += (double)slo;
        acc_ub = wave_sum(acc_ub);
        acc_lo = wave_sum(acc_lo);
        if (split) {
            if (lane == 0) {
                out.ub[o] = ubinf ? INFINITY : acc_ub;
                out.lo[o] = acc_lo;
            }
            continue;
        }
        if (lane == 0) {
            sh.s0[wv] = acc_ub;
            sh.s1[wv] = acc_lo;
        }
        __syncthreads();
        if (tid == 0) {
            double su = 0.0, sl = 0.0;
            for (int w = 0; w < W; ++w) {
                su += sh.s0[w];
                sl += sh.s1[w];
            }
            out.ub[o] = ubinf ? INFINITY : su;
            out.lo[o] = sl;
        }
    }
    if (out.counts && lane == 0) {
        unsigned long long *c = out.counts + kCounters * (blockIdx.x % kCountSlots);
        if (wv == 0 || split) atomicAdd(c + kCntCells, (unsigned long long)ncells);
        atomicAdd(c + kCntS11Screened, (unsigned long long)noff_all);
        atomicAdd(c + kCntS11Evaluated, (unsigned long long)nkeep_all);
    }
}

// ---------------------------------------------------------------------------
// S12 over rotation x translation cells, and the final bounds
// ---------------------------------------------------------------------------
//
// GMM component record in LDS, four float4 (64 bytes):
//   [0] w = R_r0 u (rotated unit vector), weight
//   [1] kappa(t0), G(kappa), cos, sin of Psi / 2 with Psi = psi_t + psi_r (eq. 25)
//   [2] kappa interval [alo, ahi] over the cell, half-width ha, coth(alo)
//   [3] G(alo), G(ahi), nu(alo), nu(ahi)
// Screen record of the component (a separate LDS array, two float4):
//   {w cos Psi, 1 - sin Psi - Lam / alo},
//   {Lam, 1 / alo, -sin Psi, ln(alo) / 2 (the far-apart cap's term)}
// vMF row, two float4 (32 bytes, global table or LDS):
//   {dx, dy, dz, kappa}, {weight, G(kappa), coth(kappa), ln(2 kappa) / 2};
// the screen's column term l = ln(weight G(kappa)) - ln(2 kappa) / 2 - ln thr is
// formed once per lane and column block from that row.
//
// Upper bound of the summand over the cube (Theorem 1 with kappa_1i(t)
// relaxed to [alo, ahi]): at the smallest angle B, and with
//   g(a) = log Z(K) - log Z(a) - log Z(b) = x(a) + phi(a),  x = K - a - b,
// x is convex in a (K is the norm of a u + b v), and phi'' <= min(1/3, 1/Kmin^2)
// with Kmin the smallest K on the interval, so a second-order expansion of phi
// at either end plus the exact x is a convex majorant whose maximum sits at an
// end; the smaller of the two expansions is used, capped by the value for
// aligned directions, min(ahi, b)(coth alo + coth b)/2, and by the bound for
// directions far apart,
//   2 G(ahi) G(b) exp(-qB alo b / (2 (alo + b)))                       (*)
// (h(K) <= 2, G increasing, K <= a + b, and a b / (a + b) increasing in a).
//
// Pair screen.  (*) also bounds the summand at the centre, so a pair whose
// weighted (*) is below a per-problem threshold thr contributes less than thr
// to either sum.  With the smaller far-apart cap, weighted, the pair is below
// thr when min(q, 2) / 2 >= (Lam_i + l_j)(1/alo + 1/b), Lam_i = ln(w_i G(ahi) /
// sqrt(alo)), l_j = ln(w_j G(b_j) / sqrt(2 b_j)) - ln thr, thr = kCullRel D / (M N).
// With q = 4 sin^2(B/2) >= 2 - 2 (d cos Psi + sin Psi), a lower bound for the
// angle B = max(0, theta - Psi) (d = cos theta; valid for Psi <= pi/2), and
// a = 1/alo, c = 1/b, that holds when
//   max((w_i cos Psi_i) . mu_j, -sin Psi_i) <= (1 - sin Psi_i - Lam_i a) - l_j c - Lam_i c - l_j a:
// a dot product, four multiply-adds and a max per pair, from the component's
// screen row and record slot (broadcast LDS reads) and per-lane vMF constants.  A pair that
// passes is dropped: it adds nothing to S12 at the centre (the upper bound
// rises by at most 2 thr) and thr to the upper bound S12hi (which stays an
// upper bound).  The pairs that remain are collected per wave in LDS and
// evaluated kBatch per lane at a time.

template <bool TOP8, int KP>
__device__ __forceinline__ void s12_pair(const float4 *__restrict__ rec, const float4 *__restrict__ scr, int a_,
                                         const float4 v0, const float4 v1, float inf, float &sub, float &shi,
                                         float (&top)[8])
{
    const float4 R0 = rec[kG12 * a_], R1 = rec[kG12 * a_ + 1], R2 = rec[kG12 * a_ + 2], R3 = rec[kG12 * a_ + 3];
    const float hla = scr[2 * a_ + 1].w;   // ln(alo) / 2
    const float b = v0.w;
    const float dx = R0.x - v0.x, dy = R0.y - v0.y, dz = R0.z - v0.z;
    const float q = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float px = R0.x + v0.x, py = R0.y + v0.y, pz = R0.z + v0.z;
    const float pp = fmaf(px, px, fmaf(py, py, pz * pz));
    const float ww = R0.w * v1.x;
    // the smallest angle over the cube: B = max(0, theta - Psi) (eq. 25)
    const float st = 0.5f * fsqrt(q), ct = 0.5f * fsqrt(pp);
    const float sB = fmaxf(st * R1.z - ct * R1.w, 0.0f);
    const float qB = 4.0f * sB * sB;
    const float alo = R2.x, ahi = R2.y, ha = R2.z;
    const float bc = b * fmaf(-0.5f, qB, 1.0f);             // b cos B
    // upper bound summand at the centre (eq. 12), from k0
    auto centre = [&](const PairK &k0) __attribute__((always_inline)) {
        const float v = ww * (fexp2(k0.x * kLog2e) * k0.hK * R1.y * v1.y);
        sub += v;
        if (TOP8) {
            // insert v into the descending list and drop the smallest: slot s
            // takes the median of its old value, v and the old value of slot
            // s - 1 (eight independent operations; a v not above the eighth
            // leaves the list unchanged)
#pragma unroll
            for (int s = 7; s > 0; --s) top[s] = __builtin_amdgcn_fmed3f(top[s - 1], v, top[s]);
            top[0] = __builtin_amdgcn_fmed3f(top[0], v, inf);
        }
    };
    // upper bound on the summand over the cube, from the majorant vT of the
    // kappa dependence: capped by the aligned and far-apart values
    auto upper = [&](float vT) __attribute__((always_inline)) {
        const float cap = 0.5f * fmin_med3(ahi, b, inf) * (R2.w + v1.z);
        // far-apart caps: 2 G G e^{-qB cf} and G G e^{-min(qB, 2) cf} / sqrt(2 alo b)
        const float cf = alo * b * frcp(2.0f * (alo + b));
        const float e2 = fmaf(-qB, cf, kLn2);
        const float eK = fmaf(-fmin_med3(qB, 2.0f, inf), cf, -(hla + v1.w));
        const float far = R3.y * v1.y * fexp2(fminf(e2, eK) * kLog2e);
        shi += ww * fminf(fminf(vT, cap), far);
    };
    if constexpr (KP == 1) {
        // the two expansions at the ends of [alo, ahi]: from k1 and k2
        auto terms = [&](const PairK &k0, const PairK &k1, const PairK &k2) __attribute__((always_inline)) {
            centre(k0);
            const float d1 = R3.z - k1.nuK * (alo + bc) * k1.invK;  // phi'(alo)
            const float d2 = R3.w - k2.nuK * (ahi + bc) * k2.invK;  // phi'(ahi)
            const float km2 =
                (-bc > alo && -bc < ahi) ? b * b * qB * fmaf(-0.25f, qB, 1.0f) : fmin_med3(k1.ks, k2.ks, inf);
            const float G = fminf(1.0f / 3.0f, frcp(km2));
            const float q2 = 2.0f * G * ha * ha;
            const float eA = fmaxf(k1.x, fmaf(2.0f * d1, ha, k2.x + q2));
            const float eB = fmaxf(k2.x, fmaf(-2.0f * d2, ha, k1.x + q2));
            const float vA = fexp2(eA * kLog2e) * k1.hK * R3.x;
            const float vB = fexp2(eB * kLog2e) * k2.hK * R3.y;
            upper(fminf(vA, vB) * v1.y);
        };
        // each K with its own branch for the small-K terms: one branch for all
        // three made the whole wave run both copies of the terms whenever one
        // lane had a small K, which late in a search costs more than it saves
        terms(pair_k(R1.x, b, q), pair_k(alo, b, qB), pair_k(ahi, b, qB));
    } else {
        centre(pair_k(R1.x, b, q));
        // the kappa interval in KP equal pieces: the same two expansions on
        // each piece, the largest piece bound (G and nu at the inner ends
        // computed here, at the outer ends from the record)
        const float wdt = (ahi - alo) * (1.0f / KP), hp = 0.5f * wdt;
        const float kmi = b * b * qB * fmaf(-0.25f, qB, 1.0f);   // K^2 where a = -b cos B
        float ks[KP + 1], xs[KP + 1], d[KP + 1], hk[KP + 1], ge[KP + 1];
#pragma unroll
        for (int p = 0; p <= KP; ++p) {
            const float e = p == 0 ? alo : (p == KP ? ahi : fmaf((float)p, wdt, alo));
            const PairK k = pair_k(e, b, qB);
            float Ge, nue;
            if (p == 0) {
                Ge = R3.x;
                nue = R3.z;
            } else if (p == KP) {
                Ge = R3.y;
                nue = R3.w;
            } else {
                yfun_f(e, &Ge, &nue);
            }
            ks[p] = k.ks;
            xs[p] = k.x;
            hk[p] = k.hK;
            ge[p] = Ge;
            d[p] = nue - k.nuK * (e + bc) * k.invK;
        }
        float best = 0.0f;
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            const float e0 = p == 0 ? alo : fmaf((float)p, wdt, alo);
            const float e1 = p == KP - 1 ? ahi : fmaf((float)(p + 1), wdt, alo);
            const float km2 = (-bc > e0 && -bc < e1) ? kmi : fmin_med3(ks[p], ks[p + 1], inf);
            const float G = fminf(1.0f / 3.0f, frcp(km2));
            const float q2 = 2.0f * G * hp * hp;
            const float eA = fmaxf(xs[p], fmaf(2.0f * d[p], hp, xs[p + 1] + q2));
            const float eB = fmaxf(xs[p + 1], fmaf(-2.0f * d[p + 1], hp, xs[p] + q2));
            const float vA = fexp2(eA * kLog2e) * hk[p] * ge[p];
            const float vB = fexp2(eB * kLog2e) * hk[p + 1] * ge[p + 1];
            best = fmaxf(best, fminf(vA, vB));
        }
        upper(best * v1.y);
    }
}

// The per-cube set-up pass (one thread per cube): set-up records and, with a
// cell table, each cube's translation cell (see cell_slot).
__global__ __launch_bounds__(256) void k_cube_setup(DevMix mx, const uint64_t *__restrict__ rkeys,
                                                    const uint64_t *__restrict__ tkeys,
                                                    const uint32_t *__restrict__ pids, int64_t n_host,
                                                    const uint32_t *__restrict__ n_dev, int n_dev_mul,
                                                    CubeSetup *__restrict__ out, CellTable cells)
{
    const int64_t n = n_dev ? (int64_t)n_dev[0] * n_dev_mul : n_host;
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cube = base + threadIdx.x;
        bool claimed = false;
        uint32_t pid = 0;
        int64_t at = 0;
        if (cube < n) {
            CubeSetup cs;
            pid = pids ? pids[cube] : 0u;
            if (pid >= (uint32_t)mx.n_prob) {
                cs = CubeSetup{};
                cs.flags = kSetupInvalid;
                out[cube] = cs;
            } else {
                cs = make_cube_setup(mx.prob[pid], rkeys[cube], tkeys[cube]);
                out[cube] = cs;
                if (cells.keys) {
                    // the cube's translation cell in the table
                    unsigned long long *tab = (unsigned long long *)(cells.keys + ((size_t)pid << cells.tbits));
                    at = (int64_t)(((size_t)pid << cells.tbits) + cell_slot(tab, cells.tbits, tkeys[cube], claimed));
                    cells.ctidx[cube] = at;
                }
            }
        }
        if (!cells.keys) continue;
        // the claiming thread lists the cell (one atomic per wave)
        const unsigned long long m = __ballot(claimed);
        if (!m) continue;
        const int leader = __ffsll((long long)m) - 1;
        uint32_t first = 0;
        if (lane == leader) first = atomicAdd(cells.count, (uint32_t)__popcll(m));
        first = __shfl(first, leader, 64);
        if (claimed) {
            const uint32_t j = first + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            cells.list_key[j] = tkeys[cube];
            cells.list_pid[j] = pid;
            cells.list_slot[j] = at;
        }
    }
}

// Five waves per SIMD fit the plain kernel's registers without spills; the
// variant that also keeps the top-8 terms (learned order, record logging) is
// held to four.
template <bool TOP8, bool VLDS, bool GREC, int KP = 1>
__global__ __launch_bounds__(64 * kMaxWaves) __attribute__((amdgpu_waves_per_eu(KP > 1 ? 4 : 5))) void k_s12(DevMix mx, const uint64_t *__restrict__ rkeys,
                                                         const uint64_t *__restrict__ tkeys,
                                                         const uint32_t *__restrict__ pids,
                                                         const int64_t *__restrict__ tidx,
                                                         const double *__restrict__ s11ub,
                                                         const double *__restrict__ s11lo, int64_t n_host,
                                                         const uint32_t *__restrict__ n_dev, int n_dev_mul,
                                                         BoundOut out, double gamma, int maxM, int maxN,
                                                         const CubeSetup *__restrict__ setup, TransRecs tr)
{
    extern __shared__ float4 lds4[];
    __shared__ BlockShared sh;
    static_assert(!(VLDS && GREC), "with global records the vMF rows are read from the global table");
    // component records: LDS, or the block's slice of the global records
    float4 *rec = GREC ? mx.grec + (int64_t)blockIdx.x * mx.grec_stride : lds4;   // kG12 per GMM component
    float4 *scr = rec + kG12 * maxM;    // two-float4 screen record per GMM component
    float4 *vrec = scr + 2 * maxM;      // vMF rows (VLDS only)
    // per wave: pairs that passed the screen
    uint32_t *plist = reinterpret_cast<uint32_t *>(GREC ? lds4 : vrec + (VLDS ? 2 * maxN : 0));
    const int tid = threadIdx.x, T = blockDim.x, W = T >> 6, wv = tid >> 6, lane = tid & 63;
    const int64_t n = n_dev ? (int64_t)n_dev[0] * n_dev_mul : n_host;
    unsigned nscr = 0, ncull_all = 0;   // per wave: pairs screened and dropped, over all cubes of the block
    unsigned nlive = 0;                 // cubes of the block that were not dropped
    for (int64_t cube = blockIdx.x; cube < n; cube += gridDim.x) {
        __syncthreads();
        const CubeSetup &cs = setup[cube];
        if (cs.flags & kSetupInvalid) {     // invalid problem index: no bound, both drop flags
            if (tid == 0) {
                out.ub[cube] = NAN;
                out.lb[cube] = NAN;
                if (out.lb_safe) out.lb_safe[cube] = NAN;
                out.flags[cube] = GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS;
            }
            continue;
        }
        const uint32_t pid = pids ? pids[cube] : 0u;
        const ProbDesc P = mx.prob[pid];
        const double *R = cs.R, *t0 = cs.t0, *tau = cs.tau;
        // the translation cell's records, when the caller has them: the full
        // records, or Lemma 3's only (kTRecLemma3)
        const int64_t ti = tidx ? tidx[cube] : cube;
        const uint32_t toff = tr.rec ? tr.off[ti] : kNoTRec;
        const bool full = toff != kNoTRec && !(toff & kTRecLemma3);
        const float4 *l3rec = toff != kNoTRec && !full ? reinterpret_cast<const float4 *>(tr.rec + (toff & ~kTRecLemma3))
                                                       : nullptr;

        // Lemma 2, per direction.  The angle-axis metric bound
        // angle(R_r p, R_s p) <= |r - s| caps every direction's rotation
        // uncertainty at min(|h_r|, pi).  Along the segment r0 + s d (d in the
        // half-width box) the image R_{r0 + s d} p moves with angular speed
        // |(J(r0 + s d) d) x R p|; with |J| <= 1 and the derivative of J along
        // a unit direction at most 1.6 while |r| <= 5.5, its length is at most
        //   |(J(r0) d) x w'| + 1.3 |d|^2,   w' = R_r0 p.
        // The first term is the norm of a linear function of d, largest at a
        // corner of the box (corners come in opposite pairs, so four suffice:
        // cs.jc), and moving w' inside the cone of half-angle psi_t around
        // w = R_r0 u adds at most 2 sin(psi_t / 2) |h_r|.
        const float hnf = cs.hn, cap = cs.cap;
        const bool per_dir = (cs.flags & kSetupPerDir) != 0;
        uint8_t flags = (uint8_t)(cs.flags & GOSMA_FLAG_DROP_ROT);
        int drop = 0, ubinf = 0;
        float psum = 0.0f, prsum = 0.0f;
        double dk = 0.0;
        for (int i = tid; i < P.M; i += T) {
            const int g = P.gmm_off + i;
            const float wi = mx.w1[g];
            // the translation part: the cell's record, or computed here
            TransRec r;
            if (full) {
                r = tr.rec[(size_t)toff + i];
            } else {
                double cd[3], rho2;
                bool inside;
                TransPrep tp = trans_interval(mx.mu + 3 * g, mx.isig2[g], t0, tau, P.zeta, cd, &rho2, &inside);
                apply_lemma3(tp, l3rec ? l3rec[i] : lemma3_record(cd, rho2, tau, inside));
                drop |= tp.drop;
                ubinf |= tp.ub_inf;
                psum += mx.pbar[g] * tp.psi;
                dk += 0.5 * (double)wi * (double)wi * tp.klo;
                r = trans_record(tp, wi, yfun(tp.kap), yfun(tp.klo));
            }
            double w[3];
            for (int a = 0; a < 3; ++a) w[a] = R[3 * a] * r.u[0] + R[3 * a + 1] * r.u[1] + R[3 * a + 2] * r.u[2];
            // the rotation uncertainty of this direction (FP32: it enters the
            // bound through FP32 records)
            float psir = cap;
            if (per_dir) {
                const float wf[3] = {(float)w[0], (float)w[1], (float)w[2]};
                float m2 = 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float *v = cs.jc[q];
                    const float x = wf[1] * v[2] - wf[2] * v[1], y = wf[2] * v[0] - wf[0] * v[2],
                                z = wf[0] * v[1] - wf[1] * v[0];
                    m2 = fmaxf(m2, fmaf(x, x, fmaf(y, y, z * z)));
                }
                psir = fminf(fsqrt(m2) + 2.0f * r.sps * hnf + 1.3f * hnf * hnf, cap);
            }
            prsum += mx.pbar[g] * psir;
            float crf, srf;
            sincos_half(0.5f * psir, &srf, &crf);
            const double crh = crf, srh = srf;
            // half of Psi = psi_t + psi_r (eq. 25), as cos/sin
            const double cps = r.cps, sps = r.sps;
            const double cP = cps * crh - sps * srh, sP = sps * crh + cps * srh;
            // pair screen rows: none dropped for Psi > pi/2 (where the bound on
            // cos B fails); Lam clamped below at -100 (a smaller threshold term
            // only screens out fewer pairs)
            {
                const float cf = (float)cP, sf = (float)sP;
                const float cPsi = cf * cf - sf * sf, sPsi = 2.0f * cf * sf;
                const float r0 = cf >= sf ? 1.0f - sPsi - r.lam * r.ia : -1e30f;
                scr[2 * i] = make_float4((float)w[0] * cPsi, (float)w[1] * cPsi, (float)w[2] * cPsi, r0);
                scr[2 * i + 1] = make_float4(r.lam, r.ia, -sPsi, r.hla);
            }
            rec[kG12 * i] = make_float4((float)w[0], (float)w[1], (float)w[2], wi);
            rec[kG12 * i + 1] = make_float4(r.kap, r.Gk, (float)cP, (float)sP);
            rec[kG12 * i + 2] = make_float4(r.klo, r.ahi, r.ha, r.cothl);
            rec[kG12 * i + 3] = make_float4(r.Gl, r.Gh, r.nul, r.nuh);
        }
        // the problem's vMF rows {mu, kappa}, {weight, G(kappa), coth kappa, ln(2 kappa) / 2}
        const float4 *__restrict__ vt = mx.vmf + 2 * (int64_t)P.vmf_off;
        if (VLDS)
            for (int j = tid; j < 2 * P.N; j += T) vrec[j] = vt[j];
        auto vrow = [&](int j, int h) __attribute__((always_inline)) -> float4 {
            if constexpr (VLDS)
                return vrec[2 * j + h];
            else
                return vt[2 * j + h];
        };
        // the sums over the components: the rotation part here, the
        // translation part from the cell's sums when it has records
        const bool own = !full;
        prsum = wave_sumf(prsum);
        if (own) {
            drop = wave_or(drop);
            ubinf = wave_or(ubinf);
            psum = wave_sumf(psum);
            dk = wave_sum(dk);
        }
        if (lane == 0) {
            sh.prsum[wv] = prsum;
            if (own) {
                sh.drop[wv] = drop;
                sh.ubinf[wv] = ubinf;
                sh.psum[wv] = psum;
                sh.dk[wv] = dk;
            }
        }
        __syncthreads();
        prsum = 0.0f;
        for (int w = 0; w < W; ++w) prsum += sh.prsum[w];
        if (own) {
            drop = 0;
            ubinf = 0;
            psum = 0.0f;
            dk = 0.0;
            for (int w = 0; w < W; ++w) {
                drop |= sh.drop[w];
                ubinf |= sh.ubinf[w];
                psum += sh.psum[w];
                dk += sh.dk[w];
            }
        } else {
            const CellSums c = tr.csum[ti];
            drop = (c.flags & kCellDrop) != 0;
            ubinf = (c.flags & kCellUbInf) != 0;
            psum = c.psum;
            dk = c.dk;
        }
        // threshold of the pair screen, per GMM-vMF pair
        const double thr = kCullRel * dk / ((double)P.M * (double)P.N);
        const float lthr = thr > 0.0 ? __builtin_amdgcn_logf((float)thr) * kLn2 : -INFINITY;
        if (drop) flags |= GOSMA_FLAG_DROP_TRANS;
        if (ubinf) flags |= GOSMA_FLAG_UB_INF;
        // branching rule (Section 5.1): the weighted means of the two uncertainties
        if (prsum >= psum) flags |= GOSMA_FLAG_SPLIT_ROT;

        const bool dropped = flags & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS);
        nlive += dropped ? 0u : 1u;
        double acc_ub = 0.0, acc_hi = 0.0;
        float top[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) top[k] = 0.0f;

        if (!dropped) {
            // Candidate pairs are offered by every lane of a wave in lockstep
            // (a lane without one offers nothing); the pairs that are not
            // screened out are appended to the wave's list and evaluated 64 at
            // a time, with FP32 runs of kRun evaluations per lane.
            uint32_t *pl = plist + kList * wv;
            int pc = 0, run = 0;
            unsigned noff = 0, nkeep = 0;   // this wave's pairs offered and kept (wave-uniform)
            float sub = 0.0f, shi = 0.0f;
            // evaluate the cnt (<= 64 kBatch) listed pairs from pl[base]
            auto evaluate = [&](int base, int cnt) __attribute__((always_inline)) {
                uint32_t e[kBatch];
#pragma unroll
                for (int k = 0; k < kBatch; ++k) {
                    const int x = 64 * k + lane;
                    e[k] = x < cnt ? pl[base + x] : 0xffffffffu;
                }
                wave_lds_sync();
#pragma unroll
                for (int k = 0; k < kBatch; ++k) {
                    if (e[k] != 0xffffffffu) {
                        const int jj = (int)(e[k] & 0xffffu);
                        s12_pair<TOP8, KP>(rec, scr, (int)(e[k] >> 16), vrow(jj, 0), vrow(jj, 1), mx.inf, sub, shi,
                                           top);
                    }
                }
                run += kBatch;
                if (run >= kRun) {
                    acc_ub += (double)sub;
                    acc_hi += (double)shi;
                    sub = shi = 0.0f;
                    run = 0;
                }
            };
            // the screen test; vm = {mu_j, l_j c_j}, vc = {c_j = 1 / b_j, l_j}: the
            // lane's vMF screen constants
            auto screened_in = [&](int a_, const float4 &vm, const float2 &vc) __attribute__((always_inline)) {
                const float4 S0 = scr[2 * a_], S1 = scr[2 * a_ + 1];
                // max(dot, -sin Psi) as a median with +inf (no operand canonicalisation)
                const float d = __builtin_amdgcn_fmed3f(fmaf(S0.x, vm.x, fmaf(S0.y, vm.y, S0.z * vm.z)), S1.z, mx.inf);
                const float rhs = fmaf(-S1.y, vc.y, fmaf(-S1.x, vc.x, S0.w - vm.w));
                return !(d <= rhs);
            };
            // append the kept pairs (mask m) to the wave's list; evaluate a full batch
            auto append = [&](bool keep, unsigned long long m, uint32_t packed) __attribute__((always_inline)) {
                nkeep += (unsigned)__popcll(m);
                if (keep) {
                    // slot = pc + kept lanes below this one (mbcnt adds to pc)
                    const uint32_t slot = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)pc));
                    pl[slot] = packed;
                }
                pc += __popcll(m);
                if (pc >= 64 * kBatch) {
                    pc -= 64 * kBatch;
                    wave_lds_sync();
                    evaluate(pc, 64 * kBatch);
                }
            };
            auto offer = [&](int a_, int jj, const float4 &vm, const float2 &vc, bool valid) __attribute__((always_inline)) {
                const bool keep = valid && screened_in(a_, vm, vc);
                noff += (unsigned)__popcll(__ballot(valid));
                append(keep, __ballot(keep), ((uint32_t)a_ << 16) | (uint32_t)jj);
            };
            for (int c = 0; c < P.n_cls; ++c) {
                const ClassRange cr = mx.cls[P.cls_off + c];
                const int ni = cr.g1 - cr.g0, nj = cr.v1 - cr.v0;
                if (ni <= 0 || nj <= 0) continue;
                const int gb = cr.g0 - P.gmm_off, vb = cr.v0 - P.vmf_off;
                if (nj % T == 0 || T % nj == 0) {
                    // each lane keeps one vMF row per column block in registers
                    // and walks the GMM rows; with T columns the row index is
                    // the same for the whole block (broadcast LDS reads)
                    const int cols = nj < T ? nj : T, g = T / cols;
                    const int jl = tid % cols, i0 = tid / cols;
                    for (int jb = 0; jb < nj; jb += cols) {
                        const int j = vb + jb + jl;
                        const float4 v0 = vrow(j, 0), v1 = vrow(j, 1);
                        const float lw = __builtin_amdgcn_logf(v1.x * v1.y) * kLn2 - v1.w;
                        const float c = frcp(v0.w), l = fmaxf(lw, -100.0f) - lthr;
                        const float4 vm = make_float4(v0.x, v0.y, v0.z, l * c);
                        const float2 vc = make_float2(c, l);
                        if (cols % 64 == 0) {
                            // the row index is the same across the wave: uniform
                            // addresses, every lane offers a pair
                            for (int i = __builtin_amdgcn_readfirstlane(i0); i < ni; i += g) {
                                const bool keep = screened_in(gb + i, vm, vc);
                                noff += 64u;
                                append(keep, __ballot(keep), ((uint32_t)(gb + i) << 16) | (uint32_t)j);
                            }
                        } else {
                            for (int ib = 0; ib < ni; ib += g) {
                                const int i = ib + i0;
                                offer(gb + min(i, ni - 1), j, vm, vc, i < ni);
                            }
                        }
                    }
                } else {
                    // flattened (i, j) rectangle of the class, T consecutive pairs per step
                    int i = tid / nj, j = tid % nj;
                    const int di = T / nj, dj = T % nj;
                    const int steps = (ni * nj + T - 1) / T;
                    for (int st = 0; st < steps; ++st) {
                        const bool valid = i < ni;
                        const int jj = vb + j;
                        const float4 v0 = vrow(jj, 0), v1 = vrow(jj, 1);
                        const float lw = __builtin_amdgcn_logf(v1.x * v1.y) * kLn2 - v1.w;
                        const float c = frcp(v0.w), l = fmaxf(lw, -100.0f) - lthr;
                        offer(gb + min(i, ni - 1), jj, make_float4(v0.x, v0.y, v0.z, l * c), make_float2(c, l), valid);
                        j += dj;
                        i += di;
                        if (j >= nj) {
                            j -= nj;
                            i += 1;
                        }
                    }
                }
            }
            // the rest of the list
            wave_lds_sync();
            if (pc > 0) evaluate(0, pc);
            acc_ub += (double)sub;
            acc_hi += (double)shi;
            if (lane == 0) acc_hi += (double)(noff - nkeep) * thr;   // dropped pairs, once per wave
            nscr += noff;
            ncull_all += noff - nkeep;
        }
        acc_ub = wave_sum(acc_ub);
        acc_hi = wave_sum(acc_hi);
        if (TOP8 && out.top8) {
            // merge the per-lane sorted lists: 8 rounds of a wave maximum of the
            // list heads (the terms are >= 0 and an emptied slot holds -1, so the
            // signed integer order of the bit patterns is the float order); the
            // lowest lane holding the maximum drops its head
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float mine = top[0];
                const float m = __int_as_float(__ockl_wfred_max_i32(__float_as_int(mine)));
                const unsigned long long ballot = __ballot(mine == m);
                const int winner = __ffsll((long long)ballot) - 1;
                if (lane == winner) {
#pragma unroll
                    for (int s = 0; s < 7; ++s) top[s] = top[s + 1];
                    top[7] = -1.0f;
                }
                if (lane == 0) sh.top[wv][k] = fmaxf(m, 0.0f);
            }
        }
        if (lane == 0) {
            sh.s0[wv] = acc_ub;
            sh.s1[wv] = acc_hi;
        }
        __syncthreads();

        if (tid == 0) {
            double sub = 0.0, shi = 0.0;
            for (int w = 0; w < W; ++w) {
                sub += sh.s0[w];
                shi += sh.s1[w];
            }
            if (TOP8 && out.top8) {
                // merge the per-wave sorted lists (4-bit heads packed in one word)
                unsigned heads = 0;
                for (int k = 0; k < 8; ++k) {
                    int bw = 0;
                    float bv = -1.0f;
                    for (int w = 0; w < W; ++w) {
                        const int h = (heads >> (4 * w)) & 15;
                        if (h < 8 && sh.top[w][h] > bv) {
                            bv = sh.top[w][h];
                            bw = w;
                        }
                    }
                    heads += 1u << (4 * bw);
                    out.top8[8 * cube + k] = bv;
                }
            }
            double ub = INFINITY, lb = INFINITY, lbs = INFINITY;
            const int64_t t = tidx ? tidx[cube] : cube;
            const double s11u = s11ub[t], s11l = s11lo[t];
            if (!dropped) {
                ub = ubinf ? INFINITY : s11u - 2.0 * sub;
                lb = s11l - 2.0 * shi;
                lbs = lb - gamma * (s11l + 2.0 * shi);
            }
            out.ub[cube] = ub;
            out.lb[cube] = lb;
            if (out.dstar_bits && ub < INFINITY) {
                // read first: most cubes do not improve d*, and skipping their
                // atomics avoids serialising every wave on one address
                unsigned long long *d = out.dstar_bits + (size_t)pid * out.dstar_stride;
                const unsigned long long u = ordered_bits(ub);
                if (u < __atomic_load_n(d, __ATOMIC_RELAXED)) atomicMin(d, u);
            }
            if (out.lb_safe) out.lb_safe[cube] = lbs;
            out.flags[cube] = flags;
            if (out.aux) {
                out.aux[4 * cube + 0] = s11u;
                out.aux[4 * cube + 1] = sub;
                out.aux[4 * cube + 2] = s11l;
                out.aux[4 * cube + 3] = shi;
            }
            if (out.psi_gap) out.psi_gap[cube] = prsum - psum;
        }
    }
    if (out.counts && lane == 0) {
        // one set of atomics per wave, spread over kCountSlots addresses
        unsigned long long *c = out.counts + kCounters * (blockIdx.x % kCountSlots);
        if (wv == 0) atomicAdd(c + kCntCubes, (unsigned long long)nlive);
        atomicAdd(c + kCntS12Screened, (unsigned long long)nscr);
        atomicAdd(c + kCntS12Evaluated, (unsigned long long)(nscr - ncull_all));
    }
}

}  // namespace

size_t s11_lds_bytes(int maxM, int waves)
{
    return sizeof(float4) * kG * (size_t)maxM + sizeof(uint32_t) * kList * (size_t)waves;
}
// With one record set per wave, so that the waves of a block can take cells
// of their own (k_s11's split_ok): only where it fits kS11SplitLds.
constexpr size_t kS11SplitLds = 65536;
size_t s11_split_lds_bytes(int maxM, int waves)
{
    return sizeof(float4) * kG * (size_t)maxM * waves + sizeof(uint32_t) * kList * (size_t)waves;
}
size_t s12_lds_bytes(int maxM, int maxN, int waves, bool vlds)
{
    return sizeof(float4) * ((kG12 + 2) * (size_t)maxM + (vlds ? 2 * (size_t)maxN : 0)) +
           sizeof(uint32_t) * kList * (size_t)waves;
}

int64_t grec_stride(int maxM, int maxN)
{
    const int64_t s11 = (int64_t)kG * maxM, s12 = (int64_t)(kG12 + 2) * maxM;
    const int64_t sma = ((int64_t)sma_lds_bytes(maxM, maxN) + 15) / 16;
    return std::max(s11, std::max(s12, sma));
}

hipError_t prepare_bound_kernels(int maxM, int maxN)
{
    // allow dynamic LDS beyond the default limit on devices that have it
    const size_t l11s = s11_split_lds_bytes(maxM, kMaxWaves);
    hipError_t e = hipFuncSetAttribute((const void *)k_s11<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)std::max(s11_lds_bytes(maxM, kMaxWaves), l11s <= kS11SplitLds ? l11s : 0));
    const int l0 = (int)s12_lds_bytes(maxM, maxN, kMaxWaves, false), l1 = (int)s12_lds_bytes(maxM, maxN, kMaxWaves, true);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<false, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, l0);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<true, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, l0);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<false, true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<true, true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<false, false, false, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, l0);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<false, false, false, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, l0);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<false, true, false, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
    if (!e) e = hipFuncSetAttribute((const void *)k_s12<false, true, false, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
    return e;
}

static bool tile_ok(const Tile &t) { return t.waves >= 1 && t.waves <= kMaxWaves && t.blocks >= 1; }

hipError_t launch_s11(const DevMix &mx, const uint64_t *tkeys, const uint32_t *pids, int64_t nt, const uint32_t *nt_dev,
                      S11Out out, int maxM, Tile tile, hipStream_t stream, const int64_t *out_idx)
{
    if (nt <= 0) return hipSuccess;
    if (!tile_ok(tile)) return hipErrorInvalidValue;
    if (mx.grec) {
        // records in global memory: at most mx.grec_blocks blocks, LDS for the pair lists only
        const unsigned g = (unsigned)std::min<int64_t>(std::min<int64_t>(tile.blocks, nt), mx.grec_blocks);
        hipLaunchKernelGGL(k_s11<true>, dim3(g), dim3(64 * tile.waves), s11_lds_bytes(0, tile.waves), stream, mx,
                           tkeys, pids, nt, nt_dev, out, maxM, out_idx, 0);
        return hipGetLastError();
    }
    const unsigned g = (unsigned)std::min<int64_t>(tile.blocks, nt);
    const size_t ls = s11_split_lds_bytes(maxM, tile.waves);
    const int split_ok = tile.waves > 1 && ls <= kS11SplitLds;
    hipLaunchKernelGGL(k_s11<false>, dim3(g), dim3(64 * tile.waves), split_ok ? ls : s11_lds_bytes(maxM, tile.waves),
                       stream, mx, tkeys, pids, nt, nt_dev, out, maxM, out_idx, split_ok);
    return hipGetLastError();
}

hipError_t launch_cube_setup(const DevMix &mx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *pids,
                             int64_t n, const uint32_t *n_dev, int n_dev_mul, CubeSetup *setup, const CellTable *cells,
                             hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const unsigned gs = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_cube_setup, dim3(gs), dim3(256), 0, stream, mx, rkeys, tkeys, pids, n, n_dev, n_dev_mul, setup,
                       cells ? *cells : CellTable{});
    return hipGetLastError();
}

hipError_t launch_s12(const DevMix &mx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *pids,
                      const int64_t *tidx, const double *s11ub, const double *s11lo, int64_t n, const uint32_t *n_dev,
                      int n_dev_mul, BoundOut out, double margin_gamma, int maxM, int maxN, bool with_top8, Tile tile,
                      CubeSetup *setup, hipStream_t stream, bool setup_done, TransRecs tr, int kpieces)
{
    if (n <= 0) return hipSuccess;
    if (!tile_ok(tile) || !setup) return hipErrorInvalidValue;
    // pieces of the kappa interval: 1, or 2 and 4 without the top-8 terms and
    // with the component records in LDS
    if (kpieces != 1 && ((kpieces != 2 && kpieces != 4) || with_top8 || mx.grec)) return hipErrorInvalidValue;
    if (!setup_done) {
        hipError_t e = launch_cube_setup(mx, rkeys, tkeys, pids, n, n_dev, n_dev_mul, setup, nullptr, stream);
        if (e) return e;
    }
    const bool grec = mx.grec != nullptr;
    const bool vlds = mx.n_prob > 1 && !grec;   // see kG
    const size_t lds = grec ? s12_lds_bytes(0, 0, tile.waves, false) : s12_lds_bytes(maxM, maxN, tile.waves, vlds);
    const unsigned g = (unsigned)std::min<int64_t>(std::min<int64_t>(tile.blocks, n), grec ? mx.grec_blocks : INT32_MAX);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(g), dim3(64 * tile.waves), lds, stream, mx, rkeys, tkeys, pids, tidx, s11ub,
                           s11lo, n, n_dev, n_dev_mul, out, margin_gamma, maxM, maxN, setup, tr);
    };
    if (grec)
        with_top8 ? go(k_s12<true, false, true>) : go(k_s12<false, false, true>);
    else if (with_top8)
        vlds ? go(k_s12<true, true, false>) : go(k_s12<true, false, false>);
    else if (kpieces == 2)
        vlds ? go(k_s12<false, true, false, 2>) : go(k_s12<false, false, false, 2>);
    else if (kpieces == 4)
        vlds ? go(k_s12<false, true, false, 4>) : go(k_s12<false, false, false, 4>);
    else
        vlds ? go(k_s12<false, true, false>) : go(k_s12<false, false, false>);
    return hipGetLastError();
}

}  // namespace gosma
