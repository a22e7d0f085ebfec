// Device core of SMA, the local optimiser of Algorithm 1 (Section 6): L-BFGS on the
// objective of Lemma 1 over the six pose parameters, one block per start.
//
// The objective f(r, t) = S11(t) - 2 S12(r, t) (eqs. 10-13, class sum eq. 17)
// and its gradient by the chain rule.  For a GMM component i let
// d_i = mu_1i - t, rho = |d_i|, kappa_i = rho^2/sigma_i^2 + 1 (eq. 13),
// u_i = d_i / rho and p_i = kappa_i u_i, with Jacobian
//   P_i = dp_i/dd_i = (rho/sigma^2 + 1/rho) I + (rho/sigma^2 - 1/rho) u u^T.
// A summand w w' Z(K)/(Z(a) Z(b)), K = |v|, has d log(summand) = (L(K)/K) v . dv
// - L(a) da - L(b) db with L(x) = coth x - 1/x.  Summing over the partners
// of component i,
//   U_i = sum_k T_ik, D_i = sum_k T_ik c_ik   (S11, v = p_i + p_k),
//   V_i = sum_j T_ij, C_i = sum_j T_ij c_ij   (S12, v = R p_i + kappa_2j mu_2j),
// with c = (L(K)/K) v, the derivative of f with respect to d_i is
//   2 P_i (D_i - R^T C_i) - 2 L(kappa_i) (2 d_i / sigma_i^2) (U_i - V_i)
// (S11 counts each ordered pair once per slot), d f/dt = -sum_i of that,
// under R -> exp([w]x) R the derivative is -2 sum_i (R p_i) x C_i, and
// d/dr = J(r)^T d/dw with J the left Jacobian of the angle-axis map.
//
// Evaluated without cancellation.  With v split into its part along the
// component's direction (u_i; w_i = R u_i for S12) and the rest v_perp,
//   P_i v = (kappa_i / rho) v_perp + 2 ((kappa_i - 1) / rho) (v . u) u,
// and the radial part of a summand's derivative combines with the kappa term
// into (2 (kappa_i - 1) / rho) T [L(K) (v . u) / K - L(kappa_i)] u, whose
// bracket is a small difference of two numbers near 1 (of order 1/kappa).
// With nu = 1 - L it is written as
//   nu(kappa_i) - nu(K) - L(K) |v x u|^2 / (K (K + v . u))     (v . u >= 0)
// (K - v . u = |v x u|^2 / (K + v . u)); for v . u < 0 the plain form has no
// cancellation.  So per component the sums are U, V (objective), the radial
// brackets Rr (S11) and Rv (S12), and the tangential vectors
//   Dt = sum_k T L(K)/K kappa_k (u_k - (u_k . u_i) u_i),
//   Ct = sum_j T L(K)/K kappa_2j (mu_2j - (mu_2j . w_i) w_i),
// and df/dd_i = 2 (kappa_i/rho) (Dt - R^T Ct) + 4 ((kappa_i - 1)/rho) (Rr - Rv) u_i,
// d/dw = -2 sum_i kappa_i w_i x Ct_i.
//
// Summands in FP32 log space: log of the summand = -a b q / (K + a + b) +
// l(K) - l(a) - l(b), l(y) = log((1 - e^{-2y}) / y), q the squared chord
// between the two directions, K^2 = (a + b)^2 - a b q; sums and the pose in
// FP64.
//
// L-BFGS (Nocedal and Wright, Numerical Optimization, Algorithm 7.4) with the
// direction followed along the path projected on the domain box and an
// Armijo backtracking line search; the constants are those of the library's
// documentation of gosma_refine.
#pragma once

#include <cmath>

#include "gosma_impl.h"

namespace gosma {
namespace sma {
namespace {

constexpr int kSmaThreads = 512;
constexpr int kSmaMaxMem = 16;
constexpr float kLn2f = 0.6931471805599453f;
constexpr float kLog2ef = 1.4426950408889634f;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * kLog2ef); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * kLn2f; }

// l(y) = log((1 - e^{-2y}) / y); below 1e-2 the series log 2 - y + y^2/6
// (error under y^4 / 180)
__device__ __forceinline__ float ell(float y)
{
    if (y < 1e-2f) return 0.69314718f - y + y * y * (1.0f / 6.0f);
    return flog((1.0f - fexp(-2.0f * y)) * frcp(y));
}

// L(K)/K = (coth K - 1/K)/K; series 1/3 - K^2/45 below 1e-2
__device__ __forceinline__ float langevin_over(float K)
{
    if (K < 1e-2f) return 1.0f / 3.0f - K * K * (1.0f / 45.0f);
    const float e = fexp(-2.0f * K);
    const float coth = (1.0f + e) * frcp(1.0f - e);
    return (coth - frcp(K)) * frcp(K);
}

// L(K) = coth K - 1/K and nu(K) = 1 - L(K) = 1/K - 2 e^{-2K} / (1 - e^{-2K});
// series L = K/3 - K^3/45 below 1e-2
__device__ __forceinline__ void langevin_nu(float K, float &L, float &nu)
{
    if (K < 1e-2f) {
        L = K * (1.0f / 3.0f - K * K * (1.0f / 45.0f));
        nu = 1.0f - L;
        return;
    }
    const float e = fexp(-2.0f * K), ie = frcp(1.0f - e), iK = frcp(K);
    nu = iK - 2.0f * e * ie;
    L = 1.0f - nu;
}

// radial bracket L(K) (v . u) / K - L(a) of a summand (see the header), from
// nu(a), K, v . u and |v x u|^2
__device__ __forceinline__ float radial_bracket(float nua, float K, float vu, float s2)
{
    float L, nuK;
    langevin_nu(K, L, nuK);
    if (vu >= 0.0f) return nua - nuK - L * s2 * frcp(K * (K + vu));
    return L * vu * frcp(K) - (1.0f - nua);
}

// Rodrigues' formula R = I + sin(th) [k]x + (1 - cos th) [k]x^2 and the left
// Jacobian J = I + A [r]x + B [r]x^2, A = (1 - cos th)/th^2, B = (th - sin th)/th^3
__device__ void rot_and_jac(const double r[3], double R[9], double J[9])
{
    const double t2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2], th = sqrt(t2);
    double s, c, A, B, sa, sb;   // R = I + sa [r]x + sb [r]x^2
    sincos(th, &s, &c);
    if (th < 1e-4) {
        sa = 1.0 - t2 / 6.0 + t2 * t2 / 120.0;
        sb = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
        A = sb;
        B = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
    } else {
        sa = s / th;
        sb = (1.0 - c) / t2;
        A = sb;
        B = (th - s) / (t2 * th);
    }
    const double K[9] = {0.0, -r[2], r[1], r[2], 0.0, -r[0], -r[1], r[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double k2 = 0.0;
            for (int k = 0; k < 3; ++k) k2 += K[3 * i + k] * K[3 * k + j];
            const double id = i == j ? 1.0 : 0.0;
            R[3 * i + j] = id + sa * K[3 * i + j] + sb * k2;
            J[3 * i + j] = id + A * K[3 * i + j] + B * k2;
        }
}

struct SmaShared {
    double x[6];          // the pose being evaluated
    double red[kSmaThreads / 64][9];
    double f, scale, g[6];
    int infeasible;
    int go;               // 1: evaluate x again (line search), 0: stop
};

// f and its gradient at sh.x for the problem P (block-wide); returns via sh.
// LDS per GMM component: u_i (3), kappa_i, w_i = R u_i (3), l(kappa_i), its
// weight and class; per vMF component: mu (3), kappa, weight, l(kappa).
__device__ void eval_pose(const DevMix &mx, const ProbDesc &P, SmaShared &sh, float4 *gA, float4 *gB, float2 *gC,
                          int *gcls, float4 *vA, float2 *vB)
{
    const int tid = threadIdx.x, T = blockDim.x;
    double R[9], J[9], x[6];
    for (int a = 0; a < 6; ++a) x[a] = sh.x[a];
    rot_and_jac(x, R, J);
    int infeas = 0;
    for (int i = tid; i < P.M; i += T) {
        const int g = P.gmm_off + i;
        const double d[3] = {mx.mu[3 * g] - x[3], mx.mu[3 * g + 1] - x[4], mx.mu[3 * g + 2] - x[5]};
        const double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        infeas |= rho < P.zeta;
        const double kap = rho * rho * mx.isig2[g] + 1.0;
        const double u[3] = {d[0] / rho, d[1] / rho, d[2] / rho};
        double w[3];
        for (int a = 0; a < 3; ++a) w[a] = R[3 * a] * u[0] + R[3 * a + 1] * u[1] + R[3 * a + 2] * u[2];
        gA[i] = make_float4((float)u[0], (float)u[1], (float)u[2], (float)kap);
        gB[i] = make_float4((float)w[0], (float)w[1], (float)w[2], ell((float)kap));
        // nu(kappa_i) = 1/kappa - 2 e / (1 - e), e = e^{-2 kappa} (kappa >= 1)
        const double e2k = exp(-2.0 * kap);
        gC[i] = make_float2(mx.w1[g], (float)(1.0 / kap - 2.0 * e2k / (1.0 - e2k)));
        int c = 0;
        while (c + 1 < P.n_cls && !(g < mx.cls[P.cls_off + c].g1)) ++c;
        gcls[i] = c;
    }
    for (int j = tid; j < P.N; j += T) {
        const float4 a = mx.vmf[2 * (int64_t)(P.vmf_off + j)], b = mx.vmf[2 * (int64_t)(P.vmf_off + j) + 1];
        vA[j] = a;
        vB[j] = make_float2(b.x, -flog(b.y));   // l(kappa) = -log G(kappa)
    }
    if (tid == 0) sh.infeasible = 0;
    __syncthreads();
    if (infeas) atomicOr(&sh.infeasible, 1);

    // S threads per GMM component (a power of two within a wave)
    int S = 1;
    while (S < 64 && 2 * S * P.M <= T) S *= 2;
    const int sub = tid & (S - 1);
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // f, scale, d/dt (3), d/dw (3), unused
    const int iters = (P.M + T / S - 1) / (T / S);
    for (int it = 0; it < iters; ++it) {
        const int i = it * (T / S) + tid / S;
        const bool live = i < P.M;
        const int ii = live ? i : P.M - 1;
        const float4 Ai = gA[ii], Bi = gB[ii];
        const float wi = gC[ii].x;
        const ClassRange cr = mx.cls[P.cls_off + gcls[ii]];
        double U = 0.0, V = 0.0;
        float Rr = 0.0f, Rv = 0.0f;
        float D[3] = {0, 0, 0}, Cc[3] = {0, 0, 0};   // tangential sums Dt, Ct
        if (live) {
            const float a = Ai.w, la = Bi.w, nua = gC[ii].y;
            for (int k = cr.g0 - P.gmm_off + sub; k < cr.g1 - P.gmm_off; k += S) {
                const float4 Ak = gA[k];
                const float b = Ak.w;
                const float dx = Ai.x - Ak.x, dy = Ai.y - Ak.y, dz = Ai.z - Ak.z;
                const float q = dx * dx + dy * dy + dz * dz;
                const float K = fsqrt(fmaxf((a + b) * (a + b) - a * b * q, 0.0f));
                const float lg = -a * b * q * frcp(K + a + b) + ell(K) - la - gB[k].w;
                const float Tk = wi * gC[k].x * fexp(lg);
                // v = kappa_i u_i + kappa_k u_k: v . u_i = a + b cos, |v x u_i|^2 = b^2 sin^2
                const float cs = 1.0f - 0.5f * q;
                const float vu = a + b * cs, s2 = b * b * q * (1.0f - 0.25f * q);
                Rr += Tk * radial_bracket(nua, K, vu, s2);
                const float c = Tk * langevin_over(K) * b;
                D[0] += c * (Ak.x - cs * Ai.x);
                D[1] += c * (Ak.y - cs * Ai.y);
                D[2] += c * (Ak.z - cs * Ai.z);
                U += (double)Tk;
            }
            for (int j = cr.v0 - P.vmf_off + sub; j < cr.v1 - P.vmf_off; j += S) {
                const float4 Aj = vA[j];
                const float2 Bj = vB[j];
                const float b = Aj.w;
                const float dx = Bi.x - Aj.x, dy = Bi.y - Aj.y, dz = Bi.z - Aj.z;
                const float q = dx * dx + dy * dy + dz * dz;
                const float K = fsqrt(fmaxf((a + b) * (a + b) - a * b * q, 0.0f));
                const float lg = -a * b * q * frcp(K + a + b) + ell(K) - la - Bj.y;
                const float Tj = wi * Bj.x * fexp(lg);
                const float cs = 1.0f - 0.5f * q;
                const float vu = a + b * cs, s2 = b * b * q * (1.0f - 0.25f * q);
                Rv += Tj * radial_bracket(nua, K, vu, s2);
                const float c = Tj * langevin_over(K) * b;
                Cc[0] += c * (Aj.x - cs * Bi.x);
                Cc[1] += c * (Aj.y - cs * Bi.y);
                Cc[2] += c * (Aj.z - cs * Bi.z);
                V += (double)Tj;
            }
        }
        // combine the S partial sums of the component (lanes sub = 0 .. S-1 are adjacent)
        for (int off = 1; off < S; off <<= 1) {
            U += __shfl_xor(U, off, 64);
            V += __shfl_xor(V, off, 64);
            Rr += __shfl_xor(Rr, off, 64);
            Rv += __shfl_xor(Rv, off, 64);
            for (int a = 0; a < 3; ++a) {
                D[a] += __shfl_xor(D[a], off, 64);
                Cc[a] += __shfl_xor(Cc[a], off, 64);
            }
        }
        if (live && sub == 0) {
            const int g = P.gmm_off + i;
            const double d[3] = {mx.mu[3 * g] - x[3], mx.mu[3 * g + 1] - x[4], mx.mu[3 * g + 2] - x[5]};
            const double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double is2 = mx.isig2[g], kap = rho * rho * is2 + 1.0;
            const double u[3] = {d[0] / rho, d[1] / rho, d[2] / rho};
            // df/dd_i = 2 (kappa/rho) (Dt - R^T Ct) + 4 ((kappa - 1)/rho) (Rr - Rv) u
            const double tg = 2.0 * kap / rho, rd = 4.0 * rho * is2 * ((double)Rr - (double)Rv);
            double w[3];
            for (int a = 0; a < 3; ++a) {
                const double E = (double)D[a] - (R[a] * Cc[0] + R[3 + a] * Cc[1] + R[6 + a] * Cc[2]);
                acc[2 + a] -= tg * E + rd * u[a];   // d/dt = -d/dd
                w[a] = R[3 * a] * u[0] + R[3 * a + 1] * u[1] + R[3 * a + 2] * u[2];
            }
            // d/dw = -2 kappa_i w_i x Ct_i
            acc[5] += -2.0 * kap * (w[1] * Cc[2] - w[2] * Cc[1]);
            acc[6] += -2.0 * kap * (w[2] * Cc[0] - w[0] * Cc[2]);
            acc[7] += -2.0 * kap * (w[0] * Cc[1] - w[1] * Cc[0]);
            acc[0] += U - 2.0 * V;
            acc[1] += U + 2.0 * V;
        }
    }
    // block sums
    const int lane = tid & 63, wv = tid >> 6;
    for (int a = 0; a < 8; ++a) {
        double v = acc[a];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sh.red[wv][a] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < T / 64; ++w)
            for (int a = 0; a < 8; ++a) s[a] += sh.red[w][a];
        sh.f = sh.infeasible ? INFINITY : s[0];
        sh.scale = s[1];
        for (int a = 0; a < 3; ++a) {
            sh.g[a] = J[a] * s[5] + J[3 + a] * s[6] + J[6 + a] * s[7];   // J^T d/dw
            sh.g[3 + a] = s[2 + a];
        }
    }
    __syncthreads();
}

// LDS of one block: the arrays eval_pose stages for a problem of M x N.
struct SmaLds {
    float4 *gA, *gB, *vA;
    float2 *gC, *vB;
    int *gcls;
};
__device__ __forceinline__ SmaLds sma_lds(float4 *base, int M, int N)
{
    SmaLds L;
    L.gA = base;
    L.gB = L.gA + M;
    L.vA = L.gB + M;
    L.gC = reinterpret_cast<float2 *>(L.vA + N);
    L.vB = L.gC + M;
    L.gcls = reinterpret_cast<int *>(L.vB + N);
    return L;
}

// L-BFGS state of a block (LDS); the block's thread 0 drives it.
struct SmaState {
    double S[kSmaMaxMem][6], Y[kSmaMaxMem][6], rho[kSmaMaxMem];
};

// Run SMA from sh.x (set by the caller before a barrier) for problem P with
// the whole block.  On return (after a barrier) thread 0 holds the result in
// x, f, g and its iteration count (-1: the start is outside the box or within
// zeta of a mean).
__device__ int sma_run(const DevMix &mx, const ProbDesc &P, SmaShared &sh, SmaState &st, const SmaLds &L,
                       int max_iters, int memory, double gtol, double ftol, double x[6], double &f, double g[6])
{
    const int tid = threadIdx.x;
    int inbox = 1;
    for (int a = 0; a < 3; ++a) {
        inbox &= sh.x[a] >= P.r_lo[a] && sh.x[a] <= P.r_lo[a] + P.r_w[a];
        inbox &= sh.x[3 + a] >= P.t_lo[a] && sh.x[3 + a] <= P.t_lo[a] + P.t_w[a];
    }
    for (int a = 0; a < 6; ++a) {
        x[a] = sh.x[a];
        g[a] = 0.0;
    }
    f = INFINITY;
    if (!inbox) return -1;   // uniform across the block
    eval_pose(mx, P, sh, L.gA, L.gB, L.gC, L.gcls, L.vA, L.vB);
    f = sh.f;
    const double scale = sh.scale;
    for (int a = 0; a < 6; ++a) g[a] = sh.g[a];
    if (!(f < INFINITY)) return -1;
    double lo[6], hi[6], al_k[kSmaMaxMem];
    for (int a = 0; a < 3; ++a) {
        lo[a] = P.r_lo[a];
        hi[a] = P.r_lo[a] + P.r_w[a];
        lo[3 + a] = P.t_lo[a];
        hi[3 + a] = P.t_lo[a] + P.t_w[a];
    }
    int it = 0, nst = 0, head = 0;
    const int m = memory < 1 ? 1 : (memory > kSmaMaxMem ? kSmaMaxMem : memory);
    for (;;) {
        double dir[6], step = 1.0;
        if (tid == 0) {
            // 1. projected-gradient stop; 2. L-BFGS direction
            bool running = it < max_iters;
            double pg = 0.0;
            for (int a = 0; a < 6; ++a) {
                double ga = g[a];
                if ((x[a] <= lo[a] && ga > 0.0) || (x[a] >= hi[a] && ga < 0.0)) ga = 0.0;
                pg = fmax(pg, fabs(ga));
            }
            if (pg <= gtol * scale) running = false;
            if (running) {
                double q[6], gn = 0.0;
                for (int a = 0; a < 6; ++a) {
                    q[a] = g[a];
                    gn += g[a] * g[a];
                }
                gn = sqrt(gn);
                for (int k = 0; k < nst; ++k) {
                    const int s = (head - 1 - k + kSmaMaxMem) % kSmaMaxMem;
                    double sq = 0.0;
                    for (int a = 0; a < 6; ++a) sq += st.S[s][a] * q[a];
                    al_k[s] = st.rho[s] * sq;
                    for (int a = 0; a < 6; ++a) q[a] -= al_k[s] * st.Y[s][a];
                }
                double h0;
                if (nst > 0) {
                    const int s = (head - 1 + kSmaMaxMem) % kSmaMaxMem;
                    double sy = 0.0, yy = 0.0;
                    for (int a = 0; a < 6; ++a) {
                        sy += st.S[s][a] * st.Y[s][a];
                        yy += st.Y[s][a] * st.Y[s][a];
                    }
                    h0 = sy / yy;
                } else {
                    h0 = fmin(1.0, 0.05 / gn);
                }
                for (int a = 0; a < 6; ++a) q[a] *= h0;
                for (int k = nst - 1; k >= 0; --k) {
                    const int s = (head - 1 - k + kSmaMaxMem) % kSmaMaxMem;
                    double yq = 0.0;
                    for (int a = 0; a < 6; ++a) yq += st.Y[s][a] * q[a];
                    const double b = st.rho[s] * yq;
                    for (int a = 0; a < 6; ++a) q[a] += (al_k[s] - b) * st.S[s][a];
                }
                double gdir = 0.0;
                for (int a = 0; a < 6; ++a) {
                    dir[a] = -q[a];
                    gdir += g[a] * dir[a];
                }
                if (!(gdir < 0.0)) {
                    const double h = fmin(1.0, 0.05 / gn);
                    for (int a = 0; a < 6; ++a) dir[a] = -h * g[a];
                    nst = 0;
                }
                for (int a = 0; a < 6; ++a) sh.x[a] = fmin(fmax(x[a] + dir[a], lo[a]), hi[a]);
            }
            sh.go = running;
        }
        __syncthreads();
        if (!sh.go) break;
        // 3. backtracking line search: the block evaluates each trial pose
        bool accepted = false;
        for (int ls = 0; ls <= 40; ++ls) {
            eval_pose(mx, P, sh, L.gA, L.gB, L.gC, L.gcls, L.vA, L.vB);
            if (tid == 0) {
                double dec = 0.0;
                for (int a = 0; a < 6; ++a) dec += g[a] * (sh.x[a] - x[a]);
                accepted = sh.f <= f + 1e-4 * dec;
                if (!accepted && ls < 40) {
                    step *= 0.5;
                    for (int a = 0; a < 6; ++a) sh.x[a] = fmin(fmax(x[a] + step * dir[a], lo[a]), hi[a]);
                }
                sh.go = accepted || ls == 40 ? 0 : 1;
            }
            __syncthreads();
            if (!sh.go) break;
        }
        if (tid == 0) {
            bool running = accepted;
            if (accepted) {
                // 4. curvature pair; 5. gain stop
                ++it;
                double sv[6], yv[6], sy = 0.0, ss = 0.0, yy = 0.0;
                for (int a = 0; a < 6; ++a) {
                    sv[a] = sh.x[a] - x[a];
                    yv[a] = sh.g[a] - g[a];
                    sy += sv[a] * yv[a];
                    ss += sv[a] * sv[a];
                    yy += yv[a] * yv[a];
                }
                const double fprev = f;
                for (int a = 0; a < 6; ++a) {
                    x[a] = sh.x[a];
                    g[a] = sh.g[a];
                }
                f = sh.f;
                if (sy > 1e-12 * sqrt(ss * yy)) {
                    for (int a = 0; a < 6; ++a) {
                        st.S[head][a] = sv[a];
                        st.Y[head][a] = yv[a];
                    }
                    st.rho[head] = 1.0 / sy;
                    head = (head + 1) % kSmaMaxMem;
                    if (nst < m) ++nst;
                }
                if (fprev - f <= ftol * (fabs(f) + scale)) running = false;
            }
            sh.go = running;
        }
        __syncthreads();
        if (!sh.go) break;
    }
    __syncthreads();
    return it;
}

}  // namespace
}  // namespace sma
}  // namespace gosma
