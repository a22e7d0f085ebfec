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
// Work mapping: one wavefront (64 lanes) per cell.  The per-component
// quantities of the cell (kappa, its interval over the cell, uncertainty
// half-angles, rotated directions, normaliser factors) are computed in FP64,
// one component per lane, and staged in LDS as FP32 structure-of-arrays.  The
// pair sums then run over the flattened (i, j) rectangle of each class, 64
// consecutive pairs per step, with FP32 arithmetic in log space and FP64
// accumulation per lane, and a wavefront shuffle reduction at the end.
//
// Summand algebra.  With G(y) = y / (1 - e^{-2y}) and h(K) = (1 - e^{-2K})/K,
//   Z(K) / (Z(a) Z(b)) = e^{K - a - b} h(K) G(a) G(b)            (eq. 2)
// and K - a - b = -a b q / (K + a + b) for the squared chord q = |u - v|^2 of
// the two directions (K^2 = (a + b)^2 - a b q), which avoids the cancellation
// of K - a - b for concentrations in the thousands.
#include <algorithm>
#include <cmath>

#include "gosma_impl.h"

namespace gosma {

namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Decode an octree key of the box with lower corner lo and widths w.
__device__ __forceinline__ void decode_key(uint64_t key, const double *lo, const double *w, double c[3],
                                           double h[3])
{
    const uint64_t mask = (1ull << 19) - 1;
    int level = (int)((key >> 57) & 63);
    double scale = ldexp(1.0, -(level + 1));
    uint64_t idx[3] = {(key >> 38) & mask, (key >> 19) & mask, key & mask};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        h[k] = w[k] * scale;
        c[k] = lo[k] + (double)(2 * idx[k] + 1) * h[k];
    }
}

// Rotation matrix of the angle-axis vector r (Section 5.1), as
// I + A [r]x + B [r]x^2 with A = sin|r|/|r|, B = (1 - cos|r|)/|r|^2.
__device__ void rotation_matrix(const double r[3], double R[9])
{
    double th2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double A, B;
    if (th2 < 1e-8) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    } else {
        double th = sqrt(th2), sh, ch;
        sincos(0.5 * th, &sh, &ch);
        A = 2.0 * sh * ch / th;
        B = 2.0 * sh * sh / th2;
    }
    // [r]x^2 = r r^T - |r|^2 I
    R[0] = 1.0 + B * (r[0] * r[0] - th2);
    R[4] = 1.0 + B * (r[1] * r[1] - th2);
    R[8] = 1.0 + B * (r[2] * r[2] - th2);
    R[1] = -A * r[2] + B * r[0] * r[1];
    R[3] = A * r[2] + B * r[0] * r[1];
    R[2] = A * r[1] + B * r[0] * r[2];
    R[6] = -A * r[1] + B * r[0] * r[2];
    R[5] = -A * r[0] + B * r[1] * r[2];
    R[7] = A * r[0] + B * r[1] * r[2];
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

__device__ TransPrep trans_prep(const double *mu, double isig2, const double t0[3], const double tau[3],
                                double zeta)
{
    TransPrep o;
    double c[3] = {mu[0] - t0[0], mu[1] - t0[1], mu[2] - t0[2]};
    double rho2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    double rho = sqrt(rho2);
    for (int k = 0; k < 3; ++k) o.u[k] = c[k] / rho;
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

    // psi_t: largest vertex angle between mu - v and mu - t0 (Lemma 3); pi if
    // mu is in the cell or any vertex angle exceeds pi/2.  For angles below
    // pi/2 the largest angle has the largest sine, |c x (s tau)|^2 / (|a|^2 |c|^2)
    // with a = c - s tau, computed without cancellation.
    bool guard = inside;
    double best_s2 = -1.0, best_c2 = 1.0;
    for (int v = 0; v < 8; ++v) {
        double st[3] = {(v & 4) ? tau[0] : -tau[0], (v & 2) ? tau[1] : -tau[1], (v & 1) ? tau[2] : -tau[2]};
        double a[3] = {c[0] - st[0], c[1] - st[1], c[2] - st[2]};
        double a2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
        double dot = rho2 - (st[0] * c[0] + st[1] * c[1] + st[2] * c[2]);
        double cr[3] = {c[1] * st[2] - c[2] * st[1], c[2] * st[0] - c[0] * st[2], c[0] * st[1] - c[1] * st[0]};
        double den = a2 * rho2;
        double s2 = (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) / den;
        if (dot < 0.0) guard = true;
        if (s2 > best_s2) {
            best_s2 = s2;
            best_c2 = dot * dot / den;
        }
    }
    if (guard) {
        o.cps = 0.0;
        o.sps = 1.0;
        o.psi = (float)kPi;
    } else {
        double sp = sqrt(best_s2), cp = sqrt(best_c2);
        double nrm = sqrt(best_s2 + best_c2);     // 1 up to rounding
        sp /= nrm;
        cp /= nrm;
        o.cps = sqrt(0.5 * (1.0 + cp));
        o.sps = sp / (2.0 * o.cps);
        o.psi = atan2f((float)sp, (float)cp);
    }
    return o;
}

__device__ __forceinline__ double G_of(double y) { return y / (-expm1(-2.0 * y)); }
__device__ __forceinline__ double coth_of(double y) { return 1.0 + 2.0 / expm1(2.0 * y); }
// nu(y) = 1 - L(y) = 1 + 1/y - coth(y), L the derivative of log Z (y >= 1 here).
__device__ __forceinline__ double nu_of(double y) { return 1.0 / y - 2.0 / expm1(2.0 * y); }

// Pair kernel pieces for concentrations a, b and squared chord q.
struct PairK {
    float x;      // K - a - b
    float K, r;   // K and 1 / (K (K + a + b))
    float invK;   // 1 / K
    float hK;     // (1 - e^{-2K}) / K
    float nuK;    // 1 + 1/K - coth K
};

__device__ __forceinline__ PairK pair_k(float a, float b, float q)
{
    PairK o;
    float s = a + b;
    float t = a * b * q;
    float K2 = fmaxf(fmaf(s, s, -t), 0.0f);
    float K = fmaxf(fsqrt(K2), 1e-20f);
    float den = K + s;
    float r = frcp(K * den);
    o.K = K;
    o.r = r;
    o.x = -t * K * r;
    o.invK = den * r;
    o.hK = o.invK;
    o.nuK = o.invK;
    if (__builtin_expect(K < 9.0f, 0)) {
        // e^{-2K} is not negligible next to 1 in FP32 below K = 9.
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
    return o;
}

// ---------------------------------------------------------------------------
// S11 over translation cells
// ---------------------------------------------------------------------------

enum S11Field { A_UX, A_UY, A_UZ, A_KAP, A_GK, A_AC, A_HA, A_GAC, A_NU, A_LAM, A_CPS, A_SPS, A_W, A_NF };

__device__ void s11_cell(DevMix mx, const uint64_t *__restrict__ tkeys, const uint32_t *__restrict__ pids,
                         int64_t cell, S11Out out, int stride, float *lds, int lane);

__global__ __launch_bounds__(64) void k_s11(DevMix mx, const uint64_t *__restrict__ tkeys,
                                            const uint32_t *__restrict__ pids, int64_t nt_host,
                                            const uint32_t *__restrict__ nt_dev, S11Out out, int stride)
{
    extern __shared__ float lds[];
    const int lane = threadIdx.x;
    const int64_t nt = nt_dev ? (int64_t)nt_dev[0] : nt_host;
    for (int64_t cell = blockIdx.x; cell < nt; cell += gridDim.x) {
        __syncthreads();
        s11_cell(mx, tkeys, pids, cell, out, stride, lds, lane);
    }
}

__device__ void s11_cell(DevMix mx, const uint64_t *__restrict__ tkeys, const uint32_t *__restrict__ pids,
                         int64_t cell, S11Out out, int stride, float *lds, int lane)
{
    const uint32_t pid = pids ? pids[cell] : 0u;
    if (pid >= (uint32_t)mx.n_prob) {     // invalid problem index: no bound
        if (lane == 0) {
            out.ub[cell] = NAN;
            out.lo[cell] = NAN;
        }
        return;
    }
    const ProbDesc P = mx.prob[pid];
    double t0[3], tau[3];
    decode_key(tkeys[cell], P.t_lo, P.t_w, t0, tau);

    // per-component prep; the diagonal (i = i') summands are added here:
    // Z(2k)/Z(k)^2 = k coth(k) / 2 at the centre, and at the low end of the
    // kappa interval for the lower bound (the angle is exactly 0 and the
    // summand increases with kappa).
    double dub = 0.0, dlo = 0.0;
    int drop = 0, ubinf = 0;
    for (int i = lane; i < P.M; i += 64) {
        int g = P.gmm_off + i;
        TransPrep tp = trans_prep(mx.mu + 3 * g, mx.isig2[g], t0, tau, P.zeta);
        drop |= tp.drop;
        ubinf |= tp.ub_inf;
        double w = mx.w1[g];
        dub += w * w * 0.5 * tp.kap * coth_of(tp.kap);
        dlo += w * w * 0.5 * tp.klo * coth_of(tp.klo);
        lds[A_UX * stride + i] = (float)tp.u[0];
        lds[A_UY * stride + i] = (float)tp.u[1];
        lds[A_UZ * stride + i] = (float)tp.u[2];
        lds[A_KAP * stride + i] = (float)tp.kap;
        lds[A_GK * stride + i] = (float)G_of(tp.kap);
        lds[A_AC * stride + i] = (float)tp.ac;
        lds[A_HA * stride + i] = (float)tp.ha;
        lds[A_GAC * stride + i] = (float)G_of(tp.ac);
        lds[A_NU * stride + i] = (float)nu_of(tp.ac);
        lds[A_LAM * stride + i] = (float)fmin(1.0 / 3.0, 1.0 / (tp.klo * tp.klo));
        lds[A_CPS * stride + i] = (float)tp.cps;
        lds[A_SPS * stride + i] = (float)tp.sps;
        lds[A_W * stride + i] = (float)w;
    }
    drop = wave_or(drop);
    ubinf = wave_or(ubinf);
    __syncthreads();
    if (drop) {
        if (lane == 0) {
            out.ub[cell] = INFINITY;
            out.lo[cell] = INFINITY;
        }
        return;
    }

    double acc_ub = dub, acc_lo = dlo;
    for (int c = 0; c < P.n_cls; ++c) {
        const ClassRange cr = mx.cls[P.cls_off + c];
        const int n = cr.g1 - cr.g0;
        if (n < 2) continue;
        const int base = cr.g0 - P.gmm_off;
        // The upper triangle (i <= i') of the class, folded into a rectangle of
        // n2/2 rows and n2 + 1 columns (n2 = n rounded up to even): folded row
        // r holds triangle rows r and n2 - 1 - r.
        const int n2 = n + (n & 1);
        const int R = n2 >> 1, C = n2 + 1;
        int r = lane / C, col = lane % C;
        const int dr = 64 / C, dc = 64 % C;
        for (; r < R;) {
            int i, i2;
            if (col < n2 - r) {
                i = r;
                i2 = r + col;
            } else {
                i = n2 - 1 - r;
                i2 = i + col - (n2 - r);
            }
            if (i2 < n && i != i2) {
                const int a_ = base + i, b_ = base + i2;
                float ux = lds[A_UX * stride + a_], uy = lds[A_UY * stride + a_], uz = lds[A_UZ * stride + a_];
                float vx = lds[A_UX * stride + b_], vy = lds[A_UY * stride + b_], vz = lds[A_UZ * stride + b_];
                float dx = ux - vx, dy = uy - vy, dz = uz - vz;
                float q = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                float px = ux + vx, py = uy + vy, pz = uz + vz;
                float pp = fmaf(px, px, fmaf(py, py, pz * pz));
                float w2 = 2.0f * lds[A_W * stride + a_] * lds[A_W * stride + b_];
                // upper bound summand at the centre
                {
                    PairK k = pair_k(lds[A_KAP * stride + a_], lds[A_KAP * stride + b_], q);
                    float v = fexp2(k.x * kLog2e) * k.hK * lds[A_GK * stride + a_] * lds[A_GK * stride + b_];
                    acc_ub += (double)(w2 * v);
                }
                // lower bound summand: angle A = min(pi, theta + psi_i + psi_i') (eq. 24)
                // via half angles: A/2 = theta/2 + (psi_i + psi_i')/2, clamped at pi/2.
                {
                    // half-angle sine and cosine from the two chords |u - v|, |u + v|
                    float st = 0.5f * fsqrt(q), ct = 0.5f * fsqrt(pp);
                    float ci = lds[A_CPS * stride + a_], si = lds[A_SPS * stride + a_];
                    float cj = lds[A_CPS * stride + b_], sj = lds[A_SPS * stride + b_];
                    float ca = ci * cj - si * sj, sa = si * cj + ci * sj;
                    float cA = ct * ca - st * sa, sA = st * ca + ct * sa;
                    sA = cA <= 0.0f ? 1.0f : sA;
                    float qA = 4.0f * sA * sA;
                    float a = lds[A_AC * stride + a_], b = lds[A_AC * stride + b_];
                    float ha = lds[A_HA * stride + a_], hb = lds[A_HA * stride + b_];
                    PairK k = pair_k(a, b, qA);
                    // gradient of g = log Z(K) - log Z(a) - log Z(b) at the box centre:
                    // g_a = (K_a - 1) + nu(a) - nu(K) K_a with
                    // K_a - 1 = b qA (a - b - K) / (2 K (K + a + b)).
                    float ka1 = 0.5f * b * qA * (a - b - k.K) * k.r;
                    float kb1 = 0.5f * a * qA * (b - a - k.K) * k.r;
                    float ga = ka1 + lds[A_NU * stride + a_] - k.nuK * (1.0f + ka1);
                    float gb = kb1 + lds[A_NU * stride + b_] - k.nuK * (1.0f + kb1);
                    float lam = fmaxf(lds[A_LAM * stride + a_], lds[A_LAM * stride + b_]);
                    float corr = -fabsf(ga) * ha - fabsf(gb) * hb - 0.5f * lam * fmaf(ha, ha, hb * hb);
                    float v = fexp2((k.x + corr) * kLog2e) * k.hK * lds[A_GAC * stride + a_] *
                              lds[A_GAC * stride + b_];
                    acc_lo += (double)(w2 * v);
                }
            }
            col += dc;
            r += dr;
            if (col >= C) {
                col -= C;
                r += 1;
            }
        }
    }
    acc_ub = wave_sum(acc_ub);
    acc_lo = wave_sum(acc_lo);
    if (lane == 0) {
        out.ub[cell] = ubinf ? INFINITY : acc_ub;
        out.lo[cell] = acc_lo;
    }
}

// ---------------------------------------------------------------------------
// S12 over rotation x translation cells, and the final bounds
// ---------------------------------------------------------------------------

enum S12Field { B_WX, B_WY, B_WZ, B_KAP, B_GK, B_AC, B_HA, B_GAC, B_NU, B_CPS, B_SPS, B_KHI, B_COTH, B_W, B_NF };
// FP64 copies of the inputs of the lower-bound exponent (see s12_lower_exponent64)
enum S12Field64 { D_WX, D_WY, D_WZ, D_CPS, D_SPS, D_AC, D_HA, D_NU, D_NF };

// Exponent of the S12 upper summand in FP64.  The FP32 path loses about
// u |x| to cancellation when x = K - a - b and the Taylor correction are both
// large (wide kappa intervals of large translation cells), so those terms are
// recomputed here from FP64 copies of their inputs.
__device__ __noinline__ float s12_lower_exponent64(const double *L64, int stride, int a_, const double *v64)
{
    const double wx = L64[D_WX * stride + a_], wy = L64[D_WY * stride + a_], wz = L64[D_WZ * stride + a_];
    const double mx = v64[0], my = v64[1], mz = v64[2], b = v64[3];
    const double dx = wx - mx, dy = wy - my, dz = wz - mz;
    const double px = wx + mx, py = wy + my, pz = wz + mz;
    const double st = 0.5 * sqrt(dx * dx + dy * dy + dz * dz), ct = 0.5 * sqrt(px * px + py * py + pz * pz);
    const double sB = fmax(st * L64[D_CPS * stride + a_] - ct * L64[D_SPS * stride + a_], 0.0);
    const double qB = 4.0 * sB * sB;
    const double a = L64[D_AC * stride + a_], ha = L64[D_HA * stride + a_];
    const double s = a + b, t = a * b * qB;
    const double K = fmax(sqrt(fmax(s * s - t, 0.0)), 1e-300);
    const double r = 1.0 / (K * (K + s));
    const double x = -t * K * r, invK = (K + s) * r;
    const double nuK = invK - 2.0 / expm1(2.0 * K);
    const double ka1 = 0.5 * b * qB * (a - b - K) * r;
    const double ga = ka1 + L64[D_NU * stride + a_] - nuK * (1.0 + ka1);
    const double b2s2 = b * b * qB * (1.0 - 0.25 * qB);
    const double iK = fmin(invK, 1e6);
    const double G2 = ha <= 0.5 * K ? fmin(1.0 / 3.0, 4.0 * iK * iK) + fmin(1.0 / 3.0, 8.0 * b2s2 * iK * iK * iK)
                                    : 2.0 / 3.0;
    return (float)(x + fabs(ga) * ha + 0.5 * G2 * ha * ha);
}

template <bool TOP8>
__device__ void s12_cube(DevMix mx, const uint64_t *__restrict__ rkeys, const uint64_t *__restrict__ tkeys,
                         const uint32_t *__restrict__ pids, const int64_t *__restrict__ tidx,
                         const double *__restrict__ s11ub, const double *__restrict__ s11lo, int64_t cube,
                         BoundOut out, double gamma, int stride, float *lds, int lane);

template <bool TOP8>
__global__ __launch_bounds__(64) void k_s12(DevMix mx, const uint64_t *__restrict__ rkeys,
                                            const uint64_t *__restrict__ tkeys, const uint32_t *__restrict__ pids,
                                            const int64_t *__restrict__ tidx, const double *__restrict__ s11ub,
                                            const double *__restrict__ s11lo, int64_t n_host,
                                            const uint32_t *__restrict__ n_dev, int n_dev_mul, BoundOut out,
                                            double gamma, int stride)
{
    extern __shared__ float lds[];
    const int lane = threadIdx.x;
    const int64_t n = n_dev ? (int64_t)n_dev[0] * n_dev_mul : n_host;
    for (int64_t cube = blockIdx.x; cube < n; cube += gridDim.x) {
        __syncthreads();
        s12_cube<TOP8>(mx, rkeys, tkeys, pids, tidx, s11ub, s11lo, cube, out, gamma, stride, lds, lane);
    }
}

template <bool TOP8>
__device__ void s12_cube(DevMix mx, const uint64_t *__restrict__ rkeys, const uint64_t *__restrict__ tkeys,
                         const uint32_t *__restrict__ pids, const int64_t *__restrict__ tidx,
                         const double *__restrict__ s11ub, const double *__restrict__ s11lo, int64_t cube,
                         BoundOut out, double gamma, int stride, float *lds, int lane)
{
    const uint32_t pid = pids ? pids[cube] : 0u;
    if (pid >= (uint32_t)mx.n_prob) {     // invalid problem index: no bound, both drop flags
        if (lane == 0) {
            out.ub[cube] = NAN;
            out.lb[cube] = NAN;
            if (out.lb_safe) out.lb_safe[cube] = NAN;
            out.flags[cube] = GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS;
        }
        return;
    }
    const ProbDesc P = mx.prob[pid];
    double r0[3], hr[3], t0[3], tau[3];
    decode_key(rkeys[cube], P.r_lo, P.r_w, r0, hr);
    decode_key(tkeys[cube], P.t_lo, P.t_w, t0, tau);

    // psi_r = min(|h_r|, pi) (Lemma 2 bounded with |angle(R_r p, R_s p)| <= |r - s|)
    double psir = fmin(sqrt(hr[0] * hr[0] + hr[1] * hr[1] + hr[2] * hr[2]), kPi);
    uint8_t flags = 0;
    {
        double nr2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double lo = r0[k] - hr[k], hi = r0[k] + hr[k];
            double nk = lo > 0.0 ? lo : (hi < 0.0 ? hi : 0.0);
            nr2 += nk * nk;
        }
        if (nr2 > kPi * kPi) flags |= GOSMA_FLAG_DROP_ROT;
    }
    double R[9];
    rotation_matrix(r0, R);
    double crh, srh;
    sincos(0.5 * psir, &srh, &crh);

    int drop = 0, ubinf = 0;
    float psum = 0.0f;
    for (int i = lane; i < P.M; i += 64) {
        int g = P.gmm_off + i;
        TransPrep tp = trans_prep(mx.mu + 3 * g, mx.isig2[g], t0, tau, P.zeta);
        drop |= tp.drop;
        ubinf |= tp.ub_inf;
        psum += mx.pbar[g] * tp.psi;
        double w[3];
        for (int a = 0; a < 3; ++a) w[a] = R[3 * a] * tp.u[0] + R[3 * a + 1] * tp.u[1] + R[3 * a + 2] * tp.u[2];
        // half of Psi = psi_t + psi_r (eq. 25), as cos/sin
        double cP = tp.cps * crh - tp.sps * srh, sP = tp.sps * crh + tp.cps * srh;
        lds[B_WX * stride + i] = (float)w[0];
        lds[B_WY * stride + i] = (float)w[1];
        lds[B_WZ * stride + i] = (float)w[2];
        lds[B_KAP * stride + i] = (float)tp.kap;
        lds[B_GK * stride + i] = (float)G_of(tp.kap);
        lds[B_AC * stride + i] = (float)tp.ac;
        lds[B_HA * stride + i] = (float)tp.ha;
        lds[B_GAC * stride + i] = (float)G_of(tp.ac);
        lds[B_NU * stride + i] = (float)nu_of(tp.ac);
        lds[B_CPS * stride + i] = (float)cP;
        lds[B_SPS * stride + i] = (float)sP;
        lds[B_KHI * stride + i] = (float)(tp.klo + 2.0 * tp.ha);
        lds[B_COTH * stride + i] = (float)coth_of(tp.klo);
        lds[B_W * stride + i] = mx.w1[g];
        double *L64 = (double *)(lds + B_NF * stride);
        L64[D_WX * stride + i] = w[0];
        L64[D_WY * stride + i] = w[1];
        L64[D_WZ * stride + i] = w[2];
        L64[D_CPS * stride + i] = cP;
        L64[D_SPS * stride + i] = sP;
        L64[D_AC * stride + i] = tp.ac;
        L64[D_HA * stride + i] = tp.ha;
        L64[D_NU * stride + i] = nu_of(tp.ac);
    }
    drop = wave_or(drop);
    ubinf = wave_or(ubinf);
    psum = wave_sumf(psum);
    if (drop) flags |= GOSMA_FLAG_DROP_TRANS;
    if (ubinf) flags |= GOSMA_FLAG_UB_INF;
    if ((double)psir >= (double)psum) flags |= GOSMA_FLAG_SPLIT_ROT;
    __syncthreads();

    const bool dropped = flags & (GOSMA_FLAG_DROP_ROT | GOSMA_FLAG_DROP_TRANS);
    double acc_ub = 0.0, acc_hi = 0.0;
    float top[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) top[k] = 0.0f;

    if (!dropped) {
        for (int c = 0; c < P.n_cls; ++c) {
            const ClassRange cr = mx.cls[P.cls_off + c];
            const int ni = cr.g1 - cr.g0, nj = cr.v1 - cr.v0;
            if (ni <= 0 || nj <= 0) continue;
            const int gbase = cr.g0 - P.gmm_off;
            int i = lane / nj, j = lane % nj;
            const int di = 64 / nj, dj = 64 % nj;
            for (; i < ni;) {
                const int a_ = gbase + i;
                const float4 v0 = mx.vmf[2 * (cr.v0 + j)];
                const float4 v1 = mx.vmf[2 * (cr.v0 + j) + 1];
                const float b = v0.w;
                const float wx = lds[B_WX * stride + a_], wy = lds[B_WY * stride + a_], wz = lds[B_WZ * stride + a_];
                float dx = wx - v0.x, dy = wy - v0.y, dz = wz - v0.z;
                float q = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                float px = wx + v0.x, py = wy + v0.y, pz = wz + v0.z;
                float pp = fmaf(px, px, fmaf(py, py, pz * pz));
                float ww = lds[B_W * stride + a_] * v1.x;
                // upper bound summand at the centre (eq. 12)
                {
                    PairK k = pair_k(lds[B_KAP * stride + a_], b, q);
                    float v = ww * fexp2(k.x * kLog2e) * k.hK * lds[B_GK * stride + a_] * v1.y;
                    acc_ub += (double)v;
                    if (TOP8 && v > top[7]) {
                        top[7] = v;
#pragma unroll
                        for (int s = 7; s > 0; --s) {
                            if (top[s] > top[s - 1]) {
                                float tmp = top[s];
                                top[s] = top[s - 1];
                                top[s - 1] = tmp;
                            }
                        }
                    }
                }
                // upper bound on the summand over the cube: B = max(0, theta - Psi) (eq. 25)
                {
                    float st = 0.5f * fsqrt(q), ct = 0.5f * fsqrt(pp);
                    float sB = fmaxf(st * lds[B_CPS * stride + a_] - ct * lds[B_SPS * stride + a_], 0.0f);
                    float qB = 4.0f * sB * sB;
                    float a = lds[B_AC * stride + a_], ha = lds[B_HA * stride + a_];
                    PairK k = pair_k(a, b, qB);
                    float ka1 = 0.5f * b * qB * (a - b - k.K) * k.r;            // K_a - 1
                    float ga = ka1 + lds[B_NU * stride + a_] - k.nuK * (1.0f + ka1);
                    // curvature bound: g'' <= min(1/3, 1/m^2) + min(1/3, (b sin B)^2/m^3),
                    // m <= K on the interval; with ha <= K/2, m >= K/2.
                    float b2s2 = b * b * qB * (1.0f - 0.25f * qB);
                    float iK = fminf(k.invK, 1e6f);
                    float G2 = ha <= 0.5f * k.K
                                   ? fminf(1.0f / 3.0f, 4.0f * iK * iK) + fminf(1.0f / 3.0f, 8.0f * b2s2 * iK * iK * iK)
                                   : 2.0f / 3.0f;
                    float corr = fabsf(ga) * ha + 0.5f * G2 * ha * ha;
                    float expo = k.x + corr;
                    if (__builtin_expect(k.x < -16.0f && expo > -60.0f, 0))
                        expo = s12_lower_exponent64((const double *)(lds + B_NF * stride), stride, a_,
                                                    mx.vmf64 + 4 * (cr.v0 + j));
                    float vT = fexp2(expo * kLog2e) * k.hK * lds[B_GAC * stride + a_] * v1.y;
                    float cap = 0.5f * fminf(lds[B_KHI * stride + a_], b) * (lds[B_COTH * stride + a_] + v1.z);
                    acc_hi += (double)(ww * fminf(vT, cap));
                }
                j += dj;
                i += di;
                if (j >= nj) {
                    j -= nj;
                    i += 1;
                }
            }
        }
    }
    acc_ub = wave_sum(acc_ub);
    acc_hi = wave_sum(acc_hi);

    if (TOP8 && out.top8) {
        // merge the per-lane sorted lists: 8 rounds of a wave maximum
        int head = 0;
        for (int k = 0; k < 8; ++k) {
            float mine = -1.0f;
#pragma unroll
            for (int s = 0; s < 8; ++s)
                if (s == head) mine = top[s];
            float m = mine;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
            // the lowest lane holding the maximum advances its list
            unsigned long long ballot = __ballot(mine == m);
            int winner = __ffsll((long long)ballot) - 1;
            if (lane == winner) head++;
            if (lane == 0) out.top8[8 * cube + k] = fmaxf(m, 0.0f);
        }
    }

    if (lane == 0) {
        double ub = INFINITY, lb = INFINITY, lbs = INFINITY;
        const int64_t t = tidx ? tidx[cube] : cube;
        double s11u = s11ub[t], s11l = s11lo[t];
        if (!dropped) {
            ub = ubinf ? INFINITY : s11u - 2.0 * acc_ub;
            lb = s11l - 2.0 * acc_hi;
            lbs = lb - gamma * (s11l + 2.0 * acc_hi);
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
            out.aux[4 * cube + 1] = acc_ub;
            out.aux[4 * cube + 2] = s11l;
            out.aux[4 * cube + 3] = acc_hi;
        }
        if (out.psi_gap) out.psi_gap[cube] = (float)(psir - (double)psum);
    }
}

}  // namespace

hipError_t launch_s11(const DevMix &mx, const uint64_t *tkeys, const uint32_t *pids, int64_t nt, const uint32_t *nt_dev,
                      S11Out out, int maxM, int grid, hipStream_t stream)
{
    if (nt <= 0) return hipSuccess;
    size_t lds = sizeof(float) * (size_t)A_NF * (size_t)maxM;
    unsigned g = (unsigned)(grid > 0 ? std::min<int64_t>(grid, nt) : nt);
    hipLaunchKernelGGL(k_s11, dim3(g), dim3(64), lds, stream, mx, tkeys, pids, nt, nt_dev, out, maxM);
    return hipGetLastError();
}

hipError_t launch_s12(const DevMix &mx, const uint64_t *rkeys, const uint64_t *tkeys, const uint32_t *pids,
                      const int64_t *tidx, const double *s11ub, const double *s11lo, int64_t n, const uint32_t *n_dev,
                      int n_dev_mul, BoundOut out, double margin_gamma, int maxM, bool with_top8, int grid,
                      hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    size_t lds = (sizeof(float) * (size_t)B_NF + sizeof(double) * (size_t)D_NF) * (size_t)maxM;
    unsigned g = (unsigned)(grid > 0 ? std::min<int64_t>(grid, n) : n);
    if (with_top8)
        hipLaunchKernelGGL(k_s12<true>, dim3(g), dim3(64), lds, stream, mx, rkeys, tkeys, pids, tidx, s11ub, s11lo, n,
                           n_dev, n_dev_mul, out, margin_gamma, maxM);
    else
        hipLaunchKernelGGL(k_s12<false>, dim3(g), dim3(64), lds, stream, mx, rkeys, tkeys, pids, tidx, s11ub, s11lo,
                           n, n_dev, n_dev_mul, out, margin_gamma, maxM);
    return hipGetLastError();
}

}  // namespace gosma
