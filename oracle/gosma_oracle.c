/*
 * gosma_oracle.c -- plain FP64 CPU oracle for GOSMA (Campbell, Petersson,
 * Kneip, Li, Gould: "The Alignment of the Spheres: Globally-Optimal Spherical
 * Mixture Alignment for Camera Pose Estimation", arXiv:1812.01232).
 *
 * TEST INFRASTRUCTURE ONLY: the reference that the GPU library is checked
 * against.  Loaded by the tests, the smoke check and the CPU-baseline leg of
 * the benchmark, never by the product path.  Shares no code with it.
 *
 * The code follows the paper's notation and order: the objective of Lemma 1
 * (Section 4, eqs. 10-13) written with the Z(.) normaliser of eq. 2 in log
 * space; the bounds of Theorem 1 (Section 5.2, eqs. 20-25) with the
 * uncertainty angles of Lemmas 2-3; the gradient of the objective and the
 * SMA local optimiser (Section 6); and Algorithm 1 (Section 6).  Where the
 * paper leaves a step open the reading taken is stated in the comment of that
 * step.
 *
 * Parity status:
 *   oracle_log_Z, oracle_vmf_pdf, oracle_pn_pdf, oracle_qpn_kappa  -- pinned
 *     (Fig. 3b table).
 *   oracle_objective, oracle_S22                                   -- pinned
 *     (sphere quadrature of the L2 distance, zero distance at the true pose,
 *      closed-form single-pair values, invariances).
 *   oracle_psi_t, oracle_psi_r                                     -- pinned
 *     (brute-force angle sampling).
 *   oracle_bounds_cube: ub pinned (= objective at the centre); lb value is
 *     "parity unpinned" (the paper's proof appendix is missing); its validity
 *     (lb <= sampled minimum) and convergence are pinned by brute force.
 *   oracle_objective_grad                                          -- pinned
 *     (central finite differences of oracle_objective).
 *   oracle_sma: pinned by first-order optimality at its result (finite
 *     differences), by never raising f, and by reaching the zero-distance
 *     ground-truth pose from nearby starts.
 *   oracle_solve: pinned on small problems by a dense pose grid with local
 *     polishing, and by recovery of the ground-truth pose.
 */
#include "gosma_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Section 3: normaliser, vMF, PN and qPN densities                   */
/* ------------------------------------------------------------------ */

/* log Z(x) for Z(x) = (e^x - e^-x) / x (eq. 2).  Written as
 * x + log(1 - e^{-2x}) - log x so that it does not overflow; Z(0) = 2 is the
 * limit at zero. */
double oracle_log_Z(double x)
{
    if (x <= 0.0) return log(2.0);
    return x + log(-expm1(-2.0 * x)) - log(x);
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
/* The angle between two vectors, atan2(|a x b|, a . b). */
static double angle3(const double *a, const double *b)
{
    double c[3];
    cross3(a, b, c);
    return atan2(norm3(c), dot3(a, b));
}

/* vMF density, eq. 1. */
double oracle_vmf_pdf(const double f[3], const double mu_hat[3], double kappa)
{
    return exp(kappa * dot3(mu_hat, f) - oracle_log_Z(kappa)) / (2.0 * M_PI);
}

/* Isotropic Projected Normal density, eq. 3, with rho = |mu|/sigma and
 * alpha = rho mu.f/|mu|; the two exponentials are merged to avoid overflow. */
double oracle_pn_pdf(const double f[3], const double mu[3], double sigma2)
{
    double nmu = norm3(mu);
    double rho = nmu / sqrt(sigma2);
    double alpha = rho * dot3(mu, f) / nmu;
    double Phi = 0.5 * erfc(-alpha / sqrt(2.0));
    double a = exp(-0.5 * rho * rho) * alpha / sqrt(2.0 * M_PI);
    double b = Phi * exp(0.5 * (alpha * alpha - rho * rho)) * (1.0 + alpha * alpha);
    return (a + b) / (2.0 * M_PI);
}

/* qPN concentration, eq. 4 / eq. 6: kappa = (|mu| / sigma)^2 + 1. */
double oracle_qpn_kappa(const double mu[3], double sigma)
{
    double r = norm3(mu) / sigma;
    return r * r + 1.0;
}

/* Rodrigues' formula R_r for an angle-axis vector r (Section 5.1). */
void oracle_rodrigues(const double r[3], double R[9])
{
    double th = norm3(r);
    for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    if (th == 0.0) return;
    double k[3] = {r[0] / th, r[1] / th, r[2] / th};
    double Kx[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
    double K2[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0;
            for (int c = 0; c < 3; ++c) s += Kx[3 * a + c] * Kx[3 * c + b];
            K2[3 * a + b] = s;
        }
    double s = sin(th), c = 1.0 - cos(th);
    for (int q = 0; q < 9; ++q) R[q] += s * Kx[q] + c * K2[q];
}

static void matvec(const double R[9], const double v[3], double out[3])
{
    for (int a = 0; a < 3; ++a) out[a] = R[3 * a] * v[0] + R[3 * a + 1] * v[1] + R[3 * a + 2] * v[2];
}
static void matTvec(const double R[9], const double v[3], double out[3])
{
    for (int a = 0; a < 3; ++a) out[a] = R[a] * v[0] + R[3 + a] * v[1] + R[6 + a] * v[2];
}

/* ------------------------------------------------------------------ */
/* Semantic classes (eq. 17): class weights phi_l = 1/|Lambda|, and   */
/* mixture weights renormalised within each class.                    */
/* ------------------------------------------------------------------ */

static int label_of(const int32_t *lab, int i) { return lab ? lab[i] : 0; }

static void class_weights(const oracle_problem *p, double *w1, double *w2)
{
    int L = p->n_labels > 0 ? p->n_labels : 1;
    double *s1 = calloc((size_t)L, sizeof(double)), *s2 = calloc((size_t)L, sizeof(double));
    for (int i = 0; i < p->M; ++i) s1[label_of(p->label1, i)] += p->phi1[i];
    for (int j = 0; j < p->N; ++j) s2[label_of(p->label2, j)] += p->phi2[j];
    for (int i = 0; i < p->M; ++i) {
        double s = s1[label_of(p->label1, i)];
        w1[i] = s > 0 ? p->phi1[i] / s : 0.0;
    }
    for (int j = 0; j < p->N; ++j) {
        double s = s2[label_of(p->label2, j)];
        w2[j] = s > 0 ? p->phi2[j] / s : 0.0;
    }
    free(s1);
    free(s2);
}

static double class_weight(const oracle_problem *p) { return 1.0 / (p->n_labels > 0 ? p->n_labels : 1); }

/* ------------------------------------------------------------------ */
/* Lemma 1: the objective f(R, t), eqs. 10-13.                        */
/* ------------------------------------------------------------------ */

double oracle_objective(const oracle_problem *p, const double r[3], const double t[3], double *S11,
                        double *S12)
{
    int M = p->M, N = p->N;
    double R[9];
    oracle_rodrigues(r, R);
    double *w1 = malloc(sizeof(double) * M), *w2 = malloc(sizeof(double) * N);
    double *u = malloc(sizeof(double) * 3 * M), *kap = malloc(sizeof(double) * M);
    class_weights(p, w1, w2);
    for (int i = 0; i < M; ++i) {
        double d[3] = {p->mu[3 * i] - t[0], p->mu[3 * i + 1] - t[1], p->mu[3 * i + 2] - t[2]};
        double n = norm3(d);
        for (int a = 0; a < 3; ++a) u[3 * i + a] = d[a] / n;          /* (mu_1i - t)/|mu_1i - t| */
        kap[i] = (n / p->sigma[i]) * (n / p->sigma[i]) + 1.0;           /* eq. 13 */
    }
    double phil = class_weight(p), s11 = 0, s12 = 0;
    for (int i = 0; i < M; ++i) {
        for (int k = 0; k < M; ++k) {
            if (label_of(p->label1, i) != label_of(p->label1, k)) continue;
            double v[3];
            for (int a = 0; a < 3; ++a) v[a] = kap[i] * u[3 * i + a] + kap[k] * u[3 * k + a];
            double K = norm3(v);                                           /* eq. 11 */
            s11 += w1[i] * w1[k] * exp(oracle_log_Z(K) - oracle_log_Z(kap[i]) - oracle_log_Z(kap[k]));
        }
        double Ru[3];
        matvec(R, u + 3 * i, Ru);
        for (int j = 0; j < N; ++j) {
            if (label_of(p->label1, i) != label_of(p->label2, j)) continue;
            double v[3];
            for (int a = 0; a < 3; ++a) v[a] = kap[i] * Ru[a] + p->kappa2[j] * p->dir2[3 * j + a];
            double K = norm3(v);                                           /* eq. 12 */
            s12 += w1[i] * w2[j] * exp(oracle_log_Z(K) - oracle_log_Z(kap[i]) - oracle_log_Z(p->kappa2[j]));
        }
    }
    free(w1); free(w2); free(u); free(kap);
    s11 *= phil;
    s12 *= phil;
    if (S11) *S11 = s11;
    if (S12) *S12 = s12;
    return s11 - 2.0 * s12;                                                 /* eq. 10, eq. 17 */
}

/* The constant S22 that eq. 10 drops from the L2 distance (eq. 15). */
double oracle_S22(const oracle_problem *p)
{
    int N = p->N;
    double *w1 = malloc(sizeof(double) * (p->M > 0 ? p->M : 1)), *w2 = malloc(sizeof(double) * N);
    class_weights(p, w1, w2);
    double s = 0;
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) {
            if (label_of(p->label2, j) != label_of(p->label2, k)) continue;
            double v[3];
            for (int a = 0; a < 3; ++a) v[a] = p->kappa2[j] * p->dir2[3 * j + a] + p->kappa2[k] * p->dir2[3 * k + a];
            s += w2[j] * w2[k] * exp(oracle_log_Z(norm3(v)) - oracle_log_Z(p->kappa2[j]) - oracle_log_Z(p->kappa2[k]));
        }
    free(w1); free(w2);
    return s * class_weight(p);
}

/* ------------------------------------------------------------------ */
/* Lemmas 2 and 3: uncertainty angles                                 */
/* ------------------------------------------------------------------ */

/* Lemma 3 (translation uncertainty angle) with a guard.  The lemma takes
 * the largest vertex angle max_v angle(p - v, p - t0), or pi when p lies in
 * the cuboid.  The vertex maximum bounds every interior point only while it
 * is at most pi/2 (the set of directions within such an angle of p - t0 is a
 * convex cone, which then contains the convex hull of the p - v); beyond
 * pi/2 this reading returns pi. */
double oracle_psi_t(const double p[3], const double t0[3], const double tau[3])
{
    double c[3] = {p[0] - t0[0], p[1] - t0[1], p[2] - t0[2]};
    if (fabs(c[0]) <= tau[0] && fabs(c[1]) <= tau[1] && fabs(c[2]) <= tau[2]) return M_PI;
    double best = 0.0;
    for (int v = 0; v < 8; ++v) {
        double a[3];
        for (int k = 0; k < 3; ++k) {
            double s = ((v >> (2 - k)) & 1) ? 1.0 : -1.0;
            a[k] = p[k] - (t0[k] + s * tau[k]);
        }
        double th = angle3(a, c);
        if (th > best) best = th;
    }
    return best > 0.5 * M_PI ? M_PI : best;
}

/* Lemma 2 (rotation uncertainty angle).  The surface maximum of the lemma is
 * not given in computable form.  The angle-axis metric inequality
 * angle(R_r p, R_s p) <= |r - s| bounds it for every direction by min(|h|, pi)
 * for a cube of half-widths h; oracle_psi_r_dir below tightens it for one
 * direction and is what the lower bound uses. */
double oracle_psi_r(const double half[3])
{
    double h = norm3(half);
    return h < M_PI ? h : M_PI;
}

/* Left Jacobian of the angle-axis parametrisation (Section 5.1):
 * d/ds exp([r + s u]x) = [J(r) u]x exp([r]x) at s = 0, with
 * J(r) = I + A [r]x + B [r]x^2, A = (1 - cos t)/t^2, B = (t - sin t)/t^3, t = |r|. */
void oracle_left_jacobian(const double r[3], double J[9])
{
    double t2 = dot3(r, r), t = sqrt(t2), A, B;
    if (t < 1e-4) {
        A = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
        B = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
    } else {
        A = (1.0 - cos(t)) / t2;
        B = (t - sin(t)) / (t2 * t);
    }
    const double K[9] = {0.0, -r[2], r[1], r[2], 0.0, -r[0], -r[1], r[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double k2 = 0.0;
            for (int k = 0; k < 3; ++k) k2 += K[3 * i + k] * K[3 * k + j];
            J[3 * i + j] = (i == j ? 1.0 : 0.0) + A * K[3 * i + j] + B * k2;
        }
}

/* Lemma 2 per direction.  For p in the cone of half-angle psi_t around a unit
 * vector, w = R_{r0} times that vector, and r = r0 + d in the cube of
 * half-widths h: the path s -> q(s) = R_{r0 + s d} p, s in [0, 1], has speed
 * |omega(s) x q(s)| with omega(s) = J(r0 + s d) d, so the angle between its
 * ends is at most the integral of
 *   |omega(0) x q(0)| + |omega(0)| |q(s) - q(0)| + |omega(s) - omega(0)|
 *   <= |(J(r0) d) x q(0)| + s |d|^2 + L s |d|^2
 * (|J| <= 1; |q(s) - q(0)| <= s |d| by the angle-axis metric bound; L bounds
 * the derivative of J along unit directions: with A' and B' the derivatives
 * of A and B, |A'| t + A + |B'| t^2 + 2 B t <= 1.595 for t <= 5.5, so L = 1.6).
 * The first term is the norm of a linear function of d, largest at a corner
 * of the box; moving q(0) within the cone changes it by at most
 * 2 sin(psi_t/2) |J(r0) d| <= 2 sin(psi_t/2) |h|.  So
 *   angle <= max over corners c of |w x J(r0) c| + 2 sin(psi_t/2) |h| + 1.3 |h|^2,
 * capped by the metric bound min(|h|, pi), which is also the value when the
 * cube leaves |r| <= 5.5. */
double oracle_psi_r_dir(const double r0[3], const double half[3], const double w[3], double psit)
{
    const double h = norm3(half);
    double cap = h < M_PI ? h : M_PI;
    if (norm3(r0) + h > 5.5) return cap;
    double J[9];
    oracle_left_jacobian(r0, J);
    static const double corner[4][3] = {{1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    double first = 0.0;
    for (int q = 0; q < 4; ++q) {
        double d[3], u[3], x[3];
        for (int k = 0; k < 3; ++k) d[k] = corner[q][k] * half[k];
        matvec(J, d, u);
        cross3(w, u, x);
        double n = norm3(x);
        if (n > first) first = n;
    }
    double b = first + 2.0 * sin(0.5 * psit) * h + 1.3 * h * h;
    return b < cap ? b : cap;
}

/* ------------------------------------------------------------------ */
/* Cubes: integer octree keys (level, ix, iy, iz) over a root box.    */
/* ------------------------------------------------------------------ */

void oracle_decode(uint64_t key, const double lo[3], const double hi[3], double centre[3], double half[3])
{
    int L = (int)((key >> 57) & 63);
    uint64_t mask = (1ull << 19) - 1;
    uint64_t idx[3] = {(key >> 38) & mask, (key >> 19) & mask, key & mask};
    for (int k = 0; k < 3; ++k) {
        half[k] = (hi[k] - lo[k]) / ldexp(1.0, L + 1);
        centre[k] = lo[k] + (2.0 * (double)idx[k] + 1.0) * half[k];
    }
}

/* K(a, b, theta) = sqrt(a^2 + b^2 + 2 a b cos theta), the form of eqs. 22-23. */
static double Kab(double a, double b, double th) { return sqrt(fmax(a * a + b * b + 2.0 * a * b * cos(th), 0.0)); }

/* The logarithm of one summand of eq. 21 for fixed concentrations a, b and
 * angle theta: g = log Z(K) - log Z(a) - log Z(b). */
static double g_term(double a, double b, double th)
{
    return oracle_log_Z(Kab(a, b, th)) - oracle_log_Z(a) - oracle_log_Z(b);
}

/* L(x) = d log Z(x) / dx = coth x - 1/x, with 0 <= L < 1 and
 * 0 < L'(x) <= min(1/3, 1/x^2). */
static double langevin(double x) { return x < 1e-6 ? x / 3.0 : 1.0 / tanh(x) - 1.0 / x; }

/* dg/da = L(K) (a + b cos theta) / K - L(a). */
static double g_da(double a, double b, double th)
{
    double K = Kab(a, b, th);
    double LK_over_K = K < 1e-6 ? 1.0 / 3.0 : langevin(K) / K;
    return LK_over_K * (a + b * cos(th)) - langevin(a);
}

/* The concentrations kappa_1i(t) in eq. 21 depend on t; the paper states that
 * this dependence "can be optimized separately" and leaves the details to an
 * appendix that is not available.  Reading used here: over the cube,
 * kappa_1i(t) is relaxed to the interval [lo, hi] it takes there, and the
 * extremum of the summand over the interval (or, for the S11 sum, over the
 * box of two intervals) is bounded with certified second-order remainders:
 * for the S11 minimum an expansion at the box centre, for the S12 maximum the
 * exact end values of the convex part K - a - b and expansions of the rest at
 * the interval ends.  With L as above:
 *   d^2 log Z(K) / da^2 = L'(K) K_a^2 + L(K) K_aa,  K_a^2 <= 1,
 *   K_aa = b^2 sin^2(theta) / K^3 >= 0,  L'(K) <= min(1/3, 1/K^2),
 *   L(K) K_aa <= min(1/3, b^2 sin^2(theta) / K^3)  (as L(K) <= K/3, K >= b sin theta),
 * and the Hessian of log Z(K(a, b)) is positive semi-definite (K is a norm
 * of a linear function of (a, b) and log Z(K) is increasing and convex in
 * K^2).  The other two terms of g are separable, -log Z(a) and -log Z(b), so
 * the Hessian of g is at least diag(-L'(a), -L'(b)). */

/* S11 summand, i != i' (eq. 21, first sum), at angle A: a lower bound on
 * min over a in [alo, ahi], b in [blo, bhi] of g(a, b, A), from the expansion
 * at the box centre c with the Hessian bound above:
 *   g(c) - |g_a| h_a - |g_b| h_b - (lambda_a h_a^2 + lambda_b h_b^2)/2,
 * lambda_a = min(1/3, 1/alo^2) >= L'(a) on the interval, lambda_b likewise. */
static double s11_lower_log(double alo, double ahi, double blo, double bhi, double A)
{
    double ac = 0.5 * (alo + ahi), ha = 0.5 * (ahi - alo);
    double bc = 0.5 * (blo + bhi), hb = 0.5 * (bhi - blo);
    double lam_a = fmin(1.0 / 3.0, 1.0 / (alo * alo)), lam_b = fmin(1.0 / 3.0, 1.0 / (blo * blo));
    return g_term(ac, bc, A) - fabs(g_da(ac, bc, A)) * ha - fabs(g_da(bc, ac, A)) * hb -
           0.5 * (lam_a * ha * ha + lam_b * hb * hb);
}

/* S12 summand (eq. 21, second sum) at angle B with b = kappa_2j fixed: the
 * ratio Z(K)/(Z(a) Z(b)) maximised over a in [alo, ahi].  Split
 *   g(a) = log Z(K) - log Z(a) - log Z(b) = x(a) + phi(a),
 *   x(a) = K(a) - a - b,   phi(a) = l(K(a)) - l(a) - l(b),   l(y) = log Z(y) - y.
 * x is convex in a (K is the norm of a u + b v for unit vectors u, v at angle
 * B).  phi has phi'' = L'(K) K_a^2 + (L(K) - 1) K_aa - L'(a) <= min(1/3, 1/K^2)
 * (the last two terms are <= 0), so with Kmin the smallest K on the interval
 * (at an end, or b sin B where a = -b cos B lies inside) and G =
 * min(1/3, 1/Kmin^2), a second-order expansion of phi at either end e gives
 *   g(a) <= x(a) + phi(e) + phi'(e)(a - e) + G (a - e)^2 / 2,
 * a convex function of a whose maximum is at one of the two ends.  The bound
 * is the smaller of the two expansions and of the value for perfectly aligned
 * directions,
 *   Z(a + b)/(Z(a) Z(b)) = a b (coth a + coth b) / (2 (a + b)) <= min(ahi, b)(coth alo + coth b)/2,
 * which bounds every angle since Z increases and K <= a + b.  A third bound
 * serves directions far apart.  The ratio decreases with the angle (K does),
 * so its largest value over angles >= B is at B, where
 *   Z(K)/(Z(a) Z(b)) = e^{K - a - b} h(K) G(a) G(b),
 * G(y) = y / (1 - e^{-2y}) increasing, h(K) = (1 - e^{-2K})/K <= min(2, 1/K),
 * and K - a - b = -a b q / (K + a + b) <= -a b q / (2 (a + b)) with
 * q = 4 sin^2(B/2) (K <= a + b; a b / (a + b) increases with a).  For
 * B <= pi/2, K^2 = a^2 + b^2 + 2 a b cos B >= 2 a b >= 2 alo b, so
 *   ratio <= G(ahi) G(b) exp(-q alo b / (2 (alo + b))) / sqrt(2 alo b);
 * for B > pi/2 the same holds with q = 2 (the value at pi/2 bounds every
 * larger angle), and also ratio <= 2 G(ahi) G(b) exp(-q alo b / (2 (alo + b))).
 * The term is the smallest of these bounds. */
static double ell(double y) { return oracle_log_Z(y) - y; }

/* The expansion bound above over a piece [e0, e1] of the kappa interval, as
 * a log: the smaller of the two end expansions. */
static double s12_expansion_log(double e0, double e1, double b, double B)
{
    const double h = 0.5 * (e1 - e0), c = cos(B);
    const double K1 = Kab(e0, b, B), K2 = Kab(e1, b, B);
    /* K - a - b = (K^2 - (a + b)^2) / (K + a + b), with 1 - cos B = 2 sin^2(B/2) */
    const double sh = sin(0.5 * B), chord2 = 4.0 * sh * sh;
    const double x1 = -e0 * b * chord2 / (K1 + e0 + b), x2 = -e1 * b * chord2 / (K2 + e1 + b);
    const double phi1 = ell(K1) - ell(e0) - ell(b), phi2 = ell(K2) - ell(e1) - ell(b);
    /* phi'(a) = (L(K) - 1) K_a - (L(a) - 1), K_a = (a + b cos B) / K */
    const double Ka1 = K1 > 0.0 ? (e0 + b * c) / K1 : 0.0, Ka2 = K2 > 0.0 ? (e1 + b * c) / K2 : 0.0;
    const double d1 = (langevin(K1) - 1.0) * Ka1 - (langevin(e0) - 1.0);
    const double d2 = (langevin(K2) - 1.0) * Ka2 - (langevin(e1) - 1.0);
    const double astar = -b * c;
    const double Kmin = (astar > e0 && astar < e1) ? b * sin(B) : fmin(K1, K2);
    const double G = Kmin > 0.0 ? fmin(1.0 / 3.0, 1.0 / (Kmin * Kmin)) : 1.0 / 3.0;
    const double q = 2.0 * G * h * h;    /* G (a - e)^2 / 2 at the far end, a - e = 2h */
    const double from_lo = phi1 + fmax(x1, x2 + 2.0 * d1 * h + q);
    const double from_hi = phi2 + fmax(x2, x1 - 2.0 * d2 * h + q);
    return fmin(from_lo, from_hi);
}

/* The term with the kappa interval split into m equal pieces: the largest of
 * the pieces' expansion bounds (each bounds the ratio on its piece, so their
 * largest bounds it on the whole interval, and it tends to the ratio's
 * maximum over the interval as the pieces shrink), capped by the aligned and
 * far-apart bounds of the whole interval.  m = 1 is the reading above. */
static double s12_upper_pieces(double alo, double ahi, double b, double B, int m)
{
    double elog = -INFINITY;
    for (int k = 0; k < m; ++k) {
        const double e0 = k == 0 ? alo : alo + (ahi - alo) * k / m;
        const double e1 = k == m - 1 ? ahi : alo + (ahi - alo) * (k + 1) / m;
        elog = fmax(elog, s12_expansion_log(e0, e1, b, B));
    }
    const double expansion = exp(elog);
    const double sh = sin(0.5 * B), chord2 = 4.0 * sh * sh;
    const double aligned = 0.5 * fmin(ahi, b) * (1.0 / tanh(alo) + 1.0 / tanh(b));
    /* log G(y) = y - log Z(y) = -ell(y) */
    const double cf = alo * b / (2.0 * (alo + b));
    const double far2 = exp(log(2.0) - ell(ahi) - ell(b) - chord2 * cf);
    const double farK = exp(-ell(ahi) - ell(b) - fmin(chord2, 2.0) * cf - 0.5 * log(2.0 * alo * b));
    return fmin(fmin(expansion, aligned), fmin(far2, farK));
}

static double s12_upper_term(double alo, double ahi, double b, double B) { return s12_upper_pieces(alo, ahi, b, B, 1); }

/* Pieces of the kappa interval of the S12 upper term in the cube bounds (1:
 * the reading above; set by oracle_set_kappa_pieces, read by every bound
 * evaluation). */
static int g_kappa_pieces = 1;

/* Test hooks for the two summand bounds above. */
double oracle_s11_lower_log(double alo, double ahi, double blo, double bhi, double A)
{
    return s11_lower_log(alo, ahi, blo, bhi, A);
}
double oracle_s12_upper_term(double alo, double ahi, double b, double B)
{
    return s12_upper_term(alo, ahi, b, B);
}
double oracle_s12_expansion_log(double e0, double e1, double b, double B)
{
    return s12_expansion_log(e0, e1, b, B);
}
double oracle_s12_upper_term_pieces(double alo, double ahi, double b, double B, int m)
{
    return s12_upper_pieces(alo, ahi, b, B, m < 1 ? 1 : m);
}
int oracle_set_kappa_pieces(int m)
{
    if (m < 1 || m > 64) return -1;
    g_kappa_pieces = m;
    return 0;
}

static int cmp_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* Theorem 1 bounds for one sub-cube C_r x C_t (Section 5.2). */
int oracle_bounds_cube(const oracle_problem *p, const oracle_domain *d, uint64_t rkey, uint64_t tkey,
                       oracle_bound *out)
{
    int M = p->M, N = p->N;
    double r0[3], hr[3], t0[3], tau[3];
    oracle_decode(rkey, d->r_lo, d->r_hi, r0, hr);
    oracle_decode(tkey, d->t_lo, d->t_hi, t0, tau);
    memset(out, 0, sizeof(*out));
    out->ub = out->lb = INFINITY;

    /* Rotation cubes are cells of the box circumscribing the radius-pi ball
     * (Section 5.1); a cell with no point in the ball holds no rotation. */
    double nearest[3];
    for (int k = 0; k < 3; ++k) {
        double lo = r0[k] - hr[k], hi = r0[k] + hr[k];
        nearest[k] = lo > 0 ? lo : (hi < 0 ? hi : 0.0);
    }
    if (norm3(nearest) > M_PI) { out->status = 1; return 0; }

    double *w1 = malloc(sizeof(double) * M), *w2 = malloc(sizeof(double) * N);
    double *c = malloc(sizeof(double) * 3 * M), *klo = malloc(sizeof(double) * M),
           *khi = malloc(sizeof(double) * M), *psit = malloc(sizeof(double) * M);
    class_weights(p, w1, w2);

    /* Per Gaussian: c_i = mu_1i - t0, the kappa interval over the cube and
     * psi_t.  The translation domain excludes points closer than zeta to any
     * mean (Section 5.1), so over feasible t the distance to mu_1i is at least
     * max(zeta, dist(mu_1i, C_t)) and at most the largest vertex distance. */
    int infeasible = 0, centre_infeasible = 0;
    double phisum = 0, psit_mean = 0;
    for (int i = 0; i < M; ++i) {
        double dmin2 = 0, dmax2 = 0;
        for (int k = 0; k < 3; ++k) {
            c[3 * i + k] = p->mu[3 * i + k] - t0[k];
            double e = fabs(c[3 * i + k]) - tau[k];
            if (e > 0) dmin2 += e * e;
            double f = fabs(c[3 * i + k]) + tau[k];
            dmax2 += f * f;
        }
        double dmin = fmax(sqrt(dmin2), d->zeta), dmax = sqrt(dmax2);
        if (dmax < d->zeta) infeasible = 1;
        if (norm3(c + 3 * i) < d->zeta) centre_infeasible = 1;
        double s2 = p->sigma[i] * p->sigma[i];
        klo[i] = dmin * dmin / s2 + 1.0;
        khi[i] = dmax * dmax / s2 + 1.0;
        psit[i] = oracle_psi_t(p->mu + 3 * i, t0, tau);
        phisum += p->phi1[i];
        psit_mean += p->phi1[i] * psit[i];
    }
    psit_mean /= phisum;
    /* Rotation uncertainty of each Gaussian's direction (Lemma 2, per
     * direction, over the cone of its translation uncertainty). */
    double R0[9];
    oracle_rodrigues(r0, R0);
    double *psir = malloc(sizeof(double) * M), psir_mean = 0;
    for (int i = 0; i < M; ++i) {
        double n = norm3(c + 3 * i), u[3], w[3];
        for (int k = 0; k < 3; ++k) u[k] = c[3 * i + k] / n;
        matvec(R0, u, w);
        psir[i] = oracle_psi_r_dir(r0, hr, w, psit[i]);
        psir_mean += p->phi1[i] * psir[i];
    }
    psir_mean /= phisum;
    out->psi_r = psir_mean;
    out->psi_t_mean = psit_mean;
    /* Branching rule: split the group with the larger angular uncertainty
     * (Section 5.1), the weighted means over the Gaussians; ties to rotation. */
    out->split_rot = out->psi_r >= psit_mean;
    if (infeasible) {
        out->status = 2;
        free(w1); free(w2); free(c); free(klo); free(khi); free(psit); free(psir);
        return 0;
    }

    /* Upper bound, eq. 20: the objective at the centre (+inf if the centre
     * is not a feasible camera position). */
    if (!centre_infeasible) {
        double S11, S12;
        out->ub = oracle_objective(p, r0, t0, &S11, &S12);
        out->s11_ub = S11;
        out->s12_ub = S12;
        /* Largest S12 pair terms at the centre (features for queue ordering). */
        double *terms = malloc(sizeof(double) * ((size_t)M * N + 8));
        int nt = 0;
        double phil = class_weight(p);
        for (int i = 0; i < M; ++i) {
            double n = norm3(c + 3 * i), u[3], Ru[3];
            for (int k = 0; k < 3; ++k) u[k] = c[3 * i + k] / n;
            matvec(R0, u, Ru);
            double ki = (n / p->sigma[i]) * (n / p->sigma[i]) + 1.0;
            for (int j = 0; j < N; ++j) {
                if (label_of(p->label1, i) != label_of(p->label2, j)) continue;
                double v[3];
                for (int k = 0; k < 3; ++k) v[k] = ki * Ru[k] + p->kappa2[j] * p->dir2[3 * j + k];
                terms[nt++] = phil * w1[i] * w2[j] *
                              exp(oracle_log_Z(norm3(v)) - oracle_log_Z(ki) - oracle_log_Z(p->kappa2[j]));
            }
        }
        qsort(terms, (size_t)nt, sizeof(double), cmp_desc);
        for (int q = 0; q < 8; ++q) out->top8[q] = q < nt ? terms[q] : 0.0;
        free(terms);
    }

    /* Lower bound, eq. 21 with the angles A (eq. 24) and B (eq. 25). */
    double phil = class_weight(p), s11lo = 0, s12hi = 0;
    for (int i = 0; i < M; ++i) {
        for (int k = 0; k < M; ++k) {
            if (label_of(p->label1, i) != label_of(p->label1, k)) continue;
            double lg;
            if (k == i) {
                /* The angle between mu_1i - t and itself is exactly 0, so the
                 * summand is Z(2 kappa)/Z(kappa)^2 = kappa coth(kappa)/2, which
                 * increases with kappa: its minimum is at the lower end. */
                lg = oracle_log_Z(2.0 * klo[i]) - 2.0 * oracle_log_Z(klo[i]);
            } else {
                double A = angle3(c + 3 * i, c + 3 * k) + psit[i] + psit[k];
                if (A > M_PI) A = M_PI;
                lg = s11_lower_log(klo[i], khi[i], klo[k], khi[k], A);
            }
            s11lo += w1[i] * w1[k] * exp(lg);
        }
        for (int j = 0; j < N; ++j) {
            if (label_of(p->label1, i) != label_of(p->label2, j)) continue;
            double Rinv_mu[3];
            matTvec(R0, p->dir2 + 3 * j, Rinv_mu);                     /* R_{r0}^{-1} mu_2j */
            double B = angle3(c + 3 * i, Rinv_mu) - psit[i] - psir[i];
            if (B < 0) B = 0;
            s12hi += w1[i] * w2[j] * s12_upper_pieces(klo[i], khi[i], p->kappa2[j], B, g_kappa_pieces);
        }
    }
    out->s11_lo = phil * s11lo;
    out->s12_hi = phil * s12hi;
    out->lb = out->s11_lo - 2.0 * out->s12_hi;
    free(w1); free(w2); free(c); free(klo); free(khi); free(psit); free(psir);
    return 0;
}

int oracle_eval_bounds(const oracle_problem *p, const oracle_domain *d, const uint64_t *rkeys,
                       const uint64_t *tkeys, int64_t n, oracle_bound *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n; ++q) oracle_bounds_cube(p, d, rkeys[q], tkeys[q], out + q);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Section 6: SMA, the local optimiser of Algorithm 1.                */
/* ------------------------------------------------------------------ */

/* Gradient of the objective of Lemma 1 (eqs. 10-13, class sum eq. 17) with
 * respect to the angle-axis rotation r and the camera centre t, by the chain
 * rule (the paper's appendix, which derives it, is not available).  For a
 * summand w w' Z(K)/(Z(a) Z(b)) write g = log Z(K) - log Z(a) - log Z(b) and
 * L(x) = d log Z / dx = coth x - 1/x.  Each GMM component i enters through
 * d_i = mu_1i - t: kappa_i = |d_i|^2/sigma_i^2 + 1 (eq. 13), u_i = d_i/|d_i|,
 * and the vector p_i = kappa_i u_i, whose Jacobian is
 *   P_i = dp_i/dd_i = (rho/sigma^2 + 1/rho) I + (rho/sigma^2 - 1/rho) u u^T,
 * rho = |d_i|, and d kappa_i / d d_i = 2 d_i / sigma_i^2.
 *   S11 summand (i, k): v = p_i + p_k, K = |v|,
 *     dg/dd_i = P_i (L(K) v / K) - L(kappa_i) 2 d_i / sigma_i^2  (and k alike).
 *   S12 summand (i, j): v = R p_i + kappa_2j mu_2j, K = |v|,
 *     dg/dd_i = P_i R^T (L(K) v / K) - L(kappa_i) 2 d_i / sigma_i^2,
 *     and under R -> exp([w]x) R, dg/dw = (L(K)/K) (R p_i) x v.
 * d/dt = -sum_i d/dd_i, and d/dr = J(r)^T d/dw with J the left Jacobian
 * (R(r + dr) = exp([J(r) dr]x) R(r) to first order). */
double oracle_objective_grad(const oracle_problem *p, const double r[3], const double t[3], double grad[6])
{
    int M = p->M, N = p->N;
    double R[9], J[9];
    oracle_rodrigues(r, R);
    oracle_left_jacobian(r, J);
    double *w1 = malloc(sizeof(double) * M), *w2 = malloc(sizeof(double) * N);
    double *pv = malloc(sizeof(double) * 3 * M), *dv = malloc(sizeof(double) * 3 * M);
    double *kap = malloc(sizeof(double) * M), *gd = calloc((size_t)(3 * M), sizeof(double));
    class_weights(p, w1, w2);
    for (int i = 0; i < M; ++i) {
        for (int a = 0; a < 3; ++a) dv[3 * i + a] = p->mu[3 * i + a] - t[a];
        double n = norm3(dv + 3 * i);
        kap[i] = (n / p->sigma[i]) * (n / p->sigma[i]) + 1.0;
        for (int a = 0; a < 3; ++a) pv[3 * i + a] = kap[i] * dv[3 * i + a] / n;
    }
    /* dg/dd_i of one summand, given c = L(K) v / K seen from component i's frame */
    #define ADD_DD(i, c, coef)                                                              \
        do {                                                                                \
            const double *d_ = dv + 3 * (i);                                                \
            double rho_ = norm3(d_), s2_ = p->sigma[i] * p->sigma[i];                       \
            double al_ = rho_ / s2_ + 1.0 / rho_, be_ = rho_ / s2_ - 1.0 / rho_;            \
            double uc_ = (d_[0] * (c)[0] + d_[1] * (c)[1] + d_[2] * (c)[2]) / rho_;         \
            double lk_ = langevin(kap[i]);                                                  \
            for (int a_ = 0; a_ < 3; ++a_)                                                  \
                gd[3 * (i) + a_] += (coef) * (al_ * (c)[a_] + be_ * uc_ * d_[a_] / rho_ -   \
                                              lk_ * 2.0 * d_[a_] / s2_);                     \
        } while (0)
    double phil = class_weight(p), f = 0.0, gw[3] = {0, 0, 0};
    for (int i = 0; i < M; ++i) {
        for (int k = 0; k < M; ++k) {
            if (label_of(p->label1, i) != label_of(p->label1, k)) continue;
            double v[3];
            for (int a = 0; a < 3; ++a) v[a] = pv[3 * i + a] + pv[3 * k + a];
            double K = norm3(v);
            double T = phil * w1[i] * w1[k] * exp(oracle_log_Z(K) - oracle_log_Z(kap[i]) - oracle_log_Z(kap[k]));
            double lk = K < 1e-6 ? 1.0 / 3.0 : langevin(K) / K, c[3];
            for (int a = 0; a < 3; ++a) c[a] = lk * v[a];
            f += T;
            ADD_DD(i, c, T);
            ADD_DD(k, c, T);
        }
        double Rp[3];
        matvec(R, pv + 3 * i, Rp);
        for (int j = 0; j < N; ++j) {
            if (label_of(p->label1, i) != label_of(p->label2, j)) continue;
            double v[3];
            for (int a = 0; a < 3; ++a) v[a] = Rp[a] + p->kappa2[j] * p->dir2[3 * j + a];
            double K = norm3(v);
            double T = phil * w1[i] * w2[j] *
                       exp(oracle_log_Z(K) - oracle_log_Z(kap[i]) - oracle_log_Z(p->kappa2[j]));
            double lk = K < 1e-6 ? 1.0 / 3.0 : langevin(K) / K, cw[3], c[3], x[3];
            for (int a = 0; a < 3; ++a) cw[a] = lk * v[a];
            matTvec(R, cw, c);                         /* R^T (L(K) v / K) */
            f -= 2.0 * T;
            ADD_DD(i, c, -2.0 * T);
            cross3(Rp, cw, x);                         /* (R p_i) x (L(K) v / K) */
            for (int a = 0; a < 3; ++a) gw[a] += -2.0 * T * x[a];
        }
    }
    #undef ADD_DD
    double gt[3] = {0, 0, 0};
    for (int i = 0; i < M; ++i)
        for (int a = 0; a < 3; ++a) gt[a] -= gd[3 * i + a];
    matTvec(J, gw, grad);                              /* d/dr = J^T d/dw */
    for (int a = 0; a < 3; ++a) grad[3 + a] = gt[a];
    free(w1); free(w2); free(pv); free(dv); free(kap); free(gd);
    return f;
}

/* The objective where the pose is allowed: +inf if the camera centre lies
 * within zeta of a Gaussian mean (the restriction of Omega_t, Section 5.1). */
static double sma_value(const oracle_problem *p, const double x[6], double zeta, double g[6])
{
    for (int i = 0; i < p->M; ++i) {
        double e[3] = {p->mu[3 * i] - x[3], p->mu[3 * i + 1] - x[4], p->mu[3 * i + 2] - x[5]};
        if (norm3(e) < zeta) return INFINITY;
    }
    return oracle_objective_grad(p, x, x + 3, g);
}

/* SMA (Section 6): minimise the objective from a start pose with L-BFGS over
 * the six pose parameters x = (r, t), kept in the domain box (rotation box x
 * translation box; the paper cites the bound-constrained L-BFGS-B).  Reading
 * taken: the L-BFGS direction (two-loop recursion of Nocedal and Wright,
 * Numerical Optimization, Algorithm 7.4, with the newest m curvature pairs and
 * the initial scaling s^T y / y^T y) is followed along the projected path
 * x+ = clamp(x + s d) onto the box, instead of L-BFGS-B's Cauchy point and
 * subspace step; trial points within zeta of a mean are infeasible.  Steps:
 *   1. stop if the projected gradient (components pointing out of the box at
 *      an active bound dropped) has infinity norm <= gtol * scale, scale =
 *      S11 + 2 S12 at the start;
 *   2. d = -H g from the stored pairs (with none stored: d = -g scaled to
 *      length at most 0.05); if g^T d >= 0, drop the pairs and take that
 *      steepest-descent step instead;
 *   3. backtrack s = 1, 1/2, 1/4, ... (at most 40 halvings) until
 *      f(x+) <= f(x) + 1e-4 g^T (x+ - x); stop if none is accepted;
 *   4. store (x+ - x, g+ - g) if s^T y > 1e-12 |s| |y|;
 *   5. stop if f fell by at most ftol (|f| + scale), or after max_iters.
 * Returns the number of iterations taken, or -1 if the start is not an allowed
 * pose. */
int oracle_sma(const oracle_problem *p, const oracle_domain *d, const double r0[3], const double t0[3],
               const oracle_sma_opts *o, double r_out[3], double t_out[3], double *f_out)
{
    enum { MAXM = 16 };
    const int m = o->memory < 1 ? 1 : (o->memory > MAXM ? MAXM : o->memory);
    double lo[6], hi[6], x[6], g[6], S[MAXM][6], Y[MAXM][6], rho[MAXM], al[MAXM];
    for (int a = 0; a < 3; ++a) {
        lo[a] = d->r_lo[a]; hi[a] = d->r_hi[a];
        lo[3 + a] = d->t_lo[a]; hi[3 + a] = d->t_hi[a];
        x[a] = r0[a]; x[3 + a] = t0[a];
    }
    for (int a = 0; a < 6; ++a)
        if (!(x[a] >= lo[a] && x[a] <= hi[a])) return -1;
    double f = sma_value(p, x, d->zeta, g);
    if (!(f < INFINITY)) return -1;
    double s11, s12;
    oracle_objective(p, x, x + 3, &s11, &s12);
    const double scale = s11 + 2.0 * s12;
    int nst = 0, head = 0, it = 0;
    while (it < o->max_iters) {
        double pg = 0.0;
        for (int a = 0; a < 6; ++a) {
            double ga = g[a];
            if ((x[a] <= lo[a] && ga > 0.0) || (x[a] >= hi[a] && ga < 0.0)) ga = 0.0;
            pg = fmax(pg, fabs(ga));
        }
        if (pg <= o->gtol * scale) break;
        double q[6], dir[6], gn = 0.0;
        for (int a = 0; a < 6; ++a) { q[a] = g[a]; gn += g[a] * g[a]; }
        gn = sqrt(gn);
        for (int k = 0; k < nst; ++k) {
            int s = (head - 1 - k + MAXM) % MAXM;
            double sq = 0.0;
            for (int a = 0; a < 6; ++a) sq += S[s][a] * q[a];
            al[s] = rho[s] * sq;
            for (int a = 0; a < 6; ++a) q[a] -= al[s] * Y[s][a];
        }
        double h0 = 1.0;
        if (nst > 0) {
            int s = (head - 1 + MAXM) % MAXM;
            double sy = 0.0, yy = 0.0;
            for (int a = 0; a < 6; ++a) { sy += S[s][a] * Y[s][a]; yy += Y[s][a] * Y[s][a]; }
            h0 = sy / yy;
        } else {
            h0 = fmin(1.0, 0.05 / gn);
        }
        for (int a = 0; a < 6; ++a) q[a] *= h0;
        for (int k = nst - 1; k >= 0; --k) {
            int s = (head - 1 - k + MAXM) % MAXM;
            double yq = 0.0;
            for (int a = 0; a < 6; ++a) yq += Y[s][a] * q[a];
            double b = rho[s] * yq;
            for (int a = 0; a < 6; ++a) q[a] += (al[s] - b) * S[s][a];
        }
        double gdir = 0.0;
        for (int a = 0; a < 6; ++a) { dir[a] = -q[a]; gdir += g[a] * dir[a]; }
        if (!(gdir < 0.0)) {
            double h = fmin(1.0, 0.05 / gn);
            for (int a = 0; a < 6; ++a) dir[a] = -h * g[a];
            nst = 0;
        }
        double step = 1.0, xn[6], gx[6], fn = INFINITY;
        int accepted = 0;
        for (int ls = 0; ls <= 40; ++ls, step *= 0.5) {
            double dec = 0.0;
            for (int a = 0; a < 6; ++a) {
                xn[a] = fmin(fmax(x[a] + step * dir[a], lo[a]), hi[a]);
                dec += g[a] * (xn[a] - x[a]);
            }
            fn = sma_value(p, xn, d->zeta, gx);
            if (fn <= f + 1e-4 * dec) { accepted = 1; break; }
        }
        if (!accepted) break;
        ++it;
        double sv[6], yv[6], sy = 0.0, ss = 0.0, yy = 0.0;
        for (int a = 0; a < 6; ++a) {
            sv[a] = xn[a] - x[a];
            yv[a] = gx[a] - g[a];
            sy += sv[a] * yv[a];
            ss += sv[a] * sv[a];
            yy += yv[a] * yv[a];
        }
        const double fprev = f;
        memcpy(x, xn, sizeof x);
        memcpy(g, gx, sizeof g);
        f = fn;
        if (sy > 1e-12 * sqrt(ss * yy)) {
            memcpy(S[head], sv, sizeof sv);
            memcpy(Y[head], yv, sizeof yv);
            rho[head] = 1.0 / sy;
            head = (head + 1) % MAXM;
            if (nst < m) ++nst;
        }
        if (fprev - f <= o->ftol * (fabs(f) + scale)) break;
    }
    for (int a = 0; a < 3; ++a) { r_out[a] = x[a]; t_out[a] = x[3 + a]; }
    *f_out = f;
    return it;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 (Section 6), with SMA when opts->sma_iters > 0.       */
/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t rkey, tkey;
    double lb, ub;
    int split_rot;
} node;

/* Best-first priority: lowest lower bound, then lowest upper bound, then key. */
static int node_less(const node *a, const node *b)
{
    if (a->lb != b->lb) return a->lb < b->lb;
    if (a->ub != b->ub) return a->ub < b->ub;
    if (a->rkey != b->rkey) return a->rkey < b->rkey;
    return a->tkey < b->tkey;
}

typedef struct { node *v; int64_t n, cap; } heap;

static void heap_push(heap *h, node x)
{
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->v = realloc(h->v, sizeof(node) * (size_t)h->cap);
    }
    int64_t i = h->n++;
    while (i > 0) {
        int64_t par = (i - 1) / 2;
        if (!node_less(&x, &h->v[par])) break;
        h->v[i] = h->v[par];
        i = par;
    }
    h->v[i] = x;
}

static node heap_pop(heap *h)
{
    node top = h->v[0], x = h->v[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        const node *best = &x;
        if (l < h->n && node_less(&h->v[l], best)) { m = l; best = &h->v[l]; }
        if (r < h->n && node_less(&h->v[r], best)) { m = r; }
        if (m == i) break;
        h->v[i] = h->v[m];
        i = m;
    }
    if (h->n > 0) h->v[i] = x;
    return top;
}

static int key_level(uint64_t k) { return (int)((k >> 57) & 63); }

/* The 8 children of a key: one level deeper, indices 2 i + bit. */
static uint64_t child_key(uint64_t k, int c)
{
    uint64_t mask = (1ull << 19) - 1;
    uint64_t L = (uint64_t)key_level(k) + 1;
    uint64_t ix = 2 * ((k >> 38) & mask) + ((c >> 2) & 1);
    uint64_t iy = 2 * ((k >> 19) & mask) + ((c >> 1) & 1);
    uint64_t iz = 2 * (k & mask) + (c & 1);
    return (L << 57) | (ix << 38) | (iy << 19) | iz;
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* SMA settings inside the search: 5 curvature pairs; stop at a projected
 * gradient of 1e-6 of the bound scale or a step gaining under 1e-9 of it. */
#define ORACLE_SMA_MEMORY 5
#define ORACLE_SMA_GTOL 1e-6
#define ORACLE_SMA_FTOL 1e-9

int oracle_solve(const oracle_problem *p, const oracle_domain *d, const oracle_opts *o, oracle_result *res)
{
    double t_start = now_s();
    memset(res, 0, sizeof(*res));
    double S22 = oracle_S22(p);
    double eps_f = o->eps * S22;          /* tolerance on f for eps on (f + S22)/S22 */
    int64_t k = o->batch_parents > 0 ? o->batch_parents : 1;
    double dstar = INFINITY, floor_lb = INFINITY;
    double best_r[3] = {0, 0, 0}, best_t[3] = {0, 0, 0};

    heap Q = {0};
    oracle_bound root;
    oracle_bounds_cube(p, d, 0, 0, &root);
    res->cubes = 1;
    if (root.ub < dstar) {
        dstar = root.ub;
        oracle_decode(0, d->r_lo, d->r_hi, best_r, (double[3]){0});
        oracle_decode(0, d->t_lo, d->t_hi, best_t, (double[3]){0});
    }
    if (root.status == 0) heap_push(&Q, (node){0, 0, root.lb, root.ub, root.split_rot});

    node *par = malloc(sizeof(node) * (size_t)k);
    uint64_t *rk = malloc(sizeof(uint64_t) * (size_t)(8 * k)), *tk = malloc(sizeof(uint64_t) * (size_t)(8 * k));
    int64_t *parent_of = malloc(sizeof(int64_t) * (size_t)(8 * k));
    oracle_bound *cb = malloc(sizeof(oracle_bound) * (size_t)(8 * k));
    int status = 1;
    double lb_global = INFINITY;
    for (;;) {
        if (Q.n == 0) { status = 1; lb_global = fmin(dstar, floor_lb); break; }
        lb_global = fmin(Q.v[0].lb, floor_lb);          /* lowest lower bound in Q */
        if (dstar - lb_global <= eps_f) { status = 0; break; }
        if ((o->max_iters > 0 && res->iters >= o->max_iters) ||
            (o->time_limit_s > 0 && now_s() - t_start > o->time_limit_s)) { status = 2; break; }
        int64_t np = 0;
        while (np < k && Q.n > 0) par[np++] = heap_pop(&Q);
        int64_t nc = 0;
        for (int64_t q = 0; q < np; ++q) {
            int rot = par[q].split_rot;
            if (rot && key_level(par[q].rkey) >= 19) rot = 0;
            if (!rot && key_level(par[q].tkey) >= 19) rot = key_level(par[q].rkey) < 19;
            if (key_level(par[q].rkey) >= 19 && key_level(par[q].tkey) >= 19) {
                if (par[q].lb < floor_lb) floor_lb = par[q].lb;   /* unsplittable: keep its bound */
                continue;
            }
            for (int ch = 0; ch < 8; ++ch) {
                rk[nc] = rot ? child_key(par[q].rkey, ch) : par[q].rkey;
                tk[nc] = rot ? par[q].tkey : child_key(par[q].tkey, ch);
                parent_of[nc++] = q;
            }
        }
        oracle_eval_bounds(p, d, rk, tk, nc, cb, o->nthreads);
        res->cubes += nc;
        /* Upper bounds first (the best child sets d*), then push every child
         * whose lower bound, raised to its parent's, is below d*. */
        int64_t best = -1;
        for (int64_t q = 0; q < nc; ++q)
            if (cb[q].status == 0 && cb[q].ub < dstar) { dstar = cb[q].ub; best = q; }
        if (best >= 0) {
            double h[3];
            oracle_decode(rk[best], d->r_lo, d->r_hi, best_r, h);
            oracle_decode(tk[best], d->t_lo, d->t_hi, best_t, h);
            if (o->sma_iters > 0) {
                /* Algorithm 1's SMA step, from the centre of the child that
                 * improved d* most in this iteration (all children of an
                 * iteration are bounded together) */
                const oracle_sma_opts so = {o->sma_iters, ORACLE_SMA_MEMORY, ORACLE_SMA_GTOL, ORACLE_SMA_FTOL};
                double rs[3], ts[3], fs;
                res->sma_runs++;
                if (oracle_sma(p, d, best_r, best_t, &so, rs, ts, &fs) >= 0 && fs < dstar) {
                    dstar = fs;
                    memcpy(best_r, rs, sizeof rs);
                    memcpy(best_t, ts, sizeof ts);
                    res->sma_improved++;
                }
            }
        }
        for (int64_t q = 0; q < nc; ++q) {
            if (cb[q].status != 0) continue;
            double lb = fmax(cb[q].lb, par[parent_of[q]].lb);
            if (lb < dstar) heap_push(&Q, (node){rk[q], tk[q], lb, cb[q].ub, cb[q].split_rot});
        }
        if (Q.n > res->max_queue) res->max_queue = Q.n;
        res->iters++;
    }
    res->status = status;
    res->f_best = dstar;
    res->lb_global = lb_global;
    res->S22 = S22;
    res->f_norm_best = (dstar + S22) / S22;
    res->lb_norm = (lb_global + S22) / S22;
    memcpy(res->r, best_r, sizeof best_r);
    memcpy(res->t, best_t, sizeof best_t);
    res->seconds = now_s() - t_start;
    free(Q.v); free(par); free(rk); free(tk); free(parent_of); free(cb);
    return 0;
}
