/*
 * gosma_oracle.h -- plain FP64 CPU oracle for the GOSMA bound evaluation and
 * branch-and-bound (Campbell et al., "The Alignment of the Spheres", 2018).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent reference the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no source with the GPU library.
 *
 * Everything is double precision, written for readability, not speed.
 * Parity status of each function is stated at its definition in the .c file.
 */
#ifndef GOSMA_ORACLE_H
#define GOSMA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A GMM (theta_1, Section 4 eq. 7) and a vMF mixture (theta_2, eq. 9).
 * Labels (eq. 17) are optional: NULL means one class. */
typedef struct {
    int M, N, n_labels;
    const double *mu;      /* M x 3 */
    const double *sigma;   /* M */
    const double *phi1;    /* M */
    const int32_t *label1; /* M or NULL */
    const double *dir2;    /* N x 3, unit */
    const double *kappa2;  /* N */
    const double *phi2;    /* N */
    const int32_t *label2; /* N or NULL */
} oracle_problem;

/* Search domain: rotation box (angle-axis), translation box, zeta. */
typedef struct {
    double r_lo[3], r_hi[3], t_lo[3], t_hi[3];
    double zeta;
} oracle_domain;

/* Per-cube bound record. */
typedef struct {
    double ub, lb;                  /* Theorem 1 bounds (+inf when dropped) */
    double s11_ub, s12_ub;          /* upper-bound pair sums at the centre */
    double s11_lo, s12_hi;          /* lower-bound pair sums */
    double psi_r, psi_t_mean;       /* branching statistics: weighted means of psi_r and psi_t */
    int32_t status;                 /* 0 ok, 1 rotation cube outside pi-ball, 2 translation infeasible */
    int32_t split_rot;              /* 1: next split is in rotation */
    double top8[8];                 /* largest S12 upper-bound pair terms, descending */
} oracle_bound;

typedef struct {
    double eps;            /* tolerance on the normalised objective (f + S22) / S22 */
    int64_t batch_parents; /* hypercubes removed from the queue per iteration */
    int64_t max_iters;
    double time_limit_s;
    int nthreads;          /* 0: OpenMP default */
    int sma_iters;         /* > 0: run SMA (oracle_sma, at most this many iterations) from the
                              best child of an iteration whenever it improves d* */
} oracle_opts;

typedef struct {
    double f_best, lb_global, f_norm_best, lb_norm, S22;
    double r[3], t[3];
    int64_t iters, cubes, max_queue;
    int32_t status;        /* 0 eps-optimal, 1 queue exhausted, 2 iteration/time cap */
    double seconds;
    int64_t sma_runs;      /* SMA runs, and how many of them lowered d* below the cube's bound */
    int64_t sma_improved;
} oracle_result;

/* SMA options (Section 6 local optimiser, oracle_sma). */
typedef struct {
    int max_iters;         /* L-BFGS iterations */
    int memory;            /* curvature pairs kept (1..16) */
    double gtol;           /* stop when |projected gradient|_inf <= gtol * (S11 + 2 S12) at the start */
    double ftol;           /* stop when a step lowers f by <= ftol * (|f| + S11 + 2 S12) */
} oracle_sma_opts;

/* Section 3 densities (for the Fig. 3b check). */
double oracle_log_Z(double x);
double oracle_vmf_pdf(const double f[3], const double mu_hat[3], double kappa);
double oracle_pn_pdf(const double f[3], const double mu[3], double sigma2);
double oracle_qpn_kappa(const double mu[3], double sigma);

void oracle_rodrigues(const double r[3], double R[9]);

/* Lemma 1 objective, semantic sum of eq. 17; also returns S11, S12, S22. */
double oracle_objective(const oracle_problem *p, const double r[3], const double t[3],
                        double *S11, double *S12);
double oracle_S22(const oracle_problem *p);

double oracle_psi_t(const double mu[3], const double t0[3], const double tau[3]);
double oracle_psi_r(const double half[3]);
void oracle_left_jacobian(const double r[3], double J[9]);
double oracle_psi_r_dir(const double r0[3], const double half[3], const double w[3], double psit);

double oracle_s11_lower_log(double alo, double ahi, double blo, double bhi, double A);
double oracle_s12_upper_term(double alo, double ahi, double b, double B);
/* The same with the kappa interval split into m equal pieces (the largest of
 * the pieces' expansion bounds, capped as above); m = 1 is the term above. */
double oracle_s12_upper_term_pieces(double alo, double ahi, double b, double B, int m);
/* The expansion bound of the S12 upper term on [e0, e1] alone, as a log. */
double oracle_s12_expansion_log(double e0, double e1, double b, double B);
/* Pieces of the kappa interval used by the cube bounds from now on (1 to 64;
 * default 1).  Returns 0, or -1 for m out of range. */
int oracle_set_kappa_pieces(int m);

void oracle_decode(uint64_t key, const double lo[3], const double hi[3], double centre[3],
                   double half[3]);

int oracle_bounds_cube(const oracle_problem *p, const oracle_domain *d, uint64_t rkey,
                       uint64_t tkey, oracle_bound *out);
int oracle_eval_bounds(const oracle_problem *p, const oracle_domain *d, const uint64_t *rkeys,
                       const uint64_t *tkeys, int64_t n, oracle_bound *out, int nthreads);

/* Gradient of the objective with respect to (r, t); returns f. */
double oracle_objective_grad(const oracle_problem *p, const double r[3], const double t[3], double grad[6]);
/* SMA from (r0, t0) inside the domain; returns iterations or -1 (start not allowed). */
int oracle_sma(const oracle_problem *p, const oracle_domain *d, const double r0[3], const double t0[3],
               const oracle_sma_opts *o, double r_out[3], double t_out[3], double *f_out);

int oracle_solve(const oracle_problem *p, const oracle_domain *d, const oracle_opts *o,
                 oracle_result *res);

/* Mixture generation (Section 7, mixgen_oracle.c): DP-means and DP-vMF-means
 * clustering and the maximum-likelihood fits. */
int oracle_dpmeans(const double *x, int64_t n, double lambda, int max_clusters, int max_passes, int32_t *z,
                   double *mu, int64_t *counts, int *passes);
int oracle_dpvmf_means(const double *x, int64_t n, double lambda, int max_clusters, int max_passes, int32_t *z,
                       double *mu, int64_t *counts, int *passes);
double oracle_vmf_kappa_ml(double rbar);
void oracle_gmm_sigma_ml(const double *x, int64_t n, const int32_t *z, const double *mu, const int64_t *counts,
                         int K, double *sigma);

#ifdef __cplusplus
}
#endif
#endif
