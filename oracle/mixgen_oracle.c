/*
 * mixgen_oracle.c -- plain FP64 CPU oracle for the mixture generation of
 * GOSMA's experiments (Section 7): the 3D point set is clustered with
 * DP-means (Kulis and Jordan, "Revisiting k-means: new algorithms via Bayesian
 * nonparametrics", ICML 2012) and the bearing vectors with DP-vMF-means
 * (Straub, Campbell, How, Fisher, "Small-variance nonparametric clustering on
 * the hypersphere", CVPR 2015), and maximum-likelihood mixtures are fitted to
 * the clusters: an isotropic Gaussian per point cluster (theta_1, eq. 7) and a
 * vMF component per bearing cluster (theta_2, eq. 9).
 *
 * TEST INFRASTRUCTURE ONLY (like gosma_oracle.c): loaded by the tests, never
 * by the product path; shares no code with the GPU library.
 *
 * Both clusterings are the serial batch algorithms, written out: a pass visits
 * the points in index order; each point takes the nearest existing cluster
 * (ties: the cluster created first), or opens a new cluster at itself when
 * even the nearest is beyond the threshold; after the pass every cluster's
 * centre is recomputed from its points and empty clusters are removed
 * (keeping the creation order).  Passes repeat until no label changes or the
 * pass limit.  DP-means starts from one cluster at the mean of all points,
 * DP-vMF-means from one cluster along their mean direction.
 *
 * Arithmetic is FP64 with each expression evaluated left to right and no
 * fused multiply-adds (ISO C, -ffp-contract=off), so that another
 * implementation that evaluates the same expressions in the same order takes
 * the same decisions; the inputs of the tests lie on a binary grid fine
 * enough that every centre sum is exact in any order.
 *
 * Parity status: oracle_dpmeans, oracle_dpvmf_means -- pinned (hand-worked
 * passes on small inputs, separated blobs recovered exactly, the limits of
 * the threshold, the objective never rising between passes);
 * oracle_vmf_kappa_ml -- pinned (closed form of A3 and its asymptotics);
 * oracle_gmm_sigma_ml -- pinned (numpy variance).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "gosma_oracle.h"

/* Squared distance |x - m|^2, summed over x, y, z in that order. */
static double dist2(const double *x, const double *m)
{
    double a = x[0] - m[0], b = x[1] - m[1], c = x[2] - m[2];
    return a * a + b * b + c * c;
}

/* Cosine x . m of a direction and a unit centre, summed in the same order. */
static double dot3m(const double *x, const double *m) { return x[0] * m[0] + x[1] * m[1] + x[2] * m[2]; }

/* The clusterings differ only in the score (DP-means: squared distance,
 * lower is better, new cluster when the best exceeds lambda; DP-vMF-means:
 * cosine, higher is better, new cluster when the best is below lambda) and
 * in how a centre follows from the sum of its points (mean; normalised sum). */
static int dp_cluster(const double *x, int64_t n, double lambda, int max_clusters, int max_passes, int spherical,
                      int32_t *z, double *mu, int64_t *counts, int *passes_out)
{
    if (n <= 0 || max_clusters < 1) return 0;
    double *sum = malloc(sizeof(double) * 3 * (size_t)(max_clusters + 1));
    int32_t *prev = malloc(sizeof(int32_t) * (size_t)n);
    /* the starting cluster: the mean of all points (normalised on the sphere) */
    double s[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) s[a] += x[3 * i + a];
    int K = 1;
    if (spherical) {
        double nr = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        for (int a = 0; a < 3; ++a) mu[a] = nr > 0.0 ? s[a] / nr : (a == 2 ? 1.0 : 0.0);
    } else {
        for (int a = 0; a < 3; ++a) mu[a] = s[a] / (double)n;
    }
    for (int64_t i = 0; i < n; ++i) prev[i] = -1;
    int pass = 0, overflow = 0;
    for (; pass < max_passes; ++pass) {
        /* one pass in index order */
        for (int64_t i = 0; i < n; ++i) {
            const double *xi = x + 3 * i;
            int best = 0;
            double bs = spherical ? dot3m(xi, mu) : dist2(xi, mu);
            for (int c = 1; c < K; ++c) {
                double sc = spherical ? dot3m(xi, mu + 3 * c) : dist2(xi, mu + 3 * c);
                if (spherical ? sc > bs : sc < bs) { bs = sc; best = c; }
            }
            if (spherical ? bs < lambda : bs > lambda) {
                if (K == max_clusters) { overflow = 1; z[i] = best; continue; }
                for (int a = 0; a < 3; ++a) mu[3 * K + a] = xi[a];
                best = K++;
            }
            z[i] = best;
        }
        /* centres from the clusters' points; empty clusters removed in order */
        for (int c = 0; c < K; ++c) {
            counts[c] = 0;
            sum[3 * c] = sum[3 * c + 1] = sum[3 * c + 2] = 0.0;
        }
        for (int64_t i = 0; i < n; ++i) {
            counts[z[i]] += 1;
            for (int a = 0; a < 3; ++a) sum[3 * z[i] + a] += x[3 * i + a];
        }
        int *remap = malloc(sizeof(int) * (size_t)K);
        int k2 = 0;
        for (int c = 0; c < K; ++c) {
            if (counts[c] == 0) { remap[c] = -1; continue; }
            remap[c] = k2;
            counts[k2] = counts[c];
            if (spherical) {
                double sx = sum[3 * c], sy = sum[3 * c + 1], sz = sum[3 * c + 2];
                double nr = sqrt(sx * sx + sy * sy + sz * sz);
                mu[3 * k2] = sx / nr;
                mu[3 * k2 + 1] = sy / nr;
                mu[3 * k2 + 2] = sz / nr;
            } else {
                for (int a = 0; a < 3; ++a) mu[3 * k2 + a] = sum[3 * c + a] / (double)counts[c];
            }
            ++k2;
        }
        K = k2;
        int changed = 0;
        for (int64_t i = 0; i < n; ++i) {
            z[i] = remap[z[i]];
            if (z[i] != prev[i]) changed = 1;
            prev[i] = z[i];
        }
        free(remap);
        if (!changed) { ++pass; break; }
    }
    free(sum);
    free(prev);
    if (passes_out) *passes_out = overflow ? -pass : pass;
    return K;
}

/* DP-means on n points x (n x 3).  Outputs: labels z (n), centres mu
 * (max_clusters x 3, first K rows used), counts (max_clusters); returns K.
 * *passes receives the passes run (negated if a pass wanted more than
 * max_clusters clusters: the point then joined its nearest cluster). */
int oracle_dpmeans(const double *x, int64_t n, double lambda, int max_clusters, int max_passes, int32_t *z,
                   double *mu, int64_t *counts, int *passes)
{
    return dp_cluster(x, n, lambda, max_clusters, max_passes, 0, z, mu, counts, passes);
}

/* DP-vMF-means on n unit vectors; lambda is the cosine below which a
 * direction opens a new cluster.  Same outputs (unit centres). */
int oracle_dpvmf_means(const double *x, int64_t n, double lambda, int max_clusters, int max_passes, int32_t *z,
                       double *mu, int64_t *counts, int *passes)
{
    return dp_cluster(x, n, lambda, max_clusters, max_passes, 1, z, mu, counts, passes);
}

/* A3(k) = coth k - 1/k, the mean resultant length of a vMF on S^2. */
static double a3(double k) { return k < 1e-6 ? k / 3.0 : 1.0 / tanh(k) - 1.0 / k; }

/* Maximum-likelihood concentration of a vMF on S^2 with mean resultant
 * length rbar: the root of A3(k) = rbar (A3 increases from 0 to 1), by
 * bisection on [0, 2 / (1 - rbar) + 1] to a relative width of 1e-15.  rbar
 * <= 0 gives 0; rbar >= 1 gives +inf. */
double oracle_vmf_kappa_ml(double rbar)
{
    if (!(rbar > 0.0)) return 0.0;
    if (rbar >= 1.0) return INFINITY;
    double lo = 0.0, hi = 2.0 / (1.0 - rbar) + 1.0;   /* A3(k) >= 1 - 1/k, so A3(hi) > rbar */
    while (hi - lo > 1e-15 * hi) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (a3(mid) < rbar) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Maximum-likelihood isotropic standard deviation of each cluster of a
 * labelling: sigma_c^2 = sum over its points of |x - mu_c|^2 / (3 n_c). */
void oracle_gmm_sigma_ml(const double *x, int64_t n, const int32_t *z, const double *mu, const int64_t *counts,
                         int K, double *sigma)
{
    double *acc = calloc((size_t)(K > 0 ? K : 1), sizeof(double));
    for (int64_t i = 0; i < n; ++i) acc[z[i]] += dist2(x + 3 * i, mu + 3 * z[i]);
    for (int c = 0; c < K; ++c) sigma[c] = counts[c] > 0 ? sqrt(acc[c] / (3.0 * (double)counts[c])) : 0.0;
    free(acc);
}
