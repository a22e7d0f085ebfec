// Per-cube pieces shared by the bound kernels and the search's branching
// kernel: octree key decoding, the rotation matrix of a rotation cell's
// centre with its left Jacobian (Section 5.1), the per-cube set-up record of
// the GMM-vMF pair kernel, and the translation-cell table lookup.
#pragma once

#include <cmath>

#include "gosma_impl.h"

namespace gosma {
namespace {

constexpr double kCubePi = 3.14159265358979323846;

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

// sin and cos in FP64 for the rotation angles of a cell: the argument is
// reduced to [-pi, pi] with one multiple of 2 pi (exact enough for the
// |x| < 1e6 of any finite domain) and both Maclaurin series are summed in
// nested form through x^27 and x^26 (truncation below 3e-15 on [-pi, pi]).
// A short fixed sequence keeps the register footprint of the per-cell set-up
// small next to the library routine.
// Series factors 1/((2k)(2k+1)) and 1/((2k-1)(2k)), k = 1..13, in constant
// memory: read with scalar loads, so the unrolled series needs no vector
// registers for its coefficients.
__constant__ double kSinF[13] = {1.0 / 6, 1.0 / 20, 1.0 / 42, 1.0 / 72, 1.0 / 110, 1.0 / 156, 1.0 / 210,
                                 1.0 / 272, 1.0 / 342, 1.0 / 420, 1.0 / 506, 1.0 / 600, 1.0 / 702};
__constant__ double kCosF[13] = {1.0 / 2, 1.0 / 12, 1.0 / 30, 1.0 / 56, 1.0 / 90, 1.0 / 132, 1.0 / 182,
                                 1.0 / 240, 1.0 / 306, 1.0 / 380, 1.0 / 462, 1.0 / 552, 1.0 / 650};

__device__ __forceinline__ void sincos_reduced(double x, double *s, double *c)
{
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    x -= kTwoPi * rint(x * (1.0 / kTwoPi));
    const double x2 = x * x;
    double ts = 1.0, tc = 1.0;
#pragma unroll
    for (int k = 12; k >= 0; --k) {
        ts = fma(-x2 * kSinF[k], ts, 1.0);
        tc = fma(-x2 * kCosF[k], tc, 1.0);
    }
    *s = x * ts;
    *c = tc;
}

// Rotation matrix of the angle-axis vector r (Section 5.1), as
// I + A [r]x + B [r]x^2 with A = sin|r|/|r|, B = (1 - cos|r|)/|r|^2; also the
// left Jacobian coefficients of the same map, J(r) = I + a [r]x + b [r]x^2 with
// a = (1 - cos|r|)/|r|^2 = B and b = (|r| - sin|r|)/|r|^3, so that
// d/ds R(r + s d) = [J(r) d]x R(r) at s = 0.
__device__ void rotation_matrix(const double r[3], double R[9], double *ja, double *jb)
{
    double th2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double A, B;
    if (th2 < 1e-8) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        *jb = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        double th = sqrt(th2), sh, ch;
        sincos_reduced(0.5 * th, &sh, &ch);
        A = 2.0 * sh * ch / th;
        B = 2.0 * sh * sh / th2;
        *jb = th < 1e-4 ? 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0 : (th - 2.0 * sh * ch) / (th2 * th);
    }
    *ja = B;
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

// Per-cube set-up of the GMM-vMF pair kernel: the two cells, the rotation
// matrix and, for Lemma 2 per direction (the reading the pair kernel states),
// the left Jacobian applied to four corners of the rotation cell's
// half-width box; flags GOSMA_FLAG_DROP_ROT (no point in the radius-pi ball)
// and kSetupPerDir (the per-direction bound applies: |r0| + |h_r| <= 5.5).
__device__ CubeSetup make_cube_setup(const ProbDesc &P, uint64_t rkey, uint64_t tkey)
{
    CubeSetup cs;
    double r0[3], hr[3];
    decode_key(rkey, P.r_lo, P.r_w, r0, hr);
    decode_key(tkey, P.t_lo, P.t_w, cs.t0, cs.tau);
    const double hn = sqrt(hr[0] * hr[0] + hr[1] * hr[1] + hr[2] * hr[2]);
    cs.hn = (float)hn;
    cs.cap = fminf(cs.hn, (float)kCubePi);
    const double rr = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
    uint32_t flags = sqrt(rr) + hn <= 5.5 ? kSetupPerDir : 0u;
    double ja, jb;
    rotation_matrix(r0, cs.R, &ja, &jb);
    for (int q = 0; q < 4; ++q) {
        const double d[3] = {hr[0], (q & 2) ? -hr[1] : hr[1], (q & 1) ? -hr[2] : hr[2]};
        // J d = d + a (r x d) + b (r (r . d) - |r|^2 d)
        const double x[3] = {r0[1] * d[2] - r0[2] * d[1], r0[2] * d[0] - r0[0] * d[2], r0[0] * d[1] - r0[1] * d[0]};
        const double rd = r0[0] * d[0] + r0[1] * d[1] + r0[2] * d[2];
        for (int k = 0; k < 3; ++k) cs.jc[q][k] = (float)(d[k] + ja * x[k] + jb * (r0[k] * rd - rr * d[k]));
    }
    // rotation cells with no point in the radius-pi ball hold no rotation
    double nr2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double lo = r0[k] - hr[k], hi = r0[k] + hr[k];
        const double nk = lo > 0.0 ? lo : (hi < 0.0 ? hi : 0.0);
        nr2 += nk * nk;
    }
    if (nr2 > kCubePi * kCubePi) flags |= GOSMA_FLAG_DROP_ROT;
    cs.flags = flags;
    cs.pad = 0;
    return cs;
}

// The slot of translation cell `key` in its problem's part of the cell table
// (2^tbits slots): linear probing from a multiplicative hash; the first
// thread to claim an empty slot stores the key (claimed), later ones find it.
// At most half of a problem's slots are ever used, so a free or matching slot
// is always found within the table.
__device__ __forceinline__ uint32_t cell_slot(unsigned long long *tab, uint32_t tbits, uint64_t key, bool &claimed)
{
    const uint32_t mask = (1u << tbits) - 1u;
    uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - tbits));
    claimed = false;
    for (uint32_t probe = 0; probe <= mask; ++probe, h = (h + 1u) & mask) {
        const unsigned long long cur = tab[h];
        if (cur == key) return h;
        if (cur != kEmptyCell) continue;
        const unsigned long long prev = atomicCAS(&tab[h], (unsigned long long)kEmptyCell, (unsigned long long)key);
        claimed = prev == kEmptyCell;
        if (claimed || prev == key) return h;
    }
    return 0;   // not reached (see above)
}


}  // namespace
}  // namespace gosma
