// csx_update.h -- the per-element separable-surrogate update (App. B, eq.
// f_update; Lemma 1), evaluated in float64.  Included by one translation unit
// each; everything has internal linkage.
#pragma once

#include "csx_internal.h"

namespace {

// Potential psi of the penalty at a neighbour difference d: adds psi(d) to R,
// psi'(d) to s and omega(d) = psi'(d)/d to w.  HUB = 0: quadratic t^2/2
// (delta is not read); HUB = 1: Huber's potential (t^2/2 inside
// |t| <= delta, linear outside).
template <int HUB>
__device__ __forceinline__ void potential(double d, double delta, double &R, double &s, double &w)
{
    const double ad = fabs(d);
    if (!HUB || ad <= delta) {
        R += 0.5 * d * d;
        s += d;
        w += 1.0;
    } else {
        R += delta * ad - 0.5 * delta * delta;
        s += d > 0.0 ? delta : -delta;
        w += delta / ad;
    }
}

// The 4 in-slice neighbours at the same q of voxel (ix, iz) with values
// l, r (x -+ 1) and u, d (z -+ 1); those outside the grid are skipped.
template <int HUB>
__device__ __forceinline__ void neighbour_terms(double fj, float l, float r, float u, float d, int ix, int iz, int nx,
                                                int nz, double delta, double &R, double &s, double &w)
{
    if (ix > 0) potential<HUB>(fj - l, delta, R, s, w);
    if (ix < nx - 1) potential<HUB>(fj - r, delta, R, s, w);
    if (iz > 0) potential<HUB>(fj - u, delta, R, s, w);
    if (iz < nz - 1) potential<HUB>(fj - d, delta, R, s, w);
}

// The quadratic potential over the 4 neighbours, branch-free: a neighbour
// outside the grid is given the centre value (difference 0 adds nothing to R
// or s) and w is the number inside, nin.  Same sums as neighbour_terms<0>.
__device__ __forceinline__ void neighbour_terms_quad(double fj, float l, float r, float u, float d, int nin, double &R,
                                                     double &s, double &w)
{
    const double dl = fj - l, dr = fj - r, du = fj - u, dd = fj - d;
    R += 0.5 * dl * dl;
    R += 0.5 * dr * dr;
    R += 0.5 * du * du;
    R += 0.5 * dd * dd;
    s += dl;
    s += dr;
    s += du;
    s += dd;
    w += (double)nin;
}

// Lemma 1's root for one element, unit weights over a symmetric neighbourhood:
//   b3 + b4 = 4 sum omega, b5 + b6 = 2 sum psi'
//   chi1 = beta (b3+b4), chi2 = b1 + beta(-fhat (b3+b4) + b5 + b6), chi3 = fhat b2
//   f = 2 chi3 / (chi2 + sqrt(chi2^2 + 4 chi1 chi3))       if chi2 > 0
//     = (-chi2 + sqrt(chi2^2 + 4 chi1 chi3)) / (2 chi1)    if chi2 <= 0, chi1 > 0
//     = fhat                                               otherwise (unseen voxel, beta = 0)
// The first form is the root multiplied through by its conjugate.  One
// division: the numerator and denominator are chosen first.
__device__ __forceinline__ float surrogate_root(double fj, double s, double w, double b1, double b2, double beta)
{
    const double b34 = 4.0 * w;
    const double chi1 = beta * b34;
    const double chi2 = b1 + beta * (-fj * b34 + 2.0 * s);
    const double chi3 = fj * b2;
    const double disc = sqrt(chi2 * chi2 + 4.0 * chi1 * chi3);
    double num = fj, den = 1.0;
    if (chi2 > 0.0) {
        num = 2.0 * chi3;
        den = chi2 + disc;
    } else if (chi1 > 0.0) {
        num = -chi2 + disc;
        den = 2.0 * chi1;
    }
    return (float)(num / den);
}

}  // namespace
