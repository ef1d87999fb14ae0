/*
 * csx_oracle.c -- plain FP64 CPU reference of the fan-beam coded-aperture
 * coherent-scatter system matrix (Odinaka et al., arXiv:1603.06400).
 *
 * TEST INFRASTRUCTURE.  Only tests/, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code, header or table
 * with the GPU library and is slow on purpose: every factor of every
 * (voxel, pixel, q) triple is evaluated from its definition, in double
 * precision, in the loop order of the paper's un-optimised algorithms
 * (Alg. 1 forward, Alg. 3 backward).
 *
 * Frame: source focal spot at the origin, fan plane y = 0, depth along +z.
 * A voxel is r = (x, 0, z); a detector pixel is r' = (x', y', det_z); the
 * scatter vector is s = r' - r; theta is the angle between r and s (Sec. II).
 * The paper's frame is the same with axes renamed (paper x -> z, paper y -> x,
 * paper z -> y).
 *
 * System matrix entry (Sec. II eq. 2; App. A):
 *   H(r', r, q) = C * Gso(r) * God(s) * T(r, r') * dtheta * S(theta, q)
 *   Gso   = |n_o . r^| / r^2   with n_o = +z         = z / (x^2 + z^2)^1.5
 *   God   = |n_d . s^| / s^2   with n_d = +z         = |s_z| / s^3
 *   dtheta = angle between the rays from r to the midpoints of the two pixel
 *            edges that bound the pixel along the out-of-fan axis (App. A)
 *   S     = q (1 + cos^2 theta) cos(theta/2) / sin^2(theta/2) * Phi(hc q / sin(theta/2))
 *   T     = binary mask value where the ray r -> r' crosses the mask plane (App. A)
 *
 * Readings of points the paper leaves open (each listed in the design notes):
 *   - Phi is a histogram of ne equal bins on [e_lo, e_hi): bin k = floor((E - e_lo)/dE),
 *     zero outside; the discretisation weights dr dq are part of C.
 *   - The mask cell of a crossing point (px, py) is column floor(px/pm) mod
 *     mask_nx and row floor(py/pm + mask_ny/2); rows outside the image are opaque.
 *   - dtheta is evaluated as atan2(|a x b|, a . b) for a, b = s -/+ (pitch/2) y^,
 *     theta from |r x r'| and r . s; both are exact identities of the angle
 *     definitions, chosen because they do not cancel at small angles.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, nz;
    double x_min, x_max, z_min, z_max;
    int nq;
    const double *q;
    int ndx, ndy;
    double det_pitch, det_z;
    double mask_z, mask_pitch;
    int mask_nx, mask_ny;
    const unsigned char *mask;
    int ne;
    double e_lo, e_hi;
    const double *phi;
    double C, hc;
} orc_geom;

/* All per-pair factors of Alg. 1's "Compute" lines. */
typedef struct {
    double Gso, God, T, dtheta, theta_sin, theta_cos, sin_half, cos_half, kappa;
} orc_pair;

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static void voxel_centre(const orc_geom *g, int j, double *x, double *z)
{
    int ix = j % g->nx, iz = j / g->nx;
    *x = g->x_min + (ix + 0.5) * (g->x_max - g->x_min) / g->nx;
    *z = g->z_min + (iz + 0.5) * (g->z_max - g->z_min) / g->nz;
}

static void pixel_centre(const orc_geom *g, int i, double *xp, double *yp)
{
    int a = i % g->ndx, b = i / g->ndx;
    *xp = (a - 0.5 * g->ndx + 0.5) * g->det_pitch;
    *yp = (b - 0.5 * g->ndy + 0.5) * g->det_pitch;
}

/* Mask transmission T(r, r'): the ray from r = (x,0,z) to r' = (xp,yp,det_z)
 * meets the plane z = mask_z at parameter t = (mask_z - z)/(det_z - z). */
static double mask_transmission(const orc_geom *g, double x, double z, double xp, double yp)
{
    double t = (g->mask_z - z) / (g->det_z - z);
    double px = x + t * (xp - x);
    double py = t * yp;
    double cx = floor(px / g->mask_pitch);
    double cy = floor(py / g->mask_pitch + 0.5 * g->mask_ny);
    if (cy < 0.0 || cy >= (double)g->mask_ny) return 0.0;
    long col = (long)cx % g->mask_nx;
    if (col < 0) col += g->mask_nx;
    return g->mask[(long)cy * g->mask_nx + col] ? 1.0 : 0.0;
}

/* Source spectrum Phi(E) as a histogram of equal bins on [e_lo, e_hi). */
static double spectrum(const orc_geom *g, double E)
{
    double de = (g->e_hi - g->e_lo) / g->ne;
    double k = floor((E - g->e_lo) / de);
    if (k < 0.0 || k >= (double)g->ne) return 0.0;
    return g->phi[(int)k];
}

static void pair_factors(const orc_geom *g, int j, int i, orc_pair *p)
{
    double x, z, xp, yp;
    voxel_centre(g, j, &x, &z);
    pixel_centre(g, i, &xp, &yp);
    double zd = g->det_z;

    /* Gso(r) = |n_o . r^| / r^2 with n_o along the central ray. */
    double r2 = x * x + z * z;
    double r = sqrt(r2);
    p->Gso = z / (r2 * r);

    /* s = r' - r and God(s) = |n_d . s^| / s^2 with n_d along the central ray. */
    double sx = xp - x, sy = yp, sz = zd - z;
    double s2 = sx * sx + sy * sy + sz * sz;
    double s = sqrt(s2);
    p->God = fabs(sz) / (s2 * s);

    /* Scatter angle theta between r and s: |r x s| = |r x r'|, r . s. */
    double cx = 0.0 * zd - z * yp;          /* (r x r')_x = r_y r'_z - r_z r'_y */
    double cy = z * xp - x * zd;            /* (r x r')_y = r_z r'_x - r_x r'_z */
    double cz = x * yp - 0.0 * xp;          /* (r x r')_z = r_x r'_y - r_y r'_x */
    double cross = sqrt(cx * cx + cy * cy + cz * cz);
    double dot = x * sx + 0.0 * sy + z * sz;
    p->theta_sin = cross / (r * s);
    p->theta_cos = dot / (r * s);
    /* half-angle: cos(theta/2) = sqrt((1+cos)/2), sin(theta/2) = sin/(2 cos(theta/2)) */
    p->cos_half = sqrt(0.5 * (1.0 + p->theta_cos));
    p->sin_half = p->theta_sin / (2.0 * p->cos_half);
    p->kappa = g->hc / p->sin_half;         /* E = kappa * q (Bragg, App. A) */

    /* dtheta: angle between a = s - (pitch/2) y^ and b = s + (pitch/2) y^,
     * |a x b| = pitch * sqrt(sx^2 + sz^2), a . b = s^2 - pitch^2/4. */
    double hp = 0.5 * g->det_pitch;
    double axb = 2.0 * hp * sqrt(sx * sx + sz * sz);
    double adb = s2 - hp * hp;
    p->dtheta = atan2(axb, adb);

    p->T = mask_transmission(g, x, z, xp, yp);
}

/* S(theta, q) of Sec. II eq. 2 for the pair's angle. */
static double spectral_factor(const orc_geom *g, const orc_pair *p, double q)
{
    double c2 = p->theta_cos * p->theta_cos;
    double E = g->hc * q / p->sin_half;
    return q * (1.0 + c2) * p->cos_half / (p->sin_half * p->sin_half) * spectrum(g, E);
}

/* Exported: the factors of one pair, for tests.
 * out = {Gso, God, T, dtheta, sin theta, cos theta, sin(theta/2), cos(theta/2), kappa} */
void orc_pair_factors(const orc_geom *g, int j, int i, double *out)
{
    orc_pair p;
    pair_factors(g, j, i, &p);
    out[0] = p.Gso; out[1] = p.God; out[2] = p.T; out[3] = p.dtheta;
    out[4] = p.theta_sin; out[5] = p.theta_cos; out[6] = p.sin_half;
    out[7] = p.cos_half; out[8] = p.kappa;
}

/* Exported: S(theta(j,i), q) for tests. */
double orc_spectral_factor(const orc_geom *g, int j, int i, double q)
{
    orc_pair p;
    pair_factors(g, j, i, &p);
    return spectral_factor(g, &p, q);
}

/* Alg. 1 for one detector point: g(r') = C sum_r Gso God T dtheta W(r, theta),
 * W(r, theta) = sum_q S(theta, q) f(r, q)  (Sec. III eqs. 3-4). */
static double forward_one(const orc_geom *g, const double *f, int i)
{
    double acc = 0.0;
    for (int j = 0; j < g->nx * g->nz; ++j) {
        orc_pair p;
        pair_factors(g, j, i, &p);
        double W = 0.0;
        const double *fj = f + (long)j * g->nq;
        for (int m = 0; m < g->nq; ++m)
            W += spectral_factor(g, &p, g->q[m]) * fj[m];
        acc += p.Gso * p.God * p.T * p.dtheta * W;
    }
    return g->C * acc;
}

/* g = A f over all pixels.  f: [nz][nx][nq], g: [ndy][ndx]. */
void orc_forward(const orc_geom *g, const double *f, double *out)
{
    int npix = g->ndx * g->ndy;
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < npix; ++i) out[i] = forward_one(g, f, i);
}

/* g at a list of pixels only. */
void orc_forward_pixels(const orc_geom *g, const double *f, const int *pix, int n, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n; ++k) out[k] = forward_one(g, f, pix[k]);
}

/* Alg. 3 for one object point: f(r, q) = C sum_r' Gso God T dtheta S(theta, q) g(r'). */
static void adjoint_one(const orc_geom *g, const double *y, int j, double *bj)
{
    int npix = g->ndx * g->ndy;
    for (int m = 0; m < g->nq; ++m) bj[m] = 0.0;
    for (int i = 0; i < npix; ++i) {
        orc_pair p;
        pair_factors(g, j, i, &p);
        double w = p.Gso * p.God * p.T * p.dtheta * y[i];
        for (int m = 0; m < g->nq; ++m)
            bj[m] += w * spectral_factor(g, &p, g->q[m]);
    }
    for (int m = 0; m < g->nq; ++m) bj[m] *= g->C;
}

/* b = A^T y over all voxels.  y: [ndy][ndx], b: [nz][nx][nq]. */
void orc_adjoint(const orc_geom *g, const double *y, double *out)
{
    int nvox = g->nx * g->nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < nvox; ++j) adjoint_one(g, y, j, out + (long)j * g->nq);
}

/* b at a list of voxels only (all q of each); out: [n][nq]. */
void orc_adjoint_voxels(const orc_geom *g, const double *y, const int *vox, int n, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n; ++k) adjoint_one(g, y, vox[k], out + (long)k * g->nq);
}

/* ---- scatter-angle interpolation (Sec. III-B) -------------------------------------
 * The spectral part of S(theta, q), q Phi(hc q / sin(theta/2)), is tabulated
 * at nt uniformly spaced angles theta_t = t * theta_max / (nt - 1) (0 at
 * theta = 0); W(r, theta) of eq. q_integral is evaluated at the table's
 * angles and interpolated to a pair's angle, nearest node (interp = 0, the
 * paper's choice) or linear (interp = 1).  The geometric angle factor
 * (1 + cos^2 theta) cos(theta/2) / sin^2(theta/2) stays exact per pair. */
typedef struct {
    int nt, interp;
    double theta_max;
} orc_sai;

static double sai_table(const orc_geom *g, const orc_sai *a, int t, double q)
{
    double th = t * a->theta_max / (a->nt - 1);
    double sh = sin(0.5 * th);
    if (sh <= 0.0) return 0.0;
    return q * spectrum(g, g->hc * q / sh);
}

/* interpolation weights of a pair's angle: nodes t0, t0 + 1 with weights w0, w1 */
static void sai_weights(const orc_sai *a, const orc_pair *p, int *t0, double *w0, double *w1)
{
    double th = 2.0 * atan2(p->sin_half, p->cos_half);
    double u = th * (a->nt - 1) / a->theta_max;
    if (a->interp == 0) {
        double k = floor(u + 0.5);
        if (k > a->nt - 1) k = a->nt - 1;
        *t0 = (int)k;
        *w0 = 1.0;
        *w1 = 0.0;
        return;
    }
    double k = floor(u);
    if (k > a->nt - 2) k = a->nt - 2;
    double fr = u - k;
    if (fr > 1.0) fr = 1.0;
    *t0 = (int)k;
    *w0 = 1.0 - fr;
    *w1 = fr;
}

/* the pair's weight without the spectrum: C Gso God T dtheta (1 + cos^2) cos(th/2) / sin^2(th/2) */
static double sai_pair_weight(const orc_geom *g, const orc_pair *p)
{
    double c2 = p->theta_cos * p->theta_cos;
    return g->C * p->Gso * p->God * p->T * p->dtheta * (1.0 + c2) * p->cos_half / (p->sin_half * p->sin_half);
}

void orc_forward_sai(const orc_geom *g, int nt, int interp, double theta_max, const double *f, double *out)
{
    orc_sai a = {nt, interp, theta_max};
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
    double *W = (double *)malloc(sizeof(double) * (size_t)nvox * nt);
#pragma omp parallel for
    for (int j = 0; j < nvox; ++j)
        for (int t = 0; t < nt; ++t) {
            double acc = 0.0;
            for (int m = 0; m < g->nq; ++m) acc += sai_table(g, &a, t, g->q[m]) * f[(long)j * g->nq + m];
            W[(long)j * nt + t] = acc;
        }
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < npix; ++i) {
        double acc = 0.0;
        for (int j = 0; j < nvox; ++j) {
            orc_pair p;
            pair_factors(g, j, i, &p);
            int t0;
            double w0, w1;
            sai_weights(&a, &p, &t0, &w0, &w1);
            double Wi = w0 * W[(long)j * nt + t0] + (w1 != 0.0 ? w1 * W[(long)j * nt + t0 + 1] : 0.0);
            acc += sai_pair_weight(g, &p) * Wi;
        }
        out[i] = acc;
    }
    free(W);
}

void orc_adjoint_sai(const orc_geom *g, int nt, int interp, double theta_max, const double *y, double *out)
{
    orc_sai a = {nt, interp, theta_max};
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < nvox; ++j) {
        double *V = (double *)calloc((size_t)nt, sizeof(double));
        for (int i = 0; i < npix; ++i) {
            orc_pair p;
            pair_factors(g, j, i, &p);
            int t0;
            double w0, w1;
            sai_weights(&a, &p, &t0, &w0, &w1);
            double c = sai_pair_weight(g, &p) * y[i];
            V[t0] += w0 * c;
            if (w1 != 0.0) V[t0 + 1] += w1 * c;
        }
        for (int m = 0; m < g->nq; ++m) {
            double acc = 0.0;
            for (int t = 0; t < nt; ++t) acc += V[t] * sai_table(g, &a, t, g->q[m]);
            out[(long)j * g->nq + m] = acc;
        }
        free(V);
    }
}

/* ---- energy-sensitive detector (App. A, eq. energy_sensitive) -------------------------
 * An energy-resolving pixel keeps the Bragg energy E = kappa q of each detected photon
 * instead of integrating over E.  On the spectrum's own energy bins, triple (i, j, q_m)
 * contributes H(i, j, q_m) f_jm to detector energy bin k = floor((kappa_ij q_m - e_lo)/dE)
 * of pixel i, and to nothing when E is outside [e_lo, e_hi) (there Phi, hence H, is 0).
 * The sum over k is the energy-integrating g of eq. energy_integrating_finite_detector.
 * Layout of the energy-resolved detector data: [ne][ndy][ndx]. */
static int energy_bin(const orc_geom *g, double E)
{
    double de = (g->e_hi - g->e_lo) / g->ne;
    double k = floor((E - g->e_lo) / de);
    if (k < 0.0 || k >= (double)g->ne) return -1;
    return (int)k;
}

void orc_forward_energy(const orc_geom *g, const double *f, double *out)
{
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
    memset(out, 0, sizeof(double) * (size_t)g->ne * npix);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < npix; ++i)
        for (int j = 0; j < nvox; ++j) {
            orc_pair p;
            pair_factors(g, j, i, &p);
            double w = g->C * p.Gso * p.God * p.T * p.dtheta;
            const double *fj = f + (long)j * g->nq;
            for (int m = 0; m < g->nq; ++m) {
                int k = energy_bin(g, p.kappa * g->q[m]);
                if (k < 0) continue;
                out[(long)k * npix + i] += w * spectral_factor(g, &p, g->q[m]) * fj[m];
            }
        }
}

/* The transpose: b_jm = sum_i H(i, j, q_m) y[k(i, j, m)][i]. */
void orc_adjoint_energy(const orc_geom *g, const double *y, double *out)
{
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < nvox; ++j) {
        double *bj = out + (long)j * g->nq;
        for (int m = 0; m < g->nq; ++m) bj[m] = 0.0;
        for (int i = 0; i < npix; ++i) {
            orc_pair p;
            pair_factors(g, j, i, &p);
            double w = g->C * p.Gso * p.God * p.T * p.dtheta;
            for (int m = 0; m < g->nq; ++m) {
                int k = energy_bin(g, p.kappa * g->q[m]);
                if (k < 0) continue;
                bj[m] += w * spectral_factor(g, &p, g->q[m]) * y[(long)k * npix + i];
            }
        }
    }
}

/* Largest scatter angle over all voxel-pixel pairs. */
double orc_max_angle(const orc_geom *g)
{
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
    double best = 0.0;
#pragma omp parallel for reduction(max : best)
    for (int j = 0; j < nvox; ++j)
        for (int i = 0; i < npix; ++i) {
            orc_pair p;
            pair_factors(g, j, i, &p);
            double th = 2.0 * atan2(p.sin_half, p.cos_half);
            if (th > best) best = th;
        }
    return best;
}

/* Dense system matrix H[i][j*nq + m] for tiny problems. */
void orc_dense(const orc_geom *g, double *H)
{
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
    long cols = (long)nvox * g->nq;
#pragma omp parallel for
    for (int i = 0; i < npix; ++i) {
        for (int j = 0; j < nvox; ++j) {
            orc_pair p;
            pair_factors(g, j, i, &p);
            double w = g->C * p.Gso * p.God * p.T * p.dtheta;
            for (int m = 0; m < g->nq; ++m)
                H[(long)i * cols + (long)j * g->nq + m] = w * spectral_factor(g, &p, g->q[m]);
        }
    }
}

/* Work census of the direct evaluation (for the throughput model):
 * counts[0] = pairs, [1] = pairs with T = 1, [2] = triples with T = 1 and
 * Phi(E) inside [e_lo, e_hi), [3] = pairs with T = 1 and at least one such q. */
void orc_census(const orc_geom *g, double *counts)
{
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
    double c1 = 0, c2 = 0, c3 = 0;
#pragma omp parallel for reduction(+ : c1, c2, c3)
    for (int i = 0; i < npix; ++i) {
        for (int j = 0; j < nvox; ++j) {
            orc_pair p;
            pair_factors(g, j, i, &p);
            if (p.T == 0.0) continue;
            c1 += 1;
            int any = 0;
            for (int m = 0; m < g->nq; ++m) {
                double E = p.kappa * g->q[m];
                double de = (g->e_hi - g->e_lo) / g->ne;
                double k = floor((E - g->e_lo) / de);
                if (k >= 0.0 && k < (double)g->ne) { c2 += 1; any = 1; }
            }
            c3 += any;
        }
    }
    counts[0] = (double)npix * nvox;
    counts[1] = c1;
    counts[2] = c2;
    counts[3] = c3;
}

/* Smallest distance (in mm) from any mask-plane crossing to a mask cell edge,
 * and from any (E - e_lo)/dE to an integer (in bins), over all pairs and q:
 * the margins that decide whether reduced-precision evaluations can flip T or
 * a spectrum bin. */
void orc_margins(const orc_geom *g, double *out)
{
    int npix = g->ndx * g->ndy, nvox = g->nx * g->nz;
    double mmask = 1e300, mbin = 1e300;
#pragma omp parallel for reduction(min : mmask, mbin)
    for (int i = 0; i < npix; ++i) {
        double xp, yp;
        pixel_centre(g, i, &xp, &yp);
        for (int j = 0; j < nvox; ++j) {
            double x, z;
            voxel_centre(g, j, &x, &z);
            double t = (g->mask_z - z) / (g->det_z - z);
            double px = (x + t * (xp - x)) / g->mask_pitch;
            double py = t * yp / g->mask_pitch + 0.5 * g->mask_ny;
            double dx = fabs(px - floor(px + 0.5)) * g->mask_pitch;
            double dy = fabs(py - floor(py + 0.5)) * g->mask_pitch;
            if (dx < mmask) mmask = dx;
            if (dy < mmask) mmask = dy;
            orc_pair p;
            pair_factors(g, j, i, &p);
            if (p.T == 0.0) continue;
            double de = (g->e_hi - g->e_lo) / g->ne;
            for (int m = 0; m < g->nq; ++m) {
                double u = (p.kappa * g->q[m] - g->e_lo) / de;
                if (u < -0.5 || u > g->ne + 0.5) continue;
                double d = fabs(u - floor(u + 0.5));
                if (d < mbin) mbin = d;
            }
        }
    }
    out[0] = mmask;
    out[1] = mbin;
}
