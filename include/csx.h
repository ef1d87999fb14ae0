/*
 * csx.h -- C ABI of the MI355X (gfx950) fan-beam coded-aperture
 * coherent-scatter reconstruction library (libcsx.so).
 *
 * The calls follow the paper's statement of the problem (Odinaka et al.,
 * arXiv:1603.06400):
 *   csx_init_geometry  -- the system description of Sec. II and App. A
 *                         (source at the origin, fan slice of voxels, secondary
 *                         mask plane, energy-integrating detector, spectrum),
 *                         with the per-voxel and spectrum tables that Alg. 2's
 *                         "Precompute" lines keep offline.
 *   csx_forward        -- Forward_project: g = A f, eqs. 1-2, evaluated exactly
 *                         as Alg. 1 defines it (no scatter-angle interpolation).
 *   csx_backproject    -- Back_project: b = A^T y, evaluated exactly as Alg. 3
 *                         defines it.
 *   csx_recon_step     -- one iteration of the EM-type algorithm (Alg. 5) for
 *                         the Poisson model y_i ~ Poisson((A f)_i + r_i) of
 *                         Sec. V with the penalised objective J = L + beta R,
 *                         closed-form update of App. B eq. f_update.
 *   csx_recon          -- Alg. 5 for n_iter iterations.
 *
 * Frame: source focal spot at the origin, fan plane y = 0, depth along +z (the
 * paper's axes renamed: paper x -> z, paper y -> x, paper z -> y).  Lengths in
 * mm, energies in keV, q in the inverse of the unit of hc (nm^-1 with
 * hc = 1.23984193 keV nm).
 *
 * Layouts (row-major, all device buffers are float32 unless stated):
 *   image  f, b : [nz][nx][nq]   voxel (ix, iz) at x = x_min + (ix+1/2) dx,
 *                                z = z_min + (iz+1/2) dz, q fastest
 *   detector g, y, r : [ndy][ndx] pixel (a, b) at x' = (a - ndx/2 + 1/2) p,
 *                                y' = (b - ndy/2 + 1/2) p, z' = det_z
 *
 * Ownership: the caller owns every data buffer; the library owns only the
 * geometry handle, its device tables and its workspace, and never frees caller
 * memory.  Device calls are asynchronous on the HIP stream passed as
 * `stream` (NULL = the default stream).  Calls that share one handle use its
 * workspace and must not run concurrently.
 *
 * Errors: every call returns a csx_status; no exception crosses the ABI.
 * Argument validation happens before any HIP call.  csx_last_error() returns
 * a thread-local message describing the last failure.
 */
#ifndef CSX_H
#define CSX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CSX_OK = 0,
    CSX_EINVAL = -1,   /* bad argument (null pointer, size, NaN, negative count) */
    CSX_EGEOM = -2,    /* descriptor violates the geometry's requirements */
    CSX_EHIP = -3,     /* a HIP runtime call failed (no device, launch error) */
    CSX_ENOMEM = -4,   /* device or host allocation failed */
    CSX_ENUMERIC = -5  /* y_i > 0 where the model mean (A f + r)_i is 0 */
} csx_status;

enum { CSX_TABLE_F32 = 0, CSX_TABLE_BF16 = 1 };

/* System description (all host memory, copied by csx_init_geometry).
 * Requirements (else CSX_EGEOM): all counts >= 1; ndy even (no pixel on the
 * fan plane, and pixel rows pair up under the y -> -y mirror); 0 < z_min <
 * z_max < mask_z < det_z; x_min < x_max; positive pitches, hc; e_lo < e_hi;
 * finite non-negative phi and C; finite positive q; mask values 0 or 1. */
typedef struct {
    int nx, nz;                   /* voxels across / along the fan's central ray */
    double x_min, x_max;          /* mm, cell-centred voxel grid */
    double z_min, z_max;          /* mm */
    int nq;                       /* momentum-transfer nodes */
    const double *q;              /* [nq] */
    int ndx, ndy;                 /* detector pixels along x, y; ndy even */
    double det_pitch;             /* mm, square pixels */
    double det_z;                 /* mm, detector plane */
    double mask_z;                /* mm, secondary-mask plane */
    double mask_pitch;            /* mm, square mask cells */
    int mask_nx;                  /* mask period along x (cells) */
    int mask_ny;                  /* mask rows, centred on y = 0; outside rows are opaque */
    const unsigned char *mask;    /* [mask_ny][mask_nx], 0 = blocked, 1 = open */
    int ne;                       /* spectrum histogram bins on [e_lo, e_hi) */
    double e_lo, e_hi;            /* keV */
    const double *phi;            /* [ne] flux per bin */
    double C;                     /* normalisation constant C of App. A */
    double hc;                    /* keV * (unit of 1/q) */
    int table_dtype;              /* CSX_TABLE_F32, or CSX_TABLE_BF16: spectrum table
                                     rounded to bfloat16 (round-to-nearest-even) and
                                     mask stored as bits; accumulation stays float32 */
} csx_geometry_desc;

typedef struct csx_geometry csx_geometry;

/* Sizes and kernel facts of a handle. */
typedef struct {
    int nvox, npix, nq;
    int symmetric_lr;             /* 1 when the x -> -x mirror is exploited */
    int table_dtype;
    int64_t workspace_bytes;      /* device memory the handle holds */
} csx_info;

/* Checks a descriptor without touching the GPU.  Returns CSX_OK, CSX_EINVAL or
 * CSX_EGEOM. */
csx_status csx_validate_desc(const csx_geometry_desc *desc);

/* Builds the device tables and workspace for one system on the current HIP
 * device.  *out receives a handle owned by the caller (free with
 * csx_free_geometry).  Synchronous. */
csx_status csx_init_geometry(const csx_geometry_desc *desc, csx_geometry **out);

/* Releases the handle and its device memory (NULL is a no-op). */
void csx_free_geometry(csx_geometry *h);

csx_status csx_get_info(const csx_geometry *h, csx_info *out);

/* Factor store (Sec. III's trade of offline against online computation,
 * taken the other way than the paper's MATLAB implementation could afford):
 * the exact operators' per-class pair factors -- kappa = hc / sin(theta/2)
 * in float64, the weight A = C Gso God dtheta (1 + cos^2 theta) cos(theta/2)
 * / sin^2(theta/2) and the four mirror pairs' mask values -- depend on the
 * geometry only, so they can be evaluated once and read back by every
 * forward and adjoint instead of being re-evaluated per call (16 bytes per
 * adjoint class record, 32 per forward record: 2.1 GB at 128^2 voxels x
 * 128^2 pixels).  The values are those the operators compute on the fly, by
 * the same code; results agree with the on-the-fly operators to float32
 * rounding.  Needs a uniform q grid whose zero-padded spectrum table (every
 * bin coordinate kappa q_m / dE + b0 an in-band class can reach at any node)
 * fits 8192 entries.  csx_init_geometry builds the store when it needs at
 * most CSX_STORE_AUTO_BYTES and a quarter of the device's free memory
 * (the paper's 28^2 x 79 q shape with its 1536 x 2048 detector: 22.8 GB).  on = 1 builds it (CSX_ENOMEM if the allocation fails,
 * CSX_EINVAL on a non-uniform q grid), on = 0 releases it; both synchronise
 * the device.  The batched, ordered-subsets and warm-start paths use the
 * store of each handle that has one; the energy-resolved and interpolated
 * operators do not read it. */
#define CSX_STORE_AUTO_BYTES (32LL << 30)
csx_status csx_set_factor_store(csx_geometry *h, int on);

/* Whether the handle holds a factor store, its device bytes and the time its
 * build took in ms (any pointer may be NULL). */
csx_status csx_get_factor_store(const csx_geometry *h, int *on, int64_t *bytes, double *build_ms);

/* Interval form of the exact operators (Alg. 1 and Alg. 3 re-associated).
 * The spectrum is a histogram, so a class's q sum depends on its Bragg
 * factor kappa = hc / sin(theta/2) only through the spectrum bin of kappa q_m
 * at each node m: the (ne + 1) nq bin thresholds kappa = beta(c, m), sorted,
 * cut the kappa axis into intervals on which the sum is constant (Sec.
 * III-B's angle table with its grid placed exactly where S changes).  The
 * forward then builds, per voxel and call, the table F_j(t) = sum_m q_m f_jm
 * Phi(bin) over the intervals t by one float64 prefix sum, and reads it once
 * per class; the adjoint sums each class's weight A T rho into float64
 * prefix sums over the intervals and takes one difference per (node, bin).
 * Bin decisions are float64 FMAs per node, as in the direct kernels; the
 * results equal the direct sums up to the order of the additions.  Set-up
 * computes per class an 8-byte record (A, mask values, interval, rank in its
 * voxel group's interval order): 0.5 GB at 128^2 x 128^2.  Applies when
 * (ne + 1) nq < 16384, a voxel group has at most 8192 classes (pixels of
 * the upper detector half) and both kernels' tables fit in LDS; csx_init_geometry
 * builds it then when it needs at most CSX_STORE_AUTO_BYTES and a quarter of
 * the free memory.  While built, csx_forward, csx_forward_noalloc,
 * csx_backproject and the solvers' full operators use it; subset and
 * energy-resolved operators do not.  on = 1 builds (CSX_EINVAL when it does
 * not apply, CSX_ENOMEM), on = 0 releases; both synchronise the device. */
csx_status csx_set_interval_operators(csx_geometry *h, int on);

/* Whether the interval operators are built, their device bytes, set-up time
 * in ms and number of kappa intervals (any pointer may be NULL). */
csx_status csx_get_interval_operators(const csx_geometry *h, int *on, int64_t *bytes, double *build_ms,
                                      int *intervals);

/* Forward_project (Sec. II eqs. 1-2; Alg. 1): g_i = sum_j sum_m H(i, j, q_m) f_jm with
 * H = C Gso God T dtheta S(theta, q).  f: device [nz][nx][nq]; g: device
 * [ndy][ndx], overwritten.  Asynchronous on `stream`. */
csx_status csx_forward(csx_geometry *h, const float *f, float *g, void *stream);

/* Largest forward partial-image buffer of csx_forward_noalloc, in floats
 * (16 MiB of device memory per GPU, held from the first csx_init_geometry on
 * that GPU until the process ends). */
#define CSX_SCRATCH_FLOATS (1 << 22)

/* csx_forward without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels and the same result, bit for bit, as
 * csx_forward; the forward's partial images (splits x q chunks x npix
 * floats, see csx_get_launch; with the interval operators one image per
 * workgroup, at most one per compute unit) go to a static device array of
 * CSX_SCRATCH_FLOATS floats instead of the handle's workspace, so the call
 * makes no hipMalloc / hipFree and records no timing events.  Returns
 * CSX_EINVAL before any HIP call when the partials exceed CSX_SCRATCH_FLOATS
 * (lower fwd_splits with csx_set_launch) or an argument is NULL.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, or two host threads) race and must be serialised by the caller;
 * no value needs to start at zero (every partial is written before it is
 * read).  f: device [nz][nx][nq]; g: device [ndy][ndx], overwritten.
 * Asynchronous on `stream`. */
csx_status csx_forward_noalloc(const csx_geometry *h, const float *f, float *g, void *stream);

/* Back_project (Alg. 3): b_jm = sum_i H(i, j, q_m) y_i.  y: device [ndy][ndx];
 * b: device [nz][nx][nq], overwritten.  Asynchronous on `stream`. */
csx_status csx_backproject(csx_geometry *h, const float *y, float *b, void *stream);

/* One iteration of Alg. 5 from f^t (in f) to f^{t+1} (written back to f):
 *   z = A f^t + r,  b2 = A^T (y / z)  (0 where y_i = 0),
 *   f^{t+1}_j = minimiser of the separable surrogate (App. B eq. f_update,
 *   Lemma 1), quadratic potential psi(t) = t^2/2, 4 in-slice neighbours
 *   (+-x, +-z) at the same q, unit weights.
 * y: device [ndy][ndx] counts (>= 0); r: device [ndy][ndx] background or NULL
 * (= 0); f: device image, in/out; beta >= 0.  J_out: NULL, or a device double
 * that receives J(f^t) = L(f^t) + beta R(f^t) in float64 (+inf when some
 * y_i > 0 has zero model mean).  The first call on a handle also computes the
 * sensitivity image b1 = A^T 1 and keeps it.  Asynchronous on `stream`: the
 * call returns before the data are seen, so it never returns CSX_ENUMERIC;
 * that condition shows only as J = +inf in *J_out (csx_recon, which
 * synchronises, returns CSX_ENUMERIC for it). */
csx_status csx_recon_step(csx_geometry *h, const float *y, const float *r, float *f,
                          double beta, double *J_out, void *stream);

/* Alg. 5 for n_iter >= 0 iterations.  init_uniform != 0 first sets
 * f^0 = sum(y) / sum(A^T 1) everywhere (f is then output only).
 * J_hist: NULL or host double[n_iter + 1] receiving J(f^0) .. J(f^n_iter).
 * Synchronises `stream` before returning.  Returns CSX_ENUMERIC if some
 * y_i > 0 met a zero model mean. */
csx_status csx_recon(csx_geometry *h, const float *y, const float *r, float *f,
                     int init_uniform, int n_iter, double beta, double *J_hist, void *stream);

/* Penalty potential psi of R(f) = sum_j sum_{k in N_j} psi(f_j - f_k) (Sec. V
 * eq. standard_EPR; 4 in-slice neighbours at the same q, w = 1).  Quadratic
 * psi(t) = t^2/2 by default; CSX_PSI_HUBER: Huber's edge-preserving potential
 * with scale delta > 0 (t^2/2 for |t| <= delta, delta |t| - delta^2/2
 * beyond), whose separable surrogate (App. B) uses psi'(t) and the curvature
 * omega(t) = psi'(t)/t.  Applies to every later csx_recon_step, csx_recon,
 * csx_recon_os and batched call on the handle and to their objectives.
 * CSX_EINVAL for an unknown kind or a bad delta. */
#define CSX_PSI_QUADRATIC 0
#define CSX_PSI_HUBER 1
csx_status csx_set_penalty(csx_geometry *h, int kind, double delta);

/* Alg. 6, ordered subsets: n_iter sweeps over the detector subsets of the
 * symmetry-preserving partition of Sec. VI.  Vertical class rz (0 <= rz <
 * rho_z) holds rows rz, rz + rho_z, ... of one half of the detector and their
 * up-down mirrors; horizontal class cy (0 <= cy < rho_y / 2) holds columns cy,
 * cy + rho_y, ... and their left-right mirrors; subset p = rz (rho_y / 2) + cy
 * is swept in increasing p (the paper leaves the order open).  Needs
 * rho_z | ndy / 2, rho_y | ndx and rho_y even (else CSX_EINVAL); the paper's
 * choice is rho_z = 8, rho_y = 16 (64 subsets).  Each sub-step uses the
 * subset's data only (forward and back projection restricted to its pixels,
 * b1_p = A_p^T 1) and the update of App. B with penalty weight beta / P.
 * Buffers and init_uniform as for csx_recon; J_hist (host, n_iter + 1, may be
 * NULL) receives the full objective J before the first and after every sweep.
 * The partition's lists and the P sensitivity images (P * nvox * nq floats)
 * are built on the first call and kept by the handle.  Synchronises `stream`. */
csx_status csx_recon_os(csx_geometry *h, const float *y, const float *r, float *f, int init_uniform,
                        int n_iter, int rho_z, int rho_y, double beta, double *J_hist, void *stream);

/* Scatter-angle interpolation (Sec. III-B; the precomputation and the
 * interpolated reads of Alg. 2 and Alg. 4).  The spectral part of S,
 * s(theta, q) = q Phi(hc q / sin(theta/2)), is tabulated at nt angles
 * theta_t = t theta_max / (nt - 1), t = 0 .. nt-1 (s = 0 at theta = 0), in
 * float32; the geometric factor (1 + cos^2 theta) cos(theta/2) / sin^2(theta/2)
 * stays exact per pair.  interp: 0 takes the nearest node (the paper's
 * choice), 1 interpolates linearly between the two nodes around the pair's
 * angle; angles beyond theta_max take the last node's value.  theta_max = 0 takes the
 * largest scatter angle of the geometry (plus 1e-7 relative).
 * nt: 2 .. CSX_SAI_MAX_NODES; theta_max: 0 or in (0, pi]; else CSX_EINVAL.
 * Builds the table on the host in float64 and keeps it, with two
 * [nvox][nt] float32 work arrays, on the handle; a later call replaces it.
 * Synchronous. */
#define CSX_SAI_MAX_NODES 2048
csx_status csx_sai_config(csx_geometry *h, int nt, int interp, double theta_max);

/* The configuration in force (CSX_EINVAL before csx_sai_config); any output
 * pointer may be NULL. */
csx_status csx_sai_info(const csx_geometry *h, int *nt, int *interp, double *theta_max);

/* Forward with interpolated angles: W = f s^T ([nvox][nq] x [nq][nt], on the
 * matrix cores), then g_i = sum_j A_ij T_ij W_j(theta_ij) with W_j read at the
 * interpolation nodes of the pair's angle.  Buffers as for csx_forward.
 * CSX_EINVAL before csx_sai_config.  Asynchronous on `stream`. */
csx_status csx_forward_sai(csx_geometry *h, const float *f, float *g, void *stream);

/* The exact transpose of csx_forward_sai: V_jt = sum_i A_ij T_ij y_i w_t(theta_ij)
 * (w_t: the pair's interpolation weight of node t), then b = V s
 * ([nvox][nt] x [nt][nq]).  V is accumulated in 64-bit fixed point scaled to
 * the launch's bound max(A) sum_i |y_i| (results do not depend on the order of
 * the adds; bins below ~2^-40 of the bound lose relative precision).  A
 * non-finite y gives NaN everywhere.  Buffers as for csx_backproject.
 * Asynchronous. */
csx_status csx_backproject_sai(csx_geometry *h, const float *y, float *b, void *stream);

/* Operators of the solver: bit CSX_OP_FORWARD_SAI makes csx_recon_step,
 * csx_recon, csx_recon_warm and csx_recon_os use the interpolated forward for
 * A f (and A_p f of a subset; objectives included), bit CSX_OP_ADJOINT_SAI
 * makes them use the interpolated adjoint for A^T rho and for the
 * sensitivities A^T 1 and A_p^T 1 (recomputed after a change).  With one bit
 * only, the adjoint is not the transpose of the forward and J need not
 * decrease.  ops != 0 needs csx_sai_config first; batches return CSX_EINVAL
 * while ops != 0.  Default 0 (exact operators). */
#define CSX_OP_FORWARD_SAI 1
#define CSX_OP_ADJOINT_SAI 2
csx_status csx_set_operator(csx_geometry *h, int ops);

/* Energy-sensitive detector (App. A, eq. energy_sensitive): an
 * energy-resolving pixel records each photon in the spectrum bin of its Bragg
 * energy E = kappa q (the detector's bins are the spectrum's ne bins on
 * [e_lo, e_hi)), so
 *   g_E[k][i] = sum_j sum_{m: bin(kappa_ij q_m) = k} H(i, j, q_m) f_jm
 * and sum_k g_E[k][i] is csx_forward's g_i.  f: device [nz][nx][nq]; gE:
 * device [ne][ndy][ndx], overwritten.  Each wave adds its triples into
 * 64-bit fixed-point histograms scaled to the launch's bound
 * max(A) max(Phi) sum_jm q_m |f_jm| (results do not depend on the order of
 * the adds); a non-finite f gives NaN everywhere.  Needs ne small enough for
 * the histograms in LDS (about ne <= 590; else CSX_EINVAL).  The first call on a handle also finds max(A) (synchronous) and
 * allocates its partial images.  Asynchronous on `stream`. */
csx_status csx_forward_energy(csx_geometry *h, const float *f, float *gE, void *stream);

/* The transpose: b_jm = sum_i H(i, j, q_m) y_E[bin(kappa_ij q_m)][i].  yE:
 * device [ne][ndy][ndx]; b: device [nz][nx][nq], overwritten.  Asynchronous
 * on `stream` (keeps a Phi-weighted copy of yE, (ne + 2) npix floats). */
csx_status csx_backproject_energy(csx_geometry *h, const float *yE, float *b, void *stream);

/* Alg. 5 on energy-resolved counts: the Poisson likelihood over every pixel
 * and energy bin, z = A_E f + r_E, b1 = A_E^T 1 (computed on the first call
 * and kept), b2 = A_E^T (y_E / z), then the update and the objective of
 * csx_recon (the handle's penalty).  yE, rE (NULL: 0): device [ne][ndy][ndx];
 * f, init_uniform (f^0 = sum(yE) / sum(b1)), n_iter, beta and J_hist as for
 * csx_recon.  Synchronises `stream`. */
csx_status csx_recon_energy(csx_geometry *h, const float *yE, const float *rE, float *f, int init_uniform,
                            int n_iter, double beta, double *J_hist, void *stream);

/* Measurement helper (not part of the method): the float32 FMA issue rate of
 * the current device in lane-operations per second, from one timed launch of
 * independent FMA chains filling every SIMD (after one warm-up launch).  The
 * operators' roofline fraction is quoted against the published rate (256 CUs
 * x 4 SIMDs x 16 lanes x 2.4 GHz) and against this measured one.  Allocates
 * and frees a small output buffer; synchronises `stream`. */
csx_status csx_valu_peak(double *lane_ops_per_s, void *stream);

/* Launch shape of a handle's operators; a tuner may change it (results do not
 * depend on it beyond float32 summation order).
 *   fwd_splits: the forward's voxel range is split over this many block rows
 *               (1..64); partial images are summed in a fixed order.  Blocks
 *               are numbered so that each of the 8 XCDs takes a contiguous
 *               share of the splits: with a multiple of 8 each XCD's L2 holds
 *               only its share of f.  Default: enough block rows for about
 *               8 waves per SIMD, and at least 8 when f is larger than 1 MB.
 *   fwd_qw, adj_qw: q lanes per chunk of the forward / adjoint (16, 32 or 64);
 *               nq is covered by ceil(nq / qw) chunks.  Default: the
 *               smallest width covering nq, at most 64; the forward's is
 *               halved while its LDS (two q f tiles beside the spectrum
 *               table) would exceed half of a compute unit's.
 *   adj_splits: the direct adjoint's pixel classes are split into this many
 *               contiguous tile ranges (1..64), one wave per voxel group, q
 *               chunk and range, the ranges' partial images summed in a fixed
 *               order: with few voxel groups (a small voxel grid) the adjoint
 *               otherwise holds too few waves to fill the device.  0 in
 *               csx_set_launch: the default, 1 when the unsplit launch holds
 *               at least 4 waves per SIMD, else enough ranges for about 12.
 *               The interval form, batches and subsets do not split. */
typedef struct {
    int fwd_splits;
    int fwd_qw;
    int adj_qw;
    int adj_splits;
} csx_launch;

csx_status csx_get_launch(const csx_geometry *h, csx_launch *out);
/* Validates the shape (CSX_EINVAL) and grows the handle's workspace if needed
 * (synchronous). */
csx_status csx_set_launch(csx_geometry *h, const csx_launch *lc);

/* A batch of independent scans reconstructed together (the batched form).
 * The scans may differ in every size.  Each iteration merges all scans'
 * forward (and adjoint) work into one launch per kernel variant, largest scans
 * first, and the whole iteration is captured once in a HIP graph and replayed.
 * The batch keeps the handles (not owned; they must outlive it, and each may
 * appear once: the scans use their handles' workspaces) and holds small device
 * job tables.  csx_batch_create returns CSX_EINVAL for n < 1, a NULL handle or
 * a repeated handle. */
typedef struct csx_batch csx_batch;

csx_status csx_batch_create(csx_geometry *const *scans, int n, csx_batch **out);
void csx_batch_free(csx_batch *b);

/* Alg. 5 for n_iter iterations on every scan k: y[k] (counts), r[k]
 * (background or NULL; r itself may be NULL), f[k] (in/out image) are device
 * buffers laid out as for csx_recon.  init_uniform != 0 starts each scan at
 * its uniform image.  J_hist: NULL or host double[n][n_iter + 1].  Synchronises
 * `stream`.  Same status conventions as csx_recon (first failing scan). */
csx_status csx_batch_recon(csx_batch *b, const float *const *y, const float *const *r,
                           float *const *f, int init_uniform, int n_iter, double beta,
                           double *J_hist, void *stream);

/* As csx_batch_recon with an iteration count per scan: n_iter[k] >= 0
 * iterations for scan k.  The run goes in stages between consecutive distinct
 * counts; a scan leaves the merged launches once it has run its count, so the
 * scans' results are still bitwise those of csx_recon.  J_hist (NULL or host
 * double[n][J_stride], J_stride >= max(n_iter) + 1): row k receives
 * J(f^0..f^n_iter[k]); its later entries are not written. */
csx_status csx_batch_recon_n(csx_batch *b, const float *const *y, const float *const *r,
                             float *const *f, int init_uniform, const int *n_iter, double beta,
                             double *J_hist, int J_stride, void *stream);

/* Kernel timing (for measurement): while enabled, every forward and adjoint
 * operator launch on this handle is bracketed by HIP events recorded on the
 * caller's stream.  csx_timing_read synchronises those events and returns the
 * summed durations (ms) and launch counts since the last enable, per operator:
 * ms[0], n[0] = forward kernels (including the split reduction), ms[1], n[1] =
 * adjoint kernels.  Off by default; enabling resets the counters. */
csx_status csx_timing_enable(csx_geometry *h, int on);
csx_status csx_timing_read(csx_geometry *h, double ms[2], int n[2]);

/* ---- Learned warm start ------------------------------------------------------
 * Not part of the paper, which starts Alg. 5 from a uniform image.  The
 * first EM factor from the uniform start, x = A^T (y / (u A 1)) / b1 (the
 * back projection, by the back projector of Sec. IV, of the count ratio,
 * divided by the sensitivity image b1 = A^T 1; u = sum(y) / sum(b1) is the
 * uniform start value), enters a small network as log(x + delta); its last
 * layer adds that input back.  The training target of a reconstruction f_T
 * made by Alg. 5 itself is log(f_T / u + delta), and the output o gives the
 * starting image by the inverse map u max(exp(min(o, 30)) - delta,
 * delta / 100) > 0, scaled so that sum(b1 f0) = sum(y) (the total every
 * unpenalised EM iterate carries).  delta in (0, 1] is chosen with the
 * network (CSX_EINVAL otherwise).  A judge (csx_recon_warm) runs Alg. 5 from both starts and keeps
 * the warm one only if its objective is lower.
 *
 * Images are [nb][h][w][c] float32 (an f image [nz][nx][nq] is one image of
 * h = nz, w = nx, c = nq channels).  Weights are [9][c_in][c_out] binary16
 * bits, tap 3 dh + dw reading input pixel (row + dh - 1, col + dw - 1); pixels
 * outside the image read 0.  The products take binary16 operands (activations
 * and output gradients rounded to nearest-even on load) and accumulate in
 * float32.  Supported (c_in, c_out): (64, 32), (32, 32), (32, 64).  All
 * pointers are device memory owned by the caller; calls are asynchronous on
 * `stream` and return CSX_EINVAL for NULL buffers, unsupported channels or
 * sizes < 1. */
typedef struct {
    const uint16_t *w[4];   /* layers 64->32, 32->32, 32->32, 32->64 (binary16) */
    const float *b[4];      /* biases [c_out] float32 */
} csx_warm_net;

/* Workspace needed by csx_conv3x3_backward_weights and csx_warm_loss for nb
 * images of h x w (0 for sizes < 1). */
size_t csx_cnn_workspace_bytes(int nb, int h, int w);

/* y = conv3x3(x, w) + bias + residual (bias and residual may be NULL; the
 * residual is [nb][h][w][cout] and must not be y), then max(y, 0) if relu. */
csx_status csx_conv3x3_forward(const float *x, const uint16_t *w, const float *bias, const float *residual,
                               float *y, int nb, int h, int w_, int cin, int cout, int relu, void *stream);

/* dx[p][i] = sum_t sum_o dy[p - off_t][o] w[t][i][o] for the layer
 * (cin -> cout) with weights w; dy has cout channels, dx cin.  If mask (a
 * [nb][h][w][cin] activation) is not NULL, dx is 0 where mask <= 0 (the ReLU
 * derivative of the layer's input). */
csx_status csx_conv3x3_backward_data(const float *dy, const uint16_t *w, const float *mask, float *dx,
                                     int nb, int h, int w_, int cin, int cout, void *stream);

/* dw[t][i][o] = sum over images and pixels p of x[p + off_t][i] dy[p][o]
 * (float32 [9][cin][cout]); dbias[o] = sum of dy[.][o] (float32 operands,
 * may be NULL).  Fixed summation order (reproducible). */
csx_status csx_conv3x3_backward_weights(const float *x, const float *dy, float *dw, float *dbias,
                                        int nb, int h, int w_, int cin, int cout, void *ws,
                                        size_t ws_bytes, void *stream);

/* Training head: *loss = sum (o - t)^2 / nb (device float64, fixed order),
 * d = dL/do = 2 (o - t) / nb; o, t, d hold nb * n_per_image floats. */
csx_status csx_warm_loss(const float *o, const float *t, int nb, int n_per_image, float *d,
                         double *loss, void *ws, size_t ws_bytes, void *stream);

/* Adam (Kingma & Ba 2015, with bias correction) on n float32 weights w with
 * moments m, v and gradient g; step counts from 1.  w16 (may be NULL)
 * receives the binary16 copy of the updated weights. */
csx_status csx_adam_step(float *w, float *m, float *v, const float *g, uint16_t *w16, int n,
                         double lr, double beta1, double beta2, double eps, int step, void *stream);

/* y = binary16(x), nearest-even. */
csx_status csx_to_half(const float *x, uint16_t *y, int n, void *stream);

/* Network input of scan h: log(x + delta) of the first multiplicative EM
 * factor from the uniform start, x = A^T (y / (u A 1)) / b1 (ratio 0 where
 * A 1 = 0, x = 0 where b1 = 0); u x is the first unpenalised EM iterate.
 * The output holds nvox * nq floats ([nz][nx][nq]).  A 1 is computed once per
 * handle. */
csx_status csx_warm_input(csx_geometry *h, const float *y, float delta, float *x, void *stream);

/* f0 = c max(exp(min(o, 30)) - delta, delta / 100), c = u s with u of the
 * counts y and s such that sum(b1 f0) = sum(y) (float64 sums, fixed order). */
csx_status csx_warm_output(csx_geometry *h, const float *y, const float *o, float delta, float *f0,
                           void *stream);

/* Training target t = log(f / u + delta) of a reconstruction f of counts y. */
csx_status csx_warm_target(csx_geometry *h, const float *y, const float *f, float delta, float *t,
                           void *stream);

/* Input, the four layers (ReLU after the first three) and output in one call
 * (needs nq = 64); activations live in a handle workspace. */
csx_status csx_warm_start(csx_geometry *h, const float *y, const csx_warm_net *net, float delta,
                          float *f0, void *stream);

/* The judge: k_judge iterations of Alg. 5 from f_warm and k_judge from the
 * uniform start; the start whose objective is lower after k_judge iterations
 * (the warm one only if strictly lower) is continued to n_iter iterations in
 * f.  J_hist (host, n_iter + 1, may be NULL) is the kept trajectory;
 * *accepted = 1 if the warm start was kept.  Costs n_iter + k_judge
 * iterations; synchronises `stream`.  0 <= k_judge <= n_iter. */
csx_status csx_recon_warm(csx_geometry *h, const float *y, const float *r, const float *f_warm, float *f,
                          int k_judge, int n_iter, double beta, double *J_hist, int *accepted,
                          void *stream);

/* Thread-local description of the last error ("" if none). */
const char *csx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CSX_H */
