// csx_internal.h -- shared definitions of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/csx.h"

#define CSX_MAX_NE 2048
#define CSX_MAX_MASK_ROWS 4096
#define CSX_MAX_MASK_PERIOD 32
#define CSX_SUM_BLOCKS 256
#define CSX_LDS_MAX (160 * 1024)   // LDS bytes one workgroup may use on gfx950
#define CSX_SPEC_MAX 8192          // largest padded spectrum table in LDS (floats, 32 KB)

csx_status csx_fail(csx_status s, const std::string &msg);

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return csx_fail(CSX_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Per-launch constants of the operator kernels.
struct KParams {
    int nvox, npix, nx, nz, nq, ndx, ndy, ne, mask_nx, mask_ny;
    int lr;              // 1: x -> -x mirror exploited (centred grids, nx and ndx even)
    int td;              // table dtype (CSX_TABLE_F32 / CSX_TABLE_BF16)
    int n_groups;        // voxel groups: pairs (j, mirror j) with LR, else single voxels
    int n_cls;           // pixel classes of the adjoint: ndx * ndy/2 (columns x upper rows)
    int n_quad;          // forward output groups: (ndx/2)*(ndy/2) with LR, else ndx*(ndy/2)
    int qw;              // q lanes per class (64, 32 or 16); 64/qw classes share a wave instruction
    int qchunks;         // ceil(nq / qw)
    float det_z, pitch, hp2;
    double hc, det_zd, pitchd;
    double band_lo, band_hi;    // class in band iff kappa q_max >= band_lo and kappa q_min < band_hi
    double b0;                  // 1 - e_lo/dE: table index = floor(kappa q/dE + b0)
    int qu;                     // 1: uniform q grid q_m = q_0 + m dq
    // spectrum table in LDS: spec_n floats, entry k of the zero-padded table
    // [0, ne+1] at position spec_lo + k, zeros elsewhere; with a uniform grid
    // the pads cover every bin coordinate a wave can reach, so its reads need
    // no clamp
    int spec_lo, spec_n;
    double a0, da;              // q_0/dE and dq/dE of a uniform grid
    double q_min, q_max;
    float half_my;
    float inv_mask_nx;          // 1 / mask_nx
    // pixel subsets (ordered subsets): when set, the forward's waves take
    // their pixel quads from quad_list[0 .. n_quad) and the adjoint's lanes
    // their pixel classes from cls_list[0 .. n_cls) (class = row r * ndx +
    // column a, pixel row ndy/2 + r); otherwise all quads and classes
    const int *quad_list = nullptr;
    const int *cls_list = nullptr;
    // the adjoint's pixel-class tiles split into asplit contiguous ranges
    // (blockIdx.z), each writing its own partial image (full adjoint only)
    int asplit = 1;
    // with a class list: the factor store in list order, the record of entry
    // e of group g at T.ra[g * ra_gs + e] and the node range of its 64-entry
    // chunk at T.ram[(g * ra_gs + e) / 64]; 0: the tile-major store
    long ra_gs = 0;
};

// Per-voxel records.  vf: {C*Gso, det_z - z} (float32); vm: {t/pm,
// (1-t) x/pm} with t = (mask_z - z)/(det_z - z) (float64, the mask-cell
// decision); vd: {x, z, x^2+z^2} (float64).
struct VoxD {
    double x, z, R2, pad;
};

struct DevTables {
    float2 *vf = nullptr;
    double2 *vm = nullptr;
    VoxD *vd = nullptr;
    double *qa = nullptr;      // [qchunks*qw] q_m/dE (0 beyond nq)
    double2 *qblk = nullptr;   // [qchunks*qw/8] {min q, max q} of each block of 8 nodes
    float *qv = nullptr;       // [qchunks*qw] q_m (0 beyond nq)
    float *phi32 = nullptr;    // [ne+2] zero-padded spectrum, float32
    uint16_t *phi16 = nullptr; // [ne+2] zero-padded spectrum, bfloat16 bits
    uint32_t *maskbits = nullptr; // [mask_ny] bit c of row r = cell (c, r)
    // factor store (uniform q grids): the pair factors of every class,
    // computed once per geometry; null when the operators evaluate them on the fly
    uint4 *ra = nullptr;       // adjoint records [n_groups][class tiles][64]: {kappa (f64), A, bits}
    uint4 *rf = nullptr;       // forward records [n_quad][voxel tiles][64][2]: {kappa1, kappa2}, {A1, A2, bits, 0}
    // node range of each record tile (a superset over its 64 lanes, both
    // forward classes): first q node in the low 16 bits, last in the high
    // 16 bits; first > last when no lane of the tile is active
    uint32_t *ram = nullptr;   // [n_groups][class tiles]
    uint32_t *rfm = nullptr;   // [n_quad][voxel tiles]
};

// Bits of a stored record: the mask values of the class's pairs, and whether
// the class is active (some pair open and kappa in band).  Adjoint: bit 0
// (y', column a), 1 (-y', a), 2 (y', -a), 3 (-y', -a), bit 4 active.
// Forward: class 1 in bits 0-3 (tau, tad, tbu, tbd) and 4 (active), class 2
// (the pixel column's mirror) in bits 8-11 and 12.
#define CSX_REC_ACT 16u

// LDS layout of an operator launch (byte offsets).
struct Lds {
    int phi, mask, tile, total;
    int hist = 0;       // energy-resolved forward: per-wave bin histograms
};

// One scan's share of a batched operator launch (device array).
struct CsxJob {
    KParams P;
    DevTables T;
    Lds L;
    const float *in;
    float *out;
    int gx, gy, gz, tps;
};

// Launch geometry of one operator for one handle.
struct OpShape {
    KParams P;          // with the operator's q chunk width
    Lds L;
    dim3 grid, block;
    int tps;            // forward: voxel tiles per split
    int nparts;         // forward: partial images (splits x q chunks)
    int variant;        // kernel template: bit 1 LR, bit 2 uniform q, bits 3+ log2 qw
    const DevTables *T = nullptr;   // tables of the launch when not the handle's own
};

struct csx_geometry {
    csx_geometry_desc d;       // copy (array pointers not kept)
    KParams P;
    DevTables t;
    int table_dtype = CSX_TABLE_F32;
    // launch shape
    int fwd_wpb = 8, adj_wpb = 4;
    csx_launch lc;
    // workspace
    float *part = nullptr;     // forward partials [part_cap] floats
    size_t part_cap = 0;
    float *gws = nullptr;      // [npix] model mean
    float *rho = nullptr;      // [npix] y / z
    float *ones = nullptr;     // [npix] 1
    float *b1 = nullptr;       // [nvox*nq] sensitivity
    float *b2 = nullptr;       // [nvox*nq]
    float *ftmp = nullptr;     // [nvox*nq]
    float *apart = nullptr;    // [adj_splits][nvox*nq] partial images of a split direct adjoint
    size_t apart_cap = 0;      // floats in apart
    double *partL = nullptr;   // per-block data-fit partials
    double *partR = nullptr;   // per-block penalty partials
    double *partS = nullptr;   // [2 * CSX_SUM_BLOCKS] partial sums of the uniform start
    double *scal = nullptr;    // [8] scalars
    double *jhist = nullptr;   // device J history (grown on demand)
    int jhist_cap = 0;
    int *partF = nullptr;      // per-block flags of the data term
    int *flags = nullptr;      // flags of the last objective: bit 0: y_i > 0 with zero
                               // mean; bit 1: y_i < 0 or NaN
    double psi_delta = 0.0;    // penalty potential: 0 quadratic, > 0 Huber scale
    void *os = nullptr;        // ordered-subsets state (csx_os.hip), on demand
    float *fplain = nullptr;   // [nvox*nq] plain-start iterate of the warm-start judge
    float *a1 = nullptr;       // [npix] A 1 (forward of the all-ones image), on demand
    float *warm = nullptr;     // activations of the warm-start network
    size_t warm_cap = 0;       // floats in warm
    void *sai = nullptr;       // scatter-angle-interpolation tables (csx_sai.hip), on demand
    void *energy = nullptr;    // energy-resolved operator buffers (csx_energy.hip), on demand
    double a_max = 0.0;        // largest pair weight A of the geometry (0: not computed yet)
    int op_sai = 0;            // solver operators: bit 0 forward, bit 1 adjoint interpolated
    std::vector<double> q_host, phi_host;   // the descriptor's q nodes and spectrum
    int nbL = 0, nbR = 0;
    int nbRu = 0;              // blocks (penalty partials) of the last update launch
    bool have_b1 = false;
    int64_t bytes = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev[2];
    int ev_used[2] = {0, 0};
    void *iv = nullptr;        // interval-form operators (csx_interval.hip), when built
    int device = 0;            // the HIP device current at csx_init_geometry
    int64_t store_bytes = 0;   // device bytes of the factor store (0: none)
    double store_ms = 0.0;     // time its build took (host clock, synchronised)
};

// operator launchers (csx_ops.hip)
csx_status csx_launch_forward(csx_geometry *h, const float *f, float *g, hipStream_t s);
csx_status csx_launch_adjoint(csx_geometry *h, const float *rho, float *b, hipStream_t s);
csx_launch csx_default_launch(const KParams &P);
int csx_default_adj_splits(const KParams &P, int adj_qw);
bool csx_launch_valid(const csx_launch &lc);
OpShape csx_forward_shape(const csx_geometry *h);
OpShape csx_adjoint_shape(const csx_geometry *h);
csx_status csx_launch_forward_batch(const CsxJob *jobs_dev, const int *begin_dev, int njobs,
                                    int nblocks, int variant, int lds_bytes, hipStream_t s);
csx_status csx_launch_adjoint_batch(const CsxJob *jobs_dev, const int *begin_dev, int njobs,
                                    int nblocks, int variant, int lds_bytes, hipStream_t s);
csx_status csx_launch_sum_parts(csx_geometry *h, int nparts, float *g, hipStream_t s);
// forward with the partial images in a caller-given buffer of part_cap floats
// (no allocation; the handle's workspace is not touched)
csx_status csx_launch_forward_parts(const csx_geometry *h, const float *f, float *part, size_t part_cap, float *g,
                                    hipStream_t s);
// subset operators: forward at the quads of a list (with its own split count)
// finished by the count ratio rho = y / (A f + r) at the subset's pixels, and
// the adjoint over the classes of a list
OpShape csx_forward_shape_list(const csx_geometry *h, const int *quads, int n_quads, int splits);
csx_status csx_launch_forward_list(csx_geometry *h, const float *f, const int *quads, int n_quads, int splits,
                                   const int *pix, int n_pix, const float *y, const float *r, float *rho,
                                   hipStream_t s);
// ra_list, ram_list, ra_gs: the factor store in the list's order (from
// csx_launch_store_list), or null for the tile-major store.
csx_status csx_launch_adjoint_list(csx_geometry *h, const float *rho, const int *cls, int n_cls, float *b,
                                   hipStream_t s, const uint4 *ra_list = nullptr, const uint32_t *ram_list = nullptr,
                                   long ra_gs = 0);
// The adjoint's factor-store records in the order of n_sub class lists of
// n_cls entries each, padded to cls_pad (a multiple of 64): out [n_groups]
// [n_sub][cls_pad], meta one node range per 64 records.
csx_status csx_launch_store_list(const csx_geometry *h, const int *cls, int n_cls, int n_sub, int cls_pad, uint4 *out,
                                 uint32_t *meta, hipStream_t s);
hipEvent_t csx_timing_event(csx_geometry *h, int op);
// interval-form exact operators (csx_interval.hip)
bool csx_iv_feasible(const KParams &P, int *lds_f, int *lds_a);
csx_status csx_iv_build(csx_geometry *h);
void csx_iv_free(csx_geometry *h);
// forward into g; partial images in part (part_cap floats) or, when part is
// null, in the handle's own buffer
csx_status csx_iv_forward(const csx_geometry *h, const float *f, float *part, size_t part_cap, float *g,
                          hipStream_t s);
csx_status csx_iv_adjoint(const csx_geometry *h, const float *rho, float *b, hipStream_t s);
// The interval forward's kernel alone (its partial images into the handle's
// buffer); csx_iv_parts gives that buffer and its image count.
csx_status csx_iv_forward_parts(const csx_geometry *h, const float *f, hipStream_t s);
void csx_iv_parts(const csx_geometry *h, const float **part, int *nparts);

// One scan's share of the batched elementwise launches: the sum of its
// interval forward's partial images into g, the count ratio, the update
// (4 q nodes per thread) into ftmp and the copy-back into f with the
// objective at J[*iter].  Each launch covers every job's blocks (job k's from
// begin[k]), each block doing what the single-scan launch's block of the same
// index does, so results are bitwise those of the single-scan launches.
struct ElemJob {
    const float *part;
    int nparts, npix;
    float *g;
    const float *y, *r;
    float *rho;
    double *partL;
    int *partF;
    int nx, nz, nq;
    const float *f, *b1, *b2;
    float *ftmp;
    double *partR;
    double delta;
    float *fdst;
    int nL, nR;
    int *flags;
    double *J;
};
csx_status csx_launch_iv_sum_batch(const ElemJob *jobs, const int *begin, int njobs, int nblocks, hipStream_t s);
// which: 0 ratio, 1 update (hub: Huber's potential), 2 copy-back + objective
csx_status csx_launch_elem_batch(int which, const ElemJob *jobs, const int *begin, int njobs, int nblocks, double beta,
                                 int hub, const int *iter, hipStream_t s);
size_t csx_iv_part_floats(const csx_geometry *h);
void csx_iv_info(const csx_geometry *h, int *on, int64_t *bytes, double *build_ms, int *intervals);
// factor store: record counts (16-byte adjoint records, 32-byte forward
// records) and the kernels that fill them from the handle's tables
void csx_store_records(const KParams &P, size_t *n_adj, size_t *n_fwd);
csx_status csx_launch_store(const csx_geometry *h, uint4 *ra, uint4 *rf, uint32_t *ram, uint32_t *rfm,
                            hipStream_t s);

// solver pieces (csx_solver.hip)
csx_status csx_launch_ratio(csx_geometry *h, const float *y, const float *r, bool want_rho,
                            hipStream_t s);
csx_status csx_launch_update(csx_geometry *h, const float *f, double beta, bool do_update,
                             hipStream_t s);
// ftmp copied back into f, and in one extra block the objective J (J[iter ? *iter : 0])
// from the partials of the preceding ratio and update launches.
csx_status csx_launch_copy_objective(csx_geometry *h, float *f, double beta, double *J, const int *iter,
                                     hipStream_t s);
csx_status csx_launch_update_ex(csx_geometry *h, const float *f, const float *b1, const float *b2,
                                double beta, float *fout, hipStream_t s);
csx_status csx_launch_objective(csx_geometry *h, double beta, double *J, const int *iter,
                                hipStream_t s);
csx_status csx_launch_iter_incr(int *iter, hipStream_t s);
csx_status csx_launch_uniform_start(csx_geometry *h, const float *y, float *f, hipStream_t s);
csx_status csx_launch_uniform_sums(csx_geometry *h, const float *y, hipStream_t s);
csx_status csx_ensure_b1(csx_geometry *h, hipStream_t s);
void csx_os_free(csx_geometry *h);
// scatter-angle interpolation (csx_sai.hip)
void csx_sai_free(csx_geometry *h);
csx_status csx_pair_weight_max(csx_geometry *h, double *out);
// energy-resolved operators (csx_ops.hip launchers, csx_energy.hip API)
size_t csx_forward_energy_floats(const csx_geometry *h, int *lds_bytes);
csx_status csx_launch_forward_energy(csx_geometry *h, const float *f, const double *sc, float *part,
                                     size_t part_cap, float *gE, hipStream_t s);
csx_status csx_launch_adjoint_energy(csx_geometry *h, const float *psi, float *b, hipStream_t s);
void csx_energy_free(csx_geometry *h);
csx_status csx_launch_forward_sai(csx_geometry *h, const float *f, float *g, hipStream_t s);
csx_status csx_launch_adjoint_sai(csx_geometry *h, const float *rho, float *b, hipStream_t s);
csx_status csx_launch_forward_sai_list(csx_geometry *h, const float *f, const int *quads, int n_quads, int splits,
                                       const int *pix, int n_pix, const float *y, const float *r, float *rho,
                                       hipStream_t s);
csx_status csx_launch_adjoint_sai_list(csx_geometry *h, const float *rho, const int *cls, int n_cls, float *b,
                                       hipStream_t s);
csx_status csx_launch_sum_ratio_list(csx_geometry *h, int nparts, const int *pix, int n_pix, const float *y,
                                     const float *r, float *rho, hipStream_t s);
csx_status csx_launch_copy(const float *src, float *dst, int n, hipStream_t s);
csx_status csx_launch_fill(float *dst, int n, float v, hipStream_t s);
csx_status csx_launch_clear_flags(csx_geometry *h, hipStream_t s);
csx_status csx_launch_ratio_n(int n, const float *g, const float *y, const float *r, float *rho, double *partL,
                              int *partF, bool want_rho, hipStream_t s);
csx_status csx_launch_objective_n(csx_geometry *h, const double *partL, int nL, const int *partF, double beta,
                                  double *J, hipStream_t s);
csx_status csx_launch_uniform_start_n(csx_geometry *h, const float *y, int ny, const float *b1, float *f,
                                      hipStream_t s);
