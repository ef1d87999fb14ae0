// csx.hip -- MI355X (gfx950) kernels and C ABI for fan-beam coded-aperture
// coherent-scatter reconstruction (Odinaka et al., arXiv:1603.06400).
//
// Operators (Sec. II eq. 2, Sec. III eqs. 3-4, Alg. 1 / Alg. 3):
//   g_i  = sum_j A_ij T_ij sum_m q_m Phi(kappa_ij q_m) f_jm         (forward)
//   b_jm = q_m sum_i A_ij T_ij Phi(kappa_ij q_m) y_i                (adjoint)
// with kappa = hc / sin(theta/2) (so E = kappa q, Bragg's law, App. A) and
//   A = C Gso God dtheta (1 + cos^2 theta) cos(theta/2) / sin^2(theta/2).
//
// Execution model (one wave64 = 64 lanes):
//  * lanes = q.  A wave owns one output group (a pair of detector pixels that
//    are mirror images under y -> -y, or one voxel) and walks the other index.
//  * per-pair factors (theta, dtheta, Gso, God, T, kappa) are evaluated with
//    one pair per lane, 64 pairs at a time; a ballot keeps the pairs whose mask
//    cell is open and whose Bragg energies can reach the spectrum band, and the
//    wave then visits only those, broadcasting kappa and the pair weight from
//    the owning lane.  The q-sum of S(theta, q) f(r, q) (the paper's W(r,theta))
//    is the lane-parallel inner step: one spectrum-table gather from LDS and one
//    FMA per lane.
//  * the mirror pixels (x', y') and (x', -y') share theta, dtheta, God and the
//    whole spectral sum (Sec. III-A, up-down mirror symmetry); only T differs,
//    so one inner step serves both.
//  * forward: voxels are split across blocks (split-K) and the partial images
//    are summed in a fixed order -- no atomics, bitwise reproducible.
//  * adjoint: output-stationary per voxel, no atomics, no cross-lane traffic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/csx.h"

#define CSX_MAX_NE 2048
#define CSX_MAX_MASK_BYTES 32768
#define CSX_MAX_MASK_BITROWS 8192

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static csx_status fail(csx_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(CSX_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

extern "C" const char *csx_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// kernel parameters
// ---------------------------------------------------------------------------
struct KParams {
    int nvox, npix, nx, nz, nq, nqpad, ndx, ndy, ne, mask_nx, mask_ny, n_ud;
    float det_z, pitch, hp2, hc;
    float b0p;               // 1 - e_lo/dE: spectrum bin + 1 = floor(kappa * q/dE + b0p)
    float ne_p1;             // ne + 1 (clamp of the padded bin index)
    float band_lo, band_hi;  // kappa q_max >= band_lo and kappa q_min < band_hi
    float q_min, q_max;
    float half_my;           // mask_ny / 2
    int mask_bytes;          // bytes of the mask table in LDS
};

struct DevTables {
    float4 *vox_a = nullptr;  // {x, z, x^2 + z^2, 1/sqrt(x^2+z^2)}
    float4 *vox_b = nullptr;  // {C Gso, t/pm, (1-t) x/pm, 0}, t = (mask_z - z)/(det_z - z)
    float *qa = nullptr;      // q_m/dE, padded with -1e30 (never in band)
    float *qv = nullptr;      // q_m, padded with 0
    float *phi32 = nullptr;   // [ne+2] zero-padded spectrum, float32
    uint16_t *phi16 = nullptr;// [ne+2] zero-padded spectrum, bfloat16 bits
    uint8_t *mask8 = nullptr; // [mask_ny][mask_nx] 0/1
    uint32_t *maskbits = nullptr; // [mask_ny] bit c = cell (c, row)
};

struct csx_geometry {
    csx_geometry_desc d;      // copy (pointers not kept)
    KParams P;
    DevTables t;
    int table_dtype = CSX_TABLE_F32;
    int qchunks = 1;
    // launch shape
    int fwd_wpb = 8, fwd_splits = 1, adj_wpb = 4;
    // workspace
    float *part = nullptr;    // forward partials [fwd_splits*qchunks][npix]
    float *gws = nullptr;     // [npix] model mean
    float *rho = nullptr;     // [npix] y / z
    float *ones = nullptr;    // [npix] 1
    float *b1 = nullptr;      // [nvox*nq] sensitivity
    float *b2 = nullptr;      // [nvox*nq]
    float *ftmp = nullptr;    // [nvox*nq]
    double *partL = nullptr;  // per-block data-fit partials
    double *partR = nullptr;  // per-block penalty partials
    double *scal = nullptr;   // [8] scalars (sums for the uniform start, J)
    double *jhist = nullptr;  // device J history (grown on demand)
    int jhist_cap = 0;
    int *flags = nullptr;     // bit 0: y_i > 0 with zero mean; bit 1: y_i < 0 or NaN
    int nbL = 0, nbR = 0;
    bool have_b1 = false;
    int64_t bytes = 0;
    // optional event timing of operator launches
    bool timing = false;
    std::vector<hipEvent_t> ev[2];   // pairs (start, stop) per operator
    int ev_used[2] = {0, 0};
};

static void release_events(csx_geometry *h);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float readlane_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

// Pair factors of voxel (va, vb) and detector point (xp, yp, det_z):
// returns kappa = hc / sin(theta/2) and A (everything but T, q and Phi).
// theta from |r x r'| and r . s; dtheta = atan2(|a x b|, a . b) for the rays
// a, b = s -/+ (pitch/2) y^ to the two pixel-edge midpoints (App. A).
__device__ __forceinline__ void pair_factors(const KParams &P, float4 va, float4 vb, float xp,
                                             float yp, float &kappa, float &A)
{
    const float x = va.x, z = va.y, R2 = va.z, Rinv = va.w;
    const float sx = xp - x;
    const float sz = P.det_z - z;
    const float h2 = fmaf(sx, sx, sz * sz);
    const float s2 = fmaf(yp, yp, h2);
    const float inv_s = __builtin_amdgcn_rsqf(s2);
    const float God = sz * inv_s * inv_s * inv_s;
    const float cy = fmaf(z, xp, -x * P.det_z);
    const float cross2 = fmaf(yp * yp, R2, cy * cy);
    const float rs = Rinv * inv_s;
    const float sin_t = __builtin_amdgcn_sqrtf(cross2) * rs;
    const float cos_t = fmaf(x, sx, z * sz) * rs;
    const float cos_h = __builtin_amdgcn_sqrtf(0.5f * (1.0f + cos_t));
    const float inv_sin_h = 2.0f * cos_h * __builtin_amdgcn_rcpf(sin_t);
    kappa = P.hc * inv_sin_h;
    const float dth = atan2f(P.pitch * __builtin_amdgcn_sqrtf(h2), s2 - P.hp2);
    A = vb.x * God * dth * fmaf(cos_t, cos_t, 1.0f) * cos_h * inv_sin_h * inv_sin_h;
}

// Mask transmission where the ray from the voxel to (xp, yp) crosses the mask
// plane: column floor(px/pm) mod mask_nx, row floor(py/pm + mask_ny/2).
template <int TD>
__device__ __forceinline__ float mask_T(const KParams &P, float4 vb, float xp, float yp,
                                        const uint8_t *s_mask8, const uint32_t *s_bits)
{
    const float cxf = floorf(fmaf(vb.y, xp, vb.z));
    const float cyf = floorf(fmaf(vb.y, yp, P.half_my));
    if (!(cyf >= 0.0f && cyf < (float)P.mask_ny)) return 0.0f;
    const int row = (int)cyf;
    int col = ((int)cxf) % P.mask_nx;
    col += (col < 0) ? P.mask_nx : 0;
    if (TD == CSX_TABLE_BF16) return (float)((s_bits[row] >> col) & 1u);
    return (float)s_mask8[row * P.mask_nx + col];
}

__device__ __forceinline__ bool in_band(const KParams &P, float kappa)
{
    return kappa * P.q_max >= P.band_lo && kappa * P.q_min < P.band_hi;
}

// padded spectrum bin index for lane constant a = q/dE
__device__ __forceinline__ uint32_t spec_index(const KParams &P, float kappa, float a)
{
    float u = fmaf(kappa, a, P.b0p);
    u = fminf(fmaxf(u, 0.0f), P.ne_p1);
    return (uint32_t)u;
}

template <int TD>
__device__ __forceinline__ float spec_lookup(const float *s_phi, const uint16_t *s_phi16, uint32_t k)
{
    if (TD == CSX_TABLE_BF16) return bf16_to_f32(s_phi16[k]);
    return s_phi[k];
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Cooperative copy of the spectrum and mask tables into LDS.
template <int TD>
__device__ __forceinline__ void stage_tables(const KParams &P, const DevTables &T, float *s_phi,
                                             uint16_t *s_phi16, uint8_t *s_mask8, uint32_t *s_bits)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    if (TD == CSX_TABLE_BF16) {
        for (int k = tid; k < P.ne + 2; k += nt) s_phi16[k] = T.phi16[k];
        for (int k = tid; k < P.mask_ny; k += nt) s_bits[k] = T.maskbits[k];
    } else {
        for (int k = tid; k < P.ne + 2; k += nt) s_phi[k] = T.phi32[k];
        for (int k = tid; k < P.mask_bytes; k += nt) s_mask8[k] = T.mask8[k];
    }
}

struct LdsLayout {
    int phi_off, mask_off, tile_off, total;
};

static LdsLayout lds_layout(const KParams &P, int td, bool with_tile)
{
    LdsLayout L;
    int off = 0;
    auto al = [](int v) { return (v + 15) & ~15; };
    L.phi_off = off;
    off += al((P.ne + 2) * (td == CSX_TABLE_BF16 ? 2 : 4));
    L.mask_off = off;
    off += al(td == CSX_TABLE_BF16 ? P.mask_ny * 4 : P.mask_bytes);
    L.tile_off = off;
    if (with_tile) off += 64 * 64 * 4;
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// K1 forward: wave = one up/down pixel pair x one 64-wide q chunk, block =
// WPB waves sharing a staged 64-voxel x 64-q tile of f; blockIdx.y = voxel
// split, blockIdx.z = q chunk.  part[(split*qchunks + qc)][pixel].
// ---------------------------------------------------------------------------
template <int TD>
__global__ void __launch_bounds__(1024) k_forward(KParams P, DevTables T, LdsLayout L,
                                                  const float *__restrict__ f,
                                                  float *__restrict__ part, int vox_per_split)
{
    extern __shared__ __align__(16) unsigned char lds[];
    float *s_phi = (float *)(lds + L.phi_off);
    uint16_t *s_phi16 = (uint16_t *)(lds + L.phi_off);
    uint8_t *s_mask8 = (uint8_t *)(lds + L.mask_off);
    uint32_t *s_bits = (uint32_t *)(lds + L.mask_off);
    float *s_f = (float *)(lds + L.tile_off);

    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int ud = blockIdx.x * wpb + (threadIdx.x >> 6);
    const int qc = blockIdx.z;
    const int m = qc * 64 + lane;
    const int j0 = blockIdx.y * vox_per_split;
    const int j1 = min(P.nvox, j0 + vox_per_split);

    stage_tables<TD>(P, T, s_phi, s_phi16, s_mask8, s_bits);

    const bool wave_on = ud < P.n_ud;
    const int a = wave_on ? ud % P.ndx : 0;
    const int bu = P.ndy / 2 + (wave_on ? ud / P.ndx : 0);
    const float xp = (float)(2 * a - P.ndx + 1) * (0.5f * P.pitch);
    const float yp = (float)(2 * bu - P.ndy + 1) * (0.5f * P.pitch);
    const float qa = T.qa[m];

    float acc_u = 0.0f, acc_d = 0.0f;
    for (int jb = j0; jb < j1; jb += 64) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < 64 * 64; idx += blockDim.x) {
            const int v = idx >> 6, l = idx & 63;
            const int jj = jb + v, mm = qc * 64 + l;
            s_f[idx] = (jj < j1 && mm < P.nq) ? f[(size_t)jj * P.nq + mm] : 0.0f;
        }
        __syncthreads();
        if (!wave_on) continue;
        const int jj = jb + lane;
        float kap = 0.0f, su = 0.0f, sd = 0.0f;
        bool act = false;
        if (jj < j1) {
            const float4 va = T.vox_a[jj], vb = T.vox_b[jj];
            const float tu = mask_T<TD>(P, vb, xp, yp, s_mask8, s_bits);
            const float td = mask_T<TD>(P, vb, xp, -yp, s_mask8, s_bits);
            if (tu != 0.0f || td != 0.0f) {
                float A;
                pair_factors(P, va, vb, xp, yp, kap, A);
                su = A * tu;
                sd = A * td;
                act = in_band(P, kap);
            }
        }
        uint64_t bal = __ballot(act);
        while (bal) {
            const int v = __builtin_ctzll(bal);
            bal &= bal - 1;
            const float k = readlane_f(kap, v);
            const float cu = readlane_f(su, v);
            const float cd = readlane_f(sd, v);
            const float ph = spec_lookup<TD>(s_phi, s_phi16, spec_index(P, k, qa));
            const float w = ph * s_f[v * 64 + lane];
            acc_u = fmaf(cu, w, acc_u);
            acc_d = fmaf(cd, w, acc_d);
        }
    }
    if (!wave_on) return;
    const float qm = T.qv[m];
    const float gu = wave_sum(acc_u * qm);
    const float gd = wave_sum(acc_d * qm);
    if (lane == 0) {
        float *dst = part + (size_t)(blockIdx.y * gridDim.z + qc) * P.npix;
        dst[bu * P.ndx + a] = gu;
        dst[(P.ndy - 1 - bu) * P.ndx + a] = gd;
    }
}

// g_i = sum_p part[p][i] in a fixed order.
__global__ void k_sum_parts(const float *__restrict__ part, int nparts, int n, float *__restrict__ g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += part[(size_t)p * n + i];
    g[i] = s;
}

// ---------------------------------------------------------------------------
// K2 adjoint: wave = one voxel x one 64-wide q chunk; walks all up/down pixel
// pairs.  b[j][m] = q_m * sum over pairs of A (T_u rho_u + T_d rho_d) Phi(kappa q_m).
// ---------------------------------------------------------------------------
template <int TD>
__global__ void __launch_bounds__(1024) k_adjoint(KParams P, DevTables T, LdsLayout L,
                                                  const float *__restrict__ rho,
                                                  float *__restrict__ b)
{
    extern __shared__ __align__(16) unsigned char lds[];
    float *s_phi = (float *)(lds + L.phi_off);
    uint16_t *s_phi16 = (uint16_t *)(lds + L.phi_off);
    uint8_t *s_mask8 = (uint8_t *)(lds + L.mask_off);
    uint32_t *s_bits = (uint32_t *)(lds + L.mask_off);

    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int j = blockIdx.x * wpb + (threadIdx.x >> 6);
    const int qc = blockIdx.y;
    const int m = qc * 64 + lane;

    stage_tables<TD>(P, T, s_phi, s_phi16, s_mask8, s_bits);
    __syncthreads();
    if (j >= P.nvox) return;

    const float4 va = T.vox_a[j], vb = T.vox_b[j];
    const float qa = T.qa[m];
    float acc = 0.0f;
    for (int pb = 0; pb < P.n_ud; pb += 64) {
        const int p = pb + lane;
        float kap = 0.0f, c = 0.0f;
        bool act = false;
        if (p < P.n_ud) {
            const int a = p % P.ndx;
            const int bu = P.ndy / 2 + p / P.ndx;
            const int bd = P.ndy - 1 - bu;
            const float xp = (float)(2 * a - P.ndx + 1) * (0.5f * P.pitch);
            const float yp = (float)(2 * bu - P.ndy + 1) * (0.5f * P.pitch);
            const float tu = mask_T<TD>(P, vb, xp, yp, s_mask8, s_bits);
            const float td = mask_T<TD>(P, vb, xp, -yp, s_mask8, s_bits);
            const float w = tu * rho[bu * P.ndx + a] + td * rho[bd * P.ndx + a];
            if (w != 0.0f) {
                float A;
                pair_factors(P, va, vb, xp, yp, kap, A);
                c = A * w;
                act = in_band(P, kap) && c != 0.0f;
            }
        }
        uint64_t bal = __ballot(act);
        while (bal) {
            const int v = __builtin_ctzll(bal);
            bal &= bal - 1;
            const float k = readlane_f(kap, v);
            const float cc = readlane_f(c, v);
            const float ph = spec_lookup<TD>(s_phi, s_phi16, spec_index(P, k, qa));
            acc = fmaf(cc, ph, acc);
        }
    }
    if (m < P.nq) b[(size_t)j * P.nq + m] = acc * T.qv[m];
}

// ---------------------------------------------------------------------------
// K3 Poisson ratio + data-fit partials (float64):
//   z = g + r, rho = y/z (0 where y = 0), L_i = z - y ln z + ln y!
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum_d(double v, double *s_red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) s_red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += s_red[k];
    }
    return t;
}

__global__ void __launch_bounds__(256) k_ratio(int n, const float *__restrict__ g,
                                               const float *__restrict__ y,
                                               const float *__restrict__ r,
                                               float *__restrict__ rho, double *__restrict__ partL,
                                               int *__restrict__ flags, int want_rho)
{
    __shared__ double s_red[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double L = 0.0;
    if (i < n) {
        const float z = g[i] + (r ? r[i] : 0.0f);
        const float yi = y[i];
        float q = 0.0f;
        if (!(yi >= 0.0f)) {
            atomicOr(flags, 2);
        } else if (yi > 0.0f) {
            if (z > 0.0f) {
                q = yi / z;
                L = (double)z - (double)yi * log((double)z) + lgamma((double)yi + 1.0);
            } else {
                atomicOr(flags, 1);
                L = INFINITY;
            }
        } else {
            L = (double)z;
        }
        if (want_rho) rho[i] = q;
    }
    const double t = block_sum_d(L, s_red);
    if (threadIdx.x == 0) partL[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// K4 separable-surrogate update (App. B, eq. f_update) for psi(t) = t^2/2,
// 4 in-slice neighbours at the same q, unit weights; evaluated in float64:
//   b3 + b4 = 4 |N_j|, b5 + b6 = 2 sum_k (fhat_j - fhat_k)
//   chi1 = beta (b3+b4), chi2 = b1 + beta(-fhat (b3+b4) + b5 + b6), chi3 = fhat b2
//   f = 2 chi3 / (chi2 + sqrt(chi2^2 + 4 chi1 chi3))       if chi2 > 0
//     = (-chi2 + sqrt(chi2^2 + 4 chi1 chi3)) / (2 chi1)    if chi2 <= 0, chi1 > 0
//     = fhat                                               otherwise (unseen voxel, beta = 0)
// The first form is Lemma 1's root multiplied through by its conjugate.
// Also accumulates R(fhat) = sum_j sum_k (fhat_j - fhat_k)^2 / 2 per block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_update(int nx, int nz, int nq, const float *__restrict__ fh,
                                                const float *__restrict__ b1,
                                                const float *__restrict__ b2, double beta,
                                                float *__restrict__ fout,
                                                double *__restrict__ partR, int do_update)
{
    __shared__ double s_red[4];
    const int n = nx * nz * nq;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double R = 0.0;
    if (e < n) {
        const int m = e % nq;
        const int j = e / nq;
        const int ix = j % nx, iz = j / nx;
        const double fj = fh[e];
        double s = 0.0, rr = 0.0;
        int cnt = 0;
        if (ix > 0) { const double d = fj - fh[e - nq]; s += d; rr += d * d; ++cnt; }
        if (ix < nx - 1) { const double d = fj - fh[e + nq]; s += d; rr += d * d; ++cnt; }
        if (iz > 0) { const double d = fj - fh[e - (size_t)nx * nq]; s += d; rr += d * d; ++cnt; }
        if (iz < nz - 1) { const double d = fj - fh[e + (size_t)nx * nq]; s += d; rr += d * d; ++cnt; }
        R = 0.5 * rr;
        if (do_update) {
            const double b34 = 4.0 * cnt;
            const double chi1 = beta * b34;
            const double chi2 = (double)b1[e] + beta * (-fj * b34 + 2.0 * s);
            const double chi3 = fj * (double)b2[e];
            double out;
            const double disc = sqrt(chi2 * chi2 + 4.0 * chi1 * chi3);
            if (chi2 > 0.0) out = 2.0 * chi3 / (chi2 + disc);
            else if (chi1 > 0.0) out = (-chi2 + disc) / (2.0 * chi1);
            else out = fj;
            fout[e] = (float)out;
        }
        (void)m;
    }
    const double t = block_sum_d(R, s_red);
    if (threadIdx.x == 0) partR[blockIdx.x] = t;
}

// K5: J = sum partL + beta * sum partR in a fixed order, one block.
__global__ void __launch_bounds__(256) k_objective(const double *__restrict__ partL, int nL,
                                                   const double *__restrict__ partR, int nR,
                                                   double beta, const int *__restrict__ flags,
                                                   double *__restrict__ J)
{
    __shared__ double s_red[4];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nL; k += blockDim.x) a += partL[k];
    for (int k = threadIdx.x; k < nR; k += blockDim.x) b += partR[k];
    const double ta = block_sum_d(a, s_red);
    __syncthreads();
    const double tb = block_sum_d(b, s_red);
    if (threadIdx.x == 0) *J = (*flags & 1) ? INFINITY : ta + beta * tb;
}

// sums for the uniform start: scal[0] = sum y, scal[1] = sum b1
__global__ void __launch_bounds__(256) k_sum2(const float *__restrict__ x, int nx_,
                                              const float *__restrict__ y, int ny_,
                                              double *__restrict__ out)
{
    __shared__ double s_red[4];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nx_; k += blockDim.x) a += x[k];
    for (int k = threadIdx.x; k < ny_; k += blockDim.x) b += y[k];
    const double ta = block_sum_d(a, s_red);
    __syncthreads();
    const double tb = block_sum_d(b, s_red);
    if (threadIdx.x == 0) { out[0] = ta; out[1] = tb; }
}

__global__ void k_fill_ratio(float *__restrict__ f, int n, const double *__restrict__ scal)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) f[e] = (float)(scal[1] > 0.0 ? scal[0] / scal[1] : 0.0);
}

__global__ void k_fill(float *__restrict__ p, int n, float v)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void k_copy(const float *__restrict__ s, float *__restrict__ d, int n)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) d[e] = s[e];
}

__global__ void k_clear_int(int *p) { *p = 0; }

// ---------------------------------------------------------------------------
// host: descriptor validation and tables
// ---------------------------------------------------------------------------
static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

extern "C" csx_status csx_validate_desc(const csx_geometry_desc *d)
{
    if (!d) return fail(CSX_EINVAL, "descriptor is NULL");
    if (d->nx < 1 || d->nz < 1 || d->nq < 1 || d->ndx < 1 || d->ndy < 1 || d->ne < 1 ||
        d->mask_nx < 1 || d->mask_ny < 1)
        return fail(CSX_EGEOM, "all counts must be >= 1");
    if (!d->q || !d->phi || !d->mask) return fail(CSX_EINVAL, "q, phi and mask must be non-NULL");
    if (d->ndy % 2 != 0) return fail(CSX_EGEOM, "ndy must be even");
    if (!(std::isfinite(d->x_min) && std::isfinite(d->x_max) && d->x_min < d->x_max))
        return fail(CSX_EGEOM, "need x_min < x_max");
    if (!(finite_pos(d->z_min) && d->z_min < d->z_max && d->z_max < d->mask_z &&
          d->mask_z < d->det_z && std::isfinite(d->det_z)))
        return fail(CSX_EGEOM, "need 0 < z_min < z_max < mask_z < det_z");
    if (!finite_pos(d->det_pitch) || !finite_pos(d->mask_pitch) || !finite_pos(d->hc))
        return fail(CSX_EGEOM, "pitches and hc must be positive");
    if (!(std::isfinite(d->e_lo) && std::isfinite(d->e_hi) && d->e_lo < d->e_hi))
        return fail(CSX_EGEOM, "need e_lo < e_hi");
    if (!(std::isfinite(d->C) && d->C >= 0.0)) return fail(CSX_EGEOM, "C must be finite and >= 0");
    if (d->ne > CSX_MAX_NE) return fail(CSX_EGEOM, "ne exceeds the LDS spectrum table");
    if (d->table_dtype != CSX_TABLE_F32 && d->table_dtype != CSX_TABLE_BF16)
        return fail(CSX_EINVAL, "unknown table_dtype");
    if (d->table_dtype == CSX_TABLE_BF16) {
        if (d->mask_nx > 32 || d->mask_ny > CSX_MAX_MASK_BITROWS)
            return fail(CSX_EGEOM, "bit-packed mask needs mask_nx <= 32 and mask_ny <= 8192");
    } else if ((long)d->mask_nx * d->mask_ny > CSX_MAX_MASK_BYTES) {
        return fail(CSX_EGEOM, "mask exceeds the LDS mask table");
    }
    const long nvox = (long)d->nx * d->nz, npix = (long)d->ndx * d->ndy;
    if (nvox * d->nq > (1L << 30) || npix > (1L << 28)) return fail(CSX_EGEOM, "problem too large");
    if (d->ndx > (1 << 20) || d->ndy > (1 << 20)) return fail(CSX_EGEOM, "detector too large");
    for (int m = 0; m < d->nq; ++m)
        if (!finite_pos(d->q[m])) return fail(CSX_EGEOM, "q nodes must be finite and > 0");
    for (int k = 0; k < d->ne; ++k)
        if (!(std::isfinite(d->phi[k]) && d->phi[k] >= 0.0))
            return fail(CSX_EGEOM, "spectrum must be finite and >= 0");
    for (long k = 0; k < (long)d->mask_nx * d->mask_ny; ++k)
        if (d->mask[k] > 1) return fail(CSX_EGEOM, "mask values must be 0 or 1");
    return CSX_OK;
}

// float32 -> bfloat16 bits, round to nearest, ties to even
static uint16_t bf16_rne(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

template <typename T>
static csx_status dev_upload(T **dst, const std::vector<T> &src, int64_t &bytes)
{
    HIP_TRY(hipMalloc((void **)dst, src.size() * sizeof(T)));
    HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    bytes += (int64_t)(src.size() * sizeof(T));
    return CSX_OK;
}

template <typename T>
static csx_status dev_alloc(T **dst, size_t n, int64_t &bytes)
{
    HIP_TRY(hipMalloc((void **)dst, n * sizeof(T)));
    bytes += (int64_t)(n * sizeof(T));
    return CSX_OK;
}

static void free_all(csx_geometry *h)
{
    void *ptrs[] = {h->t.vox_a, h->t.vox_b, h->t.qa, h->t.qv, h->t.phi32, h->t.phi16,
                    h->t.mask8, h->t.maskbits, h->part, h->gws, h->rho, h->ones, h->b1,
                    h->b2, h->ftmp, h->partL, h->partR, h->scal, h->jhist, h->flags};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

#define CSX_TRY(expr)                        \
    do {                                     \
        csx_status s_ = (expr);              \
        if (s_ != CSX_OK) {                  \
            free_all(h);                     \
            delete h;                        \
            return s_;                       \
        }                                    \
    } while (0)

extern "C" csx_status csx_init_geometry(const csx_geometry_desc *d, csx_geometry **out)
{
    if (!out) return fail(CSX_EINVAL, "out is NULL");
    *out = nullptr;
    csx_status st = csx_validate_desc(d);
    if (st != CSX_OK) return st;

    csx_geometry *h = new (std::nothrow) csx_geometry();
    if (!h) return fail(CSX_ENOMEM, "host allocation failed");
    h->d = *d;
    h->d.q = nullptr;
    h->d.phi = nullptr;
    h->d.mask = nullptr;
    h->table_dtype = d->table_dtype;

    KParams &P = h->P;
    P.nx = d->nx;
    P.nz = d->nz;
    P.nvox = d->nx * d->nz;
    P.ndx = d->ndx;
    P.ndy = d->ndy;
    P.npix = d->ndx * d->ndy;
    P.n_ud = d->ndx * (d->ndy / 2);
    P.nq = d->nq;
    h->qchunks = (d->nq + 63) / 64;
    P.nqpad = h->qchunks * 64;
    P.ne = d->ne;
    P.mask_nx = d->mask_nx;
    P.mask_ny = d->mask_ny;
    P.mask_bytes = d->mask_nx * d->mask_ny;
    P.det_z = (float)d->det_z;
    P.pitch = (float)d->det_pitch;
    P.hp2 = (float)(0.25 * d->det_pitch * d->det_pitch);
    P.hc = (float)d->hc;
    const double dE = (d->e_hi - d->e_lo) / d->ne;
    P.b0p = (float)(1.0 - d->e_lo / dE);
    P.ne_p1 = (float)(d->ne + 1);
    double qmin = d->q[0], qmax = d->q[0];
    for (int m = 1; m < d->nq; ++m) {
        qmin = std::min(qmin, d->q[m]);
        qmax = std::max(qmax, d->q[m]);
    }
    P.q_min = (float)qmin;
    P.q_max = (float)qmax;
    P.band_lo = (float)(d->e_lo * (1.0 - 1e-5));
    P.band_hi = (float)(d->e_hi * (1.0 + 1e-5));
    P.half_my = (float)(0.5 * d->mask_ny);

    // per-voxel tables (float64 on the host, stored as float32)
    std::vector<float4> va(P.nvox), vb(P.nvox);
    const double dx = (d->x_max - d->x_min) / d->nx, dz = (d->z_max - d->z_min) / d->nz;
    for (int iz = 0; iz < d->nz; ++iz)
        for (int ix = 0; ix < d->nx; ++ix) {
            const double x = d->x_min + (ix + 0.5) * dx;
            const double z = d->z_min + (iz + 0.5) * dz;
            const double R2 = x * x + z * z;
            const double R = std::sqrt(R2);
            const double t = (d->mask_z - z) / (d->det_z - z);
            const int j = iz * d->nx + ix;
            va[j] = make_float4((float)x, (float)z, (float)R2, (float)(1.0 / R));
            vb[j] = make_float4((float)(d->C * z / (R2 * R)), (float)(t / d->mask_pitch),
                                (float)((1.0 - t) * x / d->mask_pitch), 0.0f);
        }
    std::vector<float> qa(P.nqpad, -1e30f), qv(P.nqpad, 0.0f);
    for (int m = 0; m < d->nq; ++m) {
        qa[m] = (float)(d->q[m] / dE);
        qv[m] = (float)d->q[m];
    }
    std::vector<float> phi32(d->ne + 2, 0.0f);
    std::vector<uint16_t> phi16(d->ne + 2, 0);
    for (int k = 0; k < d->ne; ++k) {
        phi32[k + 1] = (float)d->phi[k];
        phi16[k + 1] = bf16_rne((float)d->phi[k]);
    }
    std::vector<uint8_t> m8(d->mask, d->mask + (size_t)d->mask_nx * d->mask_ny);
    std::vector<uint32_t> bits(d->mask_ny, 0u);
    if (d->mask_nx <= 32)
        for (int r = 0; r < d->mask_ny; ++r)
            for (int c = 0; c < d->mask_nx; ++c)
                if (d->mask[(size_t)r * d->mask_nx + c]) bits[r] |= 1u << c;

    int64_t &B = h->bytes;
    CSX_TRY(dev_upload(&h->t.vox_a, va, B));
    CSX_TRY(dev_upload(&h->t.vox_b, vb, B));
    CSX_TRY(dev_upload(&h->t.qa, qa, B));
    CSX_TRY(dev_upload(&h->t.qv, qv, B));
    CSX_TRY(dev_upload(&h->t.phi32, phi32, B));
    CSX_TRY(dev_upload(&h->t.phi16, phi16, B));
    CSX_TRY(dev_upload(&h->t.mask8, m8, B));
    CSX_TRY(dev_upload(&h->t.maskbits, bits, B));

    // launch shape: forward waves per block and voxel splits sized so that a
    // launch holds >= ~8k waves (256 CUs x 4 SIMDs x 8)
    const int n_ud_blocks = (P.n_ud + h->fwd_wpb - 1) / h->fwd_wpb;
    const int target_waves = 16384;
    int splits = std::max(1, target_waves / std::max(1, n_ud_blocks * h->fwd_wpb * h->qchunks));
    splits = std::min(splits, std::max(1, (P.nvox + 255) / 256));
    h->fwd_splits = splits;

    const size_t nimg = (size_t)P.nvox * P.nq;
    CSX_TRY(dev_alloc(&h->part, (size_t)h->fwd_splits * h->qchunks * P.npix, B));
    CSX_TRY(dev_alloc(&h->gws, P.npix, B));
    CSX_TRY(dev_alloc(&h->rho, P.npix, B));
    CSX_TRY(dev_alloc(&h->ones, P.npix, B));
    CSX_TRY(dev_alloc(&h->b1, nimg, B));
    CSX_TRY(dev_alloc(&h->b2, nimg, B));
    CSX_TRY(dev_alloc(&h->ftmp, nimg, B));
    h->nbL = (P.npix + 255) / 256;
    h->nbR = (int)((nimg + 255) / 256);
    CSX_TRY(dev_alloc(&h->partL, h->nbL, B));
    CSX_TRY(dev_alloc(&h->partR, h->nbR, B));
    CSX_TRY(dev_alloc(&h->scal, 8, B));
    CSX_TRY(dev_alloc(&h->flags, 1, B));
    {
        hipError_t e = hipGetLastError();
        (void)e;
    }
    hipLaunchKernelGGL(k_fill, dim3((P.npix + 255) / 256), dim3(256), 0, 0, h->ones, P.npix, 1.0f);
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, 0, h->flags);
    {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            free_all(h);
            delete h;
            return fail(CSX_EHIP, std::string("init: ") + hipGetErrorString(e));
        }
    }
    *out = h;
    return CSX_OK;
}

extern "C" void csx_free_geometry(csx_geometry *h)
{
    if (!h) return;
    release_events(h);
    free_all(h);
    delete h;
}

extern "C" csx_status csx_get_info(const csx_geometry *h, csx_info *out)
{
    if (!h || !out) return fail(CSX_EINVAL, "NULL argument");
    out->nvox = h->P.nvox;
    out->npix = h->P.npix;
    out->nq = h->P.nq;
    out->symmetric_lr = 0;
    out->table_dtype = h->table_dtype;
    out->workspace_bytes = h->bytes;
    return CSX_OK;
}

// ---------------------------------------------------------------------------
// optional event timing
// ---------------------------------------------------------------------------
static hipEvent_t timing_event(csx_geometry *h, int op)
{
    if (!h->timing) return nullptr;
    std::vector<hipEvent_t> &v = h->ev[op];
    if (h->ev_used[op] == (int)v.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        v.push_back(e);
    }
    return v[h->ev_used[op]++];
}

static void release_events(csx_geometry *h)
{
    for (int op = 0; op < 2; ++op) {
        for (hipEvent_t e : h->ev[op]) (void)hipEventDestroy(e);
        h->ev[op].clear();
        h->ev_used[op] = 0;
    }
}

extern "C" csx_status csx_timing_enable(csx_geometry *h, int on)
{
    if (!h) return fail(CSX_EINVAL, "NULL handle");
    HIP_TRY(hipDeviceSynchronize());
    h->ev_used[0] = h->ev_used[1] = 0;
    h->timing = on != 0;
    return CSX_OK;
}

extern "C" csx_status csx_timing_read(csx_geometry *h, double ms[2], int n[2])
{
    if (!h || !ms || !n) return fail(CSX_EINVAL, "NULL argument");
    for (int op = 0; op < 2; ++op) {
        ms[op] = 0.0;
        n[op] = h->ev_used[op] / 2;
        for (int k = 0; k + 1 < h->ev_used[op]; k += 2) {
            HIP_TRY(hipEventSynchronize(h->ev[op][k + 1]));
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, h->ev[op][k], h->ev[op][k + 1]));
            ms[op] += t;
        }
    }
    return CSX_OK;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static csx_status launch_forward(csx_geometry *h, const float *f, float *g, hipStream_t s)
{
    const KParams &P = h->P;
    const LdsLayout L = lds_layout(P, h->table_dtype, true);
    const int wpb = h->fwd_wpb;
    const int splits = h->fwd_splits;
    const int vps = (P.nvox + splits - 1) / splits;
    dim3 grid((P.n_ud + wpb - 1) / wpb, splits, h->qchunks);
    dim3 block(64 * wpb);
    const int nparts = splits * h->qchunks;
    float *dst = h->part;
    hipEvent_t e0 = timing_event(h, 0), e1 = timing_event(h, 0);
    if (e0) HIP_TRY(hipEventRecord(e0, s));
    if (h->table_dtype == CSX_TABLE_BF16)
        hipLaunchKernelGGL(k_forward<CSX_TABLE_BF16>, grid, block, L.total, s, P, h->t, L, f, dst, vps);
    else
        hipLaunchKernelGGL(k_forward<CSX_TABLE_F32>, grid, block, L.total, s, P, h->t, L, f, dst, vps);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3((P.npix + 255) / 256), dim3(256), 0, s, h->part, nparts,
                       P.npix, g);
    HIP_TRY(hipGetLastError());
    if (e1) HIP_TRY(hipEventRecord(e1, s));
    return CSX_OK;
}

static csx_status launch_adjoint(csx_geometry *h, const float *rho, float *b, hipStream_t s)
{
    const KParams &P = h->P;
    const LdsLayout L = lds_layout(P, h->table_dtype, false);
    const int wpb = h->adj_wpb;
    dim3 grid((P.nvox + wpb - 1) / wpb, h->qchunks);
    dim3 block(64 * wpb);
    hipEvent_t e0 = timing_event(h, 1), e1 = timing_event(h, 1);
    if (e0) HIP_TRY(hipEventRecord(e0, s));
    if (h->table_dtype == CSX_TABLE_BF16)
        hipLaunchKernelGGL(k_adjoint<CSX_TABLE_BF16>, grid, block, L.total, s, P, h->t, L, rho, b);
    else
        hipLaunchKernelGGL(k_adjoint<CSX_TABLE_F32>, grid, block, L.total, s, P, h->t, L, rho, b);
    HIP_TRY(hipGetLastError());
    if (e1) HIP_TRY(hipEventRecord(e1, s));
    return CSX_OK;
}

extern "C" csx_status csx_forward(csx_geometry *h, const float *f, float *g, void *stream)
{
    if (!h || !f || !g) return fail(CSX_EINVAL, "NULL argument");
    return launch_forward(h, f, g, (hipStream_t)stream);
}

extern "C" csx_status csx_backproject(csx_geometry *h, const float *y, float *b, void *stream)
{
    if (!h || !y || !b) return fail(CSX_EINVAL, "NULL argument");
    return launch_adjoint(h, y, b, (hipStream_t)stream);
}

static csx_status ensure_b1(csx_geometry *h, hipStream_t s)
{
    if (h->have_b1) return CSX_OK;
    csx_status st = launch_adjoint(h, h->ones, h->b1, s);
    if (st != CSX_OK) return st;
    h->have_b1 = true;
    return CSX_OK;
}

// z = A f + r, rho, data-fit partials
static csx_status data_term(csx_geometry *h, const float *y, const float *r, const float *f,
                            bool want_rho, hipStream_t s)
{
    csx_status st = launch_forward(h, f, h->gws, s);
    if (st != CSX_OK) return st;
    hipLaunchKernelGGL(k_ratio, dim3(h->nbL), dim3(256), 0, s, h->P.npix, h->gws, y, r, h->rho,
                       h->partL, h->flags, want_rho ? 1 : 0);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

static csx_status step_impl(csx_geometry *h, const float *y, const float *r, float *f, double beta,
                            double *J, hipStream_t s)
{
    const KParams &P = h->P;
    csx_status st = ensure_b1(h, s);
    if (st != CSX_OK) return st;
    st = data_term(h, y, r, f, true, s);
    if (st != CSX_OK) return st;
    st = launch_adjoint(h, h->rho, h->b2, s);
    if (st != CSX_OK) return st;
    const int n = P.nvox * P.nq;
    hipLaunchKernelGGL(k_update, dim3(h->nbR), dim3(256), 0, s, P.nx, P.nz, P.nq, f, h->b1, h->b2,
                       beta, h->ftmp, h->partR, 1);
    HIP_TRY(hipGetLastError());
    if (J) {
        hipLaunchKernelGGL(k_objective, dim3(1), dim3(256), 0, s, h->partL, h->nbL, h->partR,
                           h->nbR, beta, h->flags, J);
        HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_copy, dim3((n + 255) / 256), dim3(256), 0, s, h->ftmp, f, n);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

extern "C" csx_status csx_recon_step(csx_geometry *h, const float *y, const float *r, float *f,
                                     double beta, double *J_out, void *stream)
{
    if (!h || !y || !f) return fail(CSX_EINVAL, "NULL argument");
    if (!(std::isfinite(beta) && beta >= 0.0)) return fail(CSX_EINVAL, "beta must be finite and >= 0");
    return step_impl(h, y, r, f, beta, J_out, (hipStream_t)stream);
}

extern "C" csx_status csx_recon(csx_geometry *h, const float *y, const float *r, float *f,
                                int init_uniform, int n_iter, double beta, double *J_hist,
                                void *stream)
{
    if (!h || !y || !f) return fail(CSX_EINVAL, "NULL argument");
    if (n_iter < 0) return fail(CSX_EINVAL, "n_iter must be >= 0");
    if (!(std::isfinite(beta) && beta >= 0.0)) return fail(CSX_EINVAL, "beta must be finite and >= 0");
    hipStream_t s = (hipStream_t)stream;
    const KParams &P = h->P;
    const int n = P.nvox * P.nq;
    if (h->jhist_cap < n_iter + 1) {
        if (h->jhist) HIP_TRY(hipFree(h->jhist));
        h->jhist = nullptr;
        HIP_TRY(hipMalloc((void **)&h->jhist, sizeof(double) * (n_iter + 1)));
        h->jhist_cap = n_iter + 1;
    }
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, s, h->flags);
    csx_status st = ensure_b1(h, s);
    if (st != CSX_OK) return st;
    if (init_uniform) {
        hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, s, y, P.npix, h->b1, n, h->scal);
        hipLaunchKernelGGL(k_fill_ratio, dim3((n + 255) / 256), dim3(256), 0, s, f, n, h->scal);
        HIP_TRY(hipGetLastError());
    }
    for (int t = 0; t < n_iter; ++t) {
        st = step_impl(h, y, r, f, beta, h->jhist + t, s);
        if (st != CSX_OK) return st;
    }
    // J at the final iterate
    st = data_term(h, y, r, f, false, s);
    if (st != CSX_OK) return st;
    hipLaunchKernelGGL(k_update, dim3(h->nbR), dim3(256), 0, s, P.nx, P.nz, P.nq, f, h->b1, h->b2,
                       beta, h->ftmp, h->partR, 0);
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(256), 0, s, h->partL, h->nbL, h->partR, h->nbR,
                       beta, h->flags, h->jhist + n_iter);
    HIP_TRY(hipGetLastError());
    int flags = 0;
    HIP_TRY(hipMemcpyAsync(&flags, h->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    if (J_hist)
        HIP_TRY(hipMemcpyAsync(J_hist, h->jhist, sizeof(double) * (n_iter + 1),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flags & 2) return fail(CSX_EINVAL, "y holds negative or NaN counts");
    if (flags & 1) return fail(CSX_ENUMERIC, "y_i > 0 where the model mean is 0");
    return CSX_OK;
}
