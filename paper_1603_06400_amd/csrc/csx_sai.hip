// csx_sai.hip -- scatter-angle interpolation (Sec. III-B, the precompute and
// interpolate lines of Alg. 2 and Alg. 4).
//
// The spectral part of S(theta, q), s(theta, q) = q Phi(hc q / sin(theta/2)),
// is tabulated at nt uniformly spaced angles theta_t = t theta_max / (nt - 1)
// (float32, [nt][nq] and its transpose).  The geometric angle factor
// (1 + cos^2 theta) cos(theta/2) / sin^2(theta/2) stays exact in the pair
// weight A, as in the exact operators.
//
//   forward   W = f s^T, a dense [nvox x nq] x [nq x nt] product on the matrix
//             cores (v_mfma_f32_16x16x4_f32); then per pair one interpolated
//             read of W(theta_ij, j) replaces the q loop of the exact forward.
//   adjoint   per voxel, V(j, t) = sum_i A_ij T_ij rho_i w_t(theta_ij) (the
//             interpolation weights) collected in a per-wave LDS histogram,
//             then b = V s, a dense [nvox x nt] x [nt x nq] product.
//
// The histograms are 64-bit fixed point, added with LDS integer atomics into
// memory that only the adding wave touches: integer adds are associative, so
// the totals do not depend on the order of the adds and runs repeat bit for
// bit (tested).  Interpolation: nearest node (the paper's choice) or linear;
// the kernels also take a pixel subset's quad / class lists (ordered subsets).
#include "csx_device.h"

#include <cmath>
#include <new>
#include <vector>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

struct SaiState {
    int nt = 0, interp = 1;
    double theta_max = 0.0;
    float inv_dth = 0.0f;          // (nt - 1) / theta_max
    float *S = nullptr;            // [nt][nq] spectral part
    float *St = nullptr;           // [nq][nt]
    float *W = nullptr;            // W = f s^T in the tiled layout of WLayout
    float *V = nullptr;            // [nvox][nt]
    float *bpart = nullptr;        // K-split partials of b = V s [k_splits][nvox][nq]
    double *smid = nullptr;        // [nt - 1] sin(half the midpoint angle) / hc
    double *sc = nullptr;          // [2] fixed-point scale of the adjoint's histograms and its inverse
    double a_max = 0.0;            // largest pair weight A of the geometry
};

void release(SaiState *s)
{
    if (!s) return;
    void *ptrs[] = {s->S, s->St, s->W, s->V, s->bpart, s->smid, s->sc};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete s;
}

// Placement of W = f s^T for the forward: tiled by the forward's 8 x 8 voxel
// tiles, node-major inside a tile, W[set][tile][node][lane] with lane =
// 8 (iz mod 8) + (ix mod 8), so that the 64 lanes of one forward load read
// only the few node rows their tile spans.  With the x -> -x mirror the right
// half (set 1) is stored at mirrored coordinates, so a voxel and its mirror
// share tile and lane.
struct WLayout {
    int tiled = 0;       // 0: row-major C with ldc
    int nx = 0, gw = 0, ntx = 0, ntiles = 0, lr = 0, nt = 0;
};

__device__ __forceinline__ size_t w_index(const WLayout &L, int j, int t)
{
    const int iz = j / L.nx;
    int ix = j - iz * L.nx, set = 0;
    if (L.lr && ix >= L.gw) {
        set = 1;
        ix = L.nx - 1 - ix;
    }
    const int tile = (iz >> 3) * L.ntx + (ix >> 3);
    return ((((size_t)set * L.ntiles + tile) * L.nt + t) << 6) + (((iz & 7) << 3) | (ix & 7));
}

// C[M][N] = sum_k A[m][k] B[n][k]: 64 x 64 tiles, 4 waves of 16 rows, K in
// steps of 32 staged in LDS.  Lane l of v_mfma_f32_16x16x4_f32 holds A[l%16][l/16]
// and B[l/16][l%16] of its 16 x 4 / 4 x 16 operands; D[4 (l/16) + v][l%16].
__global__ void __launch_bounds__(256) k_gemm_nt(const float *__restrict__ A, int lda, const float *__restrict__ B,
                                                 int ldb, float *__restrict__ C, int ldc, int M, int N, int K,
                                                 int kspan, WLayout WL)
{
    __shared__ float sA[64][33];
    __shared__ float sB[64][33];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    // split K: block z takes [kb, ke) and writes its partial product to the
    // z-th [M][ldc] slice of C (row-major only)
    const int kb = blockIdx.z * kspan, ke = min(K, kb + kspan);
    C += (size_t)blockIdx.z * M * ldc;
    f4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += 32) {
        for (int e = tid; e < 64 * 32; e += 256) {
            const int r = e >> 5, c = e & 31;
            const int gk = k0 + c;
            const int gm = m0 + r, gn = n0 + r;
            sA[r][c] = (gm < M && gk < ke) ? A[(size_t)gm * lda + gk] : 0.f;
            sB[r][c] = (gn < N && gk < ke) ? B[(size_t)gn * ldb + gk] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 32; kk += 4) {
            const float a = sA[wave * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float b = sB[t * 16 + (lane & 15)][kk + (lane >> 4)];
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = m0 + wave * 16 + 4 * (lane >> 4) + v;
            const int col = n0 + t * 16 + (lane & 15);
            if (row < M && col < N) C[WL.tiled ? w_index(WL, row, col) : (size_t)row * ldc + col] = acc[t][v];
        }
}

__device__ __forceinline__ void stage_mask(const KParams &P, const DevTables &T, uint32_t *s_bits)
{
    for (int k = threadIdx.x; k < P.mask_ny; k += blockDim.x) s_bits[k] = T.maskbits[k];
}

// The pair's half-angle sine and weight A in float32 only (the interpolated
// operators with linear nodes need no float64 angle: a float32 angle moves an
// interpolated value by far less than the float32 rounding of the sums).
// Same identities as pair_factors: sin^2(theta/2) = |r x r'|^2 / (2 |r||s|
// (|r||s| + r.s)), dtheta = atan(pitch |s_xz| / (|s|^2 - pitch^2/4)).
__device__ __forceinline__ void pair_factors_f(const KParams &P, const VoxD &vd, float2 vf, float xp, float yp,
                                               float &sh, float &A)
{
    const float x = (float)vd.x, z = (float)vd.z, R2 = (float)vd.R2;
    const float sx = xp - x, sz = P.det_z - z;
    const float h2 = fmaf(sx, sx, sz * sz);
    const float s2 = fmaf(yp, yp, h2);
    const float dot = fmaf(x, sx, z * sz);
    const float cy = fmaf(z, xp, -x * P.det_z);
    const float cross2 = fmaf(yp * yp, R2, cy * cy);
    const float Rs2 = R2 * s2, yr = __builtin_amdgcn_rsqf(Rs2);   // 1 / (|r| |s|)
    const float Rs = Rs2 * yr;
    const float den = 2.0f * Rs * (Rs + dot);
    const float yc = __builtin_amdgcn_rsqf(cross2);          // 1 / |r x s|
    const float K2 = den * (yc * yc);                         // 1 / sin^2(theta/2)
    sh = __builtin_amdgcn_rsqf(K2);
    const float inv_s = __builtin_amdgcn_rsqf(s2);
    const float God = vf.y * inv_s * inv_s * inv_s;
    const float cos_t = dot * yr;
    // cos(theta/2) = sin(theta) / (2 sin(theta/2)), sin(theta) = |r x s| / (|r| |s|)
    const float cos_h = 0.5f * (cross2 * yc) * yr * (K2 * sh);
    const float num = P.pitch * __builtin_amdgcn_sqrtf(h2);
    const float dnm = s2 - P.hp2;
    const float tq = num * __builtin_amdgcn_rcpf(dnm);
    float dth;
    if (dnm > 0.0f && tq < 0.05f) {
        const float t2 = tq * tq;
        dth = tq * fmaf(t2, fmaf(t2, 0.2f, -1.0f / 3.0f), 1.0f);
    } else {
        dth = atan2f(num, dnm);
    }
    A = vf.x * God * dth * fmaf(cos_t, cos_t, 1.0f) * cos_h * K2;
}

// Interpolation node(s) of an angle: u = theta (nt - 1) / theta_max, from
// float32 arithmetic (error below 2e-4 spacings).  The nearest-node rule
// settles angles within 2e-3 spacings of a midpoint exactly: theta is past
// midpoint k iff sin(theta/2) >= sin(theta_k+1/2 / 2), i.e. iff
// smid[k] kappa <= 1 with smid[k] = sin(theta_k+1/2 / 2) / hc, in float64.
template <int INTERP>
__device__ __forceinline__ void nodes(float u, double kappa, const double *__restrict__ smid, int nt, int &t0,
                                      float &w0, float &w1)
{
    if (INTERP == 0) {
        t0 = min((int)(u + 0.5f), nt - 1);
        if (fabsf(u - floorf(u) - 0.5f) < 2e-3f) {
            const int k = min((int)u, nt - 2);   // the midpoint between nodes k and k + 1
            t0 = smid[k] * kappa <= 1.0 ? k + 1 : k;
        }
        w0 = 1.0f;
        w1 = 0.0f;
    } else {
        t0 = min((int)u, nt - 2);
        const float fr = fminf(u - (float)t0, 1.0f);
        w0 = 1.0f - fr;
        w1 = fr;
    }
}

// theta = 2 asin(s), s = sin(theta/2) = hc / kappa.  When every active lane
// has s <= 0.35 (theta <= 41 degrees) the odd series of asin through s^15 is
// used: coefficients (2n)! / (4^n (n!)^2 (2n + 1)), truncation below 1e-9
// relative; otherwise the library asinf.
__device__ __forceinline__ float angle_of_sine(float s)
{
    s = fminf(s, 1.0f);
    if (__ballot(s > 0.35f) != 0) return 2.0f * asinf(s);
    const float x = s * s;
    float p = 143.0f / 10240.0f;
    p = fmaf(p, x, 231.0f / 13312.0f);
    p = fmaf(p, x, 63.0f / 2816.0f);
    p = fmaf(p, x, 35.0f / 1152.0f);
    p = fmaf(p, x, 5.0f / 112.0f);
    p = fmaf(p, x, 3.0f / 40.0f);
    p = fmaf(p, x, 1.0f / 6.0f);
    return 2.0f * fmaf(s * x, p, s);
}

__device__ __forceinline__ float angle_of(const KParams &P, double kappa)
{
    return angle_of_sine((float)P.hc * __builtin_amdgcn_rcpf((float)kappa));
}

// One pair of a class: its angle's node coordinate u (for `nodes`), float64
// kappa (the nearest-node rule's midpoint test; 0 with linear nodes) and A.
template <int INTERP>
__device__ __forceinline__ void sai_pair(const KParams &P, const VoxD &vd, float2 vf, float xp, float yp,
                                         float inv_dth, float &u, double &kappa, float &A)
{
    if (INTERP == 0) {
        pair_factors(P, vd, vf, (double)xp, (double)yp, kappa, A);
        u = angle_of(P, kappa) * inv_dth;
    } else {
        float sh;
        pair_factors_f(P, vd, vf, xp, yp, sh, A);
        kappa = 0.0;
        u = angle_of_sine(sh) * inv_dth;
    }
}

// W at the nodes t0 (and t0 + 1) of one lane's column of a tiled W block
template <int INTERP>
__device__ __forceinline__ float interp_w(const float *__restrict__ Wcol, int t0, float w0, float w1)
{
    return INTERP == 0 ? Wcol[t0 << 6] : fmaf(w0, Wcol[t0 << 6], w1 * Wcol[(t0 + 1) << 6]);
}

// Forward pairs: one wave per pixel quad (as the exact forward), lanes = voxel
// groups in 8 x 8 tiles over the block row's tile range; partial images per
// block row.
template <int LR, int INTERP>
__global__ void __launch_bounds__(512) k_forward_sai(KParams P, DevTables T, Lds L, const float *__restrict__ W,
                                                     const double *__restrict__ smid, int nt, float inv_dth,
                                                     float *__restrict__ part,
                                                     int tiles_per_split)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_bits = (uint32_t *)(lds + L.mask);
    stage_mask(P, T, s_bits);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int bx, by, bz;
    xcd_block(bx, by, bz);                     // each XCD reads its splits' tiles of W
    (void)bz;
    const int quad = bx * 8 + wv;
    if (quad >= P.n_quad) return;
    const int qq = P.quad_list ? P.quad_list[quad] : quad;   // a pixel subset's quads, or all
    int a, bu;
    if (LR) {
        const int hx = P.ndx / 2;
        a = hx + qq % hx;
        bu = P.ndy / 2 + qq / hx;
    } else {
        a = qq % P.ndx;
        bu = P.ndy / 2 + qq / P.ndx;
    }
    const double xpad = pixel_coord(P, a, P.ndx);
    const double ypd = pixel_coord(P, bu, P.ndy);
    const float xpa = (float)xpad;
    const float yp = (float)ypd;
    const int gw = LR ? P.nx / 2 : P.nx;
    const int ntx = (gw + 7) / 8;
    const int ntiles = ntx * ((P.nz + 7) / 8);
    const int t0 = by * tiles_per_split;
    const int t1 = min(ntiles, t0 + tiles_per_split);
    float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
    for (int t = t0; t < t1; ++t) {
        const int ix = (t % ntx) * 8 + (lane & 7), iz = (t / ntx) * 8 + (lane >> 3);
        if (ix >= gw || iz >= P.nz) continue;
        const int j = iz * P.nx + ix;
        const VoxD vd = T.vd[j];
        const float2 vf = T.vf[j];
        const double2 vm = T.vm[j];
        const float *Wj = W + (((size_t)t * nt) << 6) + lane;
        const float *Wm = LR ? W + (((size_t)(ntiles + t) * nt) << 6) + lane : Wj;
        {
            const Cells c = mask_cells(P, vm, xpad, ypd);
            float tau = 0.0f, tad = 0.0f, tbu = 0.0f, tbd = 0.0f;
            if (c.in_rows) {
                const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
                tau = bitf(ru, c.col_a);
                tad = bitf(rd, c.col_a);
                if (LR) {
                    tbu = bitf(ru, c.col_b);
                    tbd = bitf(rd, c.col_b);
                }
            }
            if (tau + tad + tbu + tbd != 0.0f) {
                double k;
                float A, u;
                sai_pair<INTERP>(P, vd, vf, xpa, yp, inv_dth, u, k, A);
                int n0;
                float w0, w1;
                nodes<INTERP>(u, k, smid, nt, n0, w0, w1);
                const float wa = interp_w<INTERP>(Wj, n0, w0, w1);
                o0 = fmaf(A * tau, wa, o0);
                o1 = fmaf(A * tad, wa, o1);
                if (LR) {
                    const float wb = interp_w<INTERP>(Wm, n0, w0, w1);
                    o2 = fmaf(A * tbu, wb, o2);
                    o3 = fmaf(A * tbd, wb, o3);
                }
            }
        }
        if (LR) {
            const Cells c = mask_cells(P, vm, -xpad, ypd);
            float tau = 0.0f, tad = 0.0f, tbu = 0.0f, tbd = 0.0f;
            if (c.in_rows) {
                const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
                tau = bitf(ru, c.col_a);
                tad = bitf(rd, c.col_a);
                tbu = bitf(ru, c.col_b);
                tbd = bitf(rd, c.col_b);
            }
            if (tau + tad + tbu + tbd != 0.0f) {
                double k;
                float A, u;
                sai_pair<INTERP>(P, vd, vf, -xpa, yp, inv_dth, u, k, A);
                int n0;
                float w0, w1;
                nodes<INTERP>(u, k, smid, nt, n0, w0, w1);
                const float wa = interp_w<INTERP>(Wj, n0, w0, w1);
                const float wb = interp_w<INTERP>(Wm, n0, w0, w1);
                // pixel (-a) seen from voxel j is pixel (a) seen from the mirror voxel
                o0 = fmaf(A * tbu, wb, o0);
                o1 = fmaf(A * tbd, wb, o1);
                o2 = fmaf(A * tau, wa, o2);
                o3 = fmaf(A * tad, wa, o3);
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        o0 += __shfl_xor(o0, off, 64);
        o1 += __shfl_xor(o1, off, 64);
        if (LR) {
            o2 += __shfl_xor(o2, off, 64);
            o3 += __shfl_xor(o3, off, 64);
        }
    }
    if (lane == 0) {
        float *dst = part + (size_t)by * P.npix;
        const int bd = P.ndy - 1 - bu;
        dst[bu * P.ndx + a] = o0;
        dst[bd * P.ndx + a] = o1;
        if (LR) {
            const int ab = P.ndx - 1 - a;
            dst[bu * P.ndx + ab] = o2;
            dst[bd * P.ndx + ab] = o3;
        }
    }
}

// Adjoint pairs: one wave per voxel group (voxel j, and its mirror with LR),
// lanes = pixel classes in 8 x 8 tiles; the weighted ratios go to the wave's
// two angle histograms in LDS, which are then written to V.  The histograms
// hold 64-bit fixed point: a contribution v enters as floor(v 2^s) with the
// launch's scale 2^s (sc[0]; sc[1] = 2^-s) chosen so that every bin's total
// stays below 2^61 in magnitude.  Integer adds are exact and associative, so
// the totals do not depend on the order of the adds (LDS integer atomics also
// run at full rate, unlike float ones), and the truncation error, below
// 2^-61 of the bound per add, is far under float32 rounding of the result.

template <int LR, int INTERP>
__global__ void __launch_bounds__(256) k_adjoint_sai(KParams P, DevTables T, Lds L, const float *__restrict__ rho,
                                                     float *__restrict__ V, const double *__restrict__ smid, int nt,
                                                     float inv_dth, const double *__restrict__ sc)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *s_bits = (uint32_t *)(lds + L.mask);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned long long *h0 = (unsigned long long *)(lds + L.tile) + (size_t)wv * 2 * nt;
    unsigned long long *h1 = h0 + nt;
    stage_mask(P, T, s_bits);
    for (int k = lane; k < 2 * nt; k += 64) h0[k] = 0ull;
    __syncthreads();
    const int g = blockIdx.x * (blockDim.x >> 6) + wv;
    if (g >= P.n_groups) return;
    int j, j2;
    if (LR) {
        const int half = P.nx / 2;
        const int iz = g / half, ix = g % half;
        j = iz * P.nx + ix;
        j2 = iz * P.nx + (P.nx - 1 - ix);
    } else {
        j = g;
        j2 = g;
    }
    const double scale = sc[0], inv_scale = sc[1];
    const int sexp = scale_exponent(scale);
    const VoxD vd = T.vd[j];
    const float2 vf = T.vf[j];
    const double2 vm = T.vm[j];
    const int half_y = P.ndy / 2;
    const int ntx = (P.ndx + 7) / 8;
    // pixel classes (column a, upper row r): 8 x 8 tiles of the detector, or
    // 64 consecutive entries of a pixel subset's class list
    const int ntiles = P.cls_list ? (P.n_cls + 63) / 64 : ntx * ((half_y + 7) / 8);
    for (int t = 0; t < ntiles; ++t) {
        int a, r;
        if (P.cls_list) {
            const int e = t * 64 + lane;
            if (e >= P.n_cls) continue;
            const int c = P.cls_list[e];
            a = c % P.ndx;
            r = c / P.ndx;
        } else {
            a = (t % ntx) * 8 + (lane & 7);
            r = (t / ntx) * 8 + (lane >> 3);
            if (a >= P.ndx || r >= half_y) continue;
        }
        const int bu = half_y + r, bd = P.ndy - 1 - bu;
        const double xpd = pixel_coord(P, a, P.ndx);
        const double ypd = pixel_coord(P, bu, P.ndy);
        const float xp = (float)xpd;
        const float yp = (float)ypd;
        const Cells c = mask_cells(P, vm, xpd, ypd);
        if (!c.in_rows) continue;
        const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
        const float w0 = bitf(ru, c.col_a) * rho[bu * P.ndx + a] + bitf(rd, c.col_a) * rho[bd * P.ndx + a];
        float w1 = 0.0f;
        if (LR) {
            const int ab = P.ndx - 1 - a;
            w1 = bitf(ru, c.col_b) * rho[bu * P.ndx + ab] + bitf(rd, c.col_b) * rho[bd * P.ndx + ab];
        }
        if (w0 == 0.0f && w1 == 0.0f) continue;
        double k;
        float A, u;
        sai_pair<INTERP>(P, vd, vf, xp, yp, inv_dth, u, k, A);
        int n0;
        float u0, u1;
        nodes<INTERP>(u, k, smid, nt, n0, u0, u1);
        const float c0 = A * w0, c1 = A * w1;
        atomicAdd(&h0[n0], fixed_of(c0 * u0, sexp));
        if (INTERP) atomicAdd(&h0[n0 + 1], fixed_of(c0 * u1, sexp));
        if (LR) {
            atomicAdd(&h1[n0], fixed_of(c1 * u0, sexp));
            if (INTERP) atomicAdd(&h1[n0 + 1], fixed_of(c1 * u1, sexp));
        }
    }
    // scale 0 flags a non-finite bound (rho holds inf or NaN): NaN out
    const float bad = __builtin_nanf("");
    float *vj = V + (size_t)j * nt;
    for (int k = lane; k < nt; k += 64)
        vj[k] = scale != 0.0 ? (float)((double)(long long)h0[k] * inv_scale) : bad;
    if (LR) {
        float *v2 = V + (size_t)j2 * nt;
        for (int k = lane; k < nt; k += 64)
            v2[k] = scale != 0.0 ? (float)((double)(long long)h1[k] * inv_scale) : bad;
    }
}

// out = sum over z of part[z][i], in increasing z
__global__ void __launch_bounds__(256) k_sum_slices(const float *__restrict__ part, int nz, int n,
                                                    float *__restrict__ out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float v = part[i];
    for (int z = 1; z < nz; ++z) v += part[(size_t)z * n + i];
    out[i] = v;
}

// Scale of the adjoint's fixed-point histograms: with B = a_max sum_i |rho_i|
// (a_max: the largest pair weight A of the geometry) every contribution and
// every bin total is at most B in magnitude (a pixel's weights over nodes sum
// to 1); 2^s with 2^(s-61) B < 1.  One block, fixed summation order.
__global__ void __launch_bounds__(1024) k_sai_scale(const float *__restrict__ rho, int n, double a_max,
                                                    double *__restrict__ sc)
{
    __shared__ double part[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += fabs((double)rho[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < 16; ++w) tot += part[w];
        const double B = a_max * tot;
        double s0 = 1.0, s1 = 1.0;
        if (!(B < INFINITY)) {
            s0 = 0.0;                        // inf or NaN
        } else if (B > 0.0) {
            int e;
            (void)frexp(B, &e);              // B < 2^e
            s0 = ldexp(1.0, 61 - e);
            s1 = ldexp(1.0, e - 61);
        }
        sc[0] = s0;
        sc[1] = s1;
    }
}

// Largest pair weight A over all voxel-pixel pairs (the mask ignored): one
// wave per voxel group, max over its pixel classes (the mirrors share them).
template <int LR>
__global__ void __launch_bounds__(256) k_sai_amax(KParams P, DevTables T, float *__restrict__ amax)
{
    const int lane = threadIdx.x & 63;
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= P.n_groups) return;
    const int j = LR ? (g / (P.nx / 2)) * P.nx + g % (P.nx / 2) : g;
    const VoxD vd = T.vd[j];
    const float2 vf = T.vf[j];
    const int half_y = P.ndy / 2;
    float m = 0.0f;
    for (int c = lane; c < P.ndx * half_y; c += 64) {
        const int a = c % P.ndx, bu = half_y + c / P.ndx;
        const double xp = (double)((float)(2 * a - P.ndx + 1) * (0.5f * P.pitch));
        const double yp = (double)((float)(2 * bu - P.ndy + 1) * (0.5f * P.pitch));
        double k;
        float A;
        pair_factors(P, vd, vf, xp, yp, k, A);
        m = fmaxf(m, A);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if (lane == 0) amax[g] = m;
}

int al16(int v) { return (v + 15) & ~15; }

Lds sai_lds(const KParams &P, int hist_bytes)
{
    Lds L;
    int off = 0;
    L.phi = 0;
    L.mask = off;
    off += al16(P.mask_ny * 4);
    L.tile = off;
    off += hist_bytes;
    L.total = off;
    return L;
}

// The K-split count of a product: enough blocks to fill the chip when M x N
// alone gives few (K chunks of 32 otherwise run one after another in a block).
int k_splits(int M, int N, int K)
{
    const int blocks = ((M + 63) / 64) * ((N + 63) / 64);
    int z = 1;
    while (z < 8 && blocks * z < 1024 && K / (2 * z) >= 32) z *= 2;
    return z;
}

// C = A B^T; with ksplit > 1, C receives ksplit partial products (row-major,
// ldc = N) and the caller sums them.
csx_status gemm_nt(const float *A, int lda, const float *B, int ldb, float *C, int ldc, int M, int N, int K,
                   hipStream_t s, WLayout WL = WLayout{}, int ksplit = 1)
{
    const int kspan = ((K + ksplit - 1) / ksplit + 31) / 32 * 32;
    dim3 grid((M + 63) / 64, (N + 63) / 64, (K + kspan - 1) / kspan);
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, kspan, WL);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

// Largest scatter angle over the voxels and the detector's edge pixels (the
// angle seen from a voxel has no interior maximum on the detector plane).
double max_angle(const csx_geometry *h)
{
    const csx_geometry_desc &d = h->d;
    const double dx = (d.x_max - d.x_min) / d.nx, dz = (d.z_max - d.z_min) / d.nz;
    double best = 0.0;
    for (int iz = 0; iz < d.nz; ++iz)
        for (int ix = 0; ix < d.nx; ++ix) {
            const double x = d.x_min + (ix + 0.5) * dx, z = d.z_min + (iz + 0.5) * dz;
            for (int b = 0; b < d.ndy; ++b)
                for (int a = 0; a < d.ndx; ++a) {
                    if (b != 0 && b != d.ndy - 1 && a != 0 && a != d.ndx - 1) continue;
                    const double xp = (a - d.ndx / 2.0 + 0.5) * d.det_pitch;
                    const double yp = (b - d.ndy / 2.0 + 0.5) * d.det_pitch;
                    const double sx = xp - x, sy = yp, sz = d.det_z - z;
                    const double cx = -z * sy, cy = z * sx - x * sz, cz = x * sy;
                    const double cr = std::sqrt(cx * cx + cy * cy + cz * cz), dt = x * sx + z * sz;
                    best = std::max(best, std::atan2(cr, dt));
                }
        }
    return best;
}

WLayout w_layout(const KParams &P, int nt)
{
    WLayout L;
    L.tiled = 1;
    L.nx = P.nx;
    L.lr = P.lr;
    L.gw = P.lr ? P.nx / 2 : P.nx;
    L.ntx = (L.gw + 7) / 8;
    L.ntiles = L.ntx * ((P.nz + 7) / 8);
    L.nt = nt;
    return L;
}

SaiState *state(const csx_geometry *h) { return static_cast<SaiState *>(h->sai); }

}  // namespace

// max over all voxel-pixel pairs of the pair weight A (mask ignored), computed
// once per handle
csx_status csx_pair_weight_max(csx_geometry *h, double *out)
{
    if (h->a_max <= 0.0) {
        const KParams &P = h->P;
        float *am = nullptr;
        HIP_TRY(hipMalloc((void **)&am, sizeof(float) * P.n_groups));
        if (P.lr)
            hipLaunchKernelGGL(k_sai_amax<1>, dim3((P.n_groups + 3) / 4), dim3(256), 0, nullptr, P, h->t, am);
        else
            hipLaunchKernelGGL(k_sai_amax<0>, dim3((P.n_groups + 3) / 4), dim3(256), 0, nullptr, P, h->t, am);
        hipError_t e = hipGetLastError();
        std::vector<float> hm(P.n_groups);
        if (e == hipSuccess) e = hipMemcpy(hm.data(), am, sizeof(float) * P.n_groups, hipMemcpyDeviceToHost);
        (void)hipFree(am);
        if (e != hipSuccess) return csx_fail(CSX_EHIP, std::string("pair weight maximum: ") + hipGetErrorString(e));
        double m = 0.0;
        for (float v : hm) m = std::max(m, (double)v);
        h->a_max = m;
    }
    *out = h->a_max;
    return CSX_OK;
}

void csx_sai_free(csx_geometry *h)
{
    release(state(h));
    h->sai = nullptr;
}

extern "C" csx_status csx_sai_config(csx_geometry *h, int nt, int interp, double theta_max)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    if (nt < 2 || nt > CSX_SAI_MAX_NODES) return csx_fail(CSX_EINVAL, "nt must be in [2, CSX_SAI_MAX_NODES]");
    if (interp != 0 && interp != 1) return csx_fail(CSX_EINVAL, "interp must be 0 (nearest) or 1 (linear)");
    if (!(std::isfinite(theta_max) && theta_max >= 0.0) || theta_max > M_PI)
        return csx_fail(CSX_EINVAL, "theta_max must be in [0, pi] (0: the largest pair angle)");
    const csx_geometry_desc &d = h->d;
    const int nq = h->P.nq, nvox = h->P.nvox;
    double tm = theta_max > 0.0 ? theta_max : max_angle(h) * (1.0 + 1e-7);
    // spectral part of S at the table's angles, float64 then float32
    std::vector<float> S((size_t)nt * nq), St((size_t)nq * nt);
    const double de = (d.e_hi - d.e_lo) / d.ne;
    const std::vector<double> &phi = h->phi_host;
    for (int t = 0; t < nt; ++t) {
        const double sh = std::sin(0.5 * t * tm / (nt - 1));
        for (int m = 0; m < nq; ++m) {
            double v = 0.0;
            if (sh > 0.0) {
                const double q = h->q_host[m];
                const double kb = std::floor((d.hc * q / sh - d.e_lo) / de);
                if (kb >= 0.0 && kb < d.ne) v = q * phi[(int)kb];
            }
            S[(size_t)t * nq + m] = (float)v;
            St[(size_t)m * nt + t] = (float)v;
        }
    }
    std::vector<double> smid(nt - 1);
    for (int k = 0; k < nt - 1; ++k) smid[k] = std::sin(0.5 * (k + 0.5) * tm / (nt - 1)) / d.hc;
    SaiState *s = new (std::nothrow) SaiState();
    if (!s) return csx_fail(CSX_ENOMEM, "host allocation failed");
    s->nt = nt;
    s->interp = interp;
    s->theta_max = tm;
    s->inv_dth = (float)((nt - 1) / tm);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void **)&s->S, sizeof(float) * S.size());
    if (e == hipSuccess) e = hipMalloc((void **)&s->St, sizeof(float) * St.size());
    const WLayout WL = w_layout(h->P, nt);
    if (e == hipSuccess) e = hipMalloc((void **)&s->W, sizeof(float) * ((size_t)(WL.lr ? 2 : 1) * WL.ntiles * nt << 6));
    if (e == hipSuccess) e = hipMalloc((void **)&s->V, sizeof(float) * (size_t)nvox * nt);
    if (e == hipSuccess) e = hipMalloc((void **)&s->sc, sizeof(double) * 2);
    if (e == hipSuccess)
        e = hipMalloc((void **)&s->bpart, sizeof(float) * (size_t)k_splits(nvox, nq, nt) * nvox * nq);
    if (e == hipSuccess) e = hipMalloc((void **)&s->smid, sizeof(double) * smid.size());
    if (e == hipSuccess) e = hipMemcpy(s->smid, smid.data(), sizeof(double) * smid.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->S, S.data(), sizeof(float) * S.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->St, St.data(), sizeof(float) * St.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) {   // the largest pair weight, for the adjoint's fixed-point scale
        const csx_status st = csx_pair_weight_max(h, &s->a_max);
        if (st != CSX_OK) {
            release(s);
            return st;
        }
    }
    if (e != hipSuccess) {
        release(s);
        return csx_fail(CSX_EHIP, std::string("scatter-angle tables: ") + hipGetErrorString(e));
    }
    (void)hipDeviceSynchronize();
    csx_sai_free(h);
    h->sai = s;
    if (h->op_sai & CSX_OP_ADJOINT_SAI) h->have_b1 = false;   // new table, new sensitivity
    return CSX_OK;
}

extern "C" csx_status csx_sai_info(const csx_geometry *h, int *nt, int *interp, double *theta_max)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    const SaiState *s = state(h);
    if (!s) return csx_fail(CSX_EINVAL, "scatter-angle interpolation not configured");
    if (nt) *nt = s->nt;
    if (interp) *interp = s->interp;
    if (theta_max) *theta_max = s->theta_max;
    return CSX_OK;
}

namespace {

// W = f s^T, then the pairs of the quads of P (all, or a subset's list) into
// h->part; returns the number of partial images
csx_status forward_sai_parts(csx_geometry *h, const KParams &P, const float *f, int splits_req, int *nparts,
                             hipStream_t st)
{
    SaiState *s = state(h);
    if (!s) return csx_fail(CSX_EINVAL, "scatter-angle interpolation not configured");
    csx_status r = gemm_nt(f, P.nq, s->S, P.nq, s->W, s->nt, P.nvox, s->nt, P.nq, st, w_layout(P, s->nt));
    if (r != CSX_OK) return r;
    const int gw = P.lr ? P.nx / 2 : P.nx;
    const int ntiles = ((gw + 7) / 8) * ((P.nz + 7) / 8);
    const int splits = std::max(1, std::min(splits_req, ntiles));
    const int tps = (ntiles + splits - 1) / splits;
    const int nsplit = (ntiles + tps - 1) / tps;
    if ((size_t)nsplit * P.npix > h->part_cap) return csx_fail(CSX_EINVAL, "forward partials too small");
    const Lds L = sai_lds(P, 0);
    dim3 grid((P.n_quad + 7) / 8, nsplit);
    if (P.lr) {
        if (s->interp)
            hipLaunchKernelGGL((k_forward_sai<1, 1>), grid, dim3(512), L.total, st, P, h->t, L, s->W, s->smid, s->nt,
                               s->inv_dth, h->part, tps);
        else
            hipLaunchKernelGGL((k_forward_sai<1, 0>), grid, dim3(512), L.total, st, P, h->t, L, s->W, s->smid, s->nt,
                               s->inv_dth, h->part, tps);
    } else {
        if (s->interp)
            hipLaunchKernelGGL((k_forward_sai<0, 1>), grid, dim3(512), L.total, st, P, h->t, L, s->W, s->smid, s->nt,
                               s->inv_dth, h->part, tps);
        else
            hipLaunchKernelGGL((k_forward_sai<0, 0>), grid, dim3(512), L.total, st, P, h->t, L, s->W, s->smid, s->nt,
                               s->inv_dth, h->part, tps);
    }
    HIP_TRY(hipGetLastError());
    *nparts = nsplit;
    return CSX_OK;
}

csx_status adjoint_sai_impl(csx_geometry *h, const KParams &P, const float *rho, float *b, hipStream_t st)
{
    SaiState *s = state(h);
    if (!s) return csx_fail(CSX_EINVAL, "scatter-angle interpolation not configured");
    // per-wave histograms of 2 nt 64-bit words, at most 32 KiB per block
    const int wpb = std::max(1, std::min(4, 2048 / s->nt));
    const Lds L = sai_lds(P, wpb * 2 * s->nt * 8);
    dim3 grid((P.n_groups + wpb - 1) / wpb);
    hipLaunchKernelGGL(k_sai_scale, dim3(1), dim3(1024), 0, st, rho, P.npix, s->a_max, s->sc);
    if (P.lr) {
        if (s->interp)
            hipLaunchKernelGGL((k_adjoint_sai<1, 1>), grid, dim3(64 * wpb), L.total, st, P, h->t, L, rho, s->V, s->smid, s->nt,
                               s->inv_dth, s->sc);
        else
            hipLaunchKernelGGL((k_adjoint_sai<1, 0>), grid, dim3(64 * wpb), L.total, st, P, h->t, L, rho, s->V, s->smid, s->nt,
                               s->inv_dth, s->sc);
    } else {
        if (s->interp)
            hipLaunchKernelGGL((k_adjoint_sai<0, 1>), grid, dim3(64 * wpb), L.total, st, P, h->t, L, rho, s->V, s->smid, s->nt,
                               s->inv_dth, s->sc);
        else
            hipLaunchKernelGGL((k_adjoint_sai<0, 0>), grid, dim3(64 * wpb), L.total, st, P, h->t, L, rho, s->V, s->smid, s->nt,
                               s->inv_dth, s->sc);
    }
    HIP_TRY(hipGetLastError());
    const int z = k_splits(P.nvox, P.nq, s->nt);
    if (z == 1) return gemm_nt(s->V, s->nt, s->St, s->nt, b, P.nq, P.nvox, P.nq, s->nt, st);
    const int kspan = ((s->nt + z - 1) / z + 31) / 32 * 32;
    const int nz = (s->nt + kspan - 1) / kspan;       // partial products written
    csx_status r = gemm_nt(s->V, s->nt, s->St, s->nt, s->bpart, P.nq, P.nvox, P.nq, s->nt, st, WLayout{}, z);
    if (r != CSX_OK) return r;
    const int n = P.nvox * P.nq;
    hipLaunchKernelGGL(k_sum_slices, dim3((n + 255) / 256), dim3(256), 0, st, s->bpart, nz, n, b);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

}  // namespace

csx_status csx_launch_forward_sai(csx_geometry *h, const float *f, float *g, hipStream_t st)
{
    int nparts = 0;
    csx_status r = forward_sai_parts(h, h->P, f, h->lc.fwd_splits, &nparts, st);
    if (r != CSX_OK) return r;
    return csx_launch_sum_parts(h, nparts, g, st);
}

csx_status csx_launch_adjoint_sai(csx_geometry *h, const float *rho, float *b, hipStream_t st)
{
    return adjoint_sai_impl(h, h->P, rho, b, st);
}

csx_status csx_launch_forward_sai_list(csx_geometry *h, const float *f, const int *quads, int n_quads, int splits,
                                       const int *pix, int n_pix, const float *y, const float *r, float *rho,
                                       hipStream_t st)
{
    KParams P = h->P;
    P.quad_list = quads;
    P.n_quad = n_quads;
    int nparts = 0;
    csx_status e = forward_sai_parts(h, P, f, splits, &nparts, st);
    if (e != CSX_OK) return e;
    return csx_launch_sum_ratio_list(h, nparts, pix, n_pix, y, r, rho, st);
}

csx_status csx_launch_adjoint_sai_list(csx_geometry *h, const float *rho, const int *cls, int n_cls, float *b,
                                       hipStream_t st)
{
    KParams P = h->P;
    P.cls_list = cls;
    P.n_cls = n_cls;
    return adjoint_sai_impl(h, P, rho, b, st);
}

extern "C" csx_status csx_forward_sai(csx_geometry *h, const float *f, float *g, void *stream)
{
    if (!h || !f || !g) return csx_fail(CSX_EINVAL, "NULL argument");
    return csx_launch_forward_sai(h, f, g, (hipStream_t)stream);
}

extern "C" csx_status csx_backproject_sai(csx_geometry *h, const float *y, float *b, void *stream)
{
    if (!h || !y || !b) return csx_fail(CSX_EINVAL, "NULL argument");
    return csx_launch_adjoint_sai(h, y, b, (hipStream_t)stream);
}

extern "C" csx_status csx_set_operator(csx_geometry *h, int ops)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    if (ops & ~(CSX_OP_FORWARD_SAI | CSX_OP_ADJOINT_SAI)) return csx_fail(CSX_EINVAL, "unknown operator bits");
    if (ops && !state(h)) return csx_fail(CSX_EINVAL, "scatter-angle interpolation not configured");
    if ((ops ^ h->op_sai) & CSX_OP_ADJOINT_SAI) h->have_b1 = false;   // the sensitivity A^T 1 changes
    h->op_sai = ops;
    return CSX_OK;
}
