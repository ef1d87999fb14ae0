// csx_ops.hip -- forward and adjoint operators of the fan-beam coded-aperture
// coherent-scatter model on gfx950 (Odinaka et al., arXiv:1603.06400).
//
//   g_i  = sum_j A_ij T_ij sum_m q_m Phi(kappa_ij q_m) f_jm          (forward, Alg. 1)
//   b_jm = q_m sum_i A_ij T_ij Phi(kappa_ij q_m) y_i                 (adjoint, Alg. 3)
//   kappa = hc / sin(theta/2)   (E = kappa q, Bragg's law, App. A)
//   A = C Gso God dtheta (1 + cos^2 theta) cos(theta/2) / sin^2(theta/2)
//
// Work decomposition (wave64):
//  * lanes = q.  The per-q inner step (the paper's W(r, theta) = sum_q S f) is
//    one FP64 FMA for the Bragg bin coordinate, an integer clamp, one gather
//    from the spectrum table in LDS and one or two FP32 FMAs per lane.
//  * a "class" is a set of pairs that share every factor except the mask
//    transmission T: the pixel rows y' and -y' (up-down mirror, Sec. III-A)
//    and, when the voxel grid and the detector are centred with even sizes,
//    the voxel / pixel columns x and -x (left-right mirror).  One class is
//    4 pairs (2 without the left-right mirror); its four mask cells come from a
//    single crossing point, mirrored with integer arithmetic.
//  * classes are evaluated one per lane, 64 at a time; the wave compacts the
//    classes with an open cell and an in-band Bragg energy into an LDS list
//    (ballot + mbcnt) and then walks the list with 16-byte broadcast reads,
//    64/qw classes per wave instruction when nq <= 32.
//  * the spectral bin of a triple is decided in float64 (kappa in float64
//    from float32 seeds refined by one Newton step each; the bin coordinate
//    q/dE * kappa + 1 - e_lo/dE by one FP64 FMA): the same precision as the
//    float64 definition, so bin decisions agree except at float64 ties.
//  * forward: output-stationary per group of mirror pixels, voxels staged in
//    LDS per block, voxel range split across blocks with a fixed-order sum of
//    the partial images (no atomics, bitwise reproducible).
//  * adjoint: output-stationary per (voxel, mirror voxel) pair, no atomics.
#include "csx_internal.h"

namespace {

constexpr int UNROLL = 4;
constexpr int LIST_CAP = 80;   // 64 classes + padding to a multiple of slots * UNROLL

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

template <int TD>
__device__ __forceinline__ float spec(const float *s_phi, const uint16_t *s_phi16, int k)
{
    if (TD == CSX_TABLE_BF16) return bf16_to_f32(s_phi16[k]);
    return s_phi[k];
}

__device__ __forceinline__ double as_double(float lo, float hi)
{
    const uint64_t u = ((uint64_t)__float_as_uint(hi) << 32) | (uint64_t)__float_as_uint(lo);
    return __longlong_as_double((long long)u);
}

__device__ __forceinline__ float dlo(double v)
{
    return __uint_as_float((uint32_t)((uint64_t)__double_as_longlong(v)));
}

__device__ __forceinline__ float dhi(double v)
{
    return __uint_as_float((uint32_t)((uint64_t)__double_as_longlong(v) >> 32));
}

__device__ __forceinline__ int posmod(int v, int p)
{
    int r = v % p;
    return r + (r < 0 ? p : 0);
}

// Pair factors of voxel (vd, vf) and pixel (xp, yp, det_z).
//   theta: sin^2(theta/2) = |r x r'|^2 / (2 |r||s| (|r||s| + r.s))  (no cancellation)
//   kappa = hc / sin(theta/2) in float64; A in float32.
//   dtheta = angle between s - (pitch/2) y^ and s + (pitch/2) y^
//          = atan(pitch |s_xz| / (|s|^2 - pitch^2/4)).
__device__ __forceinline__ void pair_factors(const KParams &P, const VoxD &vd, float2 vf,
                                             double xp, double yp, double &kappa, float &A)
{
    const double x = vd.x, z = vd.z, R2 = vd.R2;
    const double sx = xp - x, sz = P.det_zd - z;
    const double h2 = sx * sx + sz * sz;
    const double s2 = h2 + yp * yp;
    const double dot = x * sx + z * sz;
    const double cy = z * xp - x * P.det_zd;
    const double cross2 = yp * yp * R2 + cy * cy;
    const double Rs2 = R2 * s2;
    const float rs0 = __builtin_amdgcn_sqrtf((float)Rs2);
    const double Rs = (double)rs0 + (Rs2 - (double)rs0 * (double)rs0) * (double)(0.5f * __builtin_amdgcn_rcpf(rs0));
    const double den = 2.0 * Rs * (Rs + dot);
    const float r0 = __builtin_amdgcn_rcpf((float)cross2);
    const double inv = (double)r0 * (2.0 - cross2 * (double)r0);
    const double K2 = den * inv;   // 1 / sin^2(theta/2)
    const float k0 = __builtin_amdgcn_sqrtf((float)K2);
    const double k = (double)k0 + (K2 - (double)k0 * (double)k0) * (double)(0.5f * __builtin_amdgcn_rcpf(k0));
    kappa = P.hc * k;

    const float s2f = (float)s2;
    const float inv_s = __builtin_amdgcn_rsqf(s2f);
    const float God = vf.y * inv_s * inv_s * inv_s;
    const float cos_t = (float)dot * __builtin_amdgcn_rcpf((float)Rs);
    const float cos_h = __builtin_amdgcn_sqrtf(0.5f * (1.0f + cos_t));
    const float num = P.pitch * __builtin_amdgcn_sqrtf((float)h2);
    const float dnm = s2f - P.hp2;
    const float tq = num * __builtin_amdgcn_rcpf(dnm);
    float dth;
    if (dnm > 0.0f && tq < 0.05f) {
        // atan(t) = t - t^3/3 + t^5/5 - ...; the dropped terms are < 3e-9 relative
        const float t2 = tq * tq;
        dth = tq * fmaf(t2, fmaf(t2, 0.2f, -1.0f / 3.0f), 1.0f);
    } else {
        dth = atan2f(num, dnm);
    }
    A = vf.x * God * dth * fmaf(cos_t, cos_t, 1.0f) * cos_h * (float)K2;
}

__device__ __forceinline__ bool in_band(const KParams &P, double kappa)
{
    return kappa * P.q_max >= P.band_lo && kappa * P.q_min < P.band_hi;
}

// Spectrum-table index of one triple: 1 + bin, 0 below the band, ne + 1 above.
__device__ __forceinline__ int spec_index(const KParams &P, double kappa, double qa, double qb)
{
    const double u = fma(kappa, qa, qb);
    const int k = (int)u;
    return min(max(k, 0), P.ne + 1);
}

template <int TD>
__device__ __forceinline__ void stage_tables(const KParams &P, const DevTables &T, float *s_phi,
                                             uint16_t *s_phi16, uint32_t *s_bits)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    if (TD == CSX_TABLE_BF16) {
        for (int k = tid; k < P.ne + 2; k += nt) s_phi16[k] = T.phi16[k];
    } else {
        for (int k = tid; k < P.ne + 2; k += nt) s_phi[k] = T.phi32[k];
    }
    for (int k = tid; k < P.mask_ny; k += nt) s_bits[k] = T.maskbits[k];
}

struct Lds {
    int phi, mask, list, tile, total;
};

// Mask cells of one crossing: columns of the pixel (col_a) and of its x-mirror
// seen from the mirror voxel (col_b), rows of y' (row_u) and -y' (row_d).
struct Cells {
    int col_a, col_b, row_u, row_d;
    bool in_rows;
};

__device__ __forceinline__ Cells mask_cells(const KParams &P, float2 vm, float xp, float yp)
{
    Cells c;
    const int cx = (int)floorf(fmaf(vm.x, xp, vm.y));
    const int cy = (int)floorf(fmaf(vm.x, yp, P.half_my));
    c.col_a = posmod(cx, P.mask_nx);
    c.col_b = posmod(-cx - 1, P.mask_nx);   // floor(-px) = -floor(px) - 1 off the cell edges
    c.row_u = cy;
    c.row_d = P.mask_ny - 1 - cy;           // floor(My - v) = My - 1 - floor(v)
    c.in_rows = cy >= 0 && cy < P.mask_ny;
    return c;
}

__device__ __forceinline__ float bitf(uint32_t row, int col)
{
    return (float)((row >> col) & 1u);
}

// ---------------------------------------------------------------------------
// adjoint: one wave per voxel group (voxel j, and its mirror j2 with LR) and q
// chunk; walks all pixel classes (a, b_up), b_up in the upper half.
// ---------------------------------------------------------------------------
template <int TD, int LR, int SLOTS>
__global__ void __launch_bounds__(256) k_adjoint(KParams P, DevTables T, Lds L,
                                                 const float *__restrict__ rho,
                                                 float *__restrict__ b)
{
    constexpr int QW = 64 / SLOTS;
    constexpr int STEP = SLOTS * UNROLL;
    extern __shared__ __align__(16) unsigned char lds[];
    float *s_phi = (float *)(lds + L.phi);
    uint16_t *s_phi16 = (uint16_t *)(lds + L.phi);
    uint32_t *s_bits = (uint32_t *)(lds + L.mask);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4 *s_list = (float4 *)(lds + L.list) + wv * LIST_CAP;

    stage_tables<TD>(P, T, s_phi, s_phi16, s_bits);
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
    const VoxD vd = T.vd[j];
    const float2 vf = T.vf[j];
    const float2 vm = T.vm[j];
    const int slot = lane / QW, ml = lane % QW;
    const int mq = blockIdx.y * QW + ml;
    const double qa = T.qa[mq], qb = T.qb[mq];

    float acc0 = 0.0f, acc1 = 0.0f;
    for (int pb = 0; pb < P.n_cls; pb += 64) {
        const int p = pb + lane;
        double kap = 0.0;
        float c0 = 0.0f, c1 = 0.0f;
        bool act = false;
        if (p < P.n_cls) {
            const int a = p % P.ndx;
            const int bu = P.ndy / 2 + p / P.ndx;
            const int bd = P.ndy - 1 - bu;
            const float xp = (float)(2 * a - P.ndx + 1) * (0.5f * P.pitch);
            const float yp = (float)(2 * bu - P.ndy + 1) * (0.5f * P.pitch);
            const Cells c = mask_cells(P, vm, xp, yp);
            float w0 = 0.0f, w1 = 0.0f;
            if (c.in_rows) {
                const uint32_t ru = s_bits[c.row_u], rd = s_bits[c.row_d];
                w0 = bitf(ru, c.col_a) * rho[bu * P.ndx + a] + bitf(rd, c.col_a) * rho[bd * P.ndx + a];
                if (LR) {
                    const int ab = P.ndx - 1 - a;
                    w1 = bitf(ru, c.col_b) * rho[bu * P.ndx + ab] +
                         bitf(rd, c.col_b) * rho[bd * P.ndx + ab];
                }
            }
            if (w0 != 0.0f || w1 != 0.0f) {
                float A;
                pair_factors(P, vd, vf, (double)xp, (double)yp, kap, A);
                if (in_band(P, kap)) {
                    c0 = A * w0;
                    c1 = A * w1;
                    act = c0 != 0.0f || c1 != 0.0f;
                }
            }
        }
        const uint64_t bal = __ballot(act);
        const int nact = __popcll(bal);
        const int idx = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (act) s_list[idx] = make_float4(dlo(kap), dhi(kap), c0, c1);
        const int npad = (nact + STEP - 1) / STEP * STEP;
        if (lane < npad - nact) s_list[nact + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        __builtin_amdgcn_wave_barrier();
        for (int i = 0; i < npad; i += STEP) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const float4 e = s_list[i + u * SLOTS + slot];
                const int k = spec_index(P, as_double(e.x, e.y), qa, qb);
                const float ph = spec<TD>(s_phi, s_phi16, k);
                acc0 = fmaf(e.z, ph, acc0);
                if (LR) acc1 = fmaf(e.w, ph, acc1);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (SLOTS >= 2) {
        acc0 += __shfl_xor(acc0, 32, 64);
        acc1 += __shfl_xor(acc1, 32, 64);
    }
    if (SLOTS >= 4) {
        acc0 += __shfl_xor(acc0, 16, 64);
        acc1 += __shfl_xor(acc1, 16, 64);
    }
    const int m = blockIdx.y * QW + ml;
    if (slot == 0 && m < P.nq) {
        const float qm = T.qv[mq];
        b[(size_t)j * P.nq + m] = acc0 * qm;
        if (LR) b[(size_t)j2 * P.nq + m] = acc1 * qm;
    }
}

// ---------------------------------------------------------------------------
// forward: one wave per output group (the four mirror pixels (+-x', +-y') with
// LR, else the two pixels (x', +-y')) and q chunk; the block's waves share a
// 64-voxel tile of f in LDS; blockIdx.y splits the voxel groups.
// List entry (32 B): {kappa lo, kappa hi, k0, k1}, {k2, k3, row0 offset, row1 offset}:
// outputs O0, O1 take k0, k1 times Phi f[row0]; O2, O3 take k2, k3 times Phi f[row1].
// ---------------------------------------------------------------------------
template <int TD, int LR, int SLOTS>
__global__ void __launch_bounds__(512) k_forward(KParams P, DevTables T, Lds L,
                                                 const float *__restrict__ f,
                                                 float *__restrict__ part, int groups_per_split)
{
    constexpr int QW = 64 / SLOTS;
    constexpr int STEP = SLOTS * UNROLL;
    constexpr int GB = LR ? 32 : 64;       // voxel groups per batch (64 voxels, 64 classes)
    extern __shared__ __align__(16) unsigned char lds[];
    float *s_phi = (float *)(lds + L.phi);
    uint16_t *s_phi16 = (uint16_t *)(lds + L.phi);
    uint32_t *s_bits = (uint32_t *)(lds + L.mask);
    float *s_tile = (float *)(lds + L.tile);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float4 *s_list = (float4 *)(lds + L.list) + wv * (2 * LIST_CAP);

    stage_tables<TD>(P, T, s_phi, s_phi16, s_bits);

    const int quad = blockIdx.x * (blockDim.x >> 6) + wv;
    const bool wave_on = quad < P.n_quad;
    const int qq = wave_on ? quad : 0;
    int a, bu;
    if (LR) {
        const int hx = P.ndx / 2;
        a = hx + qq % hx;
        bu = P.ndy / 2 + qq / hx;
    } else {
        a = qq % P.ndx;
        bu = P.ndy / 2 + qq / P.ndx;
    }
    const float xpa = (float)(2 * a - P.ndx + 1) * (0.5f * P.pitch);
    const float yp = (float)(2 * bu - P.ndy + 1) * (0.5f * P.pitch);
    const int slot = lane / QW, ml = lane % QW;
    const int qc = blockIdx.z;
    const int mq = qc * QW + ml;
    const double qa = T.qa[mq], qb = T.qb[mq];
    const int g0 = blockIdx.y * groups_per_split;
    const int g1 = min(P.n_groups, g0 + groups_per_split);

    float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
    for (int gb = g0; gb < g1; gb += GB) {
        __syncthreads();
        // stage 64 voxel rows x QW q of f; with LR row 2k = left voxel of group
        // gb+k and row 2k+1 its mirror
        for (int idx = threadIdx.x; idx < 64 * QW; idx += blockDim.x) {
            const int r = idx / QW, mm = idx % QW;
            int vox = -1;
            if (LR) {
                const int gg = gb + (r >> 1);
                if (gg < g1) {
                    const int half = P.nx / 2;
                    const int iz = gg / half, ix = gg % half;
                    vox = iz * P.nx + ((r & 1) ? (P.nx - 1 - ix) : ix);
                }
            } else {
                const int gg = gb + r;
                if (gg < g1) vox = gg;
            }
            const int m = qc * QW + mm;
            s_tile[idx] = (vox >= 0 && m < P.nq) ? f[(size_t)vox * P.nq + m] : 0.0f;
        }
        __syncthreads();
        if (!wave_on) continue;

        // one class per lane
        double kap = 0.0;
        float k0 = 0.0f, k1 = 0.0f, k2 = 0.0f, k3 = 0.0f;
        int r0 = 0, r1 = 0;
        bool act = false;
        {
            const int gg = LR ? (lane >> 1) : lane;
            const int g = gb + gg;
            if (g < g1) {
                const int G = LR ? (lane & 1) : 0;   // 0: pixel column a, 1: mirror column
                int j;
                if (LR) {
                    const int half = P.nx / 2;
                    j = (g / half) * P.nx + g % half;
                } else {
                    j = g;
                }
                const float xp = G ? -xpa : xpa;
                const float2 vm = T.vm[j];
                const Cells c = mask_cells(P, vm, xp, yp);
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
                    float A;
                    pair_factors(P, T.vd[j], T.vf[j], (double)xp, (double)yp, kap, A);
                    if (in_band(P, kap)) {
                        act = true;
                        const int rowA = LR ? 2 * gg : gg, rowB = 2 * gg + 1;
                        if (G == 0) {
                            k0 = A * tau; k1 = A * tad; k2 = A * tbu; k3 = A * tbd;
                            r0 = rowA; r1 = rowB;
                        } else {
                            k0 = A * tbu; k1 = A * tbd; k2 = A * tau; k3 = A * tad;
                            r0 = rowB; r1 = rowA;
                        }
                        if (!LR) r1 = r0;
                    }
                }
            }
        }
        const uint64_t bal = __ballot(act);
        const int nact = __popcll(bal);
        const int idx = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (act) {
            s_list[2 * idx] = make_float4(dlo(kap), dhi(kap), k0, k1);
            s_list[2 * idx + 1] = make_float4(k2, k3, __int_as_float(r0 * QW * 4), __int_as_float(r1 * QW * 4));
        }
        const int npad = (nact + STEP - 1) / STEP * STEP;
        if (lane < npad - nact) {
            s_list[2 * (nact + lane)] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_list[2 * (nact + lane) + 1] = make_float4(0.0f, 0.0f, __int_as_float(0), __int_as_float(0));
        }
        __builtin_amdgcn_wave_barrier();
        const unsigned char *tile_lane = (const unsigned char *)s_tile + ml * 4;
        for (int i = 0; i < npad; i += STEP) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int e = i + u * SLOTS + slot;
                const float4 e0 = s_list[2 * e];
                const float4 e1 = s_list[2 * e + 1];
                const int k = spec_index(P, as_double(e0.x, e0.y), qa, qb);
                const float ph = spec<TD>(s_phi, s_phi16, k);
                const float w0 = ph * *(const float *)(tile_lane + __float_as_int(e1.z));
                o0 = fmaf(e0.z, w0, o0);
                o1 = fmaf(e0.w, w0, o1);
                if (LR) {
                    const float w1 = ph * *(const float *)(tile_lane + __float_as_int(e1.w));
                    o2 = fmaf(e1.x, w1, o2);
                    o3 = fmaf(e1.y, w1, o3);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (!wave_on) return;
    const float qm = T.qv[mq];
    float v0 = o0 * qm, v1 = o1 * qm, v2 = o2 * qm, v3 = o3 * qm;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v0 += __shfl_xor(v0, off, 64);
        v1 += __shfl_xor(v1, off, 64);
        if (LR) {
            v2 += __shfl_xor(v2, off, 64);
            v3 += __shfl_xor(v3, off, 64);
        }
    }
    if (lane == 0) {
        float *dst = part + (size_t)(blockIdx.y * gridDim.z + qc) * P.npix;
        const int bd = P.ndy - 1 - bu;
        dst[bu * P.ndx + a] = v0;
        dst[bd * P.ndx + a] = v1;
        if (LR) {
            const int ab = P.ndx - 1 - a;
            dst[bu * P.ndx + ab] = v2;
            dst[bd * P.ndx + ab] = v3;
        }
    }
}

// g_i = sum_p part[p][i] in a fixed order.
__global__ void __launch_bounds__(256) k_sum_parts(const float *__restrict__ part, int nparts, int n,
                                                   float *__restrict__ g)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += part[(size_t)p * n + i];
    g[i] = s;
}

Lds lds_layout(const KParams &P, int td, int wpb, bool forward)
{
    auto al = [](int v) { return (v + 15) & ~15; };
    Lds L;
    int off = 0;
    L.phi = off;
    off += al((P.ne + 2) * (td == CSX_TABLE_BF16 ? 2 : 4));
    L.mask = off;
    off += al(P.mask_ny * 4);
    L.list = off;
    off += wpb * LIST_CAP * (forward ? 32 : 16);
    L.tile = off;
    if (forward) off += 64 * P.qw * 4;
    L.total = off;
    return L;
}

template <int TD, int LR, int SLOTS>
void launch_fwd_t(const csx_geometry *h, const Lds &L, dim3 grid, dim3 block, hipStream_t s,
                  const float *f, int gps)
{
    hipLaunchKernelGGL((k_forward<TD, LR, SLOTS>), grid, block, L.total, s, h->P, h->t, L, f, h->part, gps);
}

template <int TD, int LR, int SLOTS>
void launch_adj_t(const csx_geometry *h, const Lds &L, dim3 grid, dim3 block, hipStream_t s,
                  const float *rho, float *b)
{
    hipLaunchKernelGGL((k_adjoint<TD, LR, SLOTS>), grid, block, L.total, s, h->P, h->t, L, rho, b);
}

template <int TD, int LR>
void dispatch_fwd(const csx_geometry *h, const Lds &L, dim3 grid, dim3 block, hipStream_t s,
                  const float *f, int gps)
{
    switch (64 / h->P.qw) {
    case 4: launch_fwd_t<TD, LR, 4>(h, L, grid, block, s, f, gps); break;
    case 2: launch_fwd_t<TD, LR, 2>(h, L, grid, block, s, f, gps); break;
    default: launch_fwd_t<TD, LR, 1>(h, L, grid, block, s, f, gps); break;
    }
}

template <int TD, int LR>
void dispatch_adj(const csx_geometry *h, const Lds &L, dim3 grid, dim3 block, hipStream_t s,
                  const float *rho, float *b)
{
    switch (64 / h->P.qw) {
    case 4: launch_adj_t<TD, LR, 4>(h, L, grid, block, s, rho, b); break;
    case 2: launch_adj_t<TD, LR, 2>(h, L, grid, block, s, rho, b); break;
    default: launch_adj_t<TD, LR, 1>(h, L, grid, block, s, rho, b); break;
    }
}

}  // namespace

hipEvent_t csx_timing_event(csx_geometry *h, int op)
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

void csx_choose_launch(csx_geometry *h)
{
    const KParams &P = h->P;
    h->fwd_wpb = 8;
    h->adj_wpb = 4;
    const int gb = P.lr ? 32 : 64;
    const int bx = (P.n_quad + h->fwd_wpb - 1) / h->fwd_wpb;
    // split the voxel groups so that a launch holds >= ~8 waves per SIMD
    const int target_waves = 8 * 4 * 256;
    int splits = std::max(1, target_waves / std::max(1, bx * h->fwd_wpb * P.qchunks));
    const int batches = (P.n_groups + gb - 1) / gb;
    splits = std::min(splits, std::max(1, batches / 2));
    h->fwd_splits = splits;
}

csx_status csx_launch_forward(csx_geometry *h, const float *f, float *g, hipStream_t s)
{
    const KParams &P = h->P;
    const int wpb = h->fwd_wpb;
    const Lds L = lds_layout(P, h->table_dtype, wpb, true);
    const int gb = P.lr ? 32 : 64;
    const int splits = h->fwd_splits;
    int gps = (P.n_groups + splits - 1) / splits;
    gps = (gps + gb - 1) / gb * gb;
    const int nsplit = (P.n_groups + gps - 1) / gps;
    dim3 grid((P.n_quad + wpb - 1) / wpb, nsplit, P.qchunks);
    dim3 block(64 * wpb);
    hipEvent_t e0 = csx_timing_event(h, 0), e1 = csx_timing_event(h, 0);
    if (e0) HIP_TRY(hipEventRecord(e0, s));
    const bool bf = h->table_dtype == CSX_TABLE_BF16;
    if (P.lr) {
        if (bf) dispatch_fwd<CSX_TABLE_BF16, 1>(h, L, grid, block, s, f, gps);
        else dispatch_fwd<CSX_TABLE_F32, 1>(h, L, grid, block, s, f, gps);
    } else {
        if (bf) dispatch_fwd<CSX_TABLE_BF16, 0>(h, L, grid, block, s, f, gps);
        else dispatch_fwd<CSX_TABLE_F32, 0>(h, L, grid, block, s, f, gps);
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3((P.npix + 255) / 256), dim3(256), 0, s, h->part,
                       nsplit * P.qchunks, P.npix, g);
    HIP_TRY(hipGetLastError());
    if (e1) HIP_TRY(hipEventRecord(e1, s));
    return CSX_OK;
}

csx_status csx_launch_adjoint(csx_geometry *h, const float *rho, float *b, hipStream_t s)
{
    const KParams &P = h->P;
    const int wpb = h->adj_wpb;
    const Lds L = lds_layout(P, h->table_dtype, wpb, false);
    dim3 grid((P.n_groups + wpb - 1) / wpb, P.qchunks);
    dim3 block(64 * wpb);
    hipEvent_t e0 = csx_timing_event(h, 1), e1 = csx_timing_event(h, 1);
    if (e0) HIP_TRY(hipEventRecord(e0, s));
    const bool bf = h->table_dtype == CSX_TABLE_BF16;
    if (P.lr) {
        if (bf) dispatch_adj<CSX_TABLE_BF16, 1>(h, L, grid, block, s, rho, b);
        else dispatch_adj<CSX_TABLE_F32, 1>(h, L, grid, block, s, rho, b);
    } else {
        if (bf) dispatch_adj<CSX_TABLE_BF16, 0>(h, L, grid, block, s, rho, b);
        else dispatch_adj<CSX_TABLE_F32, 0>(h, L, grid, block, s, rho, b);
    }
    HIP_TRY(hipGetLastError());
    if (e1) HIP_TRY(hipEventRecord(e1, s));
    return CSX_OK;
}
