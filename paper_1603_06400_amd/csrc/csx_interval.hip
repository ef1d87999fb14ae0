// csx_interval.hip -- the exact operators in interval form.
//
// With the spectrum a histogram of ne bins (Phi = Phi_k on [e_lo + k dE,
// e_lo + (k+1) dE), 0 outside), the q sum of one class,
//     sum_m q_m Phi(kappa q_m) f_jm   (forward)   /   q_m Phi(kappa q_m) (adjoint),
// depends on kappa = hc / sin(theta/2) only through the spectrum bins that
// kappa q_m falls in, one per node.  Node m changes bin at the thresholds
// kappa = beta(c, m), c = 1 .. ne + 1, where the bin coordinate
// u_m(kappa) = fma(kappa, q_m/dE, 1 - e_lo/dE) reaches c (index c of the
// zero-padded table: 0 below the band, 1 .. ne in it, ne + 1 above).  Sorted
// over all nodes, the (ne + 1) nq thresholds cut the kappa axis into
// intervals; a class whose kappa has passed t thresholds has, at every node,
// the bin index c_m(t) = number of node m's thresholds among the first t.
// Both operators then follow from per-call scans instead of per-node loops:
//
//   forward:  F_j(t) = sum_m q_m f_jm Phi~[c_m(t)] for every interval t of
//             voxel j, built as a float64 prefix sum over the sorted
//             thresholds (passing threshold (c, m) adds q_m f_jm (Phi~[c] -
//             Phi~[c-1])); then g_i = sum_j A_ij T_ij F_j(t_ij): one table
//             read per class and voxel instead of a q loop.
//   adjoint:  with the classes of voxel j ordered by t and W_j(t) the
//             float64 prefix sum of their weights w = A T rho over classes
//             with t_i < t, the classes in bin c at node m are those with
//             interval in (pos(c, m), pos(c + 1, m)], so
//             b_jm = q_m sum_c Phi~[c] (W_j(pos(c+1, m) + 1) - W_j(pos(c, m) + 1)).
//
// This is exact: the same bin decisions (float64 FMA per node, as the
// definition's float64 evaluation) and the same factors as the direct sums;
// only the order of the additions differs.  It is Sec. III-B's angle
// interpolation with the table grid placed exactly where S changes, so no
// interpolation error remains.
//
// Set-up (once per geometry): thresholds on the host, sorted; per class an
// 8-byte record {A, bits} in mirror-pair order (LR: the classes of pixel
// columns a and ndx-1-a of upper row r side by side), bits = mask values
// (4), interval t (14), rank of the class in its voxel group's t order (14).
#include "csx_internal.h"

#include "csx_device.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int IV_THREADS = 1024;
constexpr int IV_WAVES = IV_THREADS / 64;

struct IvState {
    uint2 *rec = nullptr;       // [n_groups][n_slots] {A bits, w}
    double *coef = nullptr;     // [nt] q_m (Phi~[c] - Phi~[c-1]) of the sorted thresholds
    uint16_t *mt = nullptr;     // [nt] node m of each sorted threshold
    uint16_t *pp = nullptr;     // [nq][ne + 2] pos(c, m) + 1, c = 1 .. ne + 1
    uint16_t *bpos = nullptr;   // [n_groups][nq][ne + 1] rank of the first class of each (node, bin)
    double *qd = nullptr;       // [nq] q nodes
    float *part = nullptr;      // [nblk][npix] forward partial images
    int nt = 0;                 // thresholds, (ne + 1) nq
    int n_slots = 0;            // classes per voxel group (LR: 2 per mirror pair)
    int n_items = 0;            // work items per group: mirror pairs (LR) or classes
    int np = 1;                 // forward: work items per thread (power of 2, <= 8)
    int npa = 1;                // adjoint: work items per thread (power of 2, <= 16)
    int nblk_f = 0, nblk_a = 0;
    int lds_f = 0, lds_a = 0;
    int64_t bytes = 0;
    double build_ms = 0.0;
};

struct IvArgs {
    const uint2 *rec;
    const double *coef;
    const uint16_t *mt;
    const uint16_t *pp;
    const uint16_t *bpos;
    const double *qd;
    int nt, n_slots, n_items, ngroups;
};

__device__ __forceinline__ void group_voxels(const KParams &P, int LR, int g, int &j, int &j2)
{
    if (LR) {
        const int half = P.nx / 2;
        j = (g / half) * P.nx + g % half;
        j2 = (g / half) * P.nx + (P.nx - 1 - g % half);
    } else {
        j = g;
        j2 = g;
    }
}

// Class of work item p and slot s (0: column a, 1: its mirror): column and upper row.
__device__ __forceinline__ void item_class(const KParams &P, int LR, int p, int s, int &a, int &r)
{
    if (LR) {
        const int hx = P.ndx / 2;
        a = p % hx;
        r = p / hx;
        if (s) a = P.ndx - 1 - a;
    } else {
        a = p % P.ndx;
        r = p / P.ndx;
    }
}

// ---------------------------------------------------------------------------
// Set-up kernels
// ---------------------------------------------------------------------------

// Record of one class: A and the mask values exactly as the direct operators
// evaluate them (pair_factors, mask_cells), and the number of thresholds its
// kappa has passed, t = sum_m clamp(floor(fma(kappa, q_m/dE, b0)), 0, ne + 1).
// Inactive classes (every pair closed, or kappa out of band) get A = 0, t = 0.
template <int LR>
__global__ void __launch_bounds__(256) k_iv_records(KParams P, DevTables T, int n_slots, uint2 *__restrict__ out)
{
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)P.n_groups * n_slots) return;
    const int g = (int)(idx / n_slots), sl = (int)(idx % n_slots);
    const int p = LR ? sl >> 1 : sl, s = LR ? sl & 1 : 0;
    int j, j2;
    group_voxels(P, LR, g, j, j2);
    int a, r;
    item_class(P, LR, p, s, a, r);
    const int half_y = P.ndy / 2;
    float A = 0.0f;
    uint32_t bits = 0u, t = 0u;
    const double xp = pixel_coord(P, a, P.ndx);
    const double yp = pixel_coord(P, half_y + r, P.ndy);
    const Cells c = mask_cells(P, T.vm[j], xp, yp);
    if (c.in_rows) {
        const uint32_t ru = T.maskbits[c.row_u], rd = T.maskbits[c.row_d];
        bits = ((ru >> c.col_a) & 1u) | (((rd >> c.col_a) & 1u) << 1);
        if (LR) bits |= (((ru >> c.col_b) & 1u) << 2) | (((rd >> c.col_b) & 1u) << 3);
    }
    if (bits) {
        double k;
        pair_factors(P, T.vd[j], T.vf[j], xp, yp, k, A);
        if (in_band(P, k)) {
            const int top = P.ne + 1;
            for (int m = 0; m < P.nq; ++m) {
                const double u = floor(fma(k, T.qa[m], P.b0));
                t += (uint32_t)fmin(fmax(u, 0.0), (double)top);
            }
        } else {
            bits = 0u;
            A = 0.0f;
        }
    }
    out[idx] = make_uint2(__float_as_uint(A), bits | (t << 4));
}

// Rank of every class of a voxel group in the order of (t, slot): a bitonic
// sort of the keys (t << 14 | slot) in LDS, one block per group.  The rank
// goes to bits 18-31 of the record.
__global__ void __launch_bounds__(1024) k_iv_rank(int n_slots, int npow2, uint2 *__restrict__ rec, int nq, int ne,
                                                  const uint16_t *__restrict__ pp, uint16_t *__restrict__ bpos)
{
    extern __shared__ uint32_t keys[];
    uint2 *rg = rec + (size_t)blockIdx.x * n_slots;
    for (int i = threadIdx.x; i < npow2; i += blockDim.x)
        keys[i] = i < n_slots ? (((rg[i].y >> 4) & 0x3FFFu) << 14) | (uint32_t)i : 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= npow2; k <<= 1)
        for (int d = k >> 1; d > 0; d >>= 1) {
            for (int i = threadIdx.x; i < npow2; i += blockDim.x) {
                const int o = i ^ d;
                if (o > i) {
                    const uint32_t x = keys[i], y = keys[o];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        keys[i] = y;
                        keys[o] = x;
                    }
                }
            }
            __syncthreads();
        }
    for (int s = threadIdx.x; s < n_slots; s += blockDim.x) {
        const int i = (int)(keys[s] & 0x3FFFu);
        rg[i].y = (rg[i].y & 0x3FFFFu) | ((uint32_t)s << 18);
    }
    // bin positions of the group: for node m and bin c (1 .. ne + 1) the
    // number of classes whose interval is below pp(c, m) = pos(c, m) + 1,
    // i.e. the rank of the first class at or past that threshold
    const int nt = (ne + 1) * nq;
    uint16_t *bg = bpos + (size_t)blockIdx.x * nt;
    for (int k = threadIdx.x; k < nt; k += blockDim.x) {
        const int m = k / (ne + 1), c = 1 + k % (ne + 1);
        const uint32_t T = pp[(size_t)m * (ne + 2) + c];
        int lo = 0, hi = n_slots;          // first sorted position with t >= T
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((keys[mid] >> 14) < T) lo = mid + 1;
            else hi = mid;
        }
        bg[k] = (uint16_t)lo;
    }
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of a pair of float64 values (fixed order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 block_exclusive_scan(double a, double b, double2 *s_tot)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double ia = a, ib = b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double ua = __shfl_up(ia, d, 64), ub = __shfl_up(ib, d, 64);
        if (lane >= d) {
            ia += ua;
            ib += ub;
        }
    }
    if (lane == 63) s_tot[wv] = make_double2(ia, ib);
    __syncthreads();
    double oa = 0.0, ob = 0.0;
    for (int w = 0; w < wv; ++w) {
        oa += s_tot[w].x;
        ob += s_tot[w].y;
    }
    return make_double2(oa + ia - a, ob + ib - b);
}

// ---------------------------------------------------------------------------
// Forward: g = A f.  Block = IV_THREADS threads, a contiguous range of voxel
// groups; thread k owns work items k, k + IV_THREADS, ... (NP of them) and
// keeps their pixels' sums in registers; partial image per block.
// ---------------------------------------------------------------------------
template <int LR, int NP>
__global__ void __launch_bounds__(IV_THREADS) k_iv_forward(KParams P, IvArgs V, const float *__restrict__ f,
                                                           float *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char lds[];
    double *s_coef = (double *)lds;
    uint16_t *s_mt = (uint16_t *)(s_coef + V.nt);
    float2 *s_F = (float2 *)(lds + (((size_t)V.nt * 10 + 15) & ~(size_t)15));
    float *s_f = (float *)(s_F + V.nt + 1);
    double2 *s_tot = (double2 *)(((uintptr_t)(s_f + 2 * P.nq) + 15) & ~(uintptr_t)15);
    const int tid = threadIdx.x;
    for (int i = tid; i < V.nt; i += IV_THREADS) {
        s_coef[i] = V.coef[i];
        s_mt[i] = V.mt[i];
    }
    // groups of this block
    const int per = (V.ngroups + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(V.ngroups, g0 + per);
    // thresholds of this thread in the scan
    const int tper = (V.nt + IV_THREADS - 1) / IV_THREADS;
    const int t0 = min(V.nt, tid * tper), t1 = min(V.nt, t0 + tper);

    constexpr int NO = LR ? 4 : 2;
    float o[NP][NO];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int k = 0; k < NO; ++k) o[i][k] = 0.0f;
    // records of the thread's items, prefetched one group ahead
    uint4 nr[NP];
    auto load_rec = [&](int g) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = tid + i * IV_THREADS;
            nr[i] = make_uint4(0u, 0u, 0u, 0u);
            if (p < V.n_items && g < g1) {
                const uint2 *rg = V.rec + (size_t)g * V.n_slots;
                if (LR) {
                    nr[i] = *(const uint4 *)(rg + 2 * p);
                } else {
                    const uint2 v = rg[p];
                    nr[i] = make_uint4(v.x, v.y, 0u, 0u);
                }
            }
        }
    };
    // thread i < 2 nq carries f of the next group's voxel j (i < nq) or j2
    auto load_f = [&](int g) -> float {
        if (tid >= 2 * P.nq || g >= g1) return 0.0f;
        int j, j2;
        group_voxels(P, LR, g, j, j2);
        if (tid < P.nq) return f[(size_t)j * P.nq + tid];
        return LR ? f[(size_t)j2 * P.nq + tid - P.nq] : 0.0f;
    };
    float fv = load_f(g0);
    load_rec(g0);
    __syncthreads();
    for (int g = g0; g < g1; ++g) {
        if (tid < 2 * P.nq) s_f[tid] = fv;
        fv = load_f(g + 1);
        __syncthreads();
        // F tables of voxels j and j2: float64 prefix sums over the sorted thresholds
        double la = 0.0, lb = 0.0;
        for (int t = t0; t < t1; ++t) {
            const double c = s_coef[t];
            const int m = s_mt[t];
            la = fma(c, (double)s_f[m], la);
            lb = fma(c, (double)s_f[P.nq + m], lb);
        }
        double2 run = block_exclusive_scan(la, lb, s_tot);
        for (int t = t0; t < t1; ++t) {
            const double c = s_coef[t];
            const int m = s_mt[t];
            run.x = fma(c, (double)s_f[m], run.x);
            run.y = fma(c, (double)s_f[P.nq + m], run.y);
            s_F[t + 1] = make_float2((float)run.x, (float)run.y);
        }
        if (tid == 0) s_F[0] = make_float2(0.0f, 0.0f);
        __syncthreads();
        uint4 cr[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) cr[i] = nr[i];
        load_rec(g + 1);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            // class of column a (record x, y) and, with LR, of column ndx-1-a (z, w)
            const float A1 = __uint_as_float(cr[i].x);
            const uint32_t w1 = cr[i].y;
            const float2 F1 = s_F[(w1 >> 4) & 0x3FFFu];
            const float a1 = A1 * F1.x;
            o[i][0] = fmaf(a1, (float)(w1 & 1u), o[i][0]);           // (a, u) <- voxel j
            o[i][1] = fmaf(a1, (float)((w1 >> 1) & 1u), o[i][1]);    // (a, d) <- voxel j
            if (LR) {
                const float b1 = A1 * F1.y;
                o[i][2] = fmaf(b1, (float)((w1 >> 2) & 1u), o[i][2]);    // (-a, u) <- voxel j2
                o[i][3] = fmaf(b1, (float)((w1 >> 3) & 1u), o[i][3]);    // (-a, d) <- voxel j2
                const float A2 = __uint_as_float(cr[i].z);
                const uint32_t w2 = cr[i].w;
                const float2 F2 = s_F[(w2 >> 4) & 0x3FFFu];
                const float a2 = A2 * F2.x, b2 = A2 * F2.y;
                o[i][2] = fmaf(a2, (float)(w2 & 1u), o[i][2]);           // (-a, u) <- voxel j
                o[i][3] = fmaf(a2, (float)((w2 >> 1) & 1u), o[i][3]);    // (-a, d) <- voxel j
                o[i][0] = fmaf(b2, (float)((w2 >> 2) & 1u), o[i][0]);    // (a, u) <- voxel j2
                o[i][1] = fmaf(b2, (float)((w2 >> 3) & 1u), o[i][1]);    // (a, d) <- voxel j2
            }
        }
    }
    // partial image of this block: every pixel is written once
    float *dst = part + (size_t)blockIdx.x * P.npix;
    const int half_y = P.ndy / 2;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = tid + i * IV_THREADS;
        if (p >= V.n_items) continue;
        int a, r;
        item_class(P, LR, p, 0, a, r);
        const int bu = half_y + r, bd = P.ndy - 1 - bu;
        dst[bu * P.ndx + a] = o[i][0];
        dst[bd * P.ndx + a] = o[i][1];
        if (LR) {
            const int ab = P.ndx - 1 - a;
            dst[bu * P.ndx + ab] = o[i][2];
            dst[bd * P.ndx + ab] = o[i][3];
        }
    }
}

// g_i = sum_p part[p][i] in a fixed order: 64 pixels per block (the lanes),
// 16 slices of the partial images (the waves), each slice's loads issued
// together, then the 16 slice sums added in slice order.
__global__ void __launch_bounds__(1024) k_iv_sum(const float *__restrict__ part, int nparts, int n,
                                                 float *__restrict__ g)
{
    __shared__ float s_part[16][64];
    const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    float acc = 0.0f;
    if (i < n) {
        constexpr int U = 8;
        for (int p0 = sl; p0 < nparts; p0 += 16 * U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = p0 + 16 * u;
                v[u] = p < nparts ? part[(size_t)p * n + i] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += v[u];
        }
    }
    s_part[sl][lane] = acc;
    __syncthreads();
    if (sl == 0 && i < n) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += s_part[k][lane];
        g[i] = t;
    }
}

// ---------------------------------------------------------------------------
// Adjoint: b = A^T rho.  Block = IV_THREADS threads, a contiguous range of
// voxel groups, one group at a time: class weights into LDS at their rank,
// float64 prefix sums at every interval, then per (m, c) differences.
// ---------------------------------------------------------------------------
// Adjoint: b = A^T rho.  One block of IVA_THREADS threads per compute unit,
// a contiguous range of voxel groups, one group at a time:
//  1. every class's weights (voxel j: A (T_u rho_u + T_d rho_d); voxel j2:
//     the mirror pixels) go to LDS, in float64, at the class's rank in the
//     group's interval order;
//  2. float64 prefix sums in rank order: thread k owns ranks [k SC, (k+1) SC)
//     and stores their exclusive prefix within the chunk (XOR-swizzled within
//     the chunk against bank conflicts) and the chunk's base from a block
//     scan, so E(p) = base[p / SC] + loc[p];
//  3. the classes in bin c at node m are the ranks [P(m, c), P(m, c + 1)),
//     P from the set-up: b_jm = q_m sum_c Phi~[c] (E(P(m, c+1)) - E(P(m, c))).
// The prefix sums are float64 end to end: a bin's sum is a difference of two
// prefixes, and a bin holding only a few small weights next to large ones
// (the lowest q nodes see only the smallest angles) needs that precision to
// stay accurate relative to itself.
constexpr int IVA_THREADS = 1024;
constexpr int IVA_WAVES = IVA_THREADS / 64;
constexpr int IVA_SC = 8;           // ranks per thread chunk
constexpr int IVA_SUB = 8;          // threads per node in the gather
constexpr int IVA_MAXV = 9;         // prefetched bin positions per thread (ne <= 8 IVA_SUB)

__device__ __forceinline__ int iva_swz(int p)
{
    return (p & ~(IVA_SC - 1)) | ((p ^ (p >> 3)) & (IVA_SC - 1));
}

// PF = 1: nq <= IVA_THREADS / IVA_SUB and ne <= 8 IVA_SUB: thread (m, sub)
// owns the consecutive bins c = 1 + sub CPT .. (sub + 1) CPT of node m and
// holds their CPT + 1 bin positions in registers, loaded one group ahead.
template <int LR, int NP, int PF>
__global__ void __launch_bounds__(IVA_THREADS) k_iv_adjoint(KParams P, IvArgs V, const DevTables T,
                                                            const float *__restrict__ rho, float *__restrict__ b)
{
    extern __shared__ __align__(16) unsigned char lds[];
    double2 *s_loc = (double2 *)lds;                               // [(IVA_THREADS + 1) SC]
    double2 *s_base = s_loc + (IVA_THREADS + 1) * IVA_SC;          // [IVA_THREADS + 1]
    float *s_phi = (float *)(s_base + IVA_THREADS + 1);            // [ne + 2]
    double2 *s_tot = (double2 *)(((uintptr_t)(s_phi + P.ne + 2) + 15) & ~(uintptr_t)15);
    const int tid = threadIdx.x;
    for (int k = tid; k < P.ne + 2; k += IVA_THREADS)
        s_phi[k] = P.td == CSX_TABLE_BF16 ? bf16_to_f32(T.phi16[k]) : T.phi32[k];
    // ranks past the last class hold zero weight for every group
    for (int k = tid; k < (IVA_THREADS + 1) * IVA_SC; k += IVA_THREADS) s_loc[k] = make_double2(0.0, 0.0);
    const int per = (V.ngroups + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(V.ngroups, g0 + per);
    const int half_y = P.ndy / 2;
    const int nt = V.nt, ne1 = P.ne + 1;
    // the detector values of the thread's items are the same for every group
    float ru[NP], rd[NP], rbu[NP], rbd[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = tid + i * IVA_THREADS;
        ru[i] = rd[i] = rbu[i] = rbd[i] = 0.0f;
        if (p < V.n_items) {
            int a, r;
            item_class(P, LR, p, 0, a, r);
            const int bu = half_y + r, bd = P.ndy - 1 - bu;
            ru[i] = rho[bu * P.ndx + a];
            rd[i] = rho[bd * P.ndx + a];
            if (LR) {
                const int ab = P.ndx - 1 - a;
                rbu[i] = rho[bu * P.ndx + ab];
                rbd[i] = rho[bd * P.ndx + ab];
            }
        }
    }
    // records of the thread's items, prefetched one group ahead (item i's
    // next record is requested as soon as its current one is used)
    uint4 nr[NP];
    auto load_one = [&](int g, int i) -> uint4 {
        const int p = tid + i * IVA_THREADS;
        if (p < V.n_items && g < g1) {
            const uint2 *rg = V.rec + (size_t)g * V.n_slots;
            if (LR) return *(const uint4 *)(rg + 2 * p);
            const uint2 v = rg[p];
            return make_uint4(v.x, v.y, 0u, 0u);
        }
        return make_uint4(0u, 0u, 0u, 0u);
    };
    auto E = [&](int p) -> double2 {
        const double2 bs = s_base[p / IVA_SC];
        const double2 l = s_loc[iva_swz(p)];
        return make_double2(bs.x + l.x, bs.y + l.y);
    };
    // PF: this thread's node, first bin and bin count, and positions of the next group
    const int pm_m = tid / IVA_SUB, pm_sub = tid % IVA_SUB;
    const int cpt = (P.ne + IVA_SUB - 1) / IVA_SUB;
    const int pc0 = 1 + pm_sub * cpt, pnc = max(0, min(P.ne, pc0 + cpt - 1) - pc0 + 1);
    const bool pact = PF && pm_m < P.nq && pnc > 0;
    // positions packed two per register (low half: even k)
    constexpr int NPV = (IVA_MAXV + 1) / 2;
    uint32_t pv[PF ? NPV : 1];
    auto load_pos = [&](int g) {
        if (!PF) return;
#pragma unroll
        for (int k = 0; k < NPV; ++k) pv[k] = 0u;
        if (pact && g < g1) {
            const uint16_t *row = V.bpos + (size_t)g * nt + (size_t)pm_m * ne1 + (pc0 - 1);
#pragma unroll
            for (int k = 0; k < IVA_MAXV; ++k)
                if (k <= pnc) pv[k >> 1] |= (uint32_t)row[k] << (16 * (k & 1));
        }
    };
    auto pos = [&](int k) -> int { return (int)((pv[k >> 1] >> (16 * (k & 1))) & 0xFFFFu); };
#pragma unroll
    for (int i = 0; i < NP; ++i) nr[i] = load_one(g0, i);
    load_pos(g0);
    for (int g = g0; g < g1; ++g) {
        int j, j2;
        group_voxels(P, LR, g, j, j2);
        // 1. class weights at their rank
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const uint4 cr = nr[i];
            nr[i] = load_one(g + 1, i);
            const int p = tid + i * IVA_THREADS;
            if (p >= V.n_items) continue;
            const float A1 = __uint_as_float(cr.x);
            const uint32_t w1 = cr.y;
            const float c10 = A1 * ((float)(w1 & 1u) * ru[i] + (float)((w1 >> 1) & 1u) * rd[i]);
            float c11 = 0.0f;
            if (LR) {
                c11 = A1 * ((float)((w1 >> 2) & 1u) * rbu[i] + (float)((w1 >> 3) & 1u) * rbd[i]);
                const float A2 = __uint_as_float(cr.z);
                const uint32_t w2 = cr.w;
                const float c20 = A2 * ((float)(w2 & 1u) * rbu[i] + (float)((w2 >> 1) & 1u) * rbd[i]);
                const float c21 = A2 * ((float)((w2 >> 2) & 1u) * ru[i] + (float)((w2 >> 3) & 1u) * rd[i]);
                s_loc[iva_swz((int)(w2 >> 18))] = make_double2((double)c20, (double)c21);
            }
            s_loc[iva_swz((int)(w1 >> 18))] = make_double2((double)c10, (double)c11);
        }
        __syncthreads();
        // 2. chunk prefixes (in place) and bases
        {
            const int c0 = tid * IVA_SC;
            double la = 0.0, lb = 0.0;
#pragma unroll
            for (int k = 0; k < IVA_SC; ++k) {
                const int q = iva_swz(c0 + k);
                const double2 w = s_loc[q];
                s_loc[q] = make_double2(la, lb);
                la += w.x;
                lb += w.y;
            }
            const double2 base = block_exclusive_scan(la, lb, s_tot);
            s_base[tid] = base;
            if (tid == IVA_THREADS - 1) s_base[IVA_THREADS] = make_double2(base.x + la, base.y + lb);
        }
        __syncthreads();
        // 3. b_jm = q_m sum_c Phi~[c] (E(P(m, c+1)) - E(P(m, c))), IVA_SUB threads per node
        if (PF) {
            double sa = 0.0, sb = 0.0;
            if (pact) {
                double2 lo = E(pos(0));
#pragma unroll
                for (int k = 1; k < IVA_MAXV; ++k) {
                    if (k > pnc) break;
                    const double2 hi = E(pos(k));
                    const double ph = (double)s_phi[pc0 + k - 1];
                    sa = fma(ph, hi.x - lo.x, sa);
                    sb = fma(ph, hi.y - lo.y, sb);
                    lo = hi;
                }
            }
#pragma unroll
            for (int d = IVA_SUB / 2; d > 0; d >>= 1) {
                sa += __shfl_xor(sa, d, 64);
                sb += __shfl_xor(sb, d, 64);
            }
            if (pm_m < P.nq && pm_sub == 0) {
                const double qm = V.qd[pm_m];
                b[(size_t)j * P.nq + pm_m] = (float)(qm * sa);
                if (LR) b[(size_t)j2 * P.nq + pm_m] = (float)(qm * sb);
            }
            load_pos(g + 1);   // used after the next group's weights and prefixes
        } else {
            const uint16_t *bg = V.bpos + (size_t)g * nt;
            for (int mb = 0; mb < P.nq; mb += IVA_THREADS / IVA_SUB) {
                const int m = mb + tid / IVA_SUB, sub = tid % IVA_SUB;
                double sa = 0.0, sb = 0.0;
                if (m < P.nq) {
                    const uint16_t *pm = bg + (size_t)m * ne1;       // pm[c - 1] = P(m, c), c = 1 .. ne + 1
                    for (int c = 1 + sub; c <= P.ne; c += IVA_SUB) {
                        const double ph = (double)s_phi[c];
                        const double2 hi = E(pm[c]), lo = E(pm[c - 1]);
                        sa = fma(ph, hi.x - lo.x, sa);
                        sb = fma(ph, hi.y - lo.y, sb);
                    }
                }
#pragma unroll
                for (int d = IVA_SUB / 2; d > 0; d >>= 1) {
                    sa += __shfl_xor(sa, d, 64);
                    sb += __shfl_xor(sb, d, 64);
                }
                if (m < P.nq && sub == 0) {
                    const double qm = V.qd[m];
                    b[(size_t)j * P.nq + m] = (float)(qm * sa);
                    if (LR) b[(size_t)j2 * P.nq + m] = (float)(qm * sb);
                }
            }
        }
        __syncthreads();   // the next group's weights overwrite s_loc
    }
}

IvArgs iv_args(const csx_geometry *h, const IvState *v)
{
    IvArgs a;
    a.rec = v->rec;
    a.coef = v->coef;
    a.mt = v->mt;
    a.pp = v->pp;
    a.bpos = v->bpos;
    a.qd = v->qd;
    a.nt = v->nt;
    a.n_slots = v->n_slots;
    a.n_items = v->n_items;
    a.ngroups = h->P.n_groups;
    return a;
}

template <typename T>
csx_status iv_upload(T **dst, const std::vector<T> &src, int64_t &bytes)
{
    HIP_TRY(hipMalloc((void **)dst, src.size() * sizeof(T)));
    HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    bytes += (int64_t)(src.size() * sizeof(T));
    return CSX_OK;
}

void iv_release(IvState *v)
{
    void *ps[] = {v->rec, v->coef, v->mt, v->pp, v->bpos, v->qd, v->part};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete v;
}

}  // namespace

// Feasibility of the interval operators for a geometry: thresholds and ranks
// in 14 bits, and both kernels' LDS within one workgroup's budget.
bool csx_iv_feasible(const KParams &P, int *lds_f, int *lds_a)
{
    const long nt = (long)(P.ne + 1) * P.nq;
    const long items = P.lr ? (long)(P.ndx / 2) * (P.ndy / 2) : (long)P.ndx * (P.ndy / 2);
    const long slots = P.lr ? 2 * items : items;
    // intervals and ranks in 14 bits; the adjoint's ranks in IVA_THREADS
    // chunks of 16; one f value per forward thread
    if (nt >= 16384 || slots > IVA_SC * IVA_THREADS || items > 8L * IV_THREADS || 2 * P.nq > IV_THREADS) return false;
    const long lf = ((nt * 10 + 15) & ~15L) + (nt + 1) * 8 + 2L * P.nq * 4 + 16 + IV_WAVES * 16;
    const long la = (long)(IVA_THREADS + 1) * IVA_SC * 16 + (IVA_THREADS + 1) * 16 + (P.ne + 2) * 4 + 16 +
                    IVA_WAVES * 16;
    if (lf > CSX_LDS_MAX || la > CSX_LDS_MAX) return false;
    if (lds_f) *lds_f = (int)lf;
    if (lds_a) *lds_a = (int)la;
    return true;
}

void csx_iv_free(csx_geometry *h)
{
    if (!h->iv) return;
    IvState *v = (IvState *)h->iv;
    h->bytes -= v->bytes;
    iv_release(v);
    h->iv = nullptr;
}

csx_status csx_iv_build(csx_geometry *h)
{
    csx_iv_free(h);
    const KParams &P = h->P;
    int lds_f = 0, lds_a = 0;
    if (!csx_iv_feasible(P, &lds_f, &lds_a))
        return csx_fail(CSX_EINVAL, "interval operators: thresholds, classes or LDS beyond their limits");
    const auto t0 = std::chrono::steady_clock::now();
    IvState *v = new (std::nothrow) IvState();
    if (!v) return csx_fail(CSX_ENOMEM, "host allocation failed");
    auto bail = [&](csx_status st) {
        iv_release(v);
        return st;
    };
    const int nq = P.nq, ne = P.ne;
    const double dE = (h->d.e_hi - h->d.e_lo) / ne;
    // thresholds beta(c, m): the least kappa >= 0 with floor(fma(kappa, q_m/dE, b0)) >= c
    // (the same q_m/dE doubles as the device table)
    struct Thr {
        double beta;
        int m, c;
    };
    std::vector<Thr> L;
    L.reserve((size_t)(ne + 1) * nq);
    auto reach = [&](double k, double qa, int c) { return std::floor(std::fma(k, qa, P.b0)) >= (double)c; };
    for (int m = 0; m < nq; ++m) {
        const double qa = h->q_host[m] / dE;
        for (int c = 1; c <= ne + 1; ++c) {
            double x = std::max(0.0, ((double)c - P.b0) / qa);
            if (reach(0.0, qa, c)) {
                x = 0.0;
            } else {
                while (x > 0.0 && reach(x, qa, c)) x = std::nextafter(x, 0.0);
                while (!reach(x, qa, c)) x = std::nextafter(x, INFINITY);
            }
            L.push_back({x, m, c});
        }
    }
    std::sort(L.begin(), L.end(), [](const Thr &a, const Thr &b) {
        if (a.beta != b.beta) return a.beta < b.beta;
        if (a.m != b.m) return a.m < b.m;
        return a.c < b.c;
    });
    const int nt = (int)L.size();
    // table values as the operators use them (float32, or bfloat16 widened)
    std::vector<double> phit(ne + 2, 0.0);
    for (int k = 0; k < ne; ++k) {
        float fv = (float)h->phi_host[k];
        if (h->table_dtype == CSX_TABLE_BF16) {
            uint32_t u;
            std::memcpy(&u, &fv, 4);
            const uint32_t lsb = (u >> 16) & 1u;
            u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
            std::memcpy(&fv, &u, 4);
        }
        phit[k + 1] = (double)fv;
    }
    std::vector<double> coef(nt);
    std::vector<uint16_t> mt(nt);
    std::vector<uint16_t> pp((size_t)nq * (ne + 2), 0);
    for (int t = 0; t < nt; ++t) {
        coef[t] = h->q_host[L[t].m] * (phit[L[t].c] - phit[L[t].c - 1]);
        mt[t] = (uint16_t)L[t].m;
        pp[(size_t)L[t].m * (ne + 2) + L[t].c] = (uint16_t)(t + 1);
    }
    std::vector<double> qd(h->q_host.begin(), h->q_host.end());
    v->nt = nt;
    v->n_items = P.lr ? (P.ndx / 2) * (P.ndy / 2) : P.ndx * (P.ndy / 2);
    v->n_slots = P.lr ? 2 * v->n_items : v->n_items;
    v->np = 1;
    while (v->np * IV_THREADS < v->n_items) v->np *= 2;
    v->lds_f = lds_f;
    v->lds_a = lds_a;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus < 1)
        cus = 256;
    {
        int per = (P.n_groups + cus - 1) / cus;                  // forward: one block per compute unit
        v->nblk_f = (P.n_groups + per - 1) / per;
        v->nblk_a = v->nblk_f;                                   // adjoint: one as well
        v->npa = 1;
        while (v->npa * IVA_THREADS < v->n_items) v->npa *= 2;
    }
    csx_status st;
    if ((st = iv_upload(&v->coef, coef, v->bytes)) != CSX_OK) return bail(st);
    if ((st = iv_upload(&v->mt, mt, v->bytes)) != CSX_OK) return bail(st);
    if ((st = iv_upload(&v->pp, pp, v->bytes)) != CSX_OK) return bail(st);
    if ((st = iv_upload(&v->qd, qd, v->bytes)) != CSX_OK) return bail(st);
    const size_t nrec = (size_t)P.n_groups * v->n_slots;
    const size_t nbpos = (size_t)P.n_groups * nt;
    if (hipMalloc((void **)&v->rec, nrec * sizeof(uint2)) != hipSuccess ||
        hipMalloc((void **)&v->bpos, nbpos * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc((void **)&v->part, (size_t)v->nblk_f * P.npix * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(csx_fail(CSX_ENOMEM, "interval operators: records"));
    }
    v->bytes += (int64_t)(nrec * sizeof(uint2) + nbpos * sizeof(uint16_t) + (size_t)v->nblk_f * P.npix * sizeof(float));
    const dim3 gr((unsigned)((nrec + 255) / 256));
    if (P.lr)
        hipLaunchKernelGGL(k_iv_records<1>, gr, dim3(256), 0, nullptr, P, h->t, v->n_slots, v->rec);
    else
        hipLaunchKernelGGL(k_iv_records<0>, gr, dim3(256), 0, nullptr, P, h->t, v->n_slots, v->rec);
    int npow2 = 1;
    while (npow2 < v->n_slots) npow2 *= 2;
    hipLaunchKernelGGL(k_iv_rank, dim3(P.n_groups), dim3(1024), npow2 * 4, nullptr, v->n_slots, npow2, v->rec, nq, ne,
                       (const uint16_t *)v->pp, v->bpos);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return bail(csx_fail(CSX_EHIP, std::string("interval set-up: ") + hipGetErrorString(e)));
        const hipError_t e2 = hipDeviceSynchronize();
        if (e2 != hipSuccess) return bail(csx_fail(CSX_EHIP, std::string("interval set-up: ") + hipGetErrorString(e2)));
    }
    v->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    h->bytes += v->bytes;
    h->iv = v;
    return CSX_OK;
}

csx_status csx_iv_forward(const csx_geometry *h, const float *f, float *part, size_t part_cap, float *g,
                          hipStream_t s)
{
    const IvState *v = (const IvState *)h->iv;
    if (!part) part = v->part;
    else if ((size_t)v->nblk_f * h->P.npix > part_cap) return csx_fail(CSX_EINVAL, "forward partials exceed the buffer");
    const IvArgs a = iv_args(h, v);
    const dim3 grid(v->nblk_f), block(IV_THREADS);
#define CSX_IVF(LR_, NP_) \
    hipLaunchKernelGGL((k_iv_forward<LR_, NP_>), grid, block, v->lds_f, s, h->P, a, f, part)
    if (h->P.lr) {
        if (v->np == 1) CSX_IVF(1, 1);
        else if (v->np == 2) CSX_IVF(1, 2);
        else if (v->np == 4) CSX_IVF(1, 4);
        else CSX_IVF(1, 8);
    } else {
        if (v->np == 1) CSX_IVF(0, 1);
        else if (v->np == 2) CSX_IVF(0, 2);
        else if (v->np == 4) CSX_IVF(0, 4);
        else CSX_IVF(0, 8);
    }
#undef CSX_IVF
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_iv_sum, dim3((h->P.npix + 63) / 64), dim3(1024), 0, s, (const float *)part, v->nblk_f,
                       h->P.npix, g);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_iv_adjoint(const csx_geometry *h, const float *rho, float *b, hipStream_t s)
{
    const IvState *v = (const IvState *)h->iv;
    const IvArgs a = iv_args(h, v);
    const dim3 grid(v->nblk_a), block(IVA_THREADS);
    const bool pf = h->P.nq <= IVA_THREADS / IVA_SUB && h->P.ne <= (IVA_MAXV - 1) * IVA_SUB;
#define CSX_IVA(LR_, NP_)                                                                                     \
    do {                                                                                                      \
        if (pf)                                                                                               \
            hipLaunchKernelGGL((k_iv_adjoint<LR_, NP_, 1>), grid, block, v->lds_a, s, h->P, a, h->t, rho, b); \
        else                                                                                                  \
            hipLaunchKernelGGL((k_iv_adjoint<LR_, NP_, 0>), grid, block, v->lds_a, s, h->P, a, h->t, rho, b); \
    } while (0)
    if (h->P.lr) {
        if (v->npa == 1) CSX_IVA(1, 1);
        else if (v->npa == 2) CSX_IVA(1, 2);
        else CSX_IVA(1, 4);
    } else {
        if (v->npa == 1) CSX_IVA(0, 1);
        else if (v->npa == 2) CSX_IVA(0, 2);
        else if (v->npa == 4) CSX_IVA(0, 4);
        else CSX_IVA(0, 8);
    }
#undef CSX_IVA
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

size_t csx_iv_part_floats(const csx_geometry *h)
{
    const IvState *v = (const IvState *)h->iv;
    return v ? (size_t)v->nblk_f * h->P.npix : 0;
}

void csx_iv_info(const csx_geometry *h, int *on, int64_t *bytes, double *build_ms, int *intervals)
{
    const IvState *v = (const IvState *)h->iv;
    if (on) *on = v ? 1 : 0;
    if (bytes) *bytes = v ? v->bytes : 0;
    if (build_ms) *build_ms = v ? v->build_ms : 0.0;
    if (intervals) *intervals = v ? v->nt + 1 : 0;
}
