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

// Blocks have up to 1024 threads (the register budget is set for that); the
// launch takes the smallest of 256, 512, 1024 that covers a voxel group's
// work, so that with small detectors several blocks share a compute unit.
constexpr int IV_THREADS = 1024;
constexpr int IV_WAVES = IV_THREADS / 64;
constexpr int IVA_THREADS = 1024;
constexpr int IVA_WAVES = IVA_THREADS / 64;
constexpr int IVA_SC = 8;                                // ranks per adjoint thread
constexpr int IVA_SUB = 8;                               // adjoint gather threads per node
constexpr int IVA_NW = IVA_SC * IVA_THREADS / 32 + 1;    // words of a position bitmap (0 .. 8192)

struct IvState {
    uint2 *rec = nullptr;       // [n_groups][n_slots] {A bits, w}, slot order (forward)
    uint2 *reca = nullptr;      // [n_groups][rstride] {A bits, mask bits | slot << 4}, interval order (adjoint)
    double *coef = nullptr;     // [nt] q_m (Phi~[c] - Phi~[c-1]) of the sorted thresholds
    uint16_t *mt = nullptr;     // [nt] node m of each sorted threshold
    uint16_t *pp = nullptr;     // [nq][ne + 2] pos(c, m) + 1, c = 1 .. ne + 1
    uint16_t *emap = nullptr;   // [n_groups][nq][es] prefix-table index of P(m, c), entry c - 1
    uint8_t *emask = nullptr;   // [n_groups][nch] bit i of byte k: position 8 k + i is in the prefix table
    int *cnt = nullptr;         // [1] largest prefix-table size over the groups (set-up)
    double *qd = nullptr;       // [nq] q nodes
    float *part = nullptr;      // [nblk][npix] forward partial images
    int nt = 0;                 // thresholds, (ne + 1) nq
    int n_slots = 0;            // classes per voxel group (LR: 2 per mirror pair)
    int n_items = 0;            // work items per group: mirror pairs (LR) or classes
    int rstride = 0;            // adjoint records per group, n_slots rounded up to a chunk
    int nch = 0;                // rank chunks per group, rstride / IVA_SC
    int es = 0;                 // emap entries per node (ne + 1 rounded up to 8)
    int cap = 0;                // prefix-table entries between the two fixed ones (largest group)
    int ncell = 0;              // detector cells of the upper half (columns x rows)
    int np = 1;                 // forward: work items per thread (power of 2, <= 8)
    int th_f = 0, th_a = 0;     // threads per block of the forward and the adjoint
    int cus = 256;              // compute units of the device
    int nblk_f = 0, nblk_a = 0;
    int lds_f = 0, lds_a = 0;
    int64_t bytes = 0;
    double build_ms = 0.0;
};

struct IvArgs {
    const uint2 *rec;
    const uint2 *reca;
    const double *coef;
    const uint16_t *mt;
    const uint16_t *emap;
    const uint8_t *emask;
    const double *qd;
    int nt, n_slots, n_items, ngroups, rstride, nch, es, cap, ncell;
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

// The adjoint's tables of one voxel group, one block per group:
//  - the rank of every class in the order of (t, slot), by a bitonic sort of
//    the keys (t << 14 | slot) in LDS, and the records in that order,
//    reca[rank] = {A, i_j | i_j2 << 15}: for voxel j and (LR) j2 the index of
//    the class's detector term in the adjoint's per-call table of three
//    entries per detector cell (column, upper row) -- 3 cell + 0 for the
//    upper pixel alone, + 1 for the lower one, + 2 for both, as the mask
//    values select -- or 3 ncell, a zero entry, when both pairs are closed;
//    past n_slots, A = 0 and both indices 3 ncell;
//  - for node m and bin edge c = 1 .. ne + 1 the position P(m, c), the rank
//    of the first class whose t reaches pp(c, m) = pos(c, m) + 1 (so the
//    classes in bin c at node m are the ranks [P(m, c), P(m, c + 1)));
//  - the prefix table the adjoint keeps for the group: entry 0 is the empty
//    prefix (P = 0), entry 1 the total (P = n_slots), entries 2, 3, ... the
//    distinct positions strictly between, ascending.  emap holds each
//    P(m, c) as its table entry (row stride es, zero past c = ne + 1), and
//    emask bit i of byte k marks position 8 k + i as one of the entries.
// cnt receives the largest number of in-between entries over the groups.
template <int LR>
__global__ void __launch_bounds__(1024) k_iv_rank(KParams P, int n_slots, int npow2, int rstride, const uint2 *__restrict__ rec,
                                                  uint2 *__restrict__ reca, int nq, int ne, int es, int nch,
                                                  const uint16_t *__restrict__ pp, uint16_t *__restrict__ emap,
                                                  uint8_t *__restrict__ emask, int *__restrict__ cnt)
{
    extern __shared__ uint32_t keys[];        // [npow2], then the positions [nt] as uint16
    __shared__ uint32_t s_bits[IVA_NW];
    __shared__ uint32_t s_pre[IVA_NW];
    const int nt = (ne + 1) * nq;
    uint16_t *s_P = (uint16_t *)(keys + npow2);
    const uint2 *rg = rec + (size_t)blockIdx.x * n_slots;
    for (int i = threadIdx.x; i < npow2; i += blockDim.x)
        keys[i] = i < n_slots ? (((rg[i].y >> 4) & 0x3FFFu) << 14) | (uint32_t)i : 0xFFFFFFFFu;
    for (int w = threadIdx.x; w < IVA_NW; w += blockDim.x) s_bits[w] = 0u;
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
    uint2 *ra = reca + (size_t)blockIdx.x * rstride;
    const uint32_t Z = 3u * (uint32_t)(P.ndx * (P.ndy / 2));
    for (int r = threadIdx.x; r < rstride; r += blockDim.x) {
        uint2 v = make_uint2(0u, Z | (Z << 15));
        if (r < n_slots) {
            const uint32_t sl = keys[r] & 0x3FFFu;
            const uint2 x = rg[sl];
            const uint32_t bits = x.y & 0xFu;
            // slot 2p is column a of item p, slot 2p + 1 its mirror column
            int a, row;
            item_class(P, LR, LR ? (int)(sl >> 1) : (int)sl, LR ? (int)(sl & 1u) : 0, a, row);
            auto term = [&](uint32_t up, uint32_t dn, int col) -> uint32_t {
                if (!up && !dn) return Z;
                return 3u * (uint32_t)(row * P.ndx + col) + (up ? (dn ? 2u : 0u) : 1u);
            };
            const uint32_t i0 = term(bits & 1u, (bits >> 1) & 1u, a);
            const uint32_t i1 = LR ? term((bits >> 2) & 1u, (bits >> 3) & 1u, P.ndx - 1 - a) : Z;
            v = make_uint2(x.x, i0 | (i1 << 15));
        }
        ra[r] = v;
    }
    for (int k = threadIdx.x; k < nt; k += blockDim.x) {
        const int m = k / (ne + 1), c = 1 + k % (ne + 1);
        const uint32_t T = pp[(size_t)m * (ne + 2) + c];
        int lo = 0, hi = n_slots;          // first sorted position with t >= T
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((keys[mid] >> 14) < T) lo = mid + 1;
            else hi = mid;
        }
        s_P[k] = (uint16_t)lo;
        if (lo > 0 && lo < n_slots) atomicOr(&s_bits[lo >> 5], 1u << (lo & 31));
    }
    __syncthreads();
    // table entries before each bitmap word: one wave, 5 words per lane
    if (threadIdx.x < 64) {
        constexpr int WPL = (IVA_NW + 63) / 64;
        const int lane = threadIdx.x;
        int before[WPL], sum = 0;
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            const int w = lane * WPL + i;
            before[i] = sum;
            sum += w < IVA_NW ? __popc(s_bits[w]) : 0;
        }
        int incl = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl, d, 64);
            if (lane >= d) incl += u;
        }
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            const int w = lane * WPL + i;
            if (w < IVA_NW) s_pre[w] = (uint32_t)(incl - sum + before[i]);
        }
        if (lane == 63) atomicMax(cnt, incl);
    }
    __syncthreads();
    uint16_t *eg = emap + (size_t)blockIdx.x * nq * es;
    for (int k = threadIdx.x; k < nq * es; k += blockDim.x) {
        const int m = k / es, e = k % es;     // e = c - 1
        uint32_t v = 0u;
        if (e <= ne) {
            const uint32_t P = s_P[m * (ne + 1) + e];
            if (P >= (uint32_t)n_slots) v = 1u;
            else if (P > 0u) v = 2u + s_pre[P >> 5] + __popc(s_bits[P >> 5] & ((1u << (P & 31u)) - 1u));
        }
        eg[k] = (uint16_t)v;
    }
    uint8_t *mg = emask + (size_t)blockIdx.x * nch;
    for (int k = threadIdx.x; k < nch; k += blockDim.x) mg[k] = (uint8_t)(s_bits[k >> 2] >> (8 * (k & 3)));
}

// ---------------------------------------------------------------------------
// Wave-level scans and sums through DPP lane moves (row shifts within rows of
// 16 lanes, then the row broadcasts of lanes 15 and 31), so that no step
// waits on an LDS permute.  Lanes without a source add zero.  The order of
// the additions is fixed, so results are reproducible.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}

constexpr int DPP_SHR1 = 0x111, DPP_SHR2 = 0x112, DPP_SHR4 = 0x114, DPP_SHR8 = 0x118;
constexpr int DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_ROW_MIRROR = 0x140;

// a lane move over all rows whose lanes without a source read zero
template <int CTRL>
__device__ __forceinline__ double dppz_f64(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// inclusive scan within each row of 16 lanes
__device__ __forceinline__ double row_scan(double x)
{
    x += dppz_f64<DPP_SHR1>(x);
    x += dppz_f64<DPP_SHR2>(x);
    x += dppz_f64<DPP_SHR4>(x);
    x += dppz_f64<DPP_SHR8>(x);
    return x;
}

__device__ __forceinline__ int row_scan(int x)
{
    x += dpp_i32<DPP_SHR1, 0xf>(x);
    x += dpp_i32<DPP_SHR2, 0xf>(x);
    x += dpp_i32<DPP_SHR4, 0xf>(x);
    x += dpp_i32<DPP_SHR8, 0xf>(x);
    return x;
}

// inclusive scan over the 64 lanes of a wave
__device__ __forceinline__ double wave_scan(double x)
{
    x = row_scan(x);
    x += dpp_f64<DPP_BCAST15, 0xa>(x);
    x += dpp_f64<DPP_BCAST31, 0xc>(x);
    return x;
}

__device__ __forceinline__ int wave_scan(int x)
{
    x = row_scan(x);
    x += dpp_i32<DPP_BCAST15, 0xa>(x);
    x += dpp_i32<DPP_BCAST31, 0xc>(x);
    return x;
}

// sum over each group of 8 (W = 8) or 16 (W = 16) lanes, every lane of the
// group getting it
template <int W>
__device__ __forceinline__ double group_sum(double x)
{
    x += dppz_f64<DPP_XOR1>(x);
    x += dppz_f64<DPP_XOR2>(x);
    x += dppz_f64<DPP_HALF_MIRROR>(x);
    if (W == 16) x += dppz_f64<DPP_ROW_MIRROR>(x);
    return x;
}

__device__ __forceinline__ double read_lane(double v, int l)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum of the first wv of 16 values held by lanes 0 .. 15 of every row (v =
// value of wave lane & 15): a row scan, then lane wv - 1 read as a scalar.
__device__ __forceinline__ double sum_below(double v, int wv)
{
    const double s = row_scan(v);
    return wv > 0 ? read_lane(s, wv - 1) : 0.0;
}

__device__ __forceinline__ int sum_below(int v, int wv)
{
    const int s = row_scan(v);
    return wv > 0 ? __builtin_amdgcn_readlane(s, wv - 1) : 0;
}

// ---------------------------------------------------------------------------
// Forward: g = A f.  Block = TH <= IV_THREADS threads, a contiguous range of
// voxel groups; thread k owns work items k, k + TH, ... (NP of them) and
// keeps their pixels' sums in registers; partial image per block.
// ---------------------------------------------------------------------------
template <int LR, int NP, int TPM>
__global__ void __launch_bounds__(IV_THREADS) k_iv_forward(KParams P, IvArgs V, const float *__restrict__ f,
                                                           float *__restrict__ part)
{
    extern __shared__ __align__(16) unsigned char lds[];
    double *s_coef = (double *)lds;
    uint16_t *s_mt = (uint16_t *)(s_coef + V.nt);
    const size_t fst = ((size_t)(V.nt + 1) * 8 + 15) & ~(size_t)15;                   // bytes per F table
    float2 *s_F0 = (float2 *)(lds + (((size_t)V.nt * 10 + 15) & ~(size_t)15));      // [2][nt + 1]
    double *s_f = (double *)((unsigned char *)s_F0 + 2 * fst);                       // [2][2 nq]
    double2 *s_tot = (double2 *)(s_f + 4 * P.nq);                                    // [IV_WAVES]
    auto s_F = [&](int g) { return (float2 *)((unsigned char *)s_F0 + (g & 1) * fst); };
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int TH = blockDim.x;
    for (int i = tid; i < V.nt; i += TH) {
        s_coef[i] = V.coef[i];
        s_mt[i] = V.mt[i];
    }
    // groups of this block
    const int per = (V.ngroups + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(V.ngroups, g0 + per);
    // thresholds of this thread in the scan (at most TPM)
    const int tper = (V.nt + TH - 1) / TH;
    const int t0 = min(V.nt, tid * tper), t1 = min(V.nt, t0 + tper);

    constexpr int NO = LR ? 4 : 2;
    float o[NP][NO];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int k = 0; k < NO; ++k) o[i][k] = 0.0f;
    // records of the thread's items; group g + 1 is loaded (clamped to the
    // block's last group, items clamped to the last one) into the register
    // set that group g does not use
    auto load_rec = [&](int g, uint4 (&r)[NP]) {
        const uint2 *rg = V.rec + (size_t)min(g, g1 - 1) * V.n_slots;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int p = min(tid + i * TH, V.n_items - 1);
            if (LR) {
                r[i] = *(const uint4 *)(rg + 2 * p);
            } else {
                const uint2 v = rg[p];
                r[i] = make_uint4(v.x, v.y, 0u, 0u);
            }
        }
    };
    // thread i < 2 nq carries f of a group's voxel j (i < nq) or j2; the
    // values of group g sit in s_f[g & 1] (float64)
    auto load_f = [&](int g) -> float {
        if (tid >= 2 * P.nq || g >= g1) return 0.0f;
        int j, j2;
        group_voxels(P, LR, g, j, j2);
        if (tid < P.nq) return f[(size_t)j * P.nq + tid];
        return LR ? f[(size_t)j2 * P.nq + tid - P.nq] : 0.0f;
    };
    // F tables of group g's voxels j and j2: float64 prefix sums over the
    // sorted thresholds, in two parts around a barrier.  Part 1: the thread's
    // local sums (with at most 5 thresholds per thread their prefixes stay
    // in registers) and the wave scan of the sums, wave totals to s_tot.
    constexpr int KEEP = TPM <= 5;
    constexpr int UNR = TPM > 5 ? 4 : TPM;
    double la[KEEP ? TPM : 1], lb[KEEP ? TPM : 1];
    double sa = 0.0, sb = 0.0, ia = 0.0, ib = 0.0;
    auto scan1 = [&](int g) {
        const double *sf = s_f + (g & 1) * 2 * P.nq;
        sa = sb = 0.0;
#pragma unroll UNR
        for (int k = 0; k < TPM; ++k) {
            const bool in = t0 + k < t1;
            const double c = in ? s_coef[t0 + k] : 0.0;
            const int m = in ? (int)s_mt[t0 + k] : 0;
            sa = fma(c, sf[m], sa);
            sb = fma(c, sf[P.nq + m], sb);
            if constexpr (KEEP) {
                la[k] = sa;
                lb[k] = sb;
            }
        }
        ia = wave_scan(sa);
        ib = wave_scan(sb);
        if (lane == 63) s_tot[wv] = make_double2(ia, ib);
    };
    // Part 2 (after the barrier): the totals of the waves below, then F at
    // every threshold of the thread into s_F(g).
    auto scan2 = [&](int g) {
        const double2 t = s_tot[lane & 15];
        const double ba = sum_below(t.x, wv) + (ia - sa), bb = sum_below(t.y, wv) + (ib - sb);
        float2 *F = s_F(g);
        if constexpr (KEEP) {
#pragma unroll
            for (int k = 0; k < TPM; ++k)
                if (t0 + k < t1) F[t0 + k + 1] = make_float2((float)(ba + la[k]), (float)(bb + lb[k]));
        } else {
            const double *sf = s_f + (g & 1) * 2 * P.nq;
            double ra = 0.0, rb = 0.0;
#pragma unroll UNR
            for (int k = 0; k < TPM; ++k) {
                const bool in = t0 + k < t1;
                const double c = in ? s_coef[t0 + k] : 0.0;
                const int m = in ? (int)s_mt[t0 + k] : 0;
                ra = fma(c, sf[m], ra);
                rb = fma(c, sf[P.nq + m], rb);
                if (in) F[t0 + k + 1] = make_float2((float)(ba + ra), (float)(bb + rb));
            }
        }
        if (tid == 0) F[0] = make_float2(0.0f, 0.0f);
    };
    // One group per barrier pair: group g's class reads and the first scan
    // part of group g + 1 share an interval, the second part and the f values
    // of group g + 2 the next one.  F tables and f values are double-buffered
    // by group parity; each buffer is rewritten two barriers after its last read.
    auto group = [&](int g, const uint4 (&cr)[NP], uint4 (&nr)[NP], float &fv) {
        load_rec(g + 1, nr);
        const float2 *F = s_F(g);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            // class of column a (record x, y) and, with LR, of column ndx-1-a (z, w)
            const float A1 = __uint_as_float(cr[i].x);
            const uint32_t w1 = cr[i].y;
            const float2 F1 = F[(w1 >> 4) & 0x3FFFu];
            const float a1 = A1 * F1.x;
            o[i][0] = fmaf(a1, (float)(w1 & 1u), o[i][0]);           // (a, u) <- voxel j
            o[i][1] = fmaf(a1, (float)((w1 >> 1) & 1u), o[i][1]);    // (a, d) <- voxel j
            if (LR) {
                const float b1 = A1 * F1.y;
                o[i][2] = fmaf(b1, (float)((w1 >> 2) & 1u), o[i][2]);    // (-a, u) <- voxel j2
                o[i][3] = fmaf(b1, (float)((w1 >> 3) & 1u), o[i][3]);    // (-a, d) <- voxel j2
                const float A2 = __uint_as_float(cr[i].z);
                const uint32_t w2 = cr[i].w;
                const float2 F2 = F[(w2 >> 4) & 0x3FFFu];
                const float a2 = A2 * F2.x, b2 = A2 * F2.y;
                o[i][2] = fmaf(a2, (float)(w2 & 1u), o[i][2]);           // (-a, u) <- voxel j
                o[i][3] = fmaf(a2, (float)((w2 >> 1) & 1u), o[i][3]);    // (-a, d) <- voxel j
                o[i][0] = fmaf(b2, (float)((w2 >> 2) & 1u), o[i][0]);    // (a, u) <- voxel j2
                o[i][1] = fmaf(b2, (float)((w2 >> 3) & 1u), o[i][1]);    // (a, d) <- voxel j2
            }
        }
        const bool more = g + 1 < g1;
        if (more) scan1(g + 1);
        __syncthreads();
        if (more) scan2(g + 1);
        if (tid < 2 * P.nq) s_f[(g & 1) * 2 * P.nq + tid] = (double)fv;   // group g + 2
        fv = load_f(g + 3);
        __syncthreads();
    };
    if (g0 < g1) {
        if (tid < 2 * P.nq) {
            s_f[(g0 & 1) * 2 * P.nq + tid] = (double)load_f(g0);
            s_f[((g0 + 1) & 1) * 2 * P.nq + tid] = (double)load_f(g0 + 1);
        }
        float fv = load_f(g0 + 2);
        uint4 ra[NP], rb[NP];
        load_rec(g0, ra);
        __syncthreads();
        scan1(g0);
        __syncthreads();
        scan2(g0);
        __syncthreads();
        for (int g = g0; g < g1; g += 2) {
            group(g, ra, rb, fv);
            if (g + 1 < g1) group(g + 1, rb, ra, fv);
        }
    }
    // partial image of this block: every pixel is written once
    float *dst = part + (size_t)blockIdx.x * P.npix;
    const int half_y = P.ndy / 2;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int p = tid + i * TH;
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
// together, then the 16 slice sums added in slice order.  bx: the block.
__device__ __forceinline__ void iv_sum_body(const float *__restrict__ part, int nparts, int n, float *__restrict__ g,
                                            int bx, float (*s_part)[64])
{
    const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int i = bx * 64 + lane;
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

__global__ void __launch_bounds__(1024) k_iv_sum(const float *__restrict__ part, int nparts, int n,
                                                 float *__restrict__ g)
{
    __shared__ float s_part[16][64];
    iv_sum_body(part, nparts, n, g, blockIdx.x, s_part);
}

// The same for the jobs of a batch: block b belongs to the job whose block
// range [begin[k], begin[k + 1]) holds it.
__global__ void __launch_bounds__(1024) k_iv_sum_batch(const ElemJob *__restrict__ jobs, const int *__restrict__ begin,
                                                       int njobs)
{
    __shared__ float s_part[16][64];
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const ElemJob &J = jobs[lo];
    iv_sum_body(J.part, J.nparts, J.npix, J.g, (int)blockIdx.x - begin[lo], s_part);
}

// ---------------------------------------------------------------------------
// Adjoint: b = A^T rho.  Blocks of TH <= IVA_THREADS threads (one per compute
// unit at 128^2),
// a contiguous range of voxel groups, one group at a time, two barriers per
// group:
//  A. thread k reads the records of ranks 8k .. 8k + 7 of the group (their
//     interval order, stored so at set-up), looks up the detector values of
//     each class's pixels in LDS and forms the class's weights for voxels j
//     and j2 (A (T_u rho_u + T_d rho_d), float32 as in the direct kernels),
//     then their exclusive prefix sums within the chunk in float64
//     registers; a wave scan gives the chunk's offset within its wave;
//  B. after the wave totals are in LDS, each thread adds the totals of the
//     waves below and writes the prefix E(p) = sum of the weights of ranks
//     < p at the positions p of its chunk that some (node, bin) edge needs,
//     into a compact table (entry 0: E = 0, entry 1: the total);
//  C. the classes in bin c at node m are the ranks [P(m, c), P(m, c + 1)), so
//     b_jm = q_m sum_c Phi~[c] (E(P(m, c + 1)) - E(P(m, c))), IVA_SUB threads
//     per node, the table indices of P loaded one group ahead.
// The prefix sums are float64 end to end: a bin's sum is a difference of two
// prefixes, and a bin holding only a few small weights behind large ones
// (the lowest q nodes see only the smallest angles) needs that precision to
// stay accurate relative to itself.
// PF = 1 (nq <= 128, ne <= 64): thread (m, sub), sub < 8, owns bins
// c = 1 + 8 sub .. 8 + 8 sub of node m; PF = 2 (nq <= 64, ne <= 64): 16
// threads per node, 4 bins each, so that every wave takes part.  A thread
// holds the table indices of its bins' edges in registers (rows of es = 72
// entries, loaded one group ahead).  PF = 0: 8 threads per node walk the
// bins with stride 8, indices read when used.
template <int LR, int PF>
__global__ void __launch_bounds__(IVA_THREADS) k_iv_adjoint(KParams P, IvArgs V, const DevTables T,
                                                            const float *__restrict__ rho, float *__restrict__ b)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const size_t ntab = ((size_t)V.ncell * 3 + 1) * sizeof(float);
    float *s_tab = (float *)lds;                                     // [3 ncell + 1]
    double2 *s_E = (double2 *)(lds + ((ntab + 15) & ~(size_t)15));   // [2 + cap]
    double2 *s_wt = s_E + 2 + V.cap;                                 // [IVA_WAVES]
    int *s_wc = (int *)(s_wt + IVA_WAVES);                           // [IVA_WAVES]
    double *s_phi = (double *)(s_wc + IVA_WAVES);                    // [nphi]
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nphi = max(P.ne + 2, IVA_SC * IVA_SUB + 2);
    const int TH = blockDim.x;
    for (int k = tid; k < nphi; k += TH)
        s_phi[k] = k >= P.ne + 2 ? 0.0 : (double)(P.td == CSX_TABLE_BF16 ? bf16_to_f32(T.phi16[k]) : T.phi32[k]);
    // detector terms of every cell (column, upper row): rho_u, rho_d and
    // rho_u + rho_d, the same for every group; then the zero entry
    const int half_y = P.ndy / 2;
    for (int c = tid; c < V.ncell; c += TH) {
        const int col = c % P.ndx, bu = half_y + c / P.ndx, bd = P.ndy - 1 - bu;
        const float u = rho[bu * P.ndx + col], d = rho[bd * P.ndx + col];
        s_tab[3 * c] = u;
        s_tab[3 * c + 1] = d;
        s_tab[3 * c + 2] = u + d;
    }
    if (tid == 0) s_tab[3 * V.ncell] = 0.0f;
    if (tid == 0) s_E[0] = make_double2(0.0, 0.0);
    const int per = (V.ngroups + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(V.ngroups, g0 + per);
    if (g0 >= g1) return;
    // records and position bits of the thread's chunk; a thread past the
    // last chunk reads the last one and contributes nothing.  Group g + 1 is
    // loaded (clamped to the block's last group) into the register set that
    // group g does not use.
    const bool own = tid < V.nch;
    const int ch = own ? tid : V.nch - 1;
    auto load_chunk = [&](int g, uint4 (&r)[IVA_SC / 2], uint32_t &m) {
        const int gg = min(g, g1 - 1);
        const uint4 *src = (const uint4 *)(V.reca + (size_t)gg * V.rstride + (size_t)ch * IVA_SC);
#pragma unroll
        for (int i = 0; i < IVA_SC / 2; ++i) r[i] = src[i];
        m = V.emask[(size_t)gg * V.nch + ch];
    };
    // PF: this thread's node and bins, and the table indices of their edges
    constexpr int PSUB = PF == 2 ? 16 : IVA_SUB, PCPT = PF == 2 ? 4 : IVA_SC;
    const int pm = tid / PSUB, ps = tid % PSUB;
    const bool pact = PF && pm < P.nq;
    uint32_t ew[PCPT / 2] = {};
    uint32_t elast = 0u;
    auto load_emap = [&](int g) {
        if (PF && pact) {
            const uint16_t *row = V.emap + ((size_t)min(g, g1 - 1) * P.nq + pm) * V.es + ps * PCPT;
            if constexpr (PCPT == 8) {
                const uint4 v = *(const uint4 *)row;
                ew[0] = v.x;
                ew[1] = v.y;
                ew[2] = v.z;
                ew[3] = v.w;
            } else {
                const uint2 v = *(const uint2 *)row;
                ew[0] = v.x;
                ew[1] = v.y;
            }
            elast = row[PCPT];
        }
    };
    auto group = [&](int g, const uint4 (&cr)[IVA_SC / 2], uint32_t cm, uint4 (&nr)[IVA_SC / 2], uint32_t &nm) {
        int j, j2;
        group_voxels(P, LR, g, j, j2);
        load_chunk(g + 1, nr, nm);
        // A. weights of the chunk's classes and their prefixes within the chunk
        const uint32_t msk = own ? cm : 0u;
        double2 loc[IVA_SC];
        double la = 0.0, lb = 0.0;
#pragma unroll
        for (int i = 0; i < IVA_SC; ++i) {
            loc[i] = make_double2(la, lb);
            const float A = __uint_as_float((i & 1) ? cr[i >> 1].z : cr[i >> 1].x);
            const uint32_t w = (i & 1) ? cr[i >> 1].w : cr[i >> 1].y;
            // A (T_u rho_u + T_d rho_d) through the cell table, as the direct
            // kernels form it: the entry is rho_u, rho_d or their float32 sum
            const float c0 = A * s_tab[w & 0x7FFFu];
            const float c1 = LR ? A * s_tab[w >> 15] : 0.0f;
            la += (double)c0;
            lb += (double)c1;
        }
        if (!own) la = lb = 0.0;
        const int cn = __popc(msk);
        const double ia = wave_scan(la), ib = wave_scan(lb);
        const int ic = wave_scan(cn);
        if (lane == 63) {
            s_wt[wv] = make_double2(ia, ib);
            s_wc[wv] = ic;
        }
        __syncthreads();
        // B. prefixes at the chunk's table positions
        {
            const double2 t = s_wt[lane & 15];
            const int tc = s_wc[lane & 15];
            const double oa = sum_below(t.x, wv), ob = sum_below(t.y, wv);
            const int oc = sum_below(tc, wv);
            const double ba = oa + (ia - la), bb = ob + (ib - lb);
            int ci = 2 + oc + (ic - cn);
#pragma unroll
            for (int i = 0; i < IVA_SC; ++i)
                if ((msk >> i) & 1u) {
                    s_E[ci] = make_double2(ba + loc[i].x, bb + loc[i].y);
                    ++ci;
                }
            if (tid == TH - 1) s_E[1] = make_double2(oa + ia, ob + ib);
        }
        __syncthreads();
        // C. b_jm = q_m sum_c Phi~[c] (E(P(m, c + 1)) - E(P(m, c)))
        if constexpr (PF) {
            double sa = 0.0, sb = 0.0;
            if (pact) {
                double2 E[PCPT + 1];
#pragma unroll
                for (int k = 0; k < PCPT; ++k) E[k] = s_E[(ew[k >> 1] >> (16 * (k & 1))) & 0xFFFFu];
                E[PCPT] = s_E[elast];
#pragma unroll
                for (int k = 0; k < PCPT; ++k) {
                    const double ph = s_phi[1 + ps * PCPT + k];
                    sa = fma(ph, E[k + 1].x - E[k].x, sa);
                    sb = fma(ph, E[k + 1].y - E[k].y, sb);
                }
            }
            sa = group_sum<PSUB>(sa);
            sb = group_sum<PSUB>(sb);
            if (pact && ps == 0) {
                const double qm = V.qd[pm];
                b[(size_t)j * P.nq + pm] = (float)(qm * sa);
                if (LR) b[(size_t)j2 * P.nq + pm] = (float)(qm * sb);
            }
            load_emap(g + 1);   // used after the next group's two barriers
        } else {
            for (int mb = 0; mb < P.nq; mb += TH / IVA_SUB) {
                const int m = mb + tid / IVA_SUB, sub = tid % IVA_SUB;
                double sa = 0.0, sb = 0.0;
                if (m < P.nq) {
                    const uint16_t *em = V.emap + ((size_t)g * P.nq + m) * V.es;   // em[c - 1]: edge c
                    for (int c = 1 + sub; c <= P.ne; c += IVA_SUB) {
                        const double ph = s_phi[c];
                        const double2 hi = s_E[em[c]], lo = s_E[em[c - 1]];
                        sa = fma(ph, hi.x - lo.x, sa);
                        sb = fma(ph, hi.y - lo.y, sb);
                    }
                }
                sa = group_sum<IVA_SUB>(sa);
                sb = group_sum<IVA_SUB>(sb);
                if (m < P.nq && sub == 0) {
                    const double qm = V.qd[m];
                    b[(size_t)j * P.nq + m] = (float)(qm * sa);
                    if (LR) b[(size_t)j2 * P.nq + m] = (float)(qm * sb);
                }
            }
        }
        // the next group's phase B overwrites s_E only after its first barrier,
        // and its phase A writes s_wt only after this group's second one
    };
    uint4 ra[IVA_SC / 2], rb[IVA_SC / 2];
    uint32_t ma = 0u, mb = 0u;
    load_chunk(g0, ra, ma);
    load_emap(g0);
    __syncthreads();
    for (int g = g0; g < g1; g += 2) {
        group(g, ra, ma, rb, mb);
        if (g + 1 < g1) group(g + 1, rb, mb, ra, ma);
    }
}

IvArgs iv_args(const csx_geometry *h, const IvState *v)
{
    IvArgs a;
    a.rec = v->rec;
    a.reca = v->reca;
    a.coef = v->coef;
    a.mt = v->mt;
    a.emap = v->emap;
    a.emask = v->emask;
    a.qd = v->qd;
    a.nt = v->nt;
    a.n_slots = v->n_slots;
    a.n_items = v->n_items;
    a.ngroups = h->P.n_groups;
    a.rstride = v->rstride;
    a.nch = v->nch;
    a.es = v->es;
    a.cap = v->cap;
    a.ncell = v->ncell;
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
    void *ps[] = {v->rec, v->reca, v->coef, v->mt, v->pp, v->emap, v->emask, v->cnt, v->qd, v->part};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete v;
}

// The adjoint's gather form for blocks of th threads: 2 (16 threads of 4
// bins per node), 1 (8 threads of 8 bins) or 0 (8 threads, bins with stride
// 8, nodes in passes of th / 8).
int iva_pf(const KParams &P, int th)
{
    if (P.ne > IVA_SC * IVA_SUB) return 0;
    if (P.nq <= th / 16) return 2;
    return P.nq <= th / IVA_SUB ? 1 : 0;
}

// Blocks of a launch over n groups: as many as the compute units hold at
// once (by threads and by LDS), each taking a contiguous range of groups.
int iv_blocks(int n, int cus, int th, int lds)
{
    const int per_cu = std::max(1, std::min(IV_THREADS / th, (int)(CSX_LDS_MAX / std::max(lds, 1))));
    const int per = (n + cus * per_cu - 1) / (cus * per_cu);
    return (n + per - 1) / per;
}

// Block sizes: the smallest of 256, 512, 1024 threads that covers a group's
// rank chunks (adjoint) or its work items at <= 4 (LR) or 8 per thread, its
// f values and <= 8 thresholds per thread (forward).
int iva_threads(long nch)
{
    for (int th = 256; th <= IVA_THREADS; th *= 2)
        if (nch <= th) return th;
    return 0;
}

int iv_threads(const KParams &P, long items, long nt)
{
    const long npmax = P.lr ? 4 : 8;
    for (int th = 256; th <= IV_THREADS; th *= 2)
        if (items <= npmax * th && 2L * P.nq <= th && nt <= 8L * th) return th;
    return IV_THREADS;
}

// LDS of the adjoint with a prefix table of cap in-between entries: the
// cell table, the prefix table, wave totals and the float64 spectrum.
long iva_lds(const KParams &P, long cap)
{
    const long cells = (long)P.ndx * (P.ndy / 2);
    return (((cells * 3 + 1) * 4 + 15) & ~15L) + (2 + cap) * 16 + IVA_WAVES * 16 + IVA_WAVES * 4 +
           (long)std::max(P.ne + 2, IVA_SC * IVA_SUB + 2) * 8;
}

}  // namespace

// Feasibility of the interval operators for a geometry: thresholds and ranks
// in 14 bits, and both kernels' LDS within one workgroup's budget (the
// adjoint's with an empty prefix table; the set-up checks the real one).
bool csx_iv_feasible(const KParams &P, int *lds_f, int *lds_a)
{
    const long nt = (long)(P.ne + 1) * P.nq;
    const long items = P.lr ? (long)(P.ndx / 2) * (P.ndy / 2) : (long)P.ndx * (P.ndy / 2);
    const long slots = P.lr ? 2 * items : items;
    // intervals and slots in 14 bits, ranks in IVA_THREADS chunks of IVA_SC
    // (so the adjoint's 3 ncell + 1 cell-table entries, ncell = slots, index
    // in 15 bits), one f value per forward thread
    if (nt >= 16384 || slots > IVA_SC * IVA_THREADS || items > 8L * IV_THREADS || 2 * P.nq > IV_THREADS) return false;
    const long lf = ((nt * 10 + 15) & ~15L) + 2 * (((nt + 1) * 8 + 15) & ~15L) + 4L * P.nq * 8 + IV_WAVES * 16;
    const long la = iva_lds(P, 0);
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
    v->rstride = (v->n_slots + IVA_SC - 1) / IVA_SC * IVA_SC;
    v->nch = v->rstride / IVA_SC;
    v->th_a = iva_threads(v->nch);
    v->th_f = iv_threads(P, v->n_items, nt);
    v->es = iva_pf(P, v->th_a) ? IVA_SC * IVA_SUB + IVA_SC : (ne + 1 + 7) / 8 * 8;   // PF rows: 72, 16-byte aligned
    v->ncell = P.ndx * (P.ndy / 2);
    v->np = 1;
    while (v->np * v->th_f < v->n_items) v->np *= 2;
    v->lds_f = lds_f;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus < 1)
        cus = 256;
    v->cus = cus;
    // as many blocks as the compute units hold at once (threads and LDS),
    // each a contiguous range of groups
    v->nblk_f = iv_blocks(P.n_groups, cus, v->th_f, lds_f);
    csx_status st;
    if ((st = iv_upload(&v->coef, coef, v->bytes)) != CSX_OK) return bail(st);
    if ((st = iv_upload(&v->mt, mt, v->bytes)) != CSX_OK) return bail(st);
    if ((st = iv_upload(&v->pp, pp, v->bytes)) != CSX_OK) return bail(st);
    if ((st = iv_upload(&v->qd, qd, v->bytes)) != CSX_OK) return bail(st);
    const size_t nrec = (size_t)P.n_groups * v->n_slots;
    const size_t nreca = (size_t)P.n_groups * v->rstride;
    const size_t nemap = (size_t)P.n_groups * nq * v->es;
    const size_t nemask = (size_t)P.n_groups * v->nch;
    if (hipMalloc((void **)&v->rec, nrec * sizeof(uint2)) != hipSuccess ||
        hipMalloc((void **)&v->reca, nreca * sizeof(uint2)) != hipSuccess ||
        hipMalloc((void **)&v->emap, nemap * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc((void **)&v->emask, nemask) != hipSuccess ||
        hipMalloc((void **)&v->cnt, sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&v->part, (size_t)v->nblk_f * P.npix * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(csx_fail(CSX_ENOMEM, "interval operators: records"));
    }
    v->bytes += (int64_t)((nrec + nreca) * sizeof(uint2) + nemap * sizeof(uint16_t) + nemask + sizeof(int) +
                          (size_t)v->nblk_f * P.npix * sizeof(float));
    if (hipMemset(v->cnt, 0, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(csx_fail(CSX_EHIP, "interval set-up: clearing the table counter"));
    }
    const dim3 gr((unsigned)((nrec + 255) / 256));
    if (P.lr)
        hipLaunchKernelGGL(k_iv_records<1>, gr, dim3(256), 0, nullptr, P, h->t, v->n_slots, v->rec);
    else
        hipLaunchKernelGGL(k_iv_records<0>, gr, dim3(256), 0, nullptr, P, h->t, v->n_slots, v->rec);
    int npow2 = 1;
    while (npow2 < v->n_slots) npow2 *= 2;
    const size_t lds_rank = (size_t)npow2 * 4 + (((size_t)nt * 2 + 15) & ~(size_t)15);
#define CSX_IVR(LR_)                                                                                             \
    hipLaunchKernelGGL(k_iv_rank<LR_>, dim3(P.n_groups), dim3(1024), lds_rank, nullptr, P, v->n_slots, npow2,     \
                       v->rstride, (const uint2 *)v->rec, v->reca, nq, ne, v->es, v->nch, (const uint16_t *)v->pp, \
                       v->emap, v->emask, v->cnt)
    if (P.lr) CSX_IVR(1);
    else CSX_IVR(0);
#undef CSX_IVR
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return bail(csx_fail(CSX_EHIP, std::string("interval set-up: ") + hipGetErrorString(e)));
        const hipError_t e2 = hipDeviceSynchronize();
        if (e2 != hipSuccess) return bail(csx_fail(CSX_EHIP, std::string("interval set-up: ") + hipGetErrorString(e2)));
    }
    // the adjoint's prefix table must fit beside the cell table
    if (hipMemcpy(&v->cap, v->cnt, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return bail(csx_fail(CSX_EHIP, "interval set-up: reading the table size"));
    }
    const long la = iva_lds(P, v->cap);
    if (la > CSX_LDS_MAX)
        return bail(csx_fail(CSX_EINVAL, "interval operators: the adjoint's tables exceed LDS"));
    v->lds_a = (int)la;
    v->nblk_a = iv_blocks(P.n_groups, v->cus, v->th_a, v->lds_a);
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
    const dim3 grid(v->nblk_f), block(v->th_f);
#define CSX_IVF(LR_, NP_, TPM_) \
    hipLaunchKernelGGL((k_iv_forward<LR_, NP_, TPM_>), grid, block, v->lds_f, s, h->P, a, f, part)
#define CSX_IVF_T(LR_, NP_)               \
    do {                                  \
        if (tper <= 5) CSX_IVF(LR_, NP_, 5);      \
        else if (tper <= 8) CSX_IVF(LR_, NP_, 8); \
        else CSX_IVF(LR_, NP_, 16);       \
    } while (0)
    // thresholds per thread in the F scan
    const int tper = (v->nt + v->th_f - 1) / v->th_f;
    if (h->P.lr) {
        if (v->np == 1) CSX_IVF_T(1, 1);
        else if (v->np == 2) CSX_IVF_T(1, 2);
        else CSX_IVF_T(1, 4);
    } else {
        if (v->np == 1) CSX_IVF_T(0, 1);
        else if (v->np == 2) CSX_IVF_T(0, 2);
        else if (v->np == 4) CSX_IVF_T(0, 4);
        else CSX_IVF_T(0, 8);
    }
#undef CSX_IVF_T
#undef CSX_IVF
    HIP_TRY(hipGetLastError());
    if (!g) return CSX_OK;   // the kernel alone (csx_iv_forward_parts)
    hipLaunchKernelGGL(k_iv_sum, dim3((h->P.npix + 63) / 64), dim3(1024), 0, s, (const float *)part, v->nblk_f,
                       h->P.npix, g);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_iv_forward_parts(const csx_geometry *h, const float *f, hipStream_t s)
{
    return csx_iv_forward(h, f, nullptr, 0, nullptr, s);
}

void csx_iv_parts(const csx_geometry *h, const float **part, int *nparts)
{
    const IvState *v = (const IvState *)h->iv;
    *part = v->part;
    *nparts = v->nblk_f;
}

csx_status csx_launch_iv_sum_batch(const ElemJob *jobs, const int *begin, int njobs, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_iv_sum_batch, dim3(nblocks), dim3(1024), 0, s, jobs, begin, njobs);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_iv_adjoint(const csx_geometry *h, const float *rho, float *b, hipStream_t s)
{
    const IvState *v = (const IvState *)h->iv;
    const IvArgs a = iv_args(h, v);
    const dim3 grid(v->nblk_a), block(v->th_a);
    const int pf = iva_pf(h->P, v->th_a);
#define CSX_IVA(LR_, PF_) \
    hipLaunchKernelGGL((k_iv_adjoint<LR_, PF_>), grid, block, v->lds_a, s, h->P, a, h->t, rho, b)
    if (h->P.lr) {
        if (pf == 2) CSX_IVA(1, 2);
        else if (pf == 1) CSX_IVA(1, 1);
        else CSX_IVA(1, 0);
    } else {
        if (pf == 2) CSX_IVA(0, 2);
        else if (pf == 1) CSX_IVA(0, 1);
        else CSX_IVA(0, 0);
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
