// csx_device.h -- device helpers shared by the operator kernels (exact and
// scatter-angle-interpolated): spectrum and mask tables in LDS, the per-pair
// factors, mask cells and wave reductions.  Included by one translation unit
// each; everything has internal linkage.
#pragma once

#include "csx_internal.h"

namespace {


__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

// The spectrum table in LDS is always float32: the bfloat16 form stores the
// table in bfloat16 and widens it while staging (exact), so both forms share
// one inner loop.
__device__ __forceinline__ float spec(const float *s_phi, uint32_t k)
{
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
    // square roots from one float reciprocal square root y ~ 1/sqrt(v) each:
    // sqrt(v) ~ v y, refined by one float64 Newton step (relative error of
    // order 1e-14); y itself serves as 1/sqrt(v) in the float32 factors
    const double Rs2 = R2 * s2;
    const float yr = __builtin_amdgcn_rsqf((float)Rs2);
    const float rs0 = (float)Rs2 * yr;
    const double Rs = (double)rs0 + (Rs2 - (double)rs0 * (double)rs0) * (double)(0.5f * yr);
    const double den = 2.0 * Rs * (Rs + dot);
    const float yc = __builtin_amdgcn_rsqf((float)cross2);     // 1 / |r x s|
    const float r0 = yc * yc;
    const double inv = (double)r0 * (2.0 - cross2 * (double)r0);
    const double K2 = den * inv;   // 1 / sin^2(theta/2)
    const float yk = __builtin_amdgcn_rsqf((float)K2);
    const float k0 = (float)K2 * yk;
    const double k = (double)k0 + (K2 - (double)k0 * (double)k0) * (double)(0.5f * yk);
    kappa = P.hc * k;

    const float s2f = (float)s2;
    const float inv_s = __builtin_amdgcn_rsqf(s2f);
    const float God = vf.y * inv_s * inv_s * inv_s;
    const float cos_t = (float)dot * yr;
    // cos(theta/2) = sin(theta) / (2 sin(theta/2)), sin(theta) = |r x s| / (|r| |s|)
    const float cos_h = 0.5f * ((float)cross2 * yc) * yr * k0;
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

// Spectrum-table index of one triple: 1 + bin inside the band; outside it the
// index lands on one of the two zero pads (0 or ne + 1): a negative bin
// coordinate wraps to a large unsigned value and is clamped to ne + 1.
__device__ __forceinline__ uint32_t spec_index(double kappa, double qa, double b0, uint32_t top)
{
    const double u = fma(kappa, qa, b0);
    const uint32_t k = (uint32_t)(int)u;
    return min(k, top);
}

// Spectrum table and mask bits into LDS.  s_tab receives the P.spec_n-entry
// padded table: entry k of the zero-padded spectrum [0, ne+1] at position
// P.spec_lo + k, zeros around it.
__device__ __forceinline__ void stage_tables(const KParams &P, const DevTables &T, float *s_tab,
                                             uint32_t *s_bits)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const bool b16 = P.td == CSX_TABLE_BF16;
    for (int k = tid; k < P.spec_n; k += nt) {
        const int e = k - P.spec_lo;
        float v = 0.0f;
        if (e >= 0 && e < P.ne + 2) v = b16 ? bf16_to_f32(T.phi16[e]) : T.phi32[e];
        s_tab[k] = v;
    }
    for (int k = tid; k < P.mask_ny; k += nt) s_bits[k] = T.maskbits[k];
}

// Mask cells of one crossing: columns of the pixel (col_a) and of its x-mirror
// seen from the mirror voxel (col_b), rows of y' (row_u) and -y' (row_d).
struct Cells {
    int col_a, col_b, row_u, row_d;
    bool in_rows;
};

// v mod P for an integer-valued float v (|v| < 2^22): the quotient is taken at
// v/P + 1/(2P), half a step away from any integer, so the float rounding of
// 1/P cannot move it across one.
__device__ __forceinline__ int fmodp(const KParams &P, float v)
{
    const float qf = floorf(fmaf(v, P.inv_mask_nx, 0.5f * P.inv_mask_nx));
    return (int)fmaf(-(float)P.mask_nx, qf, v);
}

// Centre of pixel index a on an axis of n pixels: (a - n/2 + 1/2) * pitch,
// formed as (2a - n + 1) * (pitch/2), one rounding of the same real product.
__device__ __forceinline__ double pixel_coord(const KParams &P, int a, int n)
{
    return (double)(2 * a - n + 1) * (0.5 * P.pitchd);
}

// The crossing of ray r -> r' with the mask plane, in cell units:
// p = (t/pm) r' + ((1-t)/pm) (x, 0), t = (mask_z - z)/(det_z - z) (App. A).
// The cell is decided in float64 -- the precision of the definition -- so a
// crossing lands in the same cell as in the float64 evaluation except within
// float64 rounding (~1e-13 mm) of a cell edge.  vm = {t/pm, (1-t) x/pm}.
__device__ __forceinline__ Cells mask_cells(const KParams &P, double2 vm, double xp, double yp)
{
    Cells c;
    // |p| < 2^21 cells (validated), so the floors convert exactly
    const float cx = (float)floor(fma(vm.x, xp, vm.y));
    const int cy = (int)floor(fma(vm.x, yp, (double)P.half_my));
    c.col_a = fmodp(P, cx);
    c.col_b = fmodp(P, -cx - 1.0f);          // floor(-px) = -floor(px) - 1 off the cell edges
    c.row_u = cy;
    c.row_d = P.mask_ny - 1 - cy;            // floor(My - v) = My - 1 - floor(v)
    c.in_rows = cy >= 0 && cy < P.mask_ny;
    return c;
}

__device__ __forceinline__ float bitf(uint32_t row, int col)
{
    return (float)((row >> col) & 1u);
}

// Lane exchanges of the butterfly below.  dpp_row<C>: the value of another
// lane of the same 16-lane row (C = 0x100 + d: lane l + d, 0x110 + d: lane
// l - d; lanes whose source is outside the row read 0).
template <int C>
__device__ __forceinline__ float dpp_row(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), C, 0xf, 0xf, true));
}

// One butterfly step at distance D for the pair (lo, hi): lanes with bit D
// clear keep lo and add their partner's (lane l ^ D) lo, lanes with bit D set
// keep hi and add their partner's hi.  D = 32 and 16 use gfx950's lane swaps
// (lanes 32..63 of the first operand with lanes 0..31 of the second, and odd
// 16-lane rows of the first with even rows of the second), smaller D row
// shifts: no LDS traffic.
template <int D>
__device__ __forceinline__ float butterfly(float lo, float hi, bool up)
{
    if constexpr (D == 32 || D == 16) {
        const auto r = D == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                               : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        const float tu = hi + dpp_row<0x110 + D>(hi);   // partner l - D
        const float td = lo + dpp_row<0x100 + D>(lo);   // partner l + D
        return up ? tu : td;
    }
}

// Sum of v[0..N) over the 64 lanes of the wave, butterfly style: at each
// distance d the lanes with bit d set keep the upper half of their values and
// take their partner's (lane l ^ d) upper half, the others the lower halves,
// so after six steps lane l holds the total for index l >> (6 - log2 N).
template <int N, int D>
struct WaveTransposeSum {
    static __device__ __forceinline__ void run(float *v, int lane)
    {
        if constexpr (D == 0) {
            return;
        } else if constexpr (N > 1) {
            constexpr int H = N / 2;
            const bool up = (lane & D) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) v[i] = butterfly<D>(v[i], v[H + i], up);
            WaveTransposeSum<H, D / 2>::run(v, lane);
        } else {
            v[0] = butterfly<D>(v[0], v[0], (lane & D) != 0);
            WaveTransposeSum<1, D / 2>::run(v, lane);
        }
    }
};

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// Bin coordinate of q node m on a uniform q grid: u_m = u0 + m du with
// u0 = kappa q_0/dE + 1 - e_lo/dE and du = kappa dq/dE (an FP64 FMA at nodes
// 0, 8, 16, ..., one FP64 add per node between).
// Nodes whose energy can be in band satisfy 1 <= u_m < ne + 1; the returned
// range [lo, hi] (chunk-local, widened by one node each side) contains them.
__device__ __forceinline__ void band_range(const KParams &P, double u0, double du, int m0, int qw,
                                           int &lo, int &hi)
{
    // a float bound with one node of margin each side: the reciprocal's
    // rounding (and that of the float coordinates) stays far inside it
    const float fu0 = (float)u0, r = __builtin_amdgcn_rcpf((float)du);
    const float a = (1.0f - fu0) * r, b = ((float)P.ne + 1.0f - fu0) * r;
    const float l = fmaxf(floorf(a) - 1.0f - (float)m0, -1.0f);
    const float h = fminf(floorf(b) + 1.0f - (float)m0, (float)qw);
    lo = (int)l;
    hi = (int)h;
}

// Logical block of a forward launch (exact or interpolated).  The hardware deals blocks to the
// eight XCDs round-robin by linear id; the renumbering gives each XCD a
// contiguous share of the (quad group, q chunk, tile split) grid, with the
// split slowest and the q chunk next, so an XCD fetches into its own L2 only
// the part of f that its splits and q chunks cover.
__device__ __forceinline__ void xcd_block(int &bx, int &by, int &bz)
{
    const int gx = gridDim.x, gz = gridDim.z, total = gx * gridDim.y * gz;
    int lin = blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z);
    if (total % 8 == 0) lin = (lin % 8) * (total / 8) + lin / 8;
    bx = lin % gx;
    const int r = lin / gx;
    bz = r % gz;
    by = r / gz;
}

// 64-bit fixed point of a float contribution v at scale 2^s (|v| 2^s < 2^61):
// x = v 2^s is exact in float, x = hi 2^32 + lo with lo in [0, 2^32), lo
// formed by one exact FMA; rounds toward -inf (a deterministic choice).
__device__ __forceinline__ unsigned long long fixed_of(float v, int s)
{
    const float x = __builtin_ldexpf(v, s);
    const float hi = floorf(__builtin_ldexpf(x, -32));
    const float lo = fmaf(-hi, 4294967296.0f, x);
    return ((unsigned long long)(uint32_t)(int)hi << 32) + (unsigned long long)(uint32_t)lo;
}

// The exponent s of a fixed-point scale 2^s held as a double.
__device__ __forceinline__ int scale_exponent(double sc)
{
    int e;
    (void)frexp(sc, &e);
    return e - 1;
}

// 16-byte load with the non-temporal hint (streamed records that no other
// wave reads again: kept from displacing the L2-resident tables and images)
__device__ __forceinline__ uint4 load_nt(const uint4 *p)
{
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_nontemporal_load((const u32x4 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

template <int QW>
__device__ __forceinline__ int transposed_index(int lane)
{
    return QW == 64 ? lane : (QW == 32 ? (lane >> 1) : (lane >> 2));
}

}  // namespace
