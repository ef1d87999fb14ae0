// csx_energy.hip -- the energy-sensitive detector (App. A, eq. energy_sensitive).
//
// An energy-resolving pixel keeps the Bragg energy E = kappa q of each photon.
// On the spectrum's own bins, triple (i, j, q_m) adds H(i, j, q_m) f_jm to
// energy bin k = floor((kappa_ij q_m - e_lo) / dE) of pixel i:
//
//   g_E[k][i] = sum_j sum_{m : bin(kappa_ij q_m) = k} A_ij T_ij q_m Phi_k f_jm
//   b_jm      = q_m sum_i A_ij T_ij Phi(kappa_ij q_m) y_E[bin(kappa_ij q_m)][i]
//
// The kernels are the exact operators' (csx_ops.hip) in their energy mode:
// the forward adds runs of q nodes that share a bin into per-wave histograms
// (64-bit fixed point in LDS), the adjoint reads a Phi-weighted copy of the
// data at each triple's bin.  This file holds the buffers, the fixed-point
// scale and the C entry points.
#include "csx_internal.h"

#include <algorithm>
#include <cmath>
#include <new>

namespace {

struct EnergyState {
    float *part = nullptr;     // forward partial images [nparts][ne][npix]
    size_t part_cap = 0;       // floats in part
    float *psi = nullptr;      // adjoint input [ne + 2][npix]
    double *sc = nullptr;      // [2] fixed-point scale of the forward's histograms and its inverse
    double *scpart = nullptr;  // [SCALE_BLOCKS] partial sums of the scale's bound
    // Alg. 5 on energy-resolved data
    float *gE = nullptr;       // [ne][npix] model mean
    float *rhoE = nullptr;     // [ne][npix] y / z, then ones for the sensitivity
    double *partL = nullptr;   // per-block data-fit partials
    int *partF = nullptr;      // per-block flags
    float *b1 = nullptr;       // [nvox][nq] sensitivity A_E^T 1
    bool have_b1 = false;
};

EnergyState *state(const csx_geometry *h) { return static_cast<EnergyState *>(h->energy); }

__device__ __forceinline__ float table_phi(const float *phi32, const uint16_t *phi16, int td, int k)
{
    return td == CSX_TABLE_BF16 ? __uint_as_float(((uint32_t)phi16[k]) << 16) : phi32[k];
}

// Scale of the forward's fixed-point histograms: every run contribution and
// every bin total of an output pixel is at most B = a_max phi_max sum_jm q_m
// |f_jm| in magnitude (a voxel and q node reach a pixel through one bin);
// 2^s with 2^(s-61) B < 1.  Block partial sums, then one block adds them in a
// fixed order.
constexpr int SCALE_BLOCKS = 256;

__global__ void __launch_bounds__(256) k_energy_scale_part(const float *__restrict__ f, const float *__restrict__ qv,
                                                           int nvox, int nq, double *__restrict__ part)
{
    __shared__ double red[4];
    const long n = (long)nvox * nq;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)SCALE_BLOCKS * 256)
        acc += fabs((double)qv[i % nq] * (double)f[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(64) k_energy_scale(const double *__restrict__ part, double factor,
                                                     double *__restrict__ sc)
{
    double acc = 0.0;
    for (int k = threadIdx.x; k < SCALE_BLOCKS; k += 64) acc += part[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (threadIdx.x == 0) {
        const double B = factor * acc;
        double s0 = 1.0, s1 = 1.0;
        if (!(B < INFINITY)) {
            s0 = 0.0;                        // inf or NaN in f
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

// Psi[k][i] = Phi_k y_E[k - 1][i] for the table bins k = 1..ne, 0 on the pad
// planes k = 0 and ne + 1.
__global__ void __launch_bounds__(256) k_energy_psi(const float *__restrict__ y, const float *__restrict__ phi32,
                                                    const uint16_t *__restrict__ phi16, int td, int ne, int npix,
                                                    float *__restrict__ psi)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long)(ne + 2) * npix) return;
    const int k = (int)(i / npix);
    const int p = (int)(i - (long)k * npix);
    psi[i] = (k >= 1 && k <= ne) ? table_phi(phi32, phi16, td, k) * y[(long)(k - 1) * npix + p] : 0.0f;
}

csx_status ensure_state(csx_geometry *h, bool forward)
{
    EnergyState *s = state(h);
    if (!s) {
        s = new (std::nothrow) EnergyState();
        if (!s) return csx_fail(CSX_ENOMEM, "host allocation failed");
        h->energy = s;
        HIP_TRY(hipMalloc((void **)&s->sc, sizeof(double) * 2));
        HIP_TRY(hipMalloc((void **)&s->scpart, sizeof(double) * SCALE_BLOCKS));
    }
    if (forward) {
        int lds = 0;
        const size_t need = csx_forward_energy_floats(h, &lds);
        if (lds > CSX_LDS_MAX) return csx_fail(CSX_EINVAL, "energy-resolved forward: ne too large for LDS");
        if (need > s->part_cap) {
            if (s->part) HIP_TRY(hipFree(s->part));
            s->part = nullptr;
            s->part_cap = 0;
            HIP_TRY(hipMalloc((void **)&s->part, sizeof(float) * need));
            s->part_cap = need;
        }
    } else if (!s->psi) {
        HIP_TRY(hipMalloc((void **)&s->psi, sizeof(float) * (size_t)(h->P.ne + 2) * h->P.npix));
    }
    return CSX_OK;
}

}  // namespace

void csx_energy_free(csx_geometry *h)
{
    EnergyState *s = state(h);
    if (!s) return;
    void *ptrs[] = {s->part, s->psi, s->sc, s->scpart, s->gE, s->rhoE, s->partL, s->partF, s->b1};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete s;
    h->energy = nullptr;
}

extern "C" csx_status csx_forward_energy(csx_geometry *h, const float *f, float *gE, void *stream)
{
    if (!h || !f || !gE) return csx_fail(CSX_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    csx_status r = ensure_state(h, true);
    if (r != CSX_OK) return r;
    double a_max = 0.0;
    r = csx_pair_weight_max(h, &a_max);
    if (r != CSX_OK) return r;
    double phi_max = 0.0;
    for (double v : h->phi_host) phi_max = std::max(phi_max, std::fabs(v));
    // 1 + 2^-7 covers the bfloat16 rounding of the table
    const double factor = a_max * phi_max * (1.0 + 1.0 / 128.0);
    EnergyState *s = state(h);
    hipLaunchKernelGGL(k_energy_scale_part, dim3(SCALE_BLOCKS), dim3(256), 0, st, f, h->t.qv, h->P.nvox, h->P.nq,
                       s->scpart);
    hipLaunchKernelGGL(k_energy_scale, dim3(1), dim3(64), 0, st, s->scpart, factor, s->sc);
    HIP_TRY(hipGetLastError());
    return csx_launch_forward_energy(h, f, s->sc, s->part, s->part_cap, gE, st);
}

extern "C" csx_status csx_backproject_energy(csx_geometry *h, const float *yE, float *b, void *stream)
{
    if (!h || !yE || !b) return csx_fail(CSX_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    csx_status r = ensure_state(h, false);
    if (r != CSX_OK) return r;
    EnergyState *s = state(h);
    const long n = (long)(h->P.ne + 2) * h->P.npix;
    hipLaunchKernelGGL(k_energy_psi, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, yE, h->t.phi32,
                       h->t.phi16, h->P.td, h->P.ne, h->P.npix, s->psi);
    HIP_TRY(hipGetLastError());
    return csx_launch_adjoint_energy(h, s->psi, b, st);
}

namespace {

csx_status ensure_solver(csx_geometry *h)
{
    csx_status r = ensure_state(h, true);
    if (r != CSX_OK) return r;
    r = ensure_state(h, false);
    if (r != CSX_OK) return r;
    EnergyState *s = state(h);
    const size_t n = (size_t)h->P.ne * h->P.npix, nb = (n + 255) / 256;
    if (!s->gE) HIP_TRY(hipMalloc((void **)&s->gE, sizeof(float) * n));
    if (!s->rhoE) HIP_TRY(hipMalloc((void **)&s->rhoE, sizeof(float) * n));
    if (!s->partL) HIP_TRY(hipMalloc((void **)&s->partL, sizeof(double) * nb));
    if (!s->partF) HIP_TRY(hipMalloc((void **)&s->partF, sizeof(int) * nb));
    if (!s->b1) HIP_TRY(hipMalloc((void **)&s->b1, sizeof(float) * (size_t)h->P.nvox * h->P.nq));
    return CSX_OK;
}

#define EN_TRY(expr)                 \
    do {                             \
        csx_status s_ = (expr);      \
        if (s_ != CSX_OK) return s_; \
    } while (0)

}  // namespace

extern "C" csx_status csx_recon_energy(csx_geometry *h, const float *yE, const float *rE, float *f,
                                       int init_uniform, int n_iter, double beta, double *J_hist, void *stream)
{
    if (!h || !yE || !f) return csx_fail(CSX_EINVAL, "NULL argument");
    if (n_iter < 0) return csx_fail(CSX_EINVAL, "n_iter must be >= 0");
    if (!(std::isfinite(beta) && beta >= 0.0)) return csx_fail(CSX_EINVAL, "beta must be finite and >= 0");
    hipStream_t st = (hipStream_t)stream;
    EN_TRY(ensure_solver(h));
    EnergyState *s = state(h);
    const int n = h->P.ne * h->P.npix, nb = (n + 255) / 256, nimg = h->P.nvox * h->P.nq;
    if (h->jhist_cap < n_iter + 1) {
        if (h->jhist) HIP_TRY(hipFree(h->jhist));
        h->jhist = nullptr;
        h->jhist_cap = 0;
        HIP_TRY(hipMalloc((void **)&h->jhist, sizeof(double) * (n_iter + 1)));
        h->jhist_cap = n_iter + 1;
    }
    EN_TRY(csx_launch_clear_flags(h, st));
    if (!s->have_b1) {   // b1 = A_E^T 1
        EN_TRY(csx_launch_fill(s->rhoE, n, 1.0f, st));
        EN_TRY(csx_backproject_energy(h, s->rhoE, s->b1, st));
        s->have_b1 = true;
    }
    if (init_uniform) EN_TRY(csx_launch_uniform_start_n(h, yE, n, s->b1, f, st));
    for (int t = 0; t <= n_iter; ++t) {
        EN_TRY(csx_forward_energy(h, f, s->gE, st));                                    // z = A_E f (+ r)
        const bool step = t < n_iter;
        EN_TRY(csx_launch_ratio_n(n, s->gE, yE, rE, s->rhoE, s->partL, s->partF, step, st));
        if (step) {
            EN_TRY(csx_backproject_energy(h, s->rhoE, h->b2, st));                      // b2 = A_E^T (y / z)
            EN_TRY(csx_launch_update_ex(h, f, s->b1, h->b2, beta, h->ftmp, st));        // f^{t+1}, R(f^t)
        } else {
            EN_TRY(csx_launch_update(h, f, beta, false, st));                           // R(f^T)
        }
        EN_TRY(csx_launch_objective_n(h, s->partL, nb, s->partF, beta, h->jhist + t, st));
        if (step) EN_TRY(csx_launch_copy(h->ftmp, f, nimg, st));
    }
    int flags = 0;
    HIP_TRY(hipMemcpyAsync(&flags, h->flags, sizeof(int), hipMemcpyDeviceToHost, st));
    if (J_hist) HIP_TRY(hipMemcpyAsync(J_hist, h->jhist, sizeof(double) * (n_iter + 1), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (flags & 2) return csx_fail(CSX_EINVAL, "y holds negative or NaN counts");
    if (flags & 1) return csx_fail(CSX_ENUMERIC, "y_i > 0 where the model mean is 0");
    return CSX_OK;
}
