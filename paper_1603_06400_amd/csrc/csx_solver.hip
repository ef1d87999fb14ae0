// csx_solver.hip -- the Poisson data term, the separable-surrogate update
// and the float64 objective of the EM-type algorithm (Alg. 5; Sec. V; App. B).
#include "csx_internal.h"
#include "csx_update.h"

#include <cmath>

namespace {

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

// bx: the block (blockIdx.x of the single-scan launch)
__device__ __forceinline__ void ratio_body(int n, const float *__restrict__ g, const float *__restrict__ y,
                                           const float *__restrict__ r, float *__restrict__ rho,
                                           double *__restrict__ partL, int *__restrict__ partF, int want_rho,
                                           int bx, double *s_red, int &s_flag)
{
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    const int i = bx * blockDim.x + threadIdx.x;
    double L = 0.0;
    int flag = 0;
    if (i < n) {
        const float z = g[i] + (r ? r[i] : 0.0f);
        const float yi = y[i];
        float q = 0.0f;
        if (!(yi >= 0.0f)) {
            flag = 2;
        } else if (yi > 0.0f) {
            if (z > 0.0f) {
                q = yi / z;
                L = (double)z - (double)yi * log((double)z) + lgamma((double)yi + 1.0);
            } else {
                flag = 1;
                L = INFINITY;
            }
        } else {
            L = (double)z;
        }
        if (want_rho) rho[i] = q;
    }
    if (flag) atomicOr(&s_flag, flag);
    const double t = block_sum_d(L, s_red);
    if (threadIdx.x == 0) {
        partL[bx] = t;
        partF[bx] = s_flag;
    }
}

__global__ void __launch_bounds__(256) k_ratio(int n, const float *__restrict__ g,
                                               const float *__restrict__ y,
                                               const float *__restrict__ r,
                                               float *__restrict__ rho, double *__restrict__ partL,
                                               int *__restrict__ partF, int want_rho)
{
    __shared__ double s_red[4];
    __shared__ int s_flag;
    ratio_body(n, g, y, r, rho, partL, partF, want_rho, blockIdx.x, s_red, s_flag);
}

// J = sum partL + beta * sum partR in a fixed order by one block, flags
// combined (J = +inf when some y_i > 0 met a zero mean).
__device__ void objective_block(const double *__restrict__ partL, int nL, const double *__restrict__ partR, int nR,
                                const int *__restrict__ partF, double beta, int *__restrict__ flags,
                                double *__restrict__ J, const int *__restrict__ iter, double *s_red, int *s_flag)
{
    if (threadIdx.x == 0) *s_flag = 0;
    __syncthreads();
    double a = 0.0, b = 0.0;
    int fl = 0;
    for (int k = threadIdx.x; k < nL; k += blockDim.x) {
        a += partL[k];
        fl |= partF[k];
    }
    for (int k = threadIdx.x; k < nR; k += blockDim.x) b += partR[k];
    if (fl) atomicOr(s_flag, fl);
    const double ta = block_sum_d(a, s_red);
    __syncthreads();
    const double tb = block_sum_d(b, s_red);
    if (threadIdx.x == 0) {
        *flags = *s_flag;
        J[iter ? *iter : 0] = (*s_flag & 1) ? INFINITY : ta + beta * tb;
    }
}

// ---------------------------------------------------------------------------
// K4 separable-surrogate update (App. B, eq. f_update) with 4 in-slice
// neighbours at the same q and unit weights, per element as in csx_update.h;
// also accumulates R(fhat) = sum_j sum_k psi(fhat_j - fhat_k) per block.
// ---------------------------------------------------------------------------
// VEC consecutive q nodes of one voxel per thread (VEC divides nq; 16-byte
// loads and stores when VEC = 4).  HUB = 0: the quadratic potential (delta
// is not read), 1: Huber's.
template <int VEC, int HUB>
__device__ __forceinline__ void update_body(int nx, int nz, int nq, const float *__restrict__ fh,
                                            const float *__restrict__ b1, const float *__restrict__ b2, double beta,
                                            float *__restrict__ fout, double *__restrict__ partR, int do_update,
                                            double delta, int bx, double *s_red)
{
    const int n = nx * nz * nq;
    const int e0 = (bx * blockDim.x + threadIdx.x) * VEC;
    double R = 0.0;
    if (e0 < n) {
        const int j = e0 / nq;
        const int ix = j % nx, iz = j / nx;
        const size_t row = (size_t)nx * nq;
        float c[VEC], l[VEC], r[VEC], u[VEC], d[VEC];
        auto ld = [&](const float *p, float (&v)[VEC]) {
            if constexpr (VEC == 4) {
                const float4 t = *(const float4 *)p;
                v[0] = t.x;
                v[1] = t.y;
                v[2] = t.z;
                v[3] = t.w;
            } else {
                v[0] = *p;
            }
        };
        // a neighbour outside the grid reads the centre
        ld(fh + e0, c);
        ld(fh + e0 - (ix > 0 ? nq : 0), l);
        ld(fh + e0 + (ix < nx - 1 ? nq : 0), r);
        ld(fh + e0 - (iz > 0 ? row : 0), u);
        ld(fh + e0 + (iz < nz - 1 ? row : 0), d);
        const int nin = (ix > 0) + (ix < nx - 1) + (iz > 0) + (iz < nz - 1);
        float vb1[VEC], vb2[VEC], out[VEC];
        if (do_update) {
            ld(b1 + e0, vb1);
            ld(b2 + e0, vb2);
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const double fj = c[k];
            double s = 0.0, w = 0.0;
            if (HUB) neighbour_terms<1>(fj, l[k], r[k], u[k], d[k], ix, iz, nx, nz, delta, R, s, w);
            else neighbour_terms_quad(fj, l[k], r[k], u[k], d[k], nin, R, s, w);
            if (do_update) out[k] = surrogate_root(fj, s, w, vb1[k], vb2[k], beta);
        }
        if (do_update) {
            if constexpr (VEC == 4) *(float4 *)(fout + e0) = make_float4(out[0], out[1], out[2], out[3]);
            else fout[e0] = out[0];
        }
    }
    const double t = block_sum_d(R, s_red);
    if (threadIdx.x == 0) partR[bx] = t;
}

template <int VEC, int HUB>
__global__ void __launch_bounds__(256) k_update(int nx, int nz, int nq, const float *__restrict__ fh,
                                                const float *__restrict__ b1,
                                                const float *__restrict__ b2, double beta,
                                                float *__restrict__ fout,
                                                double *__restrict__ partR, int do_update, double delta)
{
    __shared__ double s_red[4];
    update_body<VEC, HUB>(nx, nz, nq, fh, b1, b2, beta, fout, partR, do_update, delta, blockIdx.x, s_red);
}

// K5: J = sum partL + beta * sum partR in a fixed order, one block; the
// per-block flags of K3 are combined into *flags (J = +inf when some y_i > 0
// met a zero mean).
__global__ void __launch_bounds__(256) k_objective(const double *__restrict__ partL, int nL,
                                                   const double *__restrict__ partR, int nR,
                                                   const int *__restrict__ partF, double beta,
                                                   int *__restrict__ flags, double *__restrict__ J,
                                                   const int *__restrict__ iter)
{
    __shared__ double s_red[4];
    __shared__ int s_flag;
    objective_block(partL, nL, partR, nR, partF, beta, flags, J, iter, s_red, &s_flag);
}

__global__ void k_iter_incr(int *iter) { *iter += 1; }

// sums for the uniform start: block partials of sum x and sum y over a
// grid-stride range, then one block adds the partials in a fixed order
// (out[0] = sum x, out[1] = sum y)
__global__ void __launch_bounds__(256) k_sum2_part(const float *__restrict__ x, int nx_,
                                                   const float *__restrict__ y, int ny_,
                                                   double *__restrict__ part)
{
    __shared__ double s_red[4];
    double a = 0.0, b = 0.0;
    const int stride = gridDim.x * blockDim.x;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nx_; k += stride) a += x[k];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ny_; k += stride) b += y[k];
    const double ta = block_sum_d(a, s_red);
    __syncthreads();
    const double tb = block_sum_d(b, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}

__global__ void __launch_bounds__(256) k_sum2_final(const double *__restrict__ part, int nb,
                                                    double *__restrict__ out)
{
    __shared__ double s_red[4];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    const double ta = block_sum_d(a, s_red);
    __syncthreads();
    const double tb = block_sum_d(b, s_red);
    if (threadIdx.x == 0) {
        out[0] = ta;
        out[1] = tb;
    }
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

__global__ void k_copy4(const float4 *__restrict__ s, float4 *__restrict__ d, int n4)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n4) d[e] = s[e];
}

// The copy of the updated image back, with one extra block (the last) that
// forms the objective from the partials of the ratio and update launches
// before it (n % 4 == 0, 16-byte aligned arrays).
__global__ void __launch_bounds__(256) k_copy4_objective(const float4 *__restrict__ s, float4 *__restrict__ d,
                                                         int n4, const double *__restrict__ partL, int nL,
                                                         const double *__restrict__ partR, int nR,
                                                         const int *__restrict__ partF, double beta,
                                                         int *__restrict__ flags, double *__restrict__ J,
                                                         const int *__restrict__ iter)
{
    if (blockIdx.x == gridDim.x - 1) {
        __shared__ double s_red[4];
        __shared__ int s_flag;
        objective_block(partL, nL, partR, nR, partF, beta, flags, J, iter, s_red, &s_flag);
        return;
    }
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n4) d[e] = s[e];
}

// The batched form's jobs (ElemJob): block b belongs to the job whose block
// range [begin[k], begin[k + 1]) holds it, and does what block b - begin[k]
// of the job's single-scan launch does.
__device__ __forceinline__ int elem_job(const int *__restrict__ begin, int njobs, int b)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_ratio_batch(const ElemJob *__restrict__ jobs, const int *__restrict__ begin,
                                                     int njobs)
{
    __shared__ double s_red[4];
    __shared__ int s_flag;
    const int k = elem_job(begin, njobs, blockIdx.x);
    const ElemJob &J = jobs[k];
    ratio_body(J.npix, J.g, J.y, J.r, J.rho, J.partL, J.partF, 1, (int)blockIdx.x - begin[k], s_red, s_flag);
}

template <int HUB>
__global__ void __launch_bounds__(256) k_update_batch(const ElemJob *__restrict__ jobs, const int *__restrict__ begin,
                                                      int njobs, double beta)
{
    __shared__ double s_red[4];
    const int k = elem_job(begin, njobs, blockIdx.x);
    const ElemJob &J = jobs[k];
    update_body<4, HUB>(J.nx, J.nz, J.nq, J.f, J.b1, J.b2, beta, J.ftmp, J.partR, 1, J.delta,
                        (int)blockIdx.x - begin[k], s_red);
}

// copy-back blocks, then the job's objective block last
__global__ void __launch_bounds__(256) k_copy4_objective_batch(const ElemJob *__restrict__ jobs,
                                                               const int *__restrict__ begin, int njobs, double beta,
                                                               const int *__restrict__ iter)
{
    const int k = elem_job(begin, njobs, blockIdx.x);
    const ElemJob &J = jobs[k];
    const int b = (int)blockIdx.x - begin[k];
    const int n4 = J.nx * J.nz * J.nq / 4;
    if (b == (n4 + 255) / 256) {
        __shared__ double s_red[4];
        __shared__ int s_flag;
        objective_block(J.partL, J.nL, J.partR, J.nR, J.partF, beta, J.flags, J.J, iter, s_red, &s_flag);
        return;
    }
    const int e = b * blockDim.x + threadIdx.x;
    if (e < n4) ((float4 *)J.fdst)[e] = ((const float4 *)J.ftmp)[e];
}

__global__ void k_clear_int(int *p) { *p = 0; }

}  // namespace

csx_status csx_launch_elem_batch(int which, const ElemJob *jobs, const int *begin, int njobs, int nblocks, double beta,
                                 int hub, const int *iter, hipStream_t s)
{
    if (which == 0) {
        hipLaunchKernelGGL(k_ratio_batch, dim3(nblocks), dim3(256), 0, s, jobs, begin, njobs);
    } else if (which == 1) {
        if (hub) hipLaunchKernelGGL(k_update_batch<1>, dim3(nblocks), dim3(256), 0, s, jobs, begin, njobs, beta);
        else hipLaunchKernelGGL(k_update_batch<0>, dim3(nblocks), dim3(256), 0, s, jobs, begin, njobs, beta);
    } else {
        hipLaunchKernelGGL(k_copy4_objective_batch, dim3(nblocks), dim3(256), 0, s, jobs, begin, njobs, beta, iter);
    }
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_ratio(csx_geometry *h, const float *y, const float *r, bool want_rho,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_ratio, dim3(h->nbL), dim3(256), 0, s, h->P.npix, h->gws, y, r, h->rho,
                       h->partL, h->partF, want_rho ? 1 : 0);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

// The update's vector width: 4 q nodes per thread when nq is a multiple of 4
// and every array is 16-byte aligned, else 1.
static int update_vec(const csx_geometry *h, const void *a, const void *b, const void *c, const void *d)
{
    const uintptr_t al = (uintptr_t)a | (uintptr_t)b | (uintptr_t)c | (uintptr_t)d;
    return (h->P.nq % 4 == 0 && (al & 15) == 0) ? 4 : 1;
}

static csx_status launch_update(csx_geometry *h, const float *f, const float *b1, const float *b2, double beta,
                                float *fout, bool do_update, hipStream_t s)
{
    const KParams &P = h->P;
    const long n = (long)P.nvox * P.nq;
    const int vec = update_vec(h, f, b1, b2, fout);
    const int nb = (int)((n + 256L * vec - 1) / (256L * vec));
    h->nbRu = nb;
#define CSX_UPD(V_, H_)                                                                                       \
    hipLaunchKernelGGL((k_update<V_, H_>), dim3(nb), dim3(256), 0, s, P.nx, P.nz, P.nq, f, b1, b2, beta, fout, \
                       h->partR, do_update ? 1 : 0, h->psi_delta)
    const bool hub = h->psi_delta > 0.0;
    if (vec == 4) {
        if (hub) CSX_UPD(4, 1);
        else CSX_UPD(4, 0);
    } else {
        if (hub) CSX_UPD(1, 1);
        else CSX_UPD(1, 0);
    }
#undef CSX_UPD
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_update(csx_geometry *h, const float *f, double beta, bool do_update,
                             hipStream_t s)
{
    return launch_update(h, f, h->b1, h->b2, beta, h->ftmp, do_update, s);
}

csx_status csx_launch_update_ex(csx_geometry *h, const float *f, const float *b1, const float *b2,
                                double beta, float *fout, hipStream_t s)
{
    return launch_update(h, f, b1, b2, beta, fout, true, s);
}

csx_status csx_launch_copy_objective(csx_geometry *h, float *f, double beta, double *J, const int *iter,
                                     hipStream_t s)
{
    const int n = h->P.nvox * h->P.nq;
    if (n % 4 != 0 || (((uintptr_t)h->ftmp | (uintptr_t)f) & 15) != 0) {
        csx_status st = csx_launch_copy(h->ftmp, f, n, s);
        if (st != CSX_OK) return st;
        return csx_launch_objective(h, beta, J, iter, s);
    }
    const int nb = (n / 4 + 255) / 256;
    hipLaunchKernelGGL(k_copy4_objective, dim3(nb + 1), dim3(256), 0, s, (const float4 *)h->ftmp, (float4 *)f, n / 4,
                       h->partL, h->nbL, h->partR, h->nbRu, h->partF, beta, h->flags, J, iter);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_objective(csx_geometry *h, double beta, double *J, const int *iter,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(256), 0, s, h->partL, h->nbL, h->partR, h->nbRu,
                       h->partF, beta, h->flags, J, iter);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_iter_incr(int *iter, hipStream_t s)
{
    hipLaunchKernelGGL(k_iter_incr, dim3(1), dim3(1), 0, s, iter);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

// scal[0] = sum(y), scal[1] = sum(b1) (float64, fixed order)
csx_status csx_launch_uniform_sums(csx_geometry *h, const float *y, hipStream_t s)
{
    const int n = h->P.nvox * h->P.nq;
    const int nb = CSX_SUM_BLOCKS;
    hipLaunchKernelGGL(k_sum2_part, dim3(nb), dim3(256), 0, s, y, h->P.npix, h->b1, n, h->partS);
    hipLaunchKernelGGL(k_sum2_final, dim3(1), dim3(256), 0, s, h->partS, nb, h->scal);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_uniform_start(csx_geometry *h, const float *y, float *f, hipStream_t s)
{
    const int n = h->P.nvox * h->P.nq;
    csx_status st = csx_launch_uniform_sums(h, y, s);
    if (st != CSX_OK) return st;
    hipLaunchKernelGGL(k_fill_ratio, dim3((n + 255) / 256), dim3(256), 0, s, f, n, h->scal);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_copy(const float *src, float *dst, int n, hipStream_t s)
{
    if (n % 4 == 0 && (((uintptr_t)src | (uintptr_t)dst) & 15) == 0)
        hipLaunchKernelGGL(k_copy4, dim3((n / 4 + 255) / 256), dim3(256), 0, s, (const float4 *)src, (float4 *)dst,
                           n / 4);
    else
        hipLaunchKernelGGL(k_copy, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_fill(float *dst, int n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, s, dst, n, v);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_clear_flags(csx_geometry *h, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_int, dim3(1), dim3(1), 0, s, h->flags);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

// Pieces of Alg. 5 on data of any length (the energy-resolved detector's
// [ne][npix] counts): the ratio and data-fit partials over n entries, the
// objective from those partials, and the uniform start from a given b1.
csx_status csx_launch_ratio_n(int n, const float *g, const float *y, const float *r, float *rho, double *partL,
                              int *partF, bool want_rho, hipStream_t s)
{
    hipLaunchKernelGGL(k_ratio, dim3((n + 255) / 256), dim3(256), 0, s, n, g, y, r, rho, partL, partF,
                       want_rho ? 1 : 0);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_objective_n(csx_geometry *h, const double *partL, int nL, const int *partF, double beta,
                                  double *J, hipStream_t s)
{
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(256), 0, s, partL, nL, h->partR, h->nbRu, partF, beta, h->flags,
                       J, nullptr);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status csx_launch_uniform_start_n(csx_geometry *h, const float *y, int ny, const float *b1, float *f,
                                      hipStream_t s)
{
    const int n = h->P.nvox * h->P.nq;
    const int nb = CSX_SUM_BLOCKS;
    hipLaunchKernelGGL(k_sum2_part, dim3(nb), dim3(256), 0, s, y, ny, b1, n, h->partS);
    hipLaunchKernelGGL(k_sum2_final, dim3(1), dim3(256), 0, s, h->partS, nb, h->scal);
    hipLaunchKernelGGL(k_fill_ratio, dim3((n + 255) / 256), dim3(256), 0, s, f, n, h->scal);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}
