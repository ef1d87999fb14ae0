// csx_api.hip -- C ABI of libcsx: descriptor validation, device tables,
// operator calls and the EM-type reconstruction loop (Alg. 5).
#include "csx_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

static thread_local std::string g_last_error;

// Static scratch of csx_forward_noalloc: the forward's partial images live in
// this file-scope device array (one copy per GPU, held until the process
// ends) instead of the handle's workspace.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in); it uses the
// device address that hipGetSymbolAddress returns, resolved once per device
// at csx_init_geometry with that device current.
static __device__ __align__(256) float scratch[CSX_SCRATCH_FLOATS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static csx_status resolve_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return csx_fail(CSX_EHIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return CSX_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return csx_fail(CSX_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (float *)p;
    return CSX_OK;
}

csx_status csx_fail(csx_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

extern "C" const char *csx_last_error(void) { return g_last_error.c_str(); }

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

extern "C" csx_status csx_validate_desc(const csx_geometry_desc *d)
{
    if (!d) return csx_fail(CSX_EINVAL, "descriptor is NULL");
    if (d->nx < 1 || d->nz < 1 || d->nq < 1 || d->ndx < 1 || d->ndy < 1 || d->ne < 1 ||
        d->mask_nx < 1 || d->mask_ny < 1)
        return csx_fail(CSX_EGEOM, "all counts must be >= 1");
    if (!d->q || !d->phi || !d->mask) return csx_fail(CSX_EINVAL, "q, phi and mask must be non-NULL");
    if (d->ndy % 2 != 0) return csx_fail(CSX_EGEOM, "ndy must be even");
    if (!(std::isfinite(d->x_min) && std::isfinite(d->x_max) && d->x_min < d->x_max))
        return csx_fail(CSX_EGEOM, "need x_min < x_max");
    if (!(finite_pos(d->z_min) && d->z_min < d->z_max && d->z_max < d->mask_z &&
          d->mask_z < d->det_z && std::isfinite(d->det_z)))
        return csx_fail(CSX_EGEOM, "need 0 < z_min < z_max < mask_z < det_z");
    if (!finite_pos(d->det_pitch) || !finite_pos(d->mask_pitch) || !finite_pos(d->hc))
        return csx_fail(CSX_EGEOM, "pitches and hc must be positive");
    if (!(std::isfinite(d->e_lo) && std::isfinite(d->e_hi) && d->e_lo < d->e_hi))
        return csx_fail(CSX_EGEOM, "need e_lo < e_hi");
    if (!(std::isfinite(d->C) && d->C >= 0.0)) return csx_fail(CSX_EGEOM, "C must be finite and >= 0");
    if (d->ne > CSX_MAX_NE) return csx_fail(CSX_EGEOM, "ne exceeds the LDS spectrum table (2048)");
    if (d->table_dtype != CSX_TABLE_F32 && d->table_dtype != CSX_TABLE_BF16)
        return csx_fail(CSX_EINVAL, "unknown table_dtype");
    if (d->mask_nx > CSX_MAX_MASK_PERIOD || d->mask_ny > CSX_MAX_MASK_ROWS)
        return csx_fail(CSX_EGEOM, "mask must have <= 32 columns and <= 4096 rows");
    // a mask crossing lies between the voxel and the pixel: its cell indices
    // are bounded by the extents, kept below 2^21 for exact float conversion
    {
        const double ext_x = std::max({std::fabs(d->x_min), std::fabs(d->x_max), 0.5 * d->ndx * d->det_pitch});
        const double ext_y = 0.5 * d->ndy * d->det_pitch;
        if (ext_x / d->mask_pitch >= 2097152.0 || ext_y / d->mask_pitch + 0.5 * d->mask_ny >= 2097152.0)
            return csx_fail(CSX_EGEOM, "mask crossings beyond 2^21 cells");
    }
    const long nvox = (long)d->nx * d->nz, npix = (long)d->ndx * d->ndy;
    if (nvox * d->nq > (1L << 30) || npix > (1L << 28)) return csx_fail(CSX_EGEOM, "problem too large");
    if (d->ndx > (1 << 20) || d->ndy > (1 << 20)) return csx_fail(CSX_EGEOM, "detector too large");
    double qmin = INFINITY, qmax = 0.0;
    for (int m = 0; m < d->nq; ++m) {
        if (!finite_pos(d->q[m])) return csx_fail(CSX_EGEOM, "q nodes must be finite and > 0");
        qmin = std::min(qmin, d->q[m]);
        qmax = std::max(qmax, d->q[m]);
    }
    // bounds the spectrum-bin coordinate of any in-band pair (int range)
    if (qmax / qmin * d->ne > 1e8) return csx_fail(CSX_EGEOM, "q range times ne too large");
    for (int k = 0; k < d->ne; ++k)
        if (!(std::isfinite(d->phi[k]) && d->phi[k] >= 0.0))
            return csx_fail(CSX_EGEOM, "spectrum must be finite and >= 0");
    for (long k = 0; k < (long)d->mask_nx * d->mask_ny; ++k)
        if (d->mask[k] > 1) return csx_fail(CSX_EGEOM, "mask values must be 0 or 1");
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

static void release_events(csx_geometry *h)
{
    for (int op = 0; op < 2; ++op) {
        for (hipEvent_t e : h->ev[op]) (void)hipEventDestroy(e);
        h->ev[op].clear();
        h->ev_used[op] = 0;
    }
}

static void free_all(csx_geometry *h)
{
    csx_iv_free(h);
    csx_os_free(h);
    csx_sai_free(h);
    csx_energy_free(h);
    void *ptrs[] = {h->t.vf, h->t.vm, h->t.vd, h->t.qa, h->t.qblk, h->t.qv, h->t.phi32,
                    h->t.phi16, h->t.maskbits, h->part, h->gws, h->rho, h->ones, h->b1,
                    h->b2, h->ftmp, h->partL, h->partR, h->partF, h->partS, h->scal, h->jhist, h->flags, h->apart,
                    h->fplain, h->warm, h->a1, h->t.ra, h->t.rf, h->t.ram, h->t.rfm};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    release_events(h);
}

// Factor store: device records of every class's pair factors (uniform q
// grids).  Builds them (on = 1) or releases them (on = 0); synchronous.
static csx_status store_set(csx_geometry *h, bool on)
{
    HIP_TRY(hipDeviceSynchronize());
    void *old[] = {h->t.ra, h->t.rf, h->t.ram, h->t.rfm};
    for (void *p : old)
        if (p) HIP_TRY(hipFree(p));
    h->t.ra = nullptr;
    h->t.rf = nullptr;
    h->t.ram = nullptr;
    h->t.rfm = nullptr;
    h->bytes -= h->store_bytes;
    h->store_bytes = 0;
    h->store_ms = 0.0;
    if (!on) return CSX_OK;
    if (!h->P.qu) return csx_fail(CSX_EINVAL, "the factor store needs a uniform q grid");
    if (h->P.nq >= 65535) return csx_fail(CSX_EINVAL, "the factor store holds q-node ranges in 16 bits");
    size_t na, nf;
    csx_store_records(h->P, &na, &nf);
    uint4 *ra = nullptr, *rf = nullptr;
    uint32_t *ram = nullptr, *rfm = nullptr;
    auto release = [&]() {
        void *ps[] = {ra, rf, ram, rfm};
        for (void *p : ps)
            if (p) (void)hipFree(p);
    };
    if (hipMalloc((void **)&ra, na * sizeof(uint4)) != hipSuccess ||
        hipMalloc((void **)&rf, nf * 2 * sizeof(uint4)) != hipSuccess ||
        hipMalloc((void **)&ram, na / 64 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&rfm, nf / 64 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return csx_fail(CSX_ENOMEM, "factor store");
    }
    const auto t0 = std::chrono::steady_clock::now();
    csx_status st = csx_launch_store(h, ra, rf, ram, rfm, nullptr);
    const hipError_t e = hipDeviceSynchronize();
    if (st == CSX_OK && e != hipSuccess) st = csx_fail(CSX_EHIP, std::string("factor store: ") + hipGetErrorString(e));
    if (st != CSX_OK) {
        release();
        return st;
    }
    h->store_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    h->t.ra = ra;
    h->t.rf = rf;
    h->t.ram = ram;
    h->t.rfm = rfm;
    h->store_bytes = (int64_t)((na + 2 * nf) * sizeof(uint4) + (na + nf) / 64 * sizeof(uint32_t));
    h->bytes += h->store_bytes;
    return CSX_OK;
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
    if (!out) return csx_fail(CSX_EINVAL, "out is NULL");
    *out = nullptr;
    csx_status st = csx_validate_desc(d);
    if (st != CSX_OK) return st;

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    st = resolve_scratch(dev);
    if (st != CSX_OK) return st;

    csx_geometry *h = new (std::nothrow) csx_geometry();
    if (!h) return csx_fail(CSX_ENOMEM, "host allocation failed");
    h->device = dev;
    h->d = *d;
    h->q_host.assign(d->q, d->q + d->nq);
    h->phi_host.assign(d->phi, d->phi + d->ne);
    h->d.q = nullptr;
    h->d.phi = nullptr;
    h->d.mask = nullptr;
    h->table_dtype = d->table_dtype;

    KParams &P = h->P;
    std::memset(&P, 0, sizeof(P));
    P.nx = d->nx;
    P.nz = d->nz;
    P.nvox = d->nx * d->nz;
    P.ndx = d->ndx;
    P.ndy = d->ndy;
    P.npix = d->ndx * d->ndy;
    P.nq = d->nq;
    P.ne = d->ne;
    P.mask_nx = d->mask_nx;
    P.mask_ny = d->mask_ny;
    P.lr = (d->x_min == -d->x_max && d->nx % 2 == 0 && d->ndx % 2 == 0) ? 1 : 0;
    P.td = d->table_dtype;
    P.n_groups = P.lr ? d->nz * (d->nx / 2) : P.nvox;
    P.n_cls = d->ndx * (d->ndy / 2);
    P.n_quad = P.lr ? (d->ndx / 2) * (d->ndy / 2) : d->ndx * (d->ndy / 2);
    P.qw = d->nq <= 16 ? 16 : (d->nq <= 32 ? 32 : 64);
    P.qchunks = (d->nq + P.qw - 1) / P.qw;
    P.det_z = (float)d->det_z;
    P.det_zd = d->det_z;
    P.pitch = (float)d->det_pitch;
    P.pitchd = d->det_pitch;
    P.hp2 = (float)(0.25 * d->det_pitch * d->det_pitch);
    P.hc = d->hc;
    const double dE = (d->e_hi - d->e_lo) / d->ne;
    double qmin = d->q[0], qmax = d->q[0];
    for (int m = 1; m < d->nq; ++m) {
        qmin = std::min(qmin, d->q[m]);
        qmax = std::max(qmax, d->q[m]);
    }
    P.q_min = qmin;
    P.q_max = qmax;
    P.band_lo = d->e_lo - 1e-9 * std::fabs(d->e_lo) - 1e-300;
    P.band_hi = d->e_hi + 1e-9 * std::fabs(d->e_hi);
    P.half_my = (float)(0.5 * d->mask_ny);
    P.inv_mask_nx = (float)(1.0 / d->mask_nx);

    // per-voxel tables; with the x -> -x mirror the coordinates are mirrored
    // exactly (x of column nx-1-i is -x of column i)
    const int nvox = P.nvox;
    std::vector<float2> vf(nvox);
    std::vector<double2> vm(nvox);
    std::vector<VoxD> vd(nvox);
    const double dx = (d->x_max - d->x_min) / d->nx, dz = (d->z_max - d->z_min) / d->nz;
    for (int iz = 0; iz < d->nz; ++iz)
        for (int ix = 0; ix < d->nx; ++ix) {
            double x = d->x_min + (ix + 0.5) * dx;
            if (P.lr && ix >= d->nx / 2) x = -(d->x_min + (d->nx - 1 - ix + 0.5) * dx);
            const double z = d->z_min + (iz + 0.5) * dz;
            const double R2 = x * x + z * z;
            const double R = std::sqrt(R2);
            const double t = (d->mask_z - z) / (d->det_z - z);
            const int j = iz * d->nx + ix;
            vf[j] = make_float2((float)(d->C * z / (R2 * R)), (float)(d->det_z - z));
            vm[j] = make_double2(t / d->mask_pitch, (1.0 - t) * x / d->mask_pitch);
            vd[j] = VoxD{x, z, R2, 0.0};
        }
    const int nqp = ((d->nq + 63) / 64) * 64;   // padded for any chunk width dividing 64
    P.b0 = 1.0 - d->e_lo / dE;
    // uniform q grid: q_m = q_0 + m dq to 1e-12 relative (then q/dE = a0 + m da)
    {
        const double dq = d->nq > 1 ? (d->q[d->nq - 1] - d->q[0]) / (d->nq - 1) : 0.0;
        bool uni = d->nq > 1 && dq > 0.0;
        for (int m = 0; m < d->nq && uni; ++m)
            uni = std::fabs(d->q[m] - (d->q[0] + m * dq)) <= 1e-12 * qmax;
        P.qu = uni ? 1 : 0;
        P.a0 = d->q[0] / dE;
        P.da = dq / dE;
        // Bin coordinates u = kappa q/dE + b0 of the uniform-grid operators: an
        // idle lane holds b0 (kappa = 0); a lane in band has kappa < band_hi/q_min
        // (the band test), so at any node up to the last padded one u stays
        // below band_hi/q_min * q_top/dE + b0.  Zero pads around the table
        // cover that range (two entries of margin each side for rounding); if
        // they would not fit, the generic path (clamped index per node) runs.
        P.spec_lo = 0;
        P.spec_n = d->ne + 2;
        if (uni) {
            const double q_top = d->q[0] + dq * (nqp - 1);
            const double u_hi = P.band_hi / qmin * (q_top / dE) + P.b0;
            const double lo = std::floor(P.b0) - 2.0, hi = std::floor(u_hi) + 2.0;
            const bool fits = qmin > 0.0 && std::isfinite(u_hi) && lo > -CSX_SPEC_MAX && hi < CSX_SPEC_MAX &&
                              std::max(0.0, -lo) + std::max((double)d->ne + 1.0, hi) + 1.0 <= CSX_SPEC_MAX;
            if (fits) {
                P.spec_lo = std::max(0, (int)-lo);
                P.spec_n = P.spec_lo + std::max(d->ne + 1, (int)hi) + 1;
            } else {
                P.qu = 0;
            }
        }
    }
    std::vector<double> qa(nqp, 0.0);
    std::vector<float> qv(nqp, 0.0f);
    for (int m = 0; m < d->nq; ++m) {
        qa[m] = d->q[m] / dE;
        qv[m] = (float)d->q[m];
    }
    // q range of each block of 8 nodes (padding blocks never in band)
    std::vector<double2> qblk(nqp / 8);
    for (int bk = 0; bk < nqp / 8; ++bk) {
        double lo = INFINITY, hi = -INFINITY;
        for (int m = bk * 8; m < bk * 8 + 8; ++m)
            if (m < d->nq) {
                lo = std::min(lo, d->q[m]);
                hi = std::max(hi, d->q[m]);
            }
        qblk[bk] = make_double2(lo, hi);
    }
    std::vector<float> phi32(d->ne + 2, 0.0f);
    std::vector<uint16_t> phi16(d->ne + 2, 0);
    for (int k = 0; k < d->ne; ++k) {
        phi32[k + 1] = (float)d->phi[k];
        phi16[k + 1] = bf16_rne((float)d->phi[k]);
    }
    std::vector<uint32_t> bits(d->mask_ny, 0u);
    for (int r = 0; r < d->mask_ny; ++r)
        for (int c = 0; c < d->mask_nx; ++c)
            if (d->mask[(size_t)r * d->mask_nx + c]) bits[r] |= 1u << c;

    int64_t &B = h->bytes;
    CSX_TRY(dev_upload(&h->t.vf, vf, B));
    CSX_TRY(dev_upload(&h->t.vm, vm, B));
    CSX_TRY(dev_upload(&h->t.vd, vd, B));
    CSX_TRY(dev_upload(&h->t.qa, qa, B));
    CSX_TRY(dev_upload(&h->t.qblk, qblk, B));
    CSX_TRY(dev_upload(&h->t.qv, qv, B));
    CSX_TRY(dev_upload(&h->t.phi32, phi32, B));
    CSX_TRY(dev_upload(&h->t.phi16, phi16, B));
    CSX_TRY(dev_upload(&h->t.maskbits, bits, B));

    h->lc = csx_default_launch(P);
    const size_t nimg = (size_t)P.nvox * P.nq;
    h->part_cap = (size_t)csx_forward_shape(h).nparts * P.npix;
    CSX_TRY(dev_alloc(&h->part, h->part_cap, B));
    CSX_TRY(dev_alloc(&h->gws, P.npix, B));
    CSX_TRY(dev_alloc(&h->rho, P.npix, B));
    CSX_TRY(dev_alloc(&h->ones, P.npix, B));
    CSX_TRY(dev_alloc(&h->b1, nimg, B));
    CSX_TRY(dev_alloc(&h->b2, nimg, B));
    CSX_TRY(dev_alloc(&h->ftmp, nimg, B));
    if (h->lc.adj_splits > 1) {
        h->apart_cap = (size_t)h->lc.adj_splits * nimg;
        CSX_TRY(dev_alloc(&h->apart, h->apart_cap, B));
    }
    h->nbL = (P.npix + 255) / 256;
    h->nbR = (int)((nimg + 255) / 256);
    CSX_TRY(dev_alloc(&h->partL, h->nbL, B));
    CSX_TRY(dev_alloc(&h->partR, h->nbR, B));
    h->nbRu = h->nbR;
    CSX_TRY(dev_alloc(&h->partF, h->nbL, B));
    CSX_TRY(dev_alloc(&h->partS, 2 * CSX_SUM_BLOCKS, B));
    CSX_TRY(dev_alloc(&h->scal, 8, B));
    CSX_TRY(dev_alloc(&h->flags, 1, B));
    CSX_TRY(csx_launch_fill(h->ones, P.npix, 1.0f, nullptr));
    CSX_TRY(csx_launch_clear_flags(h, nullptr));
    // the factor store by default when it is small beside the device's free
    // memory (at most CSX_STORE_AUTO_BYTES and a quarter of what is free)
    if (P.qu && P.nq < 65535) {
        size_t na, nf, fr = 0, tot = 0;
        csx_store_records(P, &na, &nf);
        const size_t need = (na + 2 * nf) * sizeof(uint4) + (na + nf) / 64 * sizeof(uint32_t);
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && need <= (size_t)CSX_STORE_AUTO_BYTES && need <= fr / 4) {
            const csx_status ss = store_set(h, true);
            if (ss != CSX_ENOMEM) CSX_TRY(ss);   // out of memory: the handle runs without a store
        }
    }
    // the interval-form operators by default where they apply (their records
    // are 8 bytes per class: at most CSX_STORE_AUTO_BYTES and a quarter of
    // the free memory)
    if (csx_iv_feasible(P, nullptr, nullptr)) {
        size_t fr = 0, tot = 0;
        const size_t need = (size_t)P.n_groups * P.ndx * (P.ndy / 2) * 8;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && need <= (size_t)CSX_STORE_AUTO_BYTES && need <= fr / 4) {
            const csx_status si = csx_iv_build(h);
            if (si != CSX_ENOMEM) CSX_TRY(si);
        }
    }
    {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            free_all(h);
            delete h;
            return csx_fail(CSX_EHIP, std::string("init: ") + hipGetErrorString(e));
        }
    }
    *out = h;
    return CSX_OK;
}

extern "C" void csx_free_geometry(csx_geometry *h)
{
    if (!h) return;
    free_all(h);
    delete h;
}

extern "C" csx_status csx_get_info(const csx_geometry *h, csx_info *out)
{
    if (!h || !out) return csx_fail(CSX_EINVAL, "NULL argument");
    out->nvox = h->P.nvox;
    out->npix = h->P.npix;
    out->nq = h->P.nq;
    out->symmetric_lr = h->P.lr;
    out->table_dtype = h->table_dtype;
    out->workspace_bytes = h->bytes;
    return CSX_OK;
}

extern "C" csx_status csx_get_launch(const csx_geometry *h, csx_launch *out)
{
    if (!h || !out) return csx_fail(CSX_EINVAL, "NULL argument");
    *out = h->lc;
    return CSX_OK;
}

extern "C" csx_status csx_set_launch(csx_geometry *h, const csx_launch *lc)
{
    if (!h || !lc) return csx_fail(CSX_EINVAL, "NULL argument");
    csx_launch nl = *lc;
    if (nl.adj_splits == 0) nl.adj_splits = csx_default_adj_splits(h->P, nl.adj_qw);
    if (!csx_launch_valid(nl))
        return csx_fail(CSX_EINVAL, "launch shape: qw must be 16, 32 or 64, 1 <= fwd_splits <= 64 and "
                                    "0 <= adj_splits <= 64");
    const size_t aneed = nl.adj_splits > 1 ? (size_t)nl.adj_splits * h->P.nvox * h->P.nq : 0;
    if (aneed > h->apart_cap) {
        HIP_TRY(hipDeviceSynchronize());
        float *p = nullptr;
        if (hipMalloc((void **)&p, aneed * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return csx_fail(CSX_ENOMEM, "adjoint partials");
        }
        if (h->apart) HIP_TRY(hipFree(h->apart));
        h->bytes += (int64_t)((aneed - h->apart_cap) * sizeof(float));
        h->apart = p;
        h->apart_cap = aneed;
    }
    const csx_launch old = h->lc;
    h->lc = nl;
    const size_t need = (size_t)csx_forward_shape(h).nparts * h->P.npix;
    if (need > h->part_cap) {
        HIP_TRY(hipDeviceSynchronize());
        float *p = nullptr;
        if (hipMalloc((void **)&p, need * sizeof(float)) != hipSuccess) {
            h->lc = old;
            return csx_fail(CSX_ENOMEM, "forward partials");
        }
        HIP_TRY(hipFree(h->part));
        h->bytes += (int64_t)((need - h->part_cap) * sizeof(float));
        h->part = p;
        h->part_cap = need;
    }
    return CSX_OK;
}

extern "C" csx_status csx_set_factor_store(csx_geometry *h, int on)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    if (on != 0 && on != 1) return csx_fail(CSX_EINVAL, "on must be 0 or 1");
    if (on && !h->P.qu) return csx_fail(CSX_EINVAL, "the factor store needs a uniform q grid");
    return store_set(h, on == 1);
}

extern "C" csx_status csx_set_interval_operators(csx_geometry *h, int on)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    if (on != 0 && on != 1) return csx_fail(CSX_EINVAL, "on must be 0 or 1");
    if (on && !csx_iv_feasible(h->P, nullptr, nullptr))
        return csx_fail(CSX_EINVAL, "interval operators: thresholds, classes or LDS beyond their limits");
    HIP_TRY(hipDeviceSynchronize());
    csx_iv_free(h);
    return on ? csx_iv_build(h) : CSX_OK;
}

extern "C" csx_status csx_get_interval_operators(const csx_geometry *h, int *on, int64_t *bytes, double *build_ms,
                                                 int *intervals)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    csx_iv_info(h, on, bytes, build_ms, intervals);
    return CSX_OK;
}

extern "C" csx_status csx_get_factor_store(const csx_geometry *h, int *on, int64_t *bytes, double *build_ms)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    if (on) *on = h->t.ra ? 1 : 0;
    if (bytes) *bytes = h->store_bytes;
    if (build_ms) *build_ms = h->store_ms;
    return CSX_OK;
}

extern "C" csx_status csx_timing_enable(csx_geometry *h, int on)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    HIP_TRY(hipDeviceSynchronize());
    h->ev_used[0] = h->ev_used[1] = 0;
    h->timing = on != 0;
    return CSX_OK;
}

extern "C" csx_status csx_timing_read(csx_geometry *h, double ms[2], int n[2])
{
    if (!h || !ms || !n) return csx_fail(CSX_EINVAL, "NULL argument");
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

extern "C" csx_status csx_forward(csx_geometry *h, const float *f, float *g, void *stream)
{
    if (!h || !f || !g) return csx_fail(CSX_EINVAL, "NULL argument");
    return csx_launch_forward(h, f, g, (hipStream_t)stream);
}

extern "C" csx_status csx_forward_noalloc(const csx_geometry *h, const float *f, float *g, void *stream)
{
    if (!h || !f || !g) return csx_fail(CSX_EINVAL, "NULL argument");
    const size_t need = h->iv ? csx_iv_part_floats(h) : (size_t)csx_forward_shape(h).nparts * h->P.npix;
    if (need > (size_t)CSX_SCRATCH_FLOATS)
        return csx_fail(CSX_EINVAL, "forward partials (" + std::to_string(need) + " floats) exceed the static scratch (" +
                                        std::to_string(CSX_SCRATCH_FLOATS) + " floats)");
    float *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch_ptr[h->device];
    }
    if (!p) return csx_fail(CSX_EHIP, "static scratch not resolved for the handle's device");
    return csx_launch_forward_parts(h, f, p, (size_t)CSX_SCRATCH_FLOATS, g, (hipStream_t)stream);
}

extern "C" csx_status csx_backproject(csx_geometry *h, const float *y, float *b, void *stream)
{
    if (!h || !y || !b) return csx_fail(CSX_EINVAL, "NULL argument");
    return csx_launch_adjoint(h, y, b, (hipStream_t)stream);
}

static csx_status ensure_b1(csx_geometry *h, hipStream_t s) { return csx_ensure_b1(h, s); }

// the solver's operators: exact, or interpolated in angle (csx_set_operator)
static csx_status solver_forward(csx_geometry *h, const float *f, float *g, hipStream_t s)
{
    return (h->op_sai & CSX_OP_FORWARD_SAI) ? csx_launch_forward_sai(h, f, g, s) : csx_launch_forward(h, f, g, s);
}

static csx_status solver_adjoint(csx_geometry *h, const float *rho, float *b, hipStream_t s)
{
    return (h->op_sai & CSX_OP_ADJOINT_SAI) ? csx_launch_adjoint_sai(h, rho, b, s)
                                            : csx_launch_adjoint(h, rho, b, s);
}

csx_status csx_ensure_b1(csx_geometry *h, hipStream_t s)
{
    if (h->have_b1) return CSX_OK;
    csx_status st = solver_adjoint(h, h->ones, h->b1, s);
    if (st != CSX_OK) return st;
    h->have_b1 = true;
    return CSX_OK;
}

#define ST_TRY(expr)                 \
    do {                             \
        csx_status s_ = (expr);      \
        if (s_ != CSX_OK) return s_; \
    } while (0)

static csx_status step_impl(csx_geometry *h, const float *y, const float *r, float *f, double beta,
                            double *J, hipStream_t s)
{
    ST_TRY(ensure_b1(h, s));
    ST_TRY(solver_forward(h, f, h->gws, s));                    // z = A f^t (+ r below)
    ST_TRY(csx_launch_ratio(h, y, r, true, s));                 // rho = y / z, data-fit partials
    ST_TRY(solver_adjoint(h, h->rho, h->b2, s));                // b2 = A^T rho
    ST_TRY(csx_launch_update(h, f, beta, true, s));             // f^{t+1} into ftmp, R(f^t) partials
    if (J) return csx_launch_copy_objective(h, f, beta, J, nullptr, s);   // f^{t+1} into f, J(f^t)
    return csx_launch_copy(h->ftmp, f, h->P.nvox * h->P.nq, s);
}

extern "C" csx_status csx_recon_step(csx_geometry *h, const float *y, const float *r, float *f,
                                     double beta, double *J_out, void *stream)
{
    if (!h || !y || !f) return csx_fail(CSX_EINVAL, "NULL argument");
    if (!(std::isfinite(beta) && beta >= 0.0)) return csx_fail(CSX_EINVAL, "beta must be finite and >= 0");
    return step_impl(h, y, r, f, beta, J_out, (hipStream_t)stream);
}

extern "C" csx_status csx_recon(csx_geometry *h, const float *y, const float *r, float *f,
                                int init_uniform, int n_iter, double beta, double *J_hist,
                                void *stream)
{
    if (!h || !y || !f) return csx_fail(CSX_EINVAL, "NULL argument");
    if (n_iter < 0) return csx_fail(CSX_EINVAL, "n_iter must be >= 0");
    if (!(std::isfinite(beta) && beta >= 0.0)) return csx_fail(CSX_EINVAL, "beta must be finite and >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (h->jhist_cap < n_iter + 1) {
        if (h->jhist) HIP_TRY(hipFree(h->jhist));
        h->jhist = nullptr;
        h->jhist_cap = 0;
        HIP_TRY(hipMalloc((void **)&h->jhist, sizeof(double) * (n_iter + 1)));
        h->jhist_cap = n_iter + 1;
    }
    ST_TRY(csx_launch_clear_flags(h, s));
    ST_TRY(ensure_b1(h, s));
    if (init_uniform) ST_TRY(csx_launch_uniform_start(h, y, f, s));
    for (int t = 0; t < n_iter; ++t) ST_TRY(step_impl(h, y, r, f, beta, h->jhist + t, s));
    // J at the final iterate
    ST_TRY(solver_forward(h, f, h->gws, s));
    ST_TRY(csx_launch_ratio(h, y, r, false, s));
    ST_TRY(csx_launch_update(h, f, beta, false, s));
    ST_TRY(csx_launch_objective(h, beta, h->jhist + n_iter, nullptr, s));
    int flags = 0;
    HIP_TRY(hipMemcpyAsync(&flags, h->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    if (J_hist)
        HIP_TRY(hipMemcpyAsync(J_hist, h->jhist, sizeof(double) * (n_iter + 1),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flags & 2) return csx_fail(CSX_EINVAL, "y holds negative or NaN counts");
    if (flags & 1) return csx_fail(CSX_ENUMERIC, "y_i > 0 where the model mean is 0");
    return CSX_OK;
}

extern "C" csx_status csx_recon_warm(csx_geometry *h, const float *y, const float *r, const float *f_warm,
                                     float *f, int k_judge, int n_iter, double beta, double *J_hist,
                                     int *accepted, void *stream)
{
    if (!h || !y || !f_warm || !f) return csx_fail(CSX_EINVAL, "NULL argument");
    if (k_judge < 0 || k_judge > n_iter) return csx_fail(CSX_EINVAL, "need 0 <= k_judge <= n_iter");
    if (f_warm == f) return csx_fail(CSX_EINVAL, "f_warm and f must be different buffers");
    hipStream_t s = (hipStream_t)stream;
    const int n = h->P.nvox * h->P.nq;
    if (!h->fplain) HIP_TRY(hipMalloc((void **)&h->fplain, sizeof(float) * n));
    std::vector<double> Jw(k_judge + 1), Jp(k_judge + 1), Jr(n_iter - k_judge + 1);
    // k iterations from the candidate, then k from the plain uniform start
    ST_TRY(csx_launch_copy(f_warm, f, n, s));
    ST_TRY(csx_recon(h, y, r, f, 0, k_judge, beta, Jw.data(), stream));
    ST_TRY(csx_recon(h, y, r, h->fplain, 1, k_judge, beta, Jp.data(), stream));
    const bool take = Jw[k_judge] < Jp[k_judge];
    if (!take) ST_TRY(csx_launch_copy(h->fplain, f, n, s));
    ST_TRY(csx_recon(h, y, r, f, 0, n_iter - k_judge, beta, Jr.data(), stream));
    if (J_hist) {
        const std::vector<double> &Jc = take ? Jw : Jp;
        for (int t = 0; t < k_judge; ++t) J_hist[t] = Jc[t];
        for (int t = k_judge; t <= n_iter; ++t) J_hist[t] = Jr[t - k_judge];
    }
    if (accepted) *accepted = take ? 1 : 0;
    return CSX_OK;
}

extern "C" csx_status csx_set_penalty(csx_geometry *h, int kind, double delta)
{
    if (!h) return csx_fail(CSX_EINVAL, "NULL handle");
    if (kind == CSX_PSI_QUADRATIC) {
        h->psi_delta = 0.0;
        return CSX_OK;
    }
    if (kind == CSX_PSI_HUBER) {
        if (!(std::isfinite(delta) && delta > 0.0)) return csx_fail(CSX_EINVAL, "Huber scale must be finite and > 0");
        h->psi_delta = delta;
        return CSX_OK;
    }
    return csx_fail(CSX_EINVAL, "unknown penalty potential");
}
