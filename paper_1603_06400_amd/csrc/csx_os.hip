// csx_os.hip -- ordered subsets (Alg. 6).
//
// The detector is split by the symmetry-preserving partition of Sec. VI: a
// subset is one vertical class (rows rz, rz + rho_z, ... of one half and
// their up-down mirrors) times one horizontal class (columns cy, cy + rho_y,
// ... and their left-right mirrors); subset p = rz (rho_y / 2) + cy is the
// sweep order.  Every subset is closed under both mirrors, so the operators
// run on it unchanged: the forward's waves take the subset's pixel quads from
// a list (its partial images are summed, and the count ratio formed, at the
// subset's pixels only), the adjoint's lanes the subset's pixel classes.  A
// sub-step is z_p = A_p f + r_p, rho_p = y_p / z_p, b2 = A_p^T rho_p and the closed-form
// update of App. B with b1_p = A_p^T 1 (computed once per partition) and
// penalty weight beta / P, so that one sweep applies the penalty once, like
// the data term.  The sweep alternates the image between the caller's buffer
// and the handle's scratch image; the full objective is evaluated after each
// sweep.
#include "csx_internal.h"

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

namespace {

struct OsState {
    int rho_z = 0, rho_y = 0, n_sub = 0;
    int n_quads = 0, n_cls = 0, n_pix = 0;    // per subset (balanced partition)
    int splits = 1;
    int *quads = nullptr;                     // [n_sub][n_quads]
    int *cls = nullptr;                       // [n_sub][n_cls]
    int *pix = nullptr;                       // [n_sub][n_pix]
    float *b1 = nullptr;                      // [n_sub][nvox * nq]
    int adj_op = 0;                           // CSX_OP_ADJOINT_SAI when b1 came from the interpolated adjoint
    // the adjoint's factor store in subset order (with the handle's store):
    // a subset's records of one voxel group are contiguous, so a wave's
    // 64 lanes read 1 KB in one piece instead of 64 records from 64 tiles
    uint4 *ra = nullptr;                      // [n_groups][n_sub][cls_pad]
    uint32_t *ram = nullptr;                  // node range per 64 records
    int cls_pad = 0;
};

// subset adjoint with the handle's selected operator (exact or interpolated)
csx_status adjoint_list(csx_geometry *h, const OsState *o, int p, const float *rho, float *b, hipStream_t s)
{
    const int *cls = o->cls + (size_t)p * o->n_cls;
    if (h->op_sai & CSX_OP_ADJOINT_SAI) return csx_launch_adjoint_sai_list(h, rho, cls, o->n_cls, b, s);
    if (o->ra && h->t.ra)
        return csx_launch_adjoint_list(h, rho, cls, o->n_cls, b, s, o->ra + (size_t)p * o->cls_pad,
                                       o->ram + (size_t)p * (o->cls_pad / 64), (long)o->n_sub * o->cls_pad);
    return csx_launch_adjoint_list(h, rho, cls, o->n_cls, b, s);
}

void release(OsState *o)
{
    if (!o) return;
    void *ptrs[] = {o->quads, o->cls, o->pix, o->b1, o->ra, o->ram};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete o;
}

#define OS_TRY(expr)                 \
    do {                             \
        csx_status s_ = (expr);      \
        if (s_ != CSX_OK) return s_; \
    } while (0)

// Builds the partition's lists and the per-subset sensitivity images.
csx_status build(csx_geometry *h, int rho_z, int rho_y, hipStream_t s, OsState **out)
{
    const KParams &P = h->P;
    const int ndx = P.ndx, ndy = P.ndy, hy = ndy / 2;
    std::vector<int> quads, cls, pix;
    int nq_sub = -1, nc_sub = -1, np_sub = -1;
    for (int rz = 0; rz < rho_z; ++rz) {
        std::vector<int> rows;                 // upper-half rows of the vertical class
        for (int r = rz; r < hy; r += rho_z) rows.push_back(ndy - 1 - r);
        std::sort(rows.begin(), rows.end());
        for (int cy = 0; cy < rho_y / 2; ++cy) {
            std::vector<int> cols;
            for (int c = cy; c < ndx; c += rho_y) {
                cols.push_back(c);
                cols.push_back(ndx - 1 - c);
            }
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            const size_t q0 = quads.size(), c0 = cls.size(), p0 = pix.size();
            for (int bu : rows) {
                for (int a : cols) {
                    if (P.lr) {
                        if (a >= ndx / 2) quads.push_back((bu - hy) * (ndx / 2) + (a - ndx / 2));
                    } else {
                        quads.push_back((bu - hy) * ndx + a);
                    }
                    cls.push_back((bu - hy) * ndx + a);
                    pix.push_back(bu * ndx + a);
                    pix.push_back((ndy - 1 - bu) * ndx + a);
                }
            }
            const int nq = (int)(quads.size() - q0), nc = (int)(cls.size() - c0), np = (int)(pix.size() - p0);
            if ((nq_sub >= 0 && nq != nq_sub) || (nc_sub >= 0 && nc != nc_sub) || (np_sub >= 0 && np != np_sub))
                return csx_fail(CSX_EINVAL, "unbalanced partition");
            nq_sub = nq;
            nc_sub = nc;
            np_sub = np;
        }
    }
    OsState *o = new (std::nothrow) OsState();
    if (!o) return csx_fail(CSX_ENOMEM, "host allocation failed");
    o->rho_z = rho_z;
    o->rho_y = rho_y;
    o->n_sub = rho_z * (rho_y / 2);
    o->n_quads = nq_sub;
    o->n_cls = nc_sub;
    o->n_pix = np_sub;
    // split the voxel range so that a subset's few quads still fill the chip
    o->splits = 64;
    const size_t img = (size_t)P.nvox * P.nq;
    auto fail = [&](hipError_t e) {
        release(o);
        return csx_fail(CSX_EHIP, std::string("ordered subsets: ") + hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipMalloc((void **)&o->quads, sizeof(int) * quads.size())) != hipSuccess) return fail(e);
    if ((e = hipMalloc((void **)&o->cls, sizeof(int) * cls.size())) != hipSuccess) return fail(e);
    if ((e = hipMalloc((void **)&o->pix, sizeof(int) * pix.size())) != hipSuccess) return fail(e);
    if ((e = hipMalloc((void **)&o->b1, sizeof(float) * img * o->n_sub)) != hipSuccess) return fail(e);
    if ((e = hipMemcpyAsync(o->quads, quads.data(), sizeof(int) * quads.size(), hipMemcpyHostToDevice, s)) != hipSuccess)
        return fail(e);
    if ((e = hipMemcpyAsync(o->cls, cls.data(), sizeof(int) * cls.size(), hipMemcpyHostToDevice, s)) != hipSuccess)
        return fail(e);
    if ((e = hipMemcpyAsync(o->pix, pix.data(), sizeof(int) * pix.size(), hipMemcpyHostToDevice, s)) != hipSuccess)
        return fail(e);
    // the adjoint's factor store in subset order, when the handle has a store
    // and the copy is small beside the device's free memory
    if (h->t.ra) {
        o->cls_pad = (o->n_cls + 63) / 64 * 64;
        const size_t nrec = (size_t)P.n_groups * o->n_sub * o->cls_pad;
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && nrec * sizeof(uint4) <= (size_t)CSX_STORE_AUTO_BYTES &&
            nrec * sizeof(uint4) <= fr / 4 && hipMalloc((void **)&o->ra, nrec * sizeof(uint4)) == hipSuccess &&
            hipMalloc((void **)&o->ram, nrec / 64 * sizeof(uint32_t)) == hipSuccess) {
            csx_status st = csx_launch_store_list(h, o->cls, o->n_cls, o->n_sub, o->cls_pad, o->ra, o->ram, s);
            if (st != CSX_OK) {
                release(o);
                return st;
            }
        } else {
            (void)hipGetLastError();
            if (o->ra) (void)hipFree(o->ra);
            o->ra = nullptr;
            o->ram = nullptr;
        }
    }
    for (int p = 0; p < o->n_sub; ++p) {
        csx_status st = adjoint_list(h, o, p, h->ones, o->b1 + (size_t)p * img, s);
        if (st != CSX_OK) {
            release(o);
            return st;
        }
    }
    o->adj_op = h->op_sai & CSX_OP_ADJOINT_SAI;
    *out = o;
    return CSX_OK;
}

// Grows the handle's forward partials to what the subset launches need with
// the handle's current launch shape (the stream is synchronised first).
csx_status ensure_parts(csx_geometry *h, const OsState *o, hipStream_t s)
{
    const OpShape S = csx_forward_shape_list(h, o->quads, o->n_quads, o->splits);
    const size_t need = (size_t)S.nparts * h->P.npix;
    if (need <= h->part_cap) return CSX_OK;
    HIP_TRY(hipStreamSynchronize(s));
    float *np = nullptr;
    HIP_TRY(hipMalloc((void **)&np, sizeof(float) * need));
    (void)hipFree(h->part);
    h->part = np;
    h->part_cap = need;
    return CSX_OK;
}

}  // namespace

void csx_os_free(csx_geometry *h)
{
    release(static_cast<OsState *>(h->os));
    h->os = nullptr;
}

extern "C" csx_status csx_recon_os(csx_geometry *h, const float *y, const float *r, float *f, int init_uniform,
                                   int n_iter, int rho_z, int rho_y, double beta, double *J_hist, void *stream)
{
    if (!h || !y || !f) return csx_fail(CSX_EINVAL, "NULL argument");
    if (n_iter < 0) return csx_fail(CSX_EINVAL, "n_iter must be >= 0");
    if (!(std::isfinite(beta) && beta >= 0.0)) return csx_fail(CSX_EINVAL, "beta must be finite and >= 0");
    const KParams &P = h->P;
    if (rho_z < 1 || rho_y < 2 || rho_y % 2 || (P.ndy / 2) % rho_z || P.ndx % rho_y)
        return csx_fail(CSX_EINVAL, "partition needs rho_z | ndy/2, rho_y | ndx and rho_y even");
    hipStream_t s = (hipStream_t)stream;
    if (h->jhist_cap < n_iter + 1) {
        if (h->jhist) HIP_TRY(hipFree(h->jhist));
        h->jhist = nullptr;
        h->jhist_cap = 0;
        HIP_TRY(hipMalloc((void **)&h->jhist, sizeof(double) * (n_iter + 1)));
        h->jhist_cap = n_iter + 1;
    }
    OS_TRY(csx_launch_clear_flags(h, s));
    OS_TRY(csx_ensure_b1(h, s));
    OsState *o = static_cast<OsState *>(h->os);
    const int adj_op = h->op_sai & CSX_OP_ADJOINT_SAI;   // the subset sensitivities follow the adjoint
    if (!o || o->rho_z != rho_z || o->rho_y != rho_y || o->adj_op != adj_op) {
        HIP_TRY(hipStreamSynchronize(s));
        csx_os_free(h);
        OS_TRY(build(h, rho_z, rho_y, s, &o));
        h->os = o;
    }
    OS_TRY(ensure_parts(h, o, s));
    if (init_uniform) OS_TRY(csx_launch_uniform_start(h, y, f, s));
    const size_t img = (size_t)P.nvox * P.nq;
    auto objective = [&](const float *fc, int t) -> csx_status {
        OS_TRY((h->op_sai & CSX_OP_FORWARD_SAI) ? csx_launch_forward_sai(h, fc, h->gws, s)
                                                 : csx_launch_forward(h, fc, h->gws, s));
        OS_TRY(csx_launch_ratio(h, y, r, false, s));
        OS_TRY(csx_launch_update(h, fc, beta, false, s));
        return csx_launch_objective(h, beta, h->jhist + t, nullptr, s);
    };
    OS_TRY(objective(f, 0));
    const double bp = beta / o->n_sub;
    for (int t = 0; t < n_iter; ++t) {
        float *cur = f, *nxt = h->ftmp;
        for (int p = 0; p < o->n_sub; ++p) {
            const int *qd = o->quads + (size_t)p * o->n_quads, *px = o->pix + (size_t)p * o->n_pix;
            if (h->op_sai & CSX_OP_FORWARD_SAI)
                OS_TRY(csx_launch_forward_sai_list(h, cur, qd, o->n_quads, o->splits, px, o->n_pix, y, r, h->rho, s));
            else
                OS_TRY(csx_launch_forward_list(h, cur, qd, o->n_quads, o->splits, px, o->n_pix, y, r, h->rho, s));
            OS_TRY(adjoint_list(h, o, p, h->rho, h->b2, s));
            OS_TRY(csx_launch_update_ex(h, cur, o->b1 + (size_t)p * img, h->b2, bp, nxt, s));
            std::swap(cur, nxt);
        }
        if (cur != f) OS_TRY(csx_launch_copy(cur, f, (int)img, s));
        OS_TRY(objective(f, t + 1));
    }
    int flags = 0;
    HIP_TRY(hipMemcpyAsync(&flags, h->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    if (J_hist)
        HIP_TRY(hipMemcpyAsync(J_hist, h->jhist, sizeof(double) * (n_iter + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (flags & 2) return csx_fail(CSX_EINVAL, "y holds negative or NaN counts");
    if (flags & 1) return csx_fail(CSX_ENUMERIC, "y_i > 0 where the model mean is 0");
    return CSX_OK;
}
