// csx_batch.hip -- the batched form: many independent scans (each its own
// geometry handle, any sizes) reconstructed together by Alg. 5.
//
// One iteration issues, per kernel variant, a single forward launch and a
// single adjoint launch that cover every active scan's blocks (largest scans
// first, so the small scans fill the tail), plus the per-scan float64
// data-term, update and objective kernels.  Scans whose operators take the
// interval form (csx_interval.hip) launch them per scan: each of those
// launches already spans every compute unit.  Their elementwise work (the sum
// of the forward's partial images, the count ratio, the update and the
// copy-back with the objective) runs in one launch per kernel covering every
// such scan (ElemJob tables).  The iteration is captured into a
// HIP graph on a private stream and replayed; the objective kernels index the
// J history through a device iteration counter, so the replays need no host
// work.  Scans may have their own iteration counts: the run goes in stages
// between consecutive distinct counts, each with its own graph over the scans
// still running.  Nothing in a graph is a memset.
#include "csx_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

namespace {

struct Group {
    int variant = 0;
    int lds = 0;
    int nblocks = 0;
    std::vector<int> scans;        // scan indices, largest first
    std::vector<CsxJob> jobs;      // host copy of the job table
    std::vector<int> begin;        // first block of each job
    CsxJob *jobs_dev = nullptr;
    int *begin_dev = nullptr;
};

double scan_cost(const csx_geometry *h)
{
    return (double)h->P.nvox * (double)h->P.npix * (double)h->P.nq;
}

}  // namespace

struct csx_batch {
    std::vector<csx_geometry *> h;
    std::vector<Group> fwd, adj;
    hipStream_t st = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int *iter_dev = nullptr;
    double *J_dev = nullptr;
    size_t J_cap = 0;
    // the interval-form scans' batched elementwise launches: jobs and, per
    // launch (sum, ratio, update, copy-back), each job's first block
    bool elem = false;
    int elem_hub = 0;
    std::vector<ElemJob> ej;
    std::vector<int> eb;          // [4][n]
    int enb[4] = {0, 0, 0, 0};
    ElemJob *ej_dev = nullptr;
    int *eb_dev = nullptr;
};

static void free_groups(std::vector<Group> &gs)
{
    for (Group &g : gs) {
        if (g.jobs_dev) (void)hipFree(g.jobs_dev);
        if (g.begin_dev) (void)hipFree(g.begin_dev);
        g.jobs_dev = nullptr;
        g.begin_dev = nullptr;
    }
}

extern "C" void csx_batch_free(csx_batch *b)
{
    if (!b) return;
    free_groups(b->fwd);
    free_groups(b->adj);
    if (b->iter_dev) (void)hipFree(b->iter_dev);
    if (b->ej_dev) (void)hipFree(b->ej_dev);
    if (b->eb_dev) (void)hipFree(b->eb_dev);
    if (b->J_dev) (void)hipFree(b->J_dev);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->st) (void)hipStreamDestroy(b->st);
    delete b;
}

// Groups the active scans by kernel variant of one operator and orders each
// group's scans by decreasing work.
static void make_groups(const std::vector<csx_geometry *> &hs, const std::vector<int> &active, bool forward,
                        std::vector<Group> &out)
{
    std::vector<int> order(active);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return scan_cost(hs[a]) > scan_cost(hs[b]); });
    for (int k : order) {
        if (hs[k]->iv) continue;   // interval-form operators: launched per scan
        const OpShape S = forward ? csx_forward_shape(hs[k]) : csx_adjoint_shape(hs[k]);
        Group *g = nullptr;
        for (Group &c : out)
            if (c.variant == S.variant) g = &c;
        if (!g) {
            out.emplace_back();
            g = &out.back();
            g->variant = S.variant;
        }
        g->scans.push_back(k);
    }
}

// Rebuilds the job tables of a group for the given per-scan buffers and
// uploads them (asynchronously on s).
static csx_status upload_jobs(Group &g, const std::vector<csx_geometry *> &hs, bool forward,
                              const std::vector<const float *> &in, const std::vector<float *> &out,
                              hipStream_t s)
{
    g.jobs.clear();
    g.begin.clear();
    g.lds = 0;
    g.nblocks = 0;
    for (int k : g.scans) {
        csx_geometry *h = hs[k];
        const OpShape S = forward ? csx_forward_shape(h) : csx_adjoint_shape(h);
        CsxJob J;
        std::memset(&J, 0, sizeof(J));
        J.P = S.P;
        J.T = h->t;
        J.L = S.L;
        J.in = in[k];
        J.out = forward ? h->part : out[k];
        J.gx = (int)S.grid.x;
        J.gy = (int)S.grid.y;
        J.gz = (int)S.grid.z;
        J.tps = S.tps;
        g.begin.push_back(g.nblocks);
        g.nblocks += J.gx * J.gy * J.gz;
        g.lds = std::max(g.lds, S.L.total);
        g.jobs.push_back(J);
    }
    if (!g.jobs_dev) {
        HIP_TRY(hipMalloc((void **)&g.jobs_dev, sizeof(CsxJob) * g.scans.size()));
        HIP_TRY(hipMalloc((void **)&g.begin_dev, sizeof(int) * g.scans.size()));
    }
    HIP_TRY(hipMemcpyAsync(g.jobs_dev, g.jobs.data(), sizeof(CsxJob) * g.jobs.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(g.begin_dev, g.begin.data(), sizeof(int) * g.begin.size(),
                           hipMemcpyHostToDevice, s));
    return CSX_OK;
}

static csx_status launch_group(const Group &g, bool forward, hipStream_t s)
{
    if (forward)
        return csx_launch_forward_batch(g.jobs_dev, g.begin_dev, (int)g.jobs.size(), g.nblocks,
                                        g.variant, g.lds, s);
    return csx_launch_adjoint_batch(g.jobs_dev, g.begin_dev, (int)g.jobs.size(), g.nblocks,
                                    g.variant, g.lds, s);
}

#define BT_TRY(expr)                 \
    do {                             \
        csx_status s_ = (expr);      \
        if (s_ != CSX_OK) return s_; \
    } while (0)

extern "C" csx_status csx_batch_create(csx_geometry *const *scans, int n, csx_batch **out)
{
    if (!scans || !out || n < 1) return csx_fail(CSX_EINVAL, "need >= 1 scan and an out pointer");
    *out = nullptr;
    for (int k = 0; k < n; ++k) {
        if (!scans[k]) return csx_fail(CSX_EINVAL, "NULL scan handle");
        for (int j = 0; j < k; ++j)   // scans own their workspaces: no sharing
            if (scans[j] == scans[k]) return csx_fail(CSX_EINVAL, "a handle appears twice in the batch");
    }
    csx_batch *b = new (std::nothrow) csx_batch();
    if (!b) return csx_fail(CSX_ENOMEM, "host allocation failed");
    b->h.assign(scans, scans + n);
    auto bail = [&](csx_status st) {
        csx_batch_free(b);
        return st;
    };
    if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipMalloc((void **)&b->iter_dev, sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&b->ej_dev, sizeof(ElemJob) * n) != hipSuccess ||
        hipMalloc((void **)&b->eb_dev, sizeof(int) * 4 * n) != hipSuccess)
        return bail(csx_fail(CSX_EHIP, "batch stream / events / counter / job tables"));
    *out = b;
    return CSX_OK;
}

// One Alg. 5 iteration of the active scans (the body that is captured).
static csx_status issue_iteration(csx_batch *b, const std::vector<int> &active, const float *const *y,
                                  const float *const *r, float *const *f, double beta, size_t jstride,
                                  hipStream_t s)
{
    const int n = (int)b->h.size(), nj = (int)b->ej.size();
    for (const Group &g : b->fwd) BT_TRY(launch_group(g, true, s));
    for (int k : active) {
        csx_geometry *h = b->h[k];
        if (h->iv && b->elem) {
            BT_TRY(csx_iv_forward_parts(h, f[k], s));
            continue;
        }
        if (h->iv)
            BT_TRY(csx_iv_forward(h, f[k], nullptr, 0, h->gws, s));
        else
            BT_TRY(csx_launch_sum_parts(h, csx_forward_shape(h).nparts, h->gws, s));
        BT_TRY(csx_launch_ratio(h, y[k], r ? r[k] : nullptr, true, s));
    }
    if (b->elem) {
        BT_TRY(csx_launch_iv_sum_batch(b->ej_dev, b->eb_dev, nj, b->enb[0], s));
        BT_TRY(csx_launch_elem_batch(0, b->ej_dev, b->eb_dev + n, nj, b->enb[1], beta, 0, nullptr, s));
    }
    for (const Group &g : b->adj) BT_TRY(launch_group(g, false, s));
    for (int k : active)
        if (b->h[k]->iv) BT_TRY(csx_iv_adjoint(b->h[k], b->h[k]->rho, b->h[k]->b2, s));
    if (b->elem) {
        BT_TRY(csx_launch_elem_batch(1, b->ej_dev, b->eb_dev + 2 * n, nj, b->enb[2], beta, b->elem_hub, nullptr, s));
        BT_TRY(csx_launch_elem_batch(2, b->ej_dev, b->eb_dev + 3 * n, nj, b->enb[3], beta, 0, b->iter_dev, s));
    }
    for (int k : active) {
        csx_geometry *h = b->h[k];
        if (h->iv && b->elem) continue;
        BT_TRY(csx_launch_update(h, f[k], beta, true, s));
        BT_TRY(csx_launch_copy_objective(h, f[k], beta, b->J_dev + k * jstride, b->iter_dev, s));
    }
    return csx_launch_iter_incr(b->iter_dev, s);
}

// The ElemJob tables of the active interval-form scans for this call's
// buffers, when every such scan takes the 4-node update and the 16-byte copy
// (nq % 4 == 0, aligned images) and all use one penalty; else those scans
// keep their single-scan launches.
static csx_status elem_jobs(csx_batch *b, const std::vector<int> &active, const float *const *y,
                            const float *const *r, float *const *f, size_t jstride, hipStream_t s)
{
    b->elem = false;
    b->ej.clear();
    const int n = (int)b->h.size();
    std::vector<int> ivs;
    for (int k : active)
        if (b->h[k]->iv) ivs.push_back(k);
    if (ivs.empty()) return CSX_OK;
    int hub = -1;
    for (int k : ivs) {
        const csx_geometry *h = b->h[k];
        const long ne = (long)h->P.nvox * h->P.nq;
        const uintptr_t al = (uintptr_t)f[k] | (uintptr_t)h->b1 | (uintptr_t)h->b2 | (uintptr_t)h->ftmp;
        const int hk = h->psi_delta > 0.0 ? 1 : 0;
        if (h->P.nq % 4 != 0 || ne % 4 != 0 || (al & 15) != 0 || (hub >= 0 && hk != hub)) return CSX_OK;
        hub = hk;
    }
    b->eb.assign(4 * (size_t)n, 0);
    int nb[4] = {0, 0, 0, 0};
    for (size_t i = 0; i < ivs.size(); ++i) {
        const int k = ivs[i];
        csx_geometry *h = b->h[k];
        const KParams &P = h->P;
        const int ne = P.nvox * P.nq;
        ElemJob J;
        std::memset(&J, 0, sizeof(J));
        csx_iv_parts(h, &J.part, &J.nparts);
        J.npix = P.npix;
        J.g = h->gws;
        J.y = y[k];
        J.r = r ? r[k] : nullptr;
        J.rho = h->rho;
        J.partL = h->partL;
        J.partF = h->partF;
        J.nx = P.nx;
        J.nz = P.nz;
        J.nq = P.nq;
        J.f = f[k];
        J.b1 = h->b1;
        J.b2 = h->b2;
        J.ftmp = h->ftmp;
        J.partR = h->partR;
        J.delta = h->psi_delta;
        J.fdst = f[k];
        J.nL = h->nbL;
        J.nR = (ne / 4 + 255) / 256;   // the update's blocks (4 nodes per thread)
        h->nbRu = J.nR;
        J.flags = h->flags;
        J.J = b->J_dev + (size_t)k * jstride;
        const int blocks[4] = {(P.npix + 63) / 64, h->nbL, J.nR, (ne / 4 + 255) / 256 + 1};
        for (int w = 0; w < 4; ++w) {
            b->eb[(size_t)w * n + i] = nb[w];
            nb[w] += blocks[w];
        }
        b->ej.push_back(J);
    }
    for (int w = 0; w < 4; ++w) b->enb[w] = nb[w];
    HIP_TRY(hipMemcpyAsync(b->ej_dev, b->ej.data(), sizeof(ElemJob) * b->ej.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->eb_dev, b->eb.data(), sizeof(int) * b->eb.size(), hipMemcpyHostToDevice, s));
    b->elem = true;
    b->elem_hub = hub;
    return CSX_OK;
}

// J at scan k's current iterate, stored at its iteration counter (single-scan
// launches: the same kernels and shapes as the batched ones).
static csx_status final_objective(csx_batch *b, int k, const float *y, const float *r, float *f, double beta,
                                  size_t jstride, hipStream_t s)
{
    csx_geometry *h = b->h[k];
    BT_TRY(csx_launch_forward(h, f, h->gws, s));
    BT_TRY(csx_launch_ratio(h, y, r, false, s));
    BT_TRY(csx_launch_update(h, f, beta, false, s));
    return csx_launch_objective(h, beta, b->J_dev + k * jstride, b->iter_dev, s);
}

// Replaces the groups by those of the active scans and uploads their job
// tables for this call's buffers (the stream is idle when this runs).
static csx_status regroup(csx_batch *b, const std::vector<int> &active, const float *const *f, hipStream_t s)
{
    free_groups(b->fwd);
    free_groups(b->adj);
    b->fwd.clear();
    b->adj.clear();
    make_groups(b->h, active, true, b->fwd);
    make_groups(b->h, active, false, b->adj);
    const int n = (int)b->h.size();
    std::vector<const float *> in(n);
    std::vector<float *> outp(n, nullptr);
    for (int k = 0; k < n; ++k) in[k] = f[k];
    for (Group &g : b->fwd) BT_TRY(upload_jobs(g, b->h, true, in, outp, s));
    for (int k = 0; k < n; ++k) {
        in[k] = b->h[k]->rho;
        outp[k] = b->h[k]->b2;
    }
    for (Group &g : b->adj) BT_TRY(upload_jobs(g, b->h, false, in, outp, s));
    return CSX_OK;
}

static csx_status replay(csx_batch *b, const std::vector<int> &active, const float *const *y,
                         const float *const *r, float *const *f, double beta, size_t jstride, int steps,
                         hipStream_t s)
{
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    csx_status st = issue_iteration(b, active, y, r, f, beta, jstride, s);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != CSX_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return csx_fail(CSX_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return csx_fail(CSX_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    for (int t = 0; t < steps && e == hipSuccess; ++t) e = hipGraphLaunch(exec, s);
    // the executable graph (and the streams the runtime gives its parallel
    // branches) is destroyed only once its launches have finished
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return csx_fail(CSX_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
    return CSX_OK;
}

extern "C" csx_status csx_batch_recon_n(csx_batch *b, const float *const *y, const float *const *r,
                                        float *const *f, int init_uniform, const int *n_iter, double beta,
                                        double *J_hist, int J_stride, void *stream)
{
    if (!b || !y || !f || !n_iter) return csx_fail(CSX_EINVAL, "NULL argument");
    if (!(std::isfinite(beta) && beta >= 0.0)) return csx_fail(CSX_EINVAL, "beta must be finite and >= 0");
    const int n = (int)b->h.size();
    int n_max = 0;
    for (int k = 0; k < n; ++k) {
        if (!y[k] || !f[k]) return csx_fail(CSX_EINVAL, "NULL scan buffer");
        if (b->h[k]->op_sai) return csx_fail(CSX_EINVAL, "batches use the exact operators (csx_set_operator(h, 0))");
        if (n_iter[k] < 0) return csx_fail(CSX_EINVAL, "n_iter must be >= 0");
        n_max = std::max(n_max, n_iter[k]);
    }
    if (J_hist && J_stride < n_max + 1) return csx_fail(CSX_EINVAL, "J_stride must be >= max(n_iter) + 1");
    hipStream_t cs = (hipStream_t)stream;
    hipStream_t s = b->st;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventRecord(b->ev_in, cs));
    HIP_TRY(hipStreamWaitEvent(s, b->ev_in, 0));

    const size_t jstride = (size_t)n_max + 1;
    if (b->J_cap < jstride * n) {
        if (b->J_dev) HIP_TRY(hipFree(b->J_dev));
        b->J_dev = nullptr;
        b->J_cap = 0;
        HIP_TRY(hipMalloc((void **)&b->J_dev, sizeof(double) * jstride * n));
        b->J_cap = jstride * n;
    }
    std::vector<int> all(n);
    for (int k = 0; k < n; ++k) all[k] = k;

    // sensitivity images of the scans that lack one, batched
    std::vector<int> need;
    for (int k = 0; k < n; ++k)
        if (!b->h[k]->have_b1) need.push_back(k);
    if (!need.empty()) {
        free_groups(b->adj);
        b->adj.clear();
        make_groups(b->h, need, false, b->adj);
        std::vector<const float *> in(n);
        std::vector<float *> outp(n);
        for (int k = 0; k < n; ++k) {
            in[k] = b->h[k]->ones;
            outp[k] = b->h[k]->b1;
        }
        for (Group &g : b->adj) {
            BT_TRY(upload_jobs(g, b->h, false, in, outp, s));
            BT_TRY(launch_group(g, false, s));
        }
        for (int k : need)
            if (b->h[k]->iv) BT_TRY(csx_iv_adjoint(b->h[k], b->h[k]->ones, b->h[k]->b1, s));
        for (int k : need) b->h[k]->have_b1 = true;
        HIP_TRY(hipStreamSynchronize(s));   // the job tables are rebuilt below
    }
    if (init_uniform)
        for (int k = 0; k < n; ++k) BT_TRY(csx_launch_uniform_start(b->h[k], y[k], f[k], s));
    const int zero = 0;
    HIP_TRY(hipMemcpyAsync(b->iter_dev, &zero, sizeof(int), hipMemcpyHostToDevice, s));

    // stages between consecutive distinct iteration counts; a scan leaves the
    // merged launches once it has run its own count
    std::vector<int> counts(n_iter, n_iter + n);
    std::sort(counts.begin(), counts.end());
    counts.erase(std::unique(counts.begin(), counts.end()), counts.end());
    int done = 0;
    for (int c : counts) {
        if (c > done) {
            std::vector<int> active;
            for (int k = 0; k < n; ++k)
                if (n_iter[k] >= c) active.push_back(k);
            HIP_TRY(hipStreamSynchronize(s));   // the previous job tables may still be read
            BT_TRY(regroup(b, active, f, s));
            BT_TRY(elem_jobs(b, active, y, r, f, jstride, s));
            BT_TRY(replay(b, active, y, r, f, beta, jstride, c - done, s));
            done = c;
        }
        for (int k = 0; k < n; ++k)
            if (n_iter[k] == c) BT_TRY(final_objective(b, k, y[k], r ? r[k] : nullptr, f[k], beta, jstride, s));
    }
    std::vector<int> flags(n, 0);
    for (int k = 0; k < n; ++k)
        HIP_TRY(hipMemcpyAsync(&flags[k], b->h[k]->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<double> Jh(jstride * n);
    HIP_TRY(hipMemcpyAsync(Jh.data(), b->J_dev, sizeof(double) * jstride * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventRecord(b->ev_out, s));
    HIP_TRY(hipStreamWaitEvent(cs, b->ev_out, 0));
    if (J_hist)
        for (int k = 0; k < n; ++k)
            for (int t = 0; t <= n_iter[k]; ++t) J_hist[(size_t)k * J_stride + t] = Jh[(size_t)k * jstride + t];
    for (int k = 0; k < n; ++k) {
        if (flags[k] & 2) return csx_fail(CSX_EINVAL, "scan " + std::to_string(k) + ": y holds negative or NaN counts");
        if (flags[k] & 1) return csx_fail(CSX_ENUMERIC, "scan " + std::to_string(k) + ": y_i > 0 where the model mean is 0");
    }
    return CSX_OK;
}

extern "C" csx_status csx_batch_recon(csx_batch *b, const float *const *y, const float *const *r,
                                      float *const *f, int init_uniform, int n_iter, double beta,
                                      double *J_hist, void *stream)
{
    if (!b) return csx_fail(CSX_EINVAL, "NULL argument");
    if (n_iter < 0) return csx_fail(CSX_EINVAL, "n_iter must be >= 0");
    std::vector<int> counts(b->h.size(), n_iter);
    return csx_batch_recon_n(b, y, r, f, init_uniform, counts.data(), beta, J_hist, n_iter + 1, stream);
}
