// csx_probe.hip -- measurement helper: the VALU issue rate of this GPU, from
// a kernel of independent float32 FMA chains (the ceiling the operators'
// roofline fraction is quoted against, beside the published figure).
#include "csx_internal.h"

namespace {

constexpr int PROBE_CHAINS = 8;   // independent chains per lane hide the FMA latency

__global__ void __launch_bounds__(256) k_fma_chains(int iters, float x, float y, float *__restrict__ out)
{
    float a[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = (float)(threadIdx.x + c) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = fmaf(a[c], x, y);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += a[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" csx_status csx_valu_peak(double *lane_ops_per_s, void *stream)
{
    if (!lane_ops_per_s) return csx_fail(CSX_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int blocks = 256 * 32, threads = 256, iters = 4096;
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipMalloc((void **)&out, sizeof(float) * (size_t)blocks * threads));
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // one warm-up launch, then the timed one
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        if (rep == 1) e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_fma_chains, dim3(blocks), dim3(threads), 0, s, iters, 0.999f, 1e-4f, out);
            e = hipGetLastError();
        }
        if (rep == 1 && e == hipSuccess) e = hipEventRecord(e1, s);
    }
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (e != hipSuccess) return csx_fail(CSX_EHIP, std::string("VALU probe: ") + hipGetErrorString(e));
    *lane_ops_per_s = (double)blocks * threads * iters * PROBE_CHAINS / (ms * 1e-3);
    return CSX_OK;
}
