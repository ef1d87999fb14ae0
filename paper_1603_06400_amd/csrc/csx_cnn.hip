// csx_cnn.hip -- the learned warm start's network on gfx950.
//
// Images are height x width x channels, float32 in HBM (the q bins of an
// image [nz][nx][nq] are its channels).  A 3x3 convolution is an implicit
// GEMM on the matrix cores: v_mfma_f32_16x16x16_f16 with binary16 operands
// (activations rounded to nearest-even when staged into LDS, weights held in
// binary16) and binary32 accumulation.
//
//   forward        out[p][o] = bias[o] + sum_{t,i} in[p + off_t][i] W[t][i][o]
//                  M = pixels of a 8 x 16 tile, N = output channels, K = 9 taps x input channels
//   backward data  the same kernel on the output gradient with the taps
//                  reversed and W transposed (FLIP), times the ReLU mask
//   weight grad    dW[t][i][o] = sum_p in[p + off_t][i] dout[p][o]
//                  M = input channels, N = output channels, K = pixels; split
//                  over blocks, partials summed in a fixed order
//
// Weights are [tap][c_in][c_out] with tap = 3 dh + dw reading input pixel
// (row + dh - 1, col + dw - 1); pixels outside the image read 0.  Nothing
// here uses atomics: every result is reproducible bit for bit.
#include "csx_internal.h"

#include <cmath>

namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TH = 8;             // forward tile rows (2 per wave)
constexpr int TW = 16;            // forward tile columns (one MFMA M block)
constexpr int GT = 16;            // weight-gradient pixel tile side
constexpr int WG_BLOCKS = 256;    // weight-gradient partial count (max)
constexpr int RED_BLOCKS = 256;   // loss / bias partial count
constexpr int WG_GROUP = 16;      // weight-gradient partials summed per first-stage group

__device__ inline f4 mfma16(h4 a, h4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

template <int CI, int CO>
struct FwdLds {
    static constexpr int PS = CI + 4;                       // halves per patch pixel
    static constexpr int WS = CI + 4;                       // halves per weight row
    static constexpr int patch = (TH + 2) * (TW + 2) * PS;  // halves
    static constexpr int weights = 9 * CO * WS;
    static constexpr int bytes = 2 * (patch + weights);
};

// out = conv3x3(in) (+ bias, + residual, ReLU) or, with FLIP, the transposed
// convolution of the forward layer whose weights w are [9][CO][CI] (its c_in =
// CO here), times the mask.
template <int CI, int CO, bool FLIP>
__global__ void __launch_bounds__(256)
k_conv3x3(const float *__restrict__ in, const _Float16 *__restrict__ w, const float *__restrict__ bias,
          const float *__restrict__ residual, const float *__restrict__ mask, float *__restrict__ out, int H,
          int W, int relu)
{
    using L = FwdLds<CI, CO>;
    constexpr int PW = TW + 2;
    constexpr int NT = CO / 16;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    _Float16 *sP = reinterpret_cast<_Float16 *>(lds_raw);
    _Float16 *sW = sP + L::patch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, img = blockIdx.z;
    const float *src = in + (size_t)img * H * W * CI;

    // weights -> LDS as [t][o][i] (binary16 already)
    for (int e = tid; e < 9 * CI * CO; e += 256) {
        int t, i, o;
        if (!FLIP) {
            t = e / (CI * CO);
            i = (e / CO) % CI;
            o = e % CO;
        } else {
            t = 8 - e / (CI * CO);
            o = (e / CI) % CO;
            i = e % CI;
        }
        sW[(t * CO + o) * L::WS + i] = w[e];
    }
    // input patch (TH+2) x (TW+2) x CI -> binary16, zero outside the image
    constexpr int C4 = CI / 4;
    for (int e = tid; e < (TH + 2) * PW * C4; e += 256) {
        const int c4 = e % C4, pix = e / C4;
        const int py = pix / PW, px = pix % PW;
        const int gy = y0 - 1 + py, gx = x0 - 1 + px;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *reinterpret_cast<const float4 *>(src + ((size_t)gy * W + gx) * CI + 4 * c4);
        h4 hv = {(_Float16)v.x, (_Float16)v.y, (_Float16)v.z, (_Float16)v.w};
        *reinterpret_cast<h4 *>(sP + pix * L::PS + 4 * c4) = hv;
    }
    __syncthreads();

    const int m = lane & 15, kq = lane >> 4;
    f4 acc[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
        const int dh = t / 3, dw = t % 3;
#pragma unroll
        for (int c = 0; c < CI / 16; ++c) {
            h4 A[2], B[NT];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const int r = wave * 2 + mt;
                A[mt] = *reinterpret_cast<const h4 *>(sP + ((r + dh) * PW + m + dw) * L::PS + c * 16 + 4 * kq);
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                B[nt] = *reinterpret_cast<const h4 *>(sW + (t * CO + nt * 16 + m) * L::WS + c * 16 + 4 * kq);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma16(A[mt], B[nt], acc[mt][nt]);
        }
    }
    // lane holds rows 4 kq + v (tile columns) of output channel nt*16 + m
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const int gy = y0 + wave * 2 + mt;
        if (gy >= H) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gx = x0 + 4 * kq + v;
            if (gx >= W) continue;
            const size_t base = (((size_t)img * H + gy) * W + gx) * CO;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int o = nt * 16 + m;
                float val = acc[mt][nt][v] + (bias ? bias[o] : 0.f);
                if (residual) val += residual[base + o];
                if (relu) val = fmaxf(val, 0.f);
                if (mask && !(mask[base + o] > 0.f)) val = 0.f;
                out[base + o] = val;
            }
        }
    }
}

template <int CI, int CO>
struct WgLds {
    static constexpr int XS = CI + 2;                       // halves per patch pixel
    static constexpr int DS = GT * GT + 4;                  // halves per gradient channel row
    static constexpr int patch = (GT + 2) * (GT + 2) * XS;
    static constexpr int grad = CO * DS;
    static constexpr int bytes = 2 * (patch + grad);
};

// Partial weight gradients of the pixel tiles blockIdx.x, blockIdx.x + G, ...
// part[block][t][i][o], G = gridDim.x.
template <int CI, int CO>
__global__ void __launch_bounds__(256)
k_conv3x3_wgrad(const float *__restrict__ in, const float *__restrict__ dout, float *__restrict__ part,
                int nb, int H, int W)
{
    using L = WgLds<CI, CO>;
    constexpr int PW = GT + 2;
    constexpr int NPAIR = (CI / 16) * (CO / 16);
    constexpr int PPW = NPAIR / 4;                           // (i, o) tile pairs per wave
    static_assert(NPAIR % 4 == 0, "pairs must split over 4 waves");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    _Float16 *sX = reinterpret_cast<_Float16 *>(lds_raw);
    _Float16 *sD = sX + L::patch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int tx = (W + GT - 1) / GT, ty = (H + GT - 1) / GT;
    const int ntiles = nb * tx * ty;

    f4 acc[PPW][9];
#pragma unroll
    for (int p = 0; p < PPW; ++p)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[p][t] = f4{0.f, 0.f, 0.f, 0.f};

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int img = tile / (tx * ty), rem = tile % (tx * ty);
        const int y0 = (rem / tx) * GT, x0 = (rem % tx) * GT;
        const float *xs = in + (size_t)img * H * W * CI;
        const float *ds = dout + (size_t)img * H * W * CO;
        __syncthreads();
        constexpr int C4 = CI / 4;
        for (int e = tid; e < PW * PW * C4; e += 256) {
            const int c4 = e % C4, pix = e / C4;
            const int py = pix / PW, px = pix % PW;
            const int gy = y0 - 1 + py, gx = x0 - 1 + px;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gy >= 0 && gy < H && gx >= 0 && gx < W)
                v = *reinterpret_cast<const float4 *>(xs + ((size_t)gy * W + gx) * CI + 4 * c4);
            _Float16 *d = sX + pix * L::XS + 4 * c4;
            d[0] = (_Float16)v.x;
            d[1] = (_Float16)v.y;
            d[2] = (_Float16)v.z;
            d[3] = (_Float16)v.w;
        }
        for (int e = tid; e < GT * GT * CO; e += 256) {
            const int o = e % CO, pix = e / CO;
            const int gy = y0 + pix / GT, gx = x0 + pix % GT;
            float v = 0.f;
            if (gy < H && gx < W) v = ds[((size_t)gy * W + gx) * CO + o];
            sD[o * L::DS + pix] = (_Float16)v;
        }
        __syncthreads();
#pragma unroll 1
        for (int r = 0; r < GT; ++r) {
            h4 B[PPW];
            int it[PPW];
#pragma unroll
            for (int p = 0; p < PPW; ++p) {
                const int pair = wave * PPW + p;
                it[p] = pair / (CO / 16);
                const int ot = pair % (CO / 16);
                B[p] = *reinterpret_cast<const h4 *>(sD + (ot * 16 + m) * L::DS + r * GT + 4 * kq);
            }
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dh = t / 3, dw = t % 3;
                const _Float16 *row = sX + ((r + dh) * PW + 4 * kq + dw) * L::XS;
#pragma unroll
                for (int p = 0; p < PPW; ++p) {
                    const int ci = it[p] * 16 + m;
                    h4 A = {row[ci], row[L::XS + ci], row[2 * L::XS + ci], row[3 * L::XS + ci]};
                    acc[p][t] = mfma16(A, B[p], acc[p][t]);
                }
            }
        }
    }
    // lane holds input channels it*16 + 4 kq + v of output channel ot*16 + m
    float *dst = part + (size_t)blockIdx.x * 9 * CI * CO;
#pragma unroll
    for (int p = 0; p < PPW; ++p) {
        const int pair = wave * PPW + p;
        const int it = pair / (CO / 16), ot = pair % (CO / 16);
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                dst[((size_t)t * CI + it * 16 + 4 * kq + v) * CO + ot * 16 + m] = acc[p][t][v];
    }
}

// out[g * n + e] = sum of part[k * n + e] over k in [g * per, min((g + 1) * per, nparts)),
// k ascending; g = blockIdx.y.  With gridDim.y = 1 and per = nparts it is the plain sum.
__global__ void __launch_bounds__(256) k_sum_partials(const float *__restrict__ part, int nparts, int n, int per,
                                                      float *__restrict__ out)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const int k0 = blockIdx.y * per;
    const int k1 = k0 + per < nparts ? k0 + per : nparts;
    float s = 0.f;
    for (int k = k0; k < k1; ++k) s += part[(size_t)k * n + e];
    out[(size_t)blockIdx.y * n + e] = s;
}

// Bias gradient partials: block b sums pixels [b*chunk, (b+1)*chunk) of every
// channel; part[b][o].
__global__ void __launch_bounds__(256) k_bias_part(const float *__restrict__ d, long npix, int co,
                                                   long chunk, float *__restrict__ part)
{
    __shared__ float red[256];
    const int tid = threadIdx.x;
    const int lanes = 256 / co;                 // pixel lanes per channel
    const int o = tid % co, sl = tid / co;
    const long p0 = (long)blockIdx.x * chunk;
    const long p1 = p0 + chunk < npix ? p0 + chunk : npix;
    float s = 0.f;
    if (sl < lanes)
        for (long p = p0 + sl; p < p1; p += lanes) s += d[p * co + o];
    red[tid] = s;
    __syncthreads();
    if (tid < co) {
        float t = 0.f;
        for (int k = 0; k < lanes; ++k) t += red[k * co + tid];
        part[(size_t)blockIdx.x * co + tid] = t;
    }
}

constexpr float WARM_CLAMP = 30.f;     // upper bound of o before exponentiation
constexpr float WARM_FLOOR = 0.01f;    // f0 / u >= WARM_FLOOR * delta

__device__ double block_sum_f64(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// d = 2 (o - t) / n_images; float64 partial sums of (o - t)^2.
__global__ void __launch_bounds__(256) k_head(const float *__restrict__ o, const float *__restrict__ t,
                                              long n, long chunk, float inv_images, float *__restrict__ d,
                                              double *__restrict__ part)
{
    __shared__ double red[256];
    const long e0 = (long)blockIdx.x * chunk;
    const long e1 = e0 + chunk < n ? e0 + chunk : n;
    double s = 0.0;
    for (long e = e0 + threadIdx.x; e < e1; e += 256) {
        const float r = o[e] - t[e];
        d[e] = 2.f * r * inv_images;
        s += (double)r * (double)r;
    }
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_loss_final(const double *__restrict__ part, int nparts,
                                                    double inv_images, double *__restrict__ loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) s += part[k];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) *loss = s * inv_images;
}

__global__ void __launch_bounds__(256) k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, _Float16 *__restrict__ w16, int n,
                                              float lr, float b1, float b2, float eps, float bc1, float bc2)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float we = w[e] - lr * (me / bc1) / (sqrtf(ve / bc2) + eps);
    w[e] = we;
    if (w16) w16[e] = (_Float16)we;
}

__global__ void __launch_bounds__(256) k_to_half(const float *__restrict__ x, _Float16 *__restrict__ y, int n)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n) y[e] = (_Float16)x[e];
}

// rho = y / (u A1), u = sum(y) / sum(b1) = scal[0] / scal[1]; 0 where A1 = 0
__global__ void __launch_bounds__(256) k_warm_ratio(const float *__restrict__ y, const float *__restrict__ a1,
                                                    int n, const double *__restrict__ scal, float *__restrict__ rho)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float u = (float)(scal[0] / scal[1]);
    const float z = u * a1[e];
    rho[e] = z > 0.f ? y[e] / z : 0.f;
}

// x = log(b / b1 + delta), b / b1 taken as 0 where b1 = 0
__global__ void __launch_bounds__(256) k_warm_input(float *__restrict__ x, const float *__restrict__ b1, int n,
                                                    float delta)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float s = b1[e];
    x[e] = logf((s > 0.f ? x[e] / s : 0.f) + delta);
}

// t = log(f / u + delta)
__global__ void __launch_bounds__(256) k_warm_target(const float *__restrict__ f, float *__restrict__ t, int n,
                                                     const double *__restrict__ scal, float delta)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float u = (float)(scal[0] / scal[1]);
    t[e] = logf(f[e] / u + delta);
}

// f0 = u max(exp(min(o, WARM_CLAMP)) - delta, WARM_FLOOR delta)
__global__ void __launch_bounds__(256) k_warm_output(const float *__restrict__ o, float *__restrict__ f0, int n,
                                                     const double *__restrict__ scal, float delta)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float u = (float)(scal[0] / scal[1]);
    f0[e] = u * fmaxf(expf(fminf(o[e], WARM_CLAMP)) - delta, WARM_FLOOR * delta);
}

// part[b] = sum of b1 f over block b's contiguous share (float64)
__global__ void __launch_bounds__(256) k_mass_part(const float *__restrict__ b1, const float *__restrict__ f,
                                                   long n, long chunk, double *__restrict__ part)
{
    __shared__ double red[256];
    const long e0 = (long)blockIdx.x * chunk;
    const long e1 = e0 + chunk < n ? e0 + chunk : n;
    double s = 0.0;
    for (long e = e0 + threadIdx.x; e < e1; e += 256) s += (double)b1[e] * (double)f[e];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// scal[2] = sum of the partials, fixed order
__global__ void __launch_bounds__(256) k_mass_final(const double *__restrict__ part, int nparts,
                                                    double *__restrict__ scal)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) s += part[k];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) scal[2] = s;
}

// f *= sum(y) / sum(b1 f) = scal[0] / scal[2]
__global__ void __launch_bounds__(256) k_mass_scale(float *__restrict__ f, int n, const double *__restrict__ scal)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    f[e] = (float)((double)f[e] * (scal[0] / scal[2]));
}

csx_status check_delta(float delta)
{
    if (!(delta > 0.f && delta <= 1.f)) return csx_fail(CSX_EINVAL, "delta must be in (0, 1]");
    return CSX_OK;
}

bool channels_ok(int ci, int co)
{
    return (ci == 64 && co == 32) || (ci == 32 && co == 32) || (ci == 32 && co == 64);
}

template <int CI, int CO, bool FLIP>
csx_status run_conv(const float *in, const _Float16 *w, const float *bias, const float *residual,
                    const float *mask, float *out, int nb, int H, int W, int relu, hipStream_t s)
{
    dim3 grid((W + TW - 1) / TW, (H + TH - 1) / TH, nb);
    constexpr int lds = FwdLds<CI, CO>::bytes;
    hipLaunchKernelGGL((k_conv3x3<CI, CO, FLIP>), grid, dim3(256), lds, s, in, w, bias,
                       residual, mask, out, H, W, relu);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

int wgrad_blocks(int nb, int H, int W)
{
    const long tiles = (long)nb * ((H + GT - 1) / GT) * ((W + GT - 1) / GT);
    return (int)(tiles < WG_BLOCKS ? tiles : WG_BLOCKS);
}

template <int CI, int CO>
csx_status run_wgrad(const float *in, const float *dout, float *part, int nblk, int nb, int H, int W,
                     hipStream_t s)
{
    constexpr int lds = WgLds<CI, CO>::bytes;
    hipLaunchKernelGGL((k_conv3x3_wgrad<CI, CO>), dim3(nblk), dim3(256), lds, s, in, dout,
                       part, nb, H, W);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

csx_status check_dims(int nb, int H, int W)
{
    if (nb < 1 || H < 1 || W < 1) return csx_fail(CSX_EINVAL, "image batch dimensions must be >= 1");
    if ((double)nb * H * W * 64 > 2147483647.0) return csx_fail(CSX_EINVAL, "image batch too large");
    return CSX_OK;
}

}  // namespace

// Workspace layout (floats): weight partials [nblk][9*64*32], bias partials
// [RED_BLOCKS][64], first-stage group sums [WG_BLOCKS/WG_GROUP][9*64*32]; the
// loss head uses the front as [RED_BLOCKS] doubles.
size_t csx_cnn_ws_floats(int nb, int H, int W)
{
    const size_t wg = (size_t)wgrad_blocks(nb, H, W) * 9 * 64 * 32;
    const size_t bias = (size_t)RED_BLOCKS * 64;
    const size_t groups = (size_t)((WG_BLOCKS + WG_GROUP - 1) / WG_GROUP) * 9 * 64 * 32;
    const size_t head = 2 * RED_BLOCKS;                     // doubles
    return (wg + bias + groups > head ? wg + bias + groups : head) + 64;
}

extern "C" size_t csx_cnn_workspace_bytes(int nb, int h, int w)
{
    if (nb < 1 || h < 1 || w < 1) return 0;
    return sizeof(float) * csx_cnn_ws_floats(nb, h, w);
}

extern "C" csx_status csx_conv3x3_forward(const float *x, const uint16_t *w, const float *bias,
                                          const float *residual, float *y, int nb, int h, int w_, int cin,
                                          int cout, int relu, void *stream)
{
    if (!x || !w || !y) return csx_fail(CSX_EINVAL, "NULL argument");
    if (!channels_ok(cin, cout)) return csx_fail(CSX_EINVAL, "unsupported channel pair (64,32), (32,32), (32,64)");
    csx_status st = check_dims(nb, h, w_);
    if (st != CSX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const _Float16 *wh = reinterpret_cast<const _Float16 *>(w);
    if (residual == y) return csx_fail(CSX_EINVAL, "residual and y must be different buffers");
    if (cin == 64) return run_conv<64, 32, false>(x, wh, bias, residual, nullptr, y, nb, h, w_, relu, s);
    if (cout == 32) return run_conv<32, 32, false>(x, wh, bias, residual, nullptr, y, nb, h, w_, relu, s);
    return run_conv<32, 64, false>(x, wh, bias, residual, nullptr, y, nb, h, w_, relu, s);
}

extern "C" csx_status csx_conv3x3_backward_data(const float *dy, const uint16_t *w, const float *mask, float *dx,
                                                int nb, int h, int w_, int cin, int cout, void *stream)
{
    if (!dy || !w || !dx) return csx_fail(CSX_EINVAL, "NULL argument");
    if (!channels_ok(cin, cout)) return csx_fail(CSX_EINVAL, "unsupported channel pair (64,32), (32,32), (32,64)");
    csx_status st = check_dims(nb, h, w_);
    if (st != CSX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const _Float16 *wh = reinterpret_cast<const _Float16 *>(w);
    // transposed layer: input channels = cout, output channels = cin
    if (cin == 64) return run_conv<32, 64, true>(dy, wh, nullptr, nullptr, mask, dx, nb, h, w_, 0, s);
    if (cout == 32) return run_conv<32, 32, true>(dy, wh, nullptr, nullptr, mask, dx, nb, h, w_, 0, s);
    return run_conv<64, 32, true>(dy, wh, nullptr, nullptr, mask, dx, nb, h, w_, 0, s);
}

extern "C" csx_status csx_conv3x3_backward_weights(const float *x, const float *dy, float *dw, float *dbias,
                                                   int nb, int h, int w_, int cin, int cout, void *ws,
                                                   size_t ws_bytes, void *stream)
{
    if (!x || !dy || !dw || !ws) return csx_fail(CSX_EINVAL, "NULL argument");
    if (!channels_ok(cin, cout)) return csx_fail(CSX_EINVAL, "unsupported channel pair (64,32), (32,32), (32,64)");
    csx_status st = check_dims(nb, h, w_);
    if (st != CSX_OK) return st;
    if (ws_bytes < csx_cnn_workspace_bytes(nb, h, w_)) return csx_fail(CSX_EINVAL, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    float *part = static_cast<float *>(ws);
    const int nblk = wgrad_blocks(nb, h, w_);
    if (cin == 64) st = run_wgrad<64, 32>(x, dy, part, nblk, nb, h, w_, s);
    else if (cout == 32) st = run_wgrad<32, 32>(x, dy, part, nblk, nb, h, w_, s);
    else st = run_wgrad<32, 64>(x, dy, part, nblk, nb, h, w_, s);
    if (st != CSX_OK) return st;
    // two fixed-order stages: groups of WG_GROUP partials, then the group sums
    const int n = 9 * cin * cout;
    const int ngrp = (nblk + WG_GROUP - 1) / WG_GROUP;
    float *gsum = part + (size_t)nblk * 9 * 64 * 32 + (size_t)RED_BLOCKS * 64;
    hipLaunchKernelGGL(k_sum_partials, dim3((n + 255) / 256, ngrp), dim3(256), 0, s, part, nblk, n, WG_GROUP,
                       gsum);
    hipLaunchKernelGGL(k_sum_partials, dim3((n + 255) / 256, 1), dim3(256), 0, s, gsum, ngrp, n, ngrp, dw);
    HIP_TRY(hipGetLastError());
    if (dbias) {
        const long npix = (long)nb * h * w_;
        const long chunk = (npix + RED_BLOCKS - 1) / RED_BLOCKS;
        const int nbb = (int)((npix + chunk - 1) / chunk);
        float *bpart = part + (size_t)nblk * 9 * 64 * 32;   // after the weight partials
        hipLaunchKernelGGL(k_bias_part, dim3(nbb), dim3(256), 0, s, dy, npix, cout, chunk, bpart);
        hipLaunchKernelGGL(k_sum_partials, dim3(1, 1), dim3(256), 0, s, bpart, nbb, cout, nbb, dbias);
        HIP_TRY(hipGetLastError());
    }
    return CSX_OK;
}

extern "C" csx_status csx_warm_loss(const float *o, const float *t, int nb, int n_per_image, float *d,
                                    double *loss, void *ws, size_t ws_bytes, void *stream)
{
    if (!o || !t || !d || !loss || !ws) return csx_fail(CSX_EINVAL, "NULL argument");
    if (nb < 1 || n_per_image < 1) return csx_fail(CSX_EINVAL, "sizes must be >= 1");
    if (ws_bytes < sizeof(double) * RED_BLOCKS) return csx_fail(CSX_EINVAL, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const long n = (long)nb * n_per_image;
    const long chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
    const int nbk = (int)((n + chunk - 1) / chunk);
    double *part = static_cast<double *>(ws);
    hipLaunchKernelGGL(k_head, dim3(nbk), dim3(256), 0, s, o, t, n, chunk, 1.f / (float)nb, d, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, part, nbk, 1.0 / nb, loss);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

extern "C" csx_status csx_adam_step(float *w, float *m, float *v, const float *g, uint16_t *w16, int n,
                                    double lr, double beta1, double beta2, double eps, int step, void *stream)
{
    if (!w || !m || !v || !g) return csx_fail(CSX_EINVAL, "NULL argument");
    if (n < 1 || step < 1) return csx_fail(CSX_EINVAL, "n and step must be >= 1");
    if (!(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0))
        return csx_fail(CSX_EINVAL, "Adam hyper-parameters out of range");
    const float bc1 = (float)(1.0 - std::pow(beta1, step));
    const float bc2 = (float)(1.0 - std::pow(beta2, step));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, w, m, v, g,
                       reinterpret_cast<_Float16 *>(w16), n, (float)lr, (float)beta1, (float)beta2, (float)eps,
                       bc1, bc2);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

extern "C" csx_status csx_to_half(const float *x, uint16_t *y, int n, void *stream)
{
    if (!x || !y || n < 1) return csx_fail(CSX_EINVAL, "NULL argument or n < 1");
    hipLaunchKernelGGL(k_to_half, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, x,
                       reinterpret_cast<_Float16 *>(y), n);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

extern "C" csx_status csx_warm_input(csx_geometry *h, const float *y, float delta, float *x, void *stream)
{
    if (!h || !y || !x) return csx_fail(CSX_EINVAL, "NULL argument");
    csx_status st = check_delta(delta);
    if (st != CSX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = csx_ensure_b1(h, s);
    if (st != CSX_OK) return st;
    const int n = h->P.nvox * h->P.nq, np = h->P.npix;
    if (!h->a1) {   // A 1, once per handle
        HIP_TRY(hipMalloc((void **)&h->a1, sizeof(float) * np));
        st = csx_launch_fill(h->ftmp, n, 1.f, s);
        if (st == CSX_OK) st = csx_launch_forward(h, h->ftmp, h->a1, s);
        if (st != CSX_OK) {
            (void)hipFree(h->a1);
            h->a1 = nullptr;
            return st;
        }
    }
    st = csx_launch_uniform_sums(h, y, s);
    if (st != CSX_OK) return st;
    hipLaunchKernelGGL(k_warm_ratio, dim3((np + 255) / 256), dim3(256), 0, s, y, h->a1, np, h->scal, h->rho);
    HIP_TRY(hipGetLastError());
    st = csx_launch_adjoint(h, h->rho, x, s);
    if (st != CSX_OK) return st;
    hipLaunchKernelGGL(k_warm_input, dim3((n + 255) / 256), dim3(256), 0, s, x, h->b1, n, delta);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

extern "C" csx_status csx_warm_target(csx_geometry *h, const float *y, const float *f, float delta, float *t,
                                      void *stream)
{
    if (!h || !y || !f || !t) return csx_fail(CSX_EINVAL, "NULL argument");
    csx_status st = check_delta(delta);
    if (st != CSX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = csx_ensure_b1(h, s);
    if (st != CSX_OK) return st;
    st = csx_launch_uniform_sums(h, y, s);
    if (st != CSX_OK) return st;
    const int n = h->P.nvox * h->P.nq;
    hipLaunchKernelGGL(k_warm_target, dim3((n + 255) / 256), dim3(256), 0, s, f, t, n, h->scal, delta);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

extern "C" csx_status csx_warm_output(csx_geometry *h, const float *y, const float *o, float delta, float *f0,
                                      void *stream)
{
    if (!h || !y || !o || !f0) return csx_fail(CSX_EINVAL, "NULL argument");
    csx_status st = check_delta(delta);
    if (st != CSX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    st = csx_ensure_b1(h, s);
    if (st != CSX_OK) return st;
    st = csx_launch_uniform_sums(h, y, s);
    if (st != CSX_OK) return st;
    const int n = h->P.nvox * h->P.nq;
    hipLaunchKernelGGL(k_warm_output, dim3((n + 255) / 256), dim3(256), 0, s, o, f0, n, h->scal, delta);
    const long chunk = ((long)n + CSX_SUM_BLOCKS - 1) / CSX_SUM_BLOCKS;
    const int nbk = (int)(((long)n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_mass_part, dim3(nbk), dim3(256), 0, s, h->b1, f0, (long)n, chunk, h->partS);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, s, h->partS, nbk, h->scal);
    hipLaunchKernelGGL(k_mass_scale, dim3((n + 255) / 256), dim3(256), 0, s, f0, n, h->scal);
    HIP_TRY(hipGetLastError());
    return CSX_OK;
}

extern "C" csx_status csx_warm_start(csx_geometry *h, const float *y, const csx_warm_net *net, float delta,
                                     float *f0, void *stream)
{
    if (!h || !y || !net || !f0) return csx_fail(CSX_EINVAL, "NULL argument");
    const int ch[5] = {h->P.nq, 32, 32, 32, h->P.nq};
    if (h->P.nq != 64) return csx_fail(CSX_EINVAL, "the warm-start network takes nq = 64 channels");
    for (int k = 0; k < 4; ++k)
        if (!net->w[k] || !net->b[k]) return csx_fail(CSX_EINVAL, "NULL layer pointer");
    hipStream_t s = (hipStream_t)stream;
    const int H = h->P.nz, W = h->P.nx;
    const size_t img = (size_t)H * W;
    const size_t need = img * (64 + 32 + 32 + 64);
    if (h->warm_cap < need) {
        if (h->warm) HIP_TRY(hipFree(h->warm));
        h->warm = nullptr;
        h->warm_cap = 0;
        HIP_TRY(hipMalloc((void **)&h->warm, sizeof(float) * need));
        h->warm_cap = need;
    }
    float *xin = h->warm;                 // [H][W][64] network input
    float *a = xin + img * 64, *b = a + img * 32, *o = b + img * 32;
    csx_status st = csx_warm_input(h, y, delta, xin, stream);
    if (st != CSX_OK) return st;
    const float *src[4] = {xin, a, b, a};
    float *dst[4] = {a, b, a, o};
    for (int k = 0; k < 4; ++k) {
        st = csx_conv3x3_forward(src[k], net->w[k], net->b[k], k == 3 ? xin : nullptr, dst[k], 1, H, W, ch[k],
                                 ch[k + 1], k < 3, s);
        if (st != CSX_OK) return st;
    }
    return csx_warm_output(h, y, o, delta, f0, stream);
}
