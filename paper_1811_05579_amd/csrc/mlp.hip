// mlp.hip -- training and inference kernels of the learned Newton initial
// guess (the grte_mlp_* calls of include/grte.h).
//
// Training data are rows of six binary32 values, (f_0..f_4, log(T^{n+1}/T^n)),
// written by grte_log_pairs from converged steps of the solver itself.  One
// training step on a minibatch of B rows is two kernels:
//   mlp_grad_kernel  one wavefront per 64 rows: forward and backward pass of
//                    every row in registers (binary32), the per-row vectors
//                    (h1, h2, dL/dz1, dL/dz2, x) in LDS, then each lane forms
//                    whole gradient entries as fixed-order sums over the 64
//                    rows -> per-block partial gradient (deterministic, no
//                    atomics);
//   mlp_adam_kernel  sums the partials in block order, applies Adam with bias
//                    correction to the binary32 master parameters and writes
//                    their bfloat16 copy (round to nearest even).
// The loss is the mean squared error of the standardised target.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/grte.h"
#include "mlp_common.hpp"

namespace {
constexpr int GB = 64;                 // rows per training block (one wavefront)
}

// Workspace of grte_mlp_train_noalloc: per-block partial gradients, partial
// losses and the loss history, in one file-scope device array that each device
// holds until the process ends.  In host code the array's name only stands
// for it: its address on a device comes from hipGetSymbolAddress, taken once
// per device with that device current, and kept.
constexpr int NOALLOC_MAX_BATCH = 16384;                      // rows per minibatch
constexpr int NOALLOC_MAX_BLOCKS = NOALLOC_MAX_BATCH / GB;    // 256 gradient blocks
constexpr int NOALLOC_MAX_STEPS = 65536;                      // loss-history entries
constexpr size_t NOALLOC_FLOATS =
    (size_t)NOALLOC_MAX_BLOCKS * MLP_NPARAM + NOALLOC_MAX_BLOCKS + NOALLOC_MAX_STEPS;   // 4.98 MB

static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

namespace {

constexpr int HS = MLP_H + 1;          // padded LDS row stride (conflict-free)
constexpr int NPAD = 4612;             // parameters in LDS, padded

constexpr size_t grad_lds_bytes() { return (size_t)(NPAD + 4 * GB * HS + GB * 8 + 2 * GB) * sizeof(float); }

__global__ void __launch_bounds__(GB) mlp_grad_kernel(const float *theta, const float *norm, const float *data,
                                                      long long n, long long start, int B, float *gpart,
                                                      float *lpart)
{
    extern __shared__ float sm[];
    float *sW = sm;
    float *sH1 = sW + NPAD, *sH2 = sH1 + GB * HS, *sD2 = sH2 + GB * HS, *sD1 = sD2 + GB * HS;
    float *sX = sD1 + GB * HS, *sDy = sX + GB * 8, *sL = sDy + GB;
    const int t = threadIdx.x;
    for (int e = t; e < MLP_NPARAM; e += GB) sW[e] = theta[e];
    __syncthreads();
    const int s = blockIdx.x * GB + t;
    const bool valid = s < B;
    float x[MLP_IN], tg = 0.0f;
    {
        const long long row = valid ? (start + s) % n : 0;
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) x[q] = valid ? (data[row * 6 + q] - norm[q]) / norm[MLP_IN + q] : 0.0f;
        if (valid) tg = (data[row * 6 + 5] - norm[2 * MLP_IN]) / norm[2 * MLP_IN + 1];
    }
    // forward
    float z1[MLP_H], h1[MLP_H], z2[MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) {
        float z = sW[MLP_OB1 + i];
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) z += sW[MLP_OW1 + MLP_IN * i + q] * x[q];
        z1[i] = z;
        h1[i] = gelu_f(z);
        sH1[t * HS + i] = h1[i];
    }
    float y = sW[MLP_OB3];
    for (int i = 0; i < MLP_H; ++i) {
        float z = sW[MLP_OB2 + i];
#pragma unroll
        for (int j = 0; j < MLP_H; ++j) z += sW[MLP_OW2 + MLP_H * i + j] * h1[j];
        z2[i] = z;
        const float h2 = gelu_f(z);
        sH2[t * HS + i] = h2;
        y += sW[MLP_OW3 + i] * h2;
    }
    // backward: dL/dy, dL/dz2, dL/dz1
    const float dy = valid ? 2.0f * (y - tg) / (float)B : 0.0f;
    sDy[t] = dy;
    sL[t] = valid ? (y - tg) * (y - tg) : 0.0f;
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) {
        const float d2 = dy * sW[MLP_OW3 + i] * gelu_prime_f(z2[i]);
        z2[i] = d2;
        sD2[t * HS + i] = d2;
    }
    for (int j = 0; j < MLP_H; ++j) {
        float dh = 0.0f;
#pragma unroll
        for (int i = 0; i < MLP_H; ++i) dh += sW[MLP_OW2 + MLP_H * i + j] * z2[i];
        sD1[t * HS + j] = dh * gelu_prime_f(z1[j]);
    }
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) sX[t * 8 + q] = x[q];
    __syncthreads();
    // gradient entries of this block: fixed-order sums over its rows
    float *g = gpart + (size_t)blockIdx.x * MLP_NPARAM;
    for (int e = t; e < MLP_NPARAM; e += GB) {
        float acc = 0.0f;
        if (e < MLP_OB1) {                 // W1[i, q]
            const int i = e / MLP_IN, q = e - (e / MLP_IN) * MLP_IN;
            for (int r = 0; r < GB; ++r) acc += sD1[r * HS + i] * sX[r * 8 + q];
        } else if (e < MLP_OW2) {          // b1[i]
            const int i = e - MLP_OB1;
            for (int r = 0; r < GB; ++r) acc += sD1[r * HS + i];
        } else if (e < MLP_OB2) {          // W2[i, j]
            const int i = (e - MLP_OW2) / MLP_H, j = (e - MLP_OW2) - ((e - MLP_OW2) / MLP_H) * MLP_H;
            for (int r = 0; r < GB; ++r) acc += sD2[r * HS + i] * sH1[r * HS + j];
        } else if (e < MLP_OW3) {          // b2[i]
            const int i = e - MLP_OB2;
            for (int r = 0; r < GB; ++r) acc += sD2[r * HS + i];
        } else if (e < MLP_OB3) {          // W3[i]
            const int i = e - MLP_OW3;
            for (int r = 0; r < GB; ++r) acc += sDy[r] * sH2[r * HS + i];
        } else {                           // b3
            for (int r = 0; r < GB; ++r) acc += sDy[r];
        }
        g[e] = acc;
    }
    if (t == 0) {
        float l = 0.0f;
        for (int r = 0; r < GB; ++r) l += sL[r];
        lpart[blockIdx.x] = l;
    }
}

__global__ void mlp_adam_kernel(float *theta, float *am, float *av, uint16_t *wbf, const float *gpart, int nblk,
                                const float *lpart, int B, float *lhist, int hidx, float lr, float c1, float c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && lhist) {
        float l = 0.0f;
        for (int b = 0; b < nblk; ++b) l += lpart[b];
        lhist[hidx] = l / (float)B;
    }
    if (e >= MLP_NPARAM) return;
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += gpart[(size_t)b * MLP_NPARAM + e];
    const float beta1 = 0.9f, beta2 = 0.999f;
    const float m = beta1 * am[e] + (1.0f - beta1) * g;
    const float v = beta2 * av[e] + (1.0f - beta2) * g * g;
    am[e] = m;
    av[e] = v;
    // c1 = 1 - beta1^k, c2 = 1 - beta2^k (bias correction, computed on the host in binary64)
    const float th = theta[e] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
    theta[e] = th;
    wbf[e] = f_to_bf16(th);
}

__global__ void mlp_round_kernel(const float *theta, uint16_t *wbf)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < MLP_NPARAM) wbf[e] = f_to_bf16(theta[e]);
}

// mean and standard deviation of the six columns (binary64 sums in row order)
__global__ void __launch_bounds__(256) mlp_norm_kernel(const float *data, long long n, float *norm)
{
    __shared__ double s1[256][6], s2[256][6];
    const int t = threadIdx.x;
    double a[6] = {0, 0, 0, 0, 0, 0}, b[6] = {0, 0, 0, 0, 0, 0};
    for (long long r = t; r < n; r += 256)
        for (int q = 0; q < 6; ++q) {
            const double v = data[r * 6 + q];
            a[q] += v;
            b[q] += v * v;
        }
    for (int q = 0; q < 6; ++q) {
        s1[t][q] = a[q];
        s2[t][q] = b[q];
    }
    __syncthreads();
    if (t < 6) {
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < 256; ++k) {
            sa += s1[k][t];
            sb += s2[k][t];
        }
        const double mean = sa / (double)n;
        const double var = fmax(sb / (double)n - mean * mean, 0.0);
        const double sd = var > 0.0 ? sqrt(var) : 1.0;
        if (t < 5) {
            norm[t] = (float)mean;
            norm[5 + t] = (float)sd;
        } else {
            norm[10] = (float)mean;
            norm[11] = (float)sd;
        }
    }
}

__global__ void __launch_bounds__(256) mlp_predict_kernel(const uint16_t *wbf, const float *norm, const float *data,
                                                          long long n, float *y)
{
    __shared__ uint16_t sW[MLP_NPARAM + 3];
    __shared__ float sN[MLP_NNORM];
    for (int e = threadIdx.x; e < MLP_NPARAM; e += 256) sW[e] = wbf[e];
    if (threadIdx.x < MLP_NNORM) sN[threadIdx.x] = norm[threadIdx.x];
    __syncthreads();
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    float f[MLP_IN];
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) f[q] = data[r * 6 + q];
    y[r] = mlp_eval(sW, sN, f);
}

grte_status mhip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GRTE_OK;
    fprintf(stderr, "grte_mlp: %s failed: %s\n", what, hipGetErrorString(e));
    return GRTE_E_HIP;
}

#define MCHK(x)                                                 \
    do {                                                        \
        grte_status _s = mhip((x), #x);                         \
        if (_s != GRTE_OK) return _s;                           \
    } while (0)

grte_status ensure_gpart(grte_mlp *m, int nblk)
{
    if (nblk <= m->gcap) return GRTE_OK;
    if (m->gpart) (void)hipFree(m->gpart);
    if (m->lpart) (void)hipFree(m->lpart);
    m->gpart = nullptr;
    m->lpart = nullptr;
    m->gcap = 0;
    if (hipMalloc((void **)&m->gpart, (size_t)nblk * MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->lpart, (size_t)nblk * sizeof(float)) != hipSuccess)
        return GRTE_E_NOMEM;
    m->gcap = nblk;
    return GRTE_OK;
}

grte_status grad_lds_attribute()
{
    static bool lds_set = false;
    if (!lds_set) {
        MCHK(hipFuncSetAttribute((const void *)mlp_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)grad_lds_bytes()));
        lds_set = true;
    }
    return GRTE_OK;
}

// per-block partial gradients and losses into gpart/lpart (nblk = ceil(B / GB) blocks)
grte_status launch_grad_into(grte_mlp *m, const float *data, long long n, long long start, int B, float *gpart,
                             float *lpart)
{
    grte_status st = grad_lds_attribute();
    if (st != GRTE_OK) return st;
    const int nblk = (B + GB - 1) / GB;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(GB), grad_lds_bytes(), m->stream, m->theta, m->norm, data,
                       n, start, B, gpart, lpart);
    MCHK(hipGetLastError());
    return GRTE_OK;
}

grte_status launch_grad(grte_mlp *m, const float *data, long long n, long long start, int B)
{
    const int nblk = (B + GB - 1) / GB;
    grte_status st = ensure_gpart(m, nblk);
    if (st != GRTE_OK) return st;
    return launch_grad_into(m, data, n, start, B, m->gpart, m->lpart);
}

// `steps` Adam steps on minibatches of B rows, taken cyclically from the n
// rows; the per-block partials go to gpart/lpart, the loss of step k to
// lhist[k] (device, null: not recorded).  Allocates nothing.
grte_status train_steps(grte_mlp *m, const float *data, long long n, int steps, int B, float lr, float *gpart,
                        float *lpart, float *lhist)
{
    const int nblk = (B + GB - 1) / GB;
    long long start = 0;
    for (int k = 0; k < steps; ++k) {
        grte_status st = launch_grad_into(m, data, n, start, B, gpart, lpart);
        if (st != GRTE_OK) return st;
        start = (start + B) % n;
        const int kk = ++m->adam_k;
        const float c1 = (float)(1.0 - std::pow(0.9, kk)), c2 = (float)(1.0 - std::pow(0.999, kk));
        hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, m->stream, m->theta,
                           m->am, m->av, m->wbf, gpart, nblk, lpart, B, lhist, k, lr, c1, c2);
        MCHK(hipGetLastError());
    }
    return GRTE_OK;
}

// ---- the training entry point that allocates nothing (grte_mlp_train_noalloc):
// the device address of the file-scope workspace, per device
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mutex;
float *scratch_ptr[NOALLOC_MAX_DEVICES] = {};

grte_status scratch_on_device(float **out)
{
    int dev = -1;
    MCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return GRTE_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        MCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return GRTE_E_HIP;
        scratch_ptr[dev] = (float *)p;
    }
    *out = scratch_ptr[dev];
    return GRTE_OK;
}

}  // namespace

extern "C" {

grte_status grte_mlp_destroy(grte_mlp *m)
{
    if (!m) return GRTE_OK;
    void *ps[] = {m->theta, m->wbf, m->am, m->av, m->norm, m->gpart, m->lpart, m->lhist};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete m;
    return GRTE_OK;
}

grte_status grte_mlp_create(grte_mlp **out)
{
    if (!out) return GRTE_E_INVAL;
    *out = nullptr;
    grte_mlp *m = new (std::nothrow) grte_mlp();
    if (!m) return GRTE_E_NOMEM;
    if (hipMalloc((void **)&m->theta, MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->wbf, (MLP_NPARAM + 3) * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc((void **)&m->am, MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->av, MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&m->norm, MLP_NNORM * sizeof(float)) != hipSuccess) {
        grte_mlp_destroy(m);
        return GRTE_E_NOMEM;
    }
    const float unit[MLP_NNORM] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0, 1};
    std::vector<float> z(MLP_NPARAM, 0.0f);
    if (hipMemcpy(m->theta, z.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->am, z.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->av, z.data(), MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->norm, unit, sizeof(unit), hipMemcpyHostToDevice) != hipSuccess) {
        grte_mlp_destroy(m);
        return GRTE_E_HIP;
    }
    hipLaunchKernelGGL(mlp_round_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, nullptr, m->theta, m->wbf);
    if (hipDeviceSynchronize() != hipSuccess) {
        grte_mlp_destroy(m);
        return GRTE_E_HIP;
    }
    *out = m;
    return GRTE_OK;
}

grte_status grte_mlp_set_stream(grte_mlp *m, void *hip_stream)
{
    if (!m) return GRTE_E_INVAL;
    m->stream = (hipStream_t)hip_stream;
    return GRTE_OK;
}

grte_status grte_mlp_set_params(grte_mlp *m, const float *theta)
{
    if (!m || !theta) return GRTE_E_INVAL;
    for (int e = 0; e < MLP_NPARAM; ++e)
        if (!std::isfinite(theta[e])) return GRTE_E_INVAL;
    MCHK(hipMemcpyAsync(m->theta, theta, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemsetAsync(m->am, 0, MLP_NPARAM * sizeof(float), m->stream));
    MCHK(hipMemsetAsync(m->av, 0, MLP_NPARAM * sizeof(float), m->stream));
    hipLaunchKernelGGL(mlp_round_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, m->stream, m->theta, m->wbf);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
    m->adam_k = 0;
    return GRTE_OK;
}

grte_status grte_mlp_get_params(grte_mlp *m, float *theta, unsigned short *theta_bf16)
{
    if (!m) return GRTE_E_INVAL;
    if (theta) MCHK(hipMemcpyAsync(theta, m->theta, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    if (theta_bf16)
        MCHK(hipMemcpyAsync(theta_bf16, m->wbf, MLP_NPARAM * sizeof(uint16_t), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GRTE_OK;
}

grte_status grte_mlp_set_norm(grte_mlp *m, const float *norm)
{
    if (!m || !norm) return GRTE_E_INVAL;
    for (int q = 0; q < MLP_NNORM; ++q)
        if (!std::isfinite(norm[q])) return GRTE_E_INVAL;
    for (int q = 0; q < MLP_IN; ++q)
        if (!(norm[MLP_IN + q] > 0)) return GRTE_E_INVAL;
    if (!(norm[11] > 0)) return GRTE_E_INVAL;
    MCHK(hipMemcpyAsync(m->norm, norm, MLP_NNORM * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GRTE_OK;
}

grte_status grte_mlp_get_norm(grte_mlp *m, float *norm)
{
    if (!m || !norm) return GRTE_E_INVAL;
    MCHK(hipMemcpyAsync(norm, m->norm, MLP_NNORM * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GRTE_OK;
}

grte_status grte_mlp_fit_norm(grte_mlp *m, const float *data, long long n)
{
    if (!m || !data || n < 2) return GRTE_E_INVAL;
    hipLaunchKernelGGL(mlp_norm_kernel, dim3(1), dim3(256), 0, m->stream, data, n, m->norm);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
    return GRTE_OK;
}

grte_status grte_mlp_grad(grte_mlp *m, const float *data, long long n, float *grad, float *loss)
{
    if (!m || !data || !grad || n < 1 || n > (1 << 24)) return GRTE_E_INVAL;
    const int B = (int)n;
    grte_status st = launch_grad(m, data, n, 0, B);
    if (st != GRTE_OK) return st;
    const int nblk = (B + GB - 1) / GB;
    std::vector<float> gp((size_t)nblk * MLP_NPARAM), lp(nblk);
    MCHK(hipMemcpyAsync(gp.data(), m->gpart, gp.size() * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipMemcpyAsync(lp.data(), m->lpart, lp.size() * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    for (int e = 0; e < MLP_NPARAM; ++e) {
        float g = 0.0f;
        for (int b = 0; b < nblk; ++b) g += gp[(size_t)b * MLP_NPARAM + e];
        grad[e] = g;
    }
    if (loss) {
        float l = 0.0f;
        for (int b = 0; b < nblk; ++b) l += lp[b];
        *loss = l / (float)B;
    }
    return GRTE_OK;
}

grte_status grte_mlp_train(grte_mlp *m, const float *data, long long n, int steps, int batch, float lr,
                           float *loss_hist)
{
    if (!m || !data || n < 1 || steps < 1 || batch < 1 || batch > (1 << 20) || !(lr > 0)) return GRTE_E_INVAL;
    const int B = (int)std::min<long long>(batch, n);
    const int nblk = (B + GB - 1) / GB;
    if (loss_hist && steps > m->hcap) {
        if (m->lhist) (void)hipFree(m->lhist);
        m->lhist = nullptr;
        m->hcap = 0;
        if (hipMalloc((void **)&m->lhist, (size_t)steps * sizeof(float)) != hipSuccess) return GRTE_E_NOMEM;
        m->hcap = steps;
    }
    grte_status st = ensure_gpart(m, nblk);
    if (st != GRTE_OK) return st;
    st = train_steps(m, data, n, steps, B, lr, m->gpart, m->lpart, loss_hist ? m->lhist : nullptr);
    if (st != GRTE_OK) return st;
    if (loss_hist)
        MCHK(hipMemcpyAsync(loss_hist, m->lhist, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GRTE_OK;
}

grte_status grte_mlp_train_noalloc(grte_mlp *m, const float *data, long long n, int steps, int batch, float lr,
                                   float *loss_hist)
{
    if (!m || !data || n < 1 || steps < 1 || batch < 1 || !(lr > 0)) return GRTE_E_INVAL;
    const int B = (int)std::min<long long>(batch, n);
    if (B > NOALLOC_MAX_BATCH || (loss_hist && steps > NOALLOC_MAX_STEPS)) {
        fprintf(stderr, "grte_mlp_train_noalloc: minibatch %d rows (at most %d) or %d loss-history steps "
                        "(at most %d) beyond the fixed workspace\n", B, NOALLOC_MAX_BATCH, steps, NOALLOC_MAX_STEPS);
        return GRTE_E_UNSUPPORTED;
    }
    float *ws = nullptr;
    grte_status st = scratch_on_device(&ws);
    if (st != GRTE_OK) return st;
    float *gpart = ws;                                              // NOALLOC_MAX_BLOCKS x MLP_NPARAM
    float *lpart = gpart + (size_t)NOALLOC_MAX_BLOCKS * MLP_NPARAM;  // NOALLOC_MAX_BLOCKS
    float *lhist = lpart + NOALLOC_MAX_BLOCKS;                      // NOALLOC_MAX_STEPS
    st = train_steps(m, data, n, steps, B, lr, gpart, lpart, loss_hist ? lhist : nullptr);
    if (st != GRTE_OK) return st;
    if (loss_hist)
        MCHK(hipMemcpyAsync(loss_hist, lhist, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GRTE_OK;
}

grte_status grte_mlp_predict(grte_mlp *m, const float *data, long long n, float *y)
{
    if (!m || !data || !y || n < 1) return GRTE_E_INVAL;
    hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->stream, m->wbf,
                       m->norm, data, n, y);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
    return GRTE_OK;
}

}  // extern "C"
