// diffusion.hip -- the discrete nonlinear diffusion limit on the GPU (the
// grte_diff_* calls of include/grte.h): the three-stage prediction-
// correction-projection scheme (2.7) of Tang, Wang & Zhang, its sigma/T^3
// form (2.9), and the two-stage scheme (2.8) that the paper gives as the
// counter-example (a compactly supported temperature never spreads).
//
// One step of a slab of N <= 4096 cells is one work-group of 256 threads:
//   stage 1   (U* - U^n)/dt = 4 T^3/(4 a T^3 + Cv) (1/dx^2)[F_{j+1}(U*_{j+1} - U*_j) - F_j(U*_j - U*_{j-1})]
//             with face coefficients F = a c K/(3 sigma) (harmonic sigma, mean K = T^m),
//             one tridiagonal solve (the tile solver of the AP step);
//   stage 2   a (T^4 - U^n)/dt + Cv (T - T^n)/dt = the same flux difference of U*, one
//             scalar Newton per cell (F from K^n, or from (U*)^{3/4} for the printed (2.9));
//   stage 3   U^{n+1} = (T^{n+1})^4 (the state is T).
// The two-stage scheme replaces stages 2-3 by T^{n+1} = max(U*, 0)^{1/4}; the
// limit of the alternative correction (3.14) (the remark closing Section 3)
// replaces stage 2 by the linear update
//   a (U* - U^n)/dt + Cv (T^{n+1} - T^n)/dt = the flux difference of U* (F from K^n).
// Boundaries: zero flux, or ghost temperatures one cell outside the slab with
// the boundary cell's coefficient on the boundary face.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>

#include "../../include/grte.h"
#include "solver_common.hpp"

namespace {

struct DiffArgs {
    int N, m, bc, scheme, corrK, maxit;
    double a, at, c, cv, dt, dx;
    double gUL, gUR;                  // ghost U = T^4 outside the two ends (Dirichlet)
    const double *T, *sigma0;
    double *Tout, *Ustar;
    int *stat;                        // [0] max Newton iterations, [1] cells at the cap
};

__device__ __forceinline__ double dkpow(double T, int m) { return m == 0 ? 1.0 : T * T * T; }

// a c K/(3 sigma) at interior face i (between cells i-1 and i)
__device__ __forceinline__ double face_F(const DiffArgs &A, double Kl, double Kr, int i)
{
    const double sl = A.sigma0[i - 1], sr = A.sigma0[i];
    const double sf = 2.0 * sl * sr / (sl + sr);
    return A.a * A.c * (0.5 * (Kl + Kr)) / (3.0 * sf);
}

template <int M>
__global__ void __launch_bounds__(NT) diff_kernel(DiffArgs A)
{
    extern __shared__ double smem[];
    constexpr int NP = NT * M;
    double *sLo = smem, *sUp = smem + NP, *sU = smem + 2 * NP, *sh = smem + 3 * NP;
    const int k = threadIdx.x, j0 = k * M;
    const int N = A.N;
    const double dx2 = A.dx * A.dx;
    // stage 1: tridiagonal system for U*
    double b[M], d[M], x[M];
    double Fl[M], Fr[M];              // face coefficients from K^n (left/right face of the row)
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int j = j0 + r;
        const int t = r * NT + k;
        if (j < N) {
            const double Tj = A.T[j];
            const double Kj = dkpow(Tj, A.m);
            double fl = 0.0, fr = 0.0;
            if (j >= 1) fl = face_F(A, dkpow(A.T[j - 1], A.m), Kj, j);
            else if (A.bc == 1) fl = A.a * A.c * Kj / (3.0 * A.sigma0[0]);
            if (j <= N - 2) fr = face_F(A, Kj, dkpow(A.T[j + 1], A.m), j + 1);
            else if (A.bc == 1) fr = A.a * A.c * Kj / (3.0 * A.sigma0[N - 1]);
            Fl[r] = fl;
            Fr[r] = fr;
            const double T3 = Tj * Tj * Tj;
            const double pref = A.dt * 4.0 * T3 / (4.0 * A.at * T3 + A.cv);
            // interior faces couple to the neighbour; ghost faces move to the right-hand side
            const double wl = (j >= 1) ? fl / dx2 : 0.0, wr = (j <= N - 2) ? fr / dx2 : 0.0;
            const double gl = (j == 0 && A.bc == 1) ? fl / dx2 : 0.0;
            const double gr = (j == N - 1 && A.bc == 1) ? fr / dx2 : 0.0;
            sLo[t] = -pref * wl;
            sUp[t] = -pref * wr;
            b[r] = 1.0 + pref * (wl + wr + gl + gr);
            d[r] = (Tj * Tj) * (Tj * Tj) + pref * (gl * A.gUL + gr * A.gUR);
        } else {
            Fl[r] = Fr[r] = 0.0;
            sLo[t] = sUp[t] = 0.0;
            b[r] = 1.0;
            d[r] = 0.0;
        }
    }
    __syncthreads();
    int ph = 0;
    tri_factor_solve<NT, M>(1.0, sLo, sUp, b, d, x, sh, ph);
#pragma unroll
    for (int r = 0; r < M; ++r) sU[r * NT + k] = x[r];
    __syncthreads();
    int nits = 0, nfail = 0;
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int j = j0 + r;
        if (j >= N) continue;
        const double us = x[r];
        A.Ustar[j] = us;
        const double Tj = A.T[j];
        double Tn1;
        if (A.scheme == 1) {
            Tn1 = pow(fmax(us, 0.0), 0.25);              // (2.8): projection of U* only
        } else {
            // stage 2: flux difference of U* with F from K^n or from (U*)^{3/4}
            auto Uat = [&](int jj) { return sU[(jj % M) * NT + jj / M]; };
            double fl = Fl[r], fr = Fr[r];
            if (A.m == 3 && A.corrK == 1) {
                auto ks = [&](int jj) { return pow(fmax(Uat(jj), 0.0), 0.75); };
                const double Kj = ks(j);
                fl = 0.0;
                fr = 0.0;
                if (j >= 1) fl = face_F(A, ks(j - 1), Kj, j);
                else if (A.bc == 1) fl = A.a * A.c * Kj / (3.0 * A.sigma0[0]);
                if (j <= N - 2) fr = face_F(A, Kj, ks(j + 1), j + 1);
                else if (A.bc == 1) fr = A.a * A.c * Kj / (3.0 * A.sigma0[N - 1]);
            }
            double fluxl = 0.0, fluxr = 0.0;                 // +x fluxes through the two faces
            if (j >= 1) fluxl = fl * (us - Uat(j - 1)) / A.dx;
            else if (A.bc == 1) fluxl = fl * (us - A.gUL) / A.dx;
            if (j <= N - 2) fluxr = fr * (Uat(j + 1) - us) / A.dx;
            else if (A.bc == 1) fluxr = fr * (A.gUR - us) / A.dx;
            const double rhs = A.dt * (fluxr - fluxl) / A.dx + A.at * (Tj * Tj) * (Tj * Tj) + A.cv * Tj;
            if (A.scheme == 2) {
                // (3.14): no nonlinear solve, U* in the time derivative
                Tn1 = Tj + (A.dt * (fluxr - fluxl) / A.dx - A.at * (us - (Tj * Tj) * (Tj * Tj))) / A.cv;
            } else if (A.at == 0.0) {
                Tn1 = rhs / A.cv;
            } else {
                // a_t T^4 + Cv T = rhs: convex and increasing for T >= 0; Newton from a start
                // at or above the root converges monotonically
                double T = fmax(fmax(Tj, 0.0), fmax(rhs / A.cv, pow(fmax(rhs, 0.0) / A.at, 0.25)));
                bool ok = false;
                int its = 0;
                for (; its < A.maxit;) {
                    const double T3 = T * T * T;
                    const double step = (A.at * T3 * T + A.cv * T - rhs) / (4.0 * A.at * T3 + A.cv);
                    T -= step;
                    ++its;
                    if (fabs(step) <= 0x1p-50 * fmax(fabs(T), 1e-300)) { ok = true; break; }
                }
                nits = max(nits, its);
                if (!ok) ++nfail;
                Tn1 = T;
            }
        }
        A.Tout[j] = Tn1;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nits = max(nits, __shfl_xor(nits, o, 64));
        nfail += __shfl_xor(nfail, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&A.stat[0], nits);
        if (nfail) atomicAdd(&A.stat[1], nfail);
    }
}

__global__ void diff_clear(int *stat)
{
    if (threadIdx.x < 2) stat[threadIdx.x] = 0;
}

int diff_rows(int N)
{
    int M = 2;
    while (NT * M < N) M *= 2;
    return M;
}

template <int M>
size_t diff_lds() { return (size_t)(3 * NT * M + tile_scratch<NT>()) * sizeof(double); }

}  // namespace

struct grte_diff {
    int N = 0, M = 2, m = 0, bc = 0;
    double L = 1, a = 1, c = 1, cv = 1, gTL = 0, gTR = 0;
    hipStream_t stream = nullptr;
    double *T = nullptr, *T2 = nullptr, *sigma0 = nullptr, *Ustar = nullptr;
    int *stat = nullptr;
};

namespace {

template <int M>
grte_status diff_launch(grte_diff *dd, const DiffArgs &A)
{
    const size_t lds = diff_lds<M>();
    if (hipFuncSetAttribute((const void *)diff_kernel<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
        return GRTE_E_HIP;
    hipLaunchKernelGGL(diff_kernel<M>, dim3(1), dim3(NT), lds, dd->stream, A);
    return hipGetLastError() == hipSuccess ? GRTE_OK : GRTE_E_HIP;
}

grte_status dcopy(grte_diff *dd, void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    if (hipMemcpyAsync(dst, src, bytes, kind, dd->stream) != hipSuccess) return GRTE_E_HIP;
    if (kind != hipMemcpyDeviceToDevice && hipStreamSynchronize(dd->stream) != hipSuccess) return GRTE_E_HIP;
    return GRTE_OK;
}

}  // namespace

extern "C" {

grte_status grte_diff_destroy(grte_diff *dd)
{
    if (!dd) return GRTE_OK;
    void *ps[] = {dd->T, dd->T2, dd->sigma0, dd->Ustar, dd->stat};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete dd;
    return GRTE_OK;
}

grte_status grte_diff_create(const grte_diff_problem *pb, grte_diff **out)
{
    if (!out) return GRTE_E_INVAL;
    *out = nullptr;
    if (!pb || pb->nx < 2 || !(pb->length > 0) || !(pb->a > 0) || !(pb->c > 0) || !(pb->cv > 0) ||
        (pb->opacity_law != 0 && pb->opacity_law != 3) || (pb->boundary != 0 && pb->boundary != 1) ||
        !(pb->ghost_left >= 0) || !(pb->ghost_right >= 0))
        return GRTE_E_INVAL;
    if (pb->nx > NT * MAX_M) return GRTE_E_UNSUPPORTED;
    grte_diff *dd = new (std::nothrow) grte_diff();
    if (!dd) return GRTE_E_NOMEM;
    dd->N = pb->nx;
    dd->M = diff_rows(pb->nx);
    dd->m = pb->opacity_law;
    dd->bc = pb->boundary;
    dd->L = pb->length;
    dd->a = pb->a;
    dd->c = pb->c;
    dd->cv = pb->cv;
    dd->gTL = pb->ghost_left;
    dd->gTR = pb->ghost_right;
    const size_t N = dd->N;
    if (hipMalloc((void **)&dd->T, N * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dd->T2, N * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dd->sigma0, N * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dd->Ustar, N * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dd->stat, 2 * sizeof(int)) != hipSuccess) {
        grte_diff_destroy(dd);
        return GRTE_E_NOMEM;
    }
    if (hipMemset(dd->T, 0, N * sizeof(double)) != hipSuccess || hipMemset(dd->Ustar, 0, N * sizeof(double)) != hipSuccess) {
        grte_diff_destroy(dd);
        return GRTE_E_HIP;
    }
    *out = dd;
    return GRTE_OK;
}

grte_status grte_diff_set_stream(grte_diff *dd, void *hip_stream)
{
    if (!dd) return GRTE_E_INVAL;
    dd->stream = (hipStream_t)hip_stream;
    return GRTE_OK;
}

grte_status grte_diff_set_opacity(grte_diff *dd, const double *sigma0, int on_device)
{
    if (!dd || !sigma0) return GRTE_E_INVAL;
    if (!on_device)
        for (int j = 0; j < dd->N; ++j)
            if (!(sigma0[j] > 0) || !std::isfinite(sigma0[j])) return GRTE_E_INVAL;
    return dcopy(dd, dd->sigma0, sigma0, dd->N * sizeof(double),
                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
}

grte_status grte_diff_set_state(grte_diff *dd, const double *T, int on_device)
{
    if (!dd || !T) return GRTE_E_INVAL;
    if (!on_device)
        for (int j = 0; j < dd->N; ++j)
            if (!(T[j] >= 0) || !std::isfinite(T[j])) return GRTE_E_INVAL;
    return dcopy(dd, dd->T, T, dd->N * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
}

grte_status grte_diff_get_state(grte_diff *dd, double *T, double *Ustar, int on_device)
{
    if (!dd) return GRTE_E_INVAL;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    grte_status s = GRTE_OK;
    if (T) s = dcopy(dd, T, dd->T, dd->N * sizeof(double), k);
    if (s == GRTE_OK && Ustar) s = dcopy(dd, Ustar, dd->Ustar, dd->N * sizeof(double), k);
    return s;
}

grte_status grte_diff_step(grte_diff *dd, double dt, int scheme, int corr_K, double a_time, int *newton_its)
{
    if (!dd || !(dt > 0) || !std::isfinite(dt) || scheme < 0 || scheme > 2 || (corr_K != 0 && corr_K != 1) ||
        !std::isfinite(a_time))
        return GRTE_E_INVAL;
    DiffArgs A{};
    A.N = dd->N;
    A.m = dd->m;
    A.bc = dd->bc;
    A.scheme = scheme;
    A.corrK = corr_K;
    A.maxit = 200;
    A.a = dd->a;
    A.at = a_time < 0 ? dd->a : a_time;
    A.c = dd->c;
    A.cv = dd->cv;
    A.dt = dt;
    A.dx = dd->L / dd->N;
    const double gl2 = dd->gTL * dd->gTL, gr2 = dd->gTR * dd->gTR;
    A.gUL = gl2 * gl2;
    A.gUR = gr2 * gr2;
    A.T = dd->T;
    A.sigma0 = dd->sigma0;
    A.Tout = dd->T2;
    A.Ustar = dd->Ustar;
    A.stat = dd->stat;
    hipLaunchKernelGGL(diff_clear, dim3(1), dim3(64), 0, dd->stream, dd->stat);
    grte_status st;
    switch (dd->M) {
    case 2: st = diff_launch<2>(dd, A); break;
    case 4: st = diff_launch<4>(dd, A); break;
    case 8: st = diff_launch<8>(dd, A); break;
    default: st = diff_launch<16>(dd, A); break;
    }
    if (st != GRTE_OK) return st;
    std::swap(dd->T, dd->T2);
    if (!newton_its) return GRTE_OK;
    int h[2];
    if (hipMemcpyAsync(h, dd->stat, sizeof(h), hipMemcpyDeviceToHost, dd->stream) != hipSuccess ||
        hipStreamSynchronize(dd->stream) != hipSuccess)
        return GRTE_E_HIP;
    *newton_its = h[0];
    return h[1] ? GRTE_E_NOCONV : GRTE_OK;
}

}  // extern "C"
