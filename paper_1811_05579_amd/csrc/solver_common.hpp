// solver_common.hpp -- device building blocks shared by the single-instance
// and the batched AP-step kernels (tridiagonal factor/solve in one
// work-group, block reductions, grid barrier, node relations).
#pragma once
#include <hip/hip_runtime.h>

namespace {

constexpr int NT = 256;          // threads per work-group of the tridiagonal solvers
constexpr int LOGNT = 8;
constexpr int MAX_M = 16;        // rows per thread -> N <= NT * MAX_M = 4096
constexpr int MAX_N = NT * MAX_M;
constexpr int MAX_P = 64;
constexpr int BAR_STRIDE = 16;   // 64-bit barrier flags, one 128-byte line per work-group

// -------------------------------------------------------------------------
// tile tridiagonal solver: factor once, solve for many right-hand sides
// -------------------------------------------------------------------------
// A system of up to W*M rows is solved by a tile of W threads: the whole
// work-group (W = 256) or one wavefront (W = 64).  Row j is owned by tile
// thread k = j / M as its row r = j % M; all per-row data live in
// "position" order t = r * W + k (conflict-free LDS, coalesced global
// traffic).  The systems solved here have off-diagonals that are a scalar
// multiple of two LDS-resident arrays, a_j = s Lo[t], c_j = s Up[t] (zero where
// a row has no neighbour, and in padding rows), and a per-row diagonal b_j.
// Each chunk's interior rows 0..M-2 are eliminated by Thomas' algorithm; the
// chunk's last rows z_k form a tridiagonal system of W rows solved by
// parallel cyclic reduction (through LDS for W = 256, through wavefront
// shuffles for W = 64).  What does not depend on the right-hand side -- the
// interior pivots and the PCR multipliers -- is computed once by tri_factor and
// kept in registers; tri_solve then costs four short FMA recurrences and one
// PCR sweep on the right-hand side only.
template <int W>
struct TileLog;
template <>
struct TileLog<64> { static constexpr int v = 6; };
template <>
struct TileLog<256> { static constexpr int v = 8; };

template <int W>
__device__ __forceinline__ int tile_lane() { return (W == 64) ? (threadIdx.x & 63) : threadIdx.x; }

template <int W>
__device__ __forceinline__ void tile_sync()
{
    if constexpr (W == 256) __syncthreads();
}

// value of tile thread k + o (o may be negative); `dflt` outside the tile
template <int W>
__device__ __forceinline__ double tile_nb(double v, int o, double dflt, double *sh)
{
    const int k = tile_lane<W>();
    const bool in = (k + o >= 0) && (k + o < W);
    if constexpr (W == 64) {
        const double r = __shfl(v, k + o, 64);
        return in ? r : dflt;
    } else {
        sh[k] = v;
        __syncthreads();
        const double r = in ? sh[k + o] : dflt;
        __syncthreads();
        return r;
    }
}

template <int W, int M>
struct TriFac {
    double inv[M - 1];          // reciprocal pivots of the interior rows
    double k1[TileLog<W>::v], k2[TileLog<W>::v];
    double invB;
};

template <int W, int M>
__device__ __forceinline__ void tri_factor(double s, const double *Lo, const double *Up,
                                           const double (&b)[M], TriFac<W, M> &F, double *sh)
{
    static_assert(M >= 2, "at least two rows per thread");
    constexpr int L = TileLog<W>::v;
    const int k = tile_lane<W>();
    double Q[M - 1], R[M - 1];   // responses of the interior to z_{k-1} (Q) and z_k (R)
    double cprev;
    {
        const double a0 = s * Lo[k], c0 = s * Up[k];
        const double inv = 1.0 / b[0];
        F.inv[0] = inv;
        cprev = (M > 2) ? c0 * inv : 0.0;
        Q[0] = -a0 * inv;
        R[0] = (M == 2) ? -c0 * inv : 0.0;
    }
#pragma unroll
    for (int r = 1; r < M - 1; ++r) {
        const double ar = s * Lo[r * W + k], cr = s * Up[r * W + k];
        const double inv = 1.0 / (b[r] - ar * cprev);
        F.inv[r] = inv;
        Q[r] = -ar * Q[r - 1] * inv;
        R[r] = ((r == M - 2 ? -cr : 0.0) - ar * R[r - 1]) * inv;
        cprev = (r < M - 2) ? cr * inv : 0.0;
    }
#pragma unroll
    for (int r = M - 3; r >= 0; --r) {
        const double cp = s * Up[r * W + k] * F.inv[r];
        Q[r] -= cp * Q[r + 1];
        R[r] -= cp * R[r + 1];
    }
    const double ae = s * Lo[(M - 1) * W + k], ce = s * Up[(M - 1) * W + k];
    const double Qn = tile_nb<W>(Q[0], 1, 0.0, sh);
    const double Rn = tile_nb<W>(R[0], 1, 0.0, sh);
    double Aa = ae * Q[M - 2];
    double Bb = ae * R[M - 2] + b[M - 1] + ce * Qn;
    double Cc = ce * Rn;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int st = 1 << l;
        double Am, Bm, Cm, Ap, Bp, Cp;
        if constexpr (W == 64) {
            Am = tile_nb<W>(Aa, -st, 0.0, sh);
            Bm = tile_nb<W>(Bb, -st, 1.0, sh);
            Cm = tile_nb<W>(Cc, -st, 0.0, sh);
            Ap = tile_nb<W>(Aa, st, 0.0, sh);
            Bp = tile_nb<W>(Bb, st, 1.0, sh);
            Cp = tile_nb<W>(Cc, st, 0.0, sh);
        } else {
            double *sA = sh, *sB = sh + W, *sC = sh + 2 * W;
            sA[k] = Aa;
            sB[k] = Bb;
            sC[k] = Cc;
            __syncthreads();
            Am = 0.0; Bm = 1.0; Cm = 0.0; Ap = 0.0; Bp = 1.0; Cp = 0.0;
            if (k >= st) { Am = sA[k - st]; Bm = sB[k - st]; Cm = sC[k - st]; }
            if (k + st < W) { Ap = sA[k + st]; Bp = sB[k + st]; Cp = sC[k + st]; }
            __syncthreads();
        }
        const double k1 = Aa / Bm, k2 = Cc / Bp;
        F.k1[l] = k1;
        F.k2[l] = k2;
        Aa = -Am * k1;
        Cc = -Cp * k2;
        Bb = Bb - Cm * k1 - Ap * k2;
    }
    F.invB = 1.0 / Bb;
}

// forward elimination + back substitution over the interior rows 0..M-2
template <int W, int M>
__device__ __forceinline__ void tri_interior(double s, const double *Lo, const double *Up,
                                             const TriFac<W, M> &F, double (&y)[M - 1])
{
    const int k = tile_lane<W>();
    y[0] = y[0] * F.inv[0];
#pragma unroll
    for (int r = 1; r < M - 1; ++r) y[r] = (y[r] - s * Lo[r * W + k] * y[r - 1]) * F.inv[r];
#pragma unroll
    for (int r = M - 3; r >= 0; --r) y[r] -= s * Up[r * W + k] * F.inv[r] * y[r + 1];
}

template <int W, int M>
__device__ __forceinline__ void tri_solve(double s, const double *Lo, const double *Up, const TriFac<W, M> &F,
                                          const double (&d)[M], double (&x)[M], double *sh)
{
    constexpr int L = TileLog<W>::v;
    const int k = tile_lane<W>();
    // interior particular solution with z_{k-1} = z_k = 0
    double y[M - 1];
#pragma unroll
    for (int r = 0; r < M - 1; ++r) y[r] = d[r];
    tri_interior<W, M>(s, Lo, Up, F, y);
    // the last interior row is not changed by back substitution
    const double ylast = y[M - 2];
    double D, yn;
    if constexpr (W == 64) {
        yn = tile_nb<W>(y[0], 1, 0.0, sh);
    } else {
        sh[k] = y[0];
        __syncthreads();
        yn = (k + 1 < W) ? sh[k + 1] : 0.0;
    }
    D = d[M - 1] - s * Lo[(M - 1) * W + k] * ylast - s * Up[(M - 1) * W + k] * yn;
    // PCR on the right-hand side (two LDS buffers: one barrier per level)
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int st = 1 << l;
        double Dm, Dp;
        if constexpr (W == 64) {
            Dm = tile_nb<W>(D, -st, 0.0, sh);
            Dp = tile_nb<W>(D, st, 0.0, sh);
        } else {
            double *bf = sh + W * (1 + (l & 1));
            bf[k] = D;
            __syncthreads();
            Dm = (k >= st) ? bf[k - st] : 0.0;
            Dp = (k + st < W) ? bf[k + st] : 0.0;
        }
        D = D - F.k1[l] * Dm - F.k2[l] * Dp;
    }
    const double z = D * F.invB;
    double zl;
    if constexpr (W == 64) {
        zl = tile_nb<W>(z, -1, 0.0, sh);
    } else {
        sh[k] = z;
        __syncthreads();
        zl = (k > 0) ? sh[k - 1] : 0.0;
        __syncthreads();
    }
    // interior again, now with the neighbouring chunk values folded in
#pragma unroll
    for (int r = 0; r < M - 1; ++r) y[r] = d[r];
    y[0] -= s * Lo[k] * zl;
    y[M - 2] -= s * Up[(M - 2) * W + k] * z;
    tri_interior<W, M>(s, Lo, Up, F, y);
#pragma unroll
    for (int r = 0; r < M - 1; ++r) x[r] = y[r];
    x[M - 1] = z;
}

// max over the tile of two values at once (fixed order; same result in every tile thread)
template <int W>
__device__ __forceinline__ void tile_max2(double &a, double &b, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a = fmax(a, __shfl_xor(a, o, 64));
        b = fmax(b, __shfl_xor(b, o, 64));
    }
    if constexpr (W == 256) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            sh[w] = a;
            sh[8 + w] = b;
        }
        __syncthreads();
        a = sh[0];
        b = sh[8];
#pragma unroll
        for (int q = 1; q < W / 64; ++q) {
            a = fmax(a, sh[q]);
            b = fmax(b, sh[8 + q]);
        }
        __syncthreads();
    }
}

// block-wide max of a non-negative value (fixed order; result in every thread)
__device__ __forceinline__ double block_max(double v, double *sh)
{
    const int k = threadIdx.x;
    sh[k] = v;
    __syncthreads();
#pragma unroll 1
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (k < s) sh[k] = fmax(sh[k], sh[k + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// -------------------------------------------------------------------------
// grid barrier for a cooperative launch (all work-groups co-resident)
// -------------------------------------------------------------------------
// Every work-group publishes the generation number in its own flag (no
// contended counter); lanes of wave 0 watch one flag each.  Each thread makes
// its own global writes visible at agent scope before the work-group
// barrier, and the flag store is a release, so the writes are visible on every
// XCD to a work-group that has observed the flag and executed the acquire.
// The wait is bounded: on a timeout, or when another work-group has already
// reported one, the error flag is raised and false is returned so that every
// work-group leaves the iteration instead of hanging the device.
__device__ __forceinline__ bool grid_barrier(unsigned long long *flags, unsigned long long gen, int *err)
{
    __shared__ int s_fail;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        s_fail = 0;
        __hip_atomic_store(&flags[(size_t)blockIdx.x * BAR_STRIDE], gen, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x < 64) {
        bool fail = false;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += 64) {
            unsigned spins = 0;
            while (__hip_atomic_load(&flags[(size_t)b * BAR_STRIDE], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT) < gen) {
                if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                    ++spins > (1u << 20)) {
                    fail = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (fail) {
            atomicOr(err, 1);
            s_fail = 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_fail == 0;
}

__device__ __forceinline__ double kpow(double T, int m) { return m == 0 ? 1.0 : T * T * T; }

// position of row j in the per-thread-chunk ("position") order used by the
// tridiagonal solvers: t = (j % M) * NT + j / M
__device__ __forceinline__ int row_pos(int j, int M) { return (j % M) * NT + j / M; }

__device__ __forceinline__ double node_flux(const double *Eall, const double *O, const double *Aw,
                                            const double *Bc, double mu, int N, int P, int i, int p)
{
    // interior node i (1..N-1): O_i = Aw_i O^n_i - Bc_i mu (E_i - E_{i-1})
    return Aw[i] * O[(size_t)i * P + p] - Bc[i] * mu * (Eall[(size_t)i * P + p] - Eall[(size_t)(i - 1) * P + p]);
}

__device__ __forceinline__ double node_any(const double *Eall, const double *O, const double *Aw,
                                           const double *Bc, double mu, double bl, double br, double eps,
                                           int N, int P, int i, int p)
{
    if (i >= 1 && i <= N - 1) return node_flux(Eall, O, Aw, Bc, mu, N, P, i, p);
    if (i == 0)   // inflow relation (4.7) at x = 0
        return 2.0 / eps * (bl - Eall[p]) - node_flux(Eall, O, Aw, Bc, mu, N, P, 1, p);
    // i == N, (4.7) at x = L
    return 2.0 / eps * (Eall[(size_t)(N - 1) * P + p] - br) - node_flux(Eall, O, Aw, Bc, mu, N, P, N - 1, p);
}

}  // namespace
