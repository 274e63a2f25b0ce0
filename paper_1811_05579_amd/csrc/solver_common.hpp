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
//
// Partitioned elimination: each thread eliminates the interior rows 0..M-2 of
// its chunk (Thomas), which leaves one unknown per chunk -- its last row z_k --
// in a "reduced" tridiagonal system of W rows.  In a wavefront tile the reduced
// system has one row per lane and is solved by parallel cyclic reduction
// through lane shuffles.  In a work-group tile the reduced rows are published
// in LDS once (one barrier) and every wavefront then solves the whole
// 256-row reduced system redundantly, as a wavefront tile with four rows per
// lane, so that each wave obtains the z values it needs without a second
// barrier.  What does not depend on the right-hand side (interior pivots,
// reduced coefficients, PCR multipliers) is computed by tri_factor; tri_solve
// costs two short FMA recurrences per thread, one LDS exchange with one
// barrier (work-group tiles), and one shuffle PCR sweep.

template <int W>
__device__ __forceinline__ int tile_lane() { return (W == 64) ? (threadIdx.x & 63) : threadIdx.x; }

// value of lane l + o of this wavefront (o may be negative); `dflt` outside the wave
__device__ __forceinline__ double wave_nb(double v, int o, double dflt)
{
    const int l = threadIdx.x & 63;
    const bool in = (l + o >= 0) && (l + o < 64);
    const double r = __shfl(v, l + o, 64);
    return in ? r : dflt;
}

// LDS scratch (doubles) of a work-group tile's solver, sh[0, 14 W + 16):
//   tri_factor        sh[0, 5W)            reduced-row exchange
//   tri_solve         sh[5W + 2W ph, +2W)  right-hand-side exchange, two buffers
//   tri_factor_solve  sh[7W ph, +7W)       both at once, two buffers
//   tile_max2         sh[14W, 14W + 16)
// (the `ph` buffers alternate so that one barrier per call suffices; a kernel
// uses either tri_factor/tri_solve or tri_factor_solve on one scratch area).
// Wavefront tiles need no scratch.  A work-group factorisation also keeps its
// reduced-system data in LDS (red_doubles(), one region per live
// factorisation, passed to tri_factor).
template <int W>
constexpr int tile_scratch() { return W == 256 ? 14 * W + 16 : 16; }
constexpr int RED_FIELDS = 28;                 // per lane: ra, rc, rce (4 each), inv (3), k1, k2 (6 each), invB
constexpr int red_doubles() { return RED_FIELDS * 64; }

// parallel cyclic reduction of a 64-row tridiagonal (row l in lane l)
struct WavePcr {
    double k1[6], k2[6];
    double invB;
};

__device__ __forceinline__ void wave_pcr_factor(double Aa, double Bb, double Cc, WavePcr &F)
{
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const int st = 1 << l;
        const double Am = wave_nb(Aa, -st, 0.0), Bm = wave_nb(Bb, -st, 1.0), Cm = wave_nb(Cc, -st, 0.0);
        const double Ap = wave_nb(Aa, st, 0.0), Bp = wave_nb(Bb, st, 1.0), Cp = wave_nb(Cc, st, 0.0);
        const double k1 = Aa / Bm, k2 = Cc / Bp;
        F.k1[l] = k1;
        F.k2[l] = k2;
        Aa = -Am * k1;
        Cc = -Cp * k2;
        Bb = Bb - Cm * k1 - Ap * k2;
    }
    F.invB = 1.0 / Bb;
}

__device__ __forceinline__ double wave_pcr_solve(double D, const WavePcr &F)
{
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const int st = 1 << l;
        const double Dm = wave_nb(D, -st, 0.0), Dp = wave_nb(D, st, 0.0);
        D = D - F.k1[l] * Dm - F.k2[l] * Dp;
    }
    return D * F.invB;
}

// interior rows 0..M-2 of one chunk with off-diagonals a[], c[] and diagonal
// b[]: reciprocal pivots, and the responses of the interior to the previous
// chunk's last unknown (Q) and to this chunk's last unknown (R)
template <int M, class GetA, class GetC>
__device__ __forceinline__ void chunk_factor(GetA a, GetC c, const double (&b)[M], double (&inv)[M - 1],
                                             double (&Q)[M - 1], double (&R)[M - 1])
{
    static_assert(M >= 2, "at least two rows per thread");
    double cprev;
    {
        const double iv = 1.0 / b[0];
        inv[0] = iv;
        cprev = (M > 2) ? c(0) * iv : 0.0;
        Q[0] = -a(0) * iv;
        R[0] = (M == 2) ? -c(0) * iv : 0.0;
    }
#pragma unroll
    for (int r = 1; r < M - 1; ++r) {
        const double ar = a(r), cr = c(r);
        const double iv = 1.0 / (b[r] - ar * cprev);
        inv[r] = iv;
        Q[r] = -ar * Q[r - 1] * iv;
        R[r] = ((r == M - 2 ? -cr : 0.0) - ar * R[r - 1]) * iv;
        cprev = (r < M - 2) ? cr * iv : 0.0;
    }
#pragma unroll
    for (int r = M - 3; r >= 0; --r) {
        const double cp = c(r) * inv[r];
        Q[r] -= cp * Q[r + 1];
        R[r] -= cp * R[r + 1];
    }
}

// forward elimination + back substitution over the interior rows 0..M-2
template <int M, class GetA, class GetC>
__device__ __forceinline__ void chunk_interior(GetA a, GetC c, const double (&inv)[M - 1], double (&y)[M - 1])
{
    y[0] = y[0] * inv[0];
#pragma unroll
    for (int r = 1; r < M - 1; ++r) y[r] = (y[r] - a(r) * y[r - 1]) * inv[r];
#pragma unroll
    for (int r = M - 3; r >= 0; --r) y[r] -= c(r) * inv[r] * y[r + 1];
}

// ---- wavefront tile, off-diagonals given by accessors a(r), c(r) of the lane's rows
template <int M>
struct WaveFac {
    double inv[M - 1];
    WavePcr pcr;
};

template <int M, class GetA, class GetC>
__device__ __forceinline__ void wave_factor(GetA a, GetC c, const double (&b)[M], WaveFac<M> &F)
{
    double Q[M - 1], R[M - 1];
    chunk_factor<M>(a, c, b, F.inv, Q, R);
    const double Qn = wave_nb(Q[0], 1, 0.0), Rn = wave_nb(R[0], 1, 0.0);
    const double ae = a(M - 1), ce = c(M - 1);
    wave_pcr_factor(ae * Q[M - 2], ae * R[M - 2] + b[M - 1] + ce * Qn, ce * Rn, F.pcr);
}

template <int M, class GetA, class GetC>
__device__ __forceinline__ void wave_solve(GetA a, GetC c, const WaveFac<M> &F, const double (&d)[M],
                                           double (&x)[M])
{
    double y[M - 1];
#pragma unroll
    for (int r = 0; r < M - 1; ++r) y[r] = d[r];
    chunk_interior<M>(a, c, F.inv, y);
    const double yn = wave_nb(y[0], 1, 0.0);
    const double z = wave_pcr_solve(d[M - 1] - a(M - 1) * y[M - 2] - c(M - 1) * yn, F.pcr);
    const double zl = wave_nb(z, -1, 0.0);
#pragma unroll
    for (int r = 0; r < M - 1; ++r) y[r] = d[r];
    y[0] -= a(0) * zl;
    y[M - 2] -= c(M - 2) * z;
    chunk_interior<M>(a, c, F.inv, y);
#pragma unroll
    for (int r = 0; r < M - 1; ++r) x[r] = y[r];
    x[M - 1] = z;
}

// ---- the tile solver used by the kernels
template <int W, int M>
struct TriFac;

template <int M>
struct TriFac<64, M> {
    WaveFac<M> w;
};

template <int M>
struct TriFac<256, M> {
    double inv[M - 1];        // interior pivots of this thread's chunk
    double *red;              // LDS: the 256-row reduced system, four rows per lane (identical in every
                              // wave): field f of lane l at red[64 f + l]
};

// reduced-system data of one lane, kept in registers while it is used
struct RedFac {
    double ra[4], rc[4];      // off-diagonals of the lane's four reduced rows
    double rce[4];            // last-row super-diagonal c_e of the chunks of those rows
    WaveFac<4> w;             // their wavefront factorisation
};

__device__ __forceinline__ void red_store(const RedFac &R, double *red)
{
    const int l = threadIdx.x & 63;
    double v[RED_FIELDS];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = R.ra[i];
        v[4 + i] = R.rc[i];
        v[8 + i] = R.rce[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) v[12 + i] = R.w.inv[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        v[15 + i] = R.w.pcr.k1[i];
        v[21 + i] = R.w.pcr.k2[i];
    }
    v[27] = R.w.pcr.invB;
#pragma unroll
    for (int f = 0; f < RED_FIELDS; ++f) red[64 * f + l] = v[f];
}

__device__ __forceinline__ void red_load(const double *red, RedFac &R)
{
    const int l = threadIdx.x & 63;
    double v[RED_FIELDS];
#pragma unroll
    for (int f = 0; f < RED_FIELDS; ++f) v[f] = red[64 * f + l];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        R.ra[i] = v[i];
        R.rc[i] = v[4 + i];
        R.rce[i] = v[8 + i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) R.w.inv[i] = v[12 + i];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        R.w.pcr.k1[i] = v[15 + i];
        R.w.pcr.k2[i] = v[21 + i];
    }
    R.w.pcr.invB = v[27];
}

// Factor.  LDS use (work-group tiles): sh[0, 5W) and the reduced-system region
// `red` (red_doubles()), which must stay untouched while the factorisation is
// used.  Every wave writes the same values to `red` and reads back its own
// writes, so no barrier is needed after it.  The caller must separate two
// factorisations that share sh (or red) by a barrier (a solve in between
// provides one).
template <int W, int M>
__device__ __forceinline__ void tri_factor(double s, const double *Lo, const double *Up, const double (&b)[M],
                                           TriFac<W, M> &F, double *sh, double *red = nullptr)
{
    const int k = tile_lane<W>();
    auto a = [&](int r) { return s * Lo[r * W + k]; };
    auto c = [&](int r) { return s * Up[r * W + k]; };
    if constexpr (W == 64) {
        wave_factor<M>(a, c, b, F.w);
    } else {
        double Q[M - 1], R[M - 1];
        chunk_factor<M>(a, c, b, F.inv, Q, R);
        double *fA = sh, *fB = sh + W, *fC = sh + 2 * W, *fQ = sh + 3 * W, *fR = sh + 4 * W;
        const double ae = a(M - 1), ce = c(M - 1);
        fA[k] = ae * Q[M - 2];
        fB[k] = ae * R[M - 2] + b[M - 1];
        fC[k] = ce;
        fQ[k] = Q[0];
        fR[k] = R[0];
        __syncthreads();
        // reduced row kk = 4 l + i couples z_{kk-1}, z_kk, z_{kk+1}
        const int l = threadIdx.x & 63;
        RedFac RF;
        double rb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = 4 * l + i;
            const double cek = fC[kk];
            const double qn = (kk + 1 < W) ? fQ[kk + 1] : 0.0;
            const double rn = (kk + 1 < W) ? fR[kk + 1] : 0.0;
            RF.ra[i] = fA[kk];
            rb[i] = fB[kk] + cek * qn;
            RF.rc[i] = cek * rn;
            RF.rce[i] = cek;
        }
        wave_factor<4>([&](int r) { return RF.ra[r]; }, [&](int r) { return RF.rc[r]; }, rb, RF.w);
        red_store(RF, red);
        F.red = red;
    }
}

// Solve T x = d.  LDS use (work-group tiles): sh[5W, 9W), alternating halves
// selected by `ph` (flipped by every call), so that one barrier per solve
// suffices.
template <int W, int M>
__device__ __forceinline__ void tri_solve(double s, const double *Lo, const double *Up, const TriFac<W, M> &F,
                                          const double (&d)[M], double (&x)[M], double *sh, int &ph)
{
    const int k = tile_lane<W>();
    auto a = [&](int r) { return s * Lo[r * W + k]; };
    auto c = [&](int r) { return s * Up[r * W + k]; };
    if constexpr (W == 64) {
        wave_solve<M>(a, c, F.w, d, x);
    } else {
        double y[M - 1];
#pragma unroll
        for (int r = 0; r < M - 1; ++r) y[r] = d[r];
        chunk_interior<M>(a, c, F.inv, y);
        double *bf = sh + 5 * W + 2 * W * ph;
        ph ^= 1;
        bf[k] = d[M - 1] - a(M - 1) * y[M - 2];
        bf[W + k] = y[0];
        __syncthreads();
        const int l = threadIdx.x & 63;
        RedFac RF;
        red_load(F.red, RF);
        double Dr[4], zr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = 4 * l + i;
            const double yn = (kk + 1 < W) ? bf[W + kk + 1] : 0.0;
            Dr[i] = bf[kk] - RF.rce[i] * yn;
        }
        wave_solve<4>([&](int r) { return RF.ra[r]; }, [&](int r) { return RF.rc[r]; }, RF.w, Dr, zr);
        // z_k and z_{k-1} from the lanes that hold them (the same lanes in every wave)
        const int src = k >> 2, sub = k & 3;
        const double z0 = __shfl(zr[0], src, 64), z1 = __shfl(zr[1], src, 64);
        const double z2 = __shfl(zr[2], src, 64), z3 = __shfl(zr[3], src, 64);
        const double zp = __shfl(zr[3], src > 0 ? src - 1 : 0, 64);
        const double z = sub == 0 ? z0 : sub == 1 ? z1 : sub == 2 ? z2 : z3;
        const double zl = sub == 0 ? (k > 0 ? zp : 0.0) : sub == 1 ? z0 : sub == 2 ? z1 : z2;
#pragma unroll
        for (int r = 0; r < M - 1; ++r) y[r] = d[r];
        y[0] -= a(0) * zl;
        y[M - 2] -= c(M - 2) * z;
        chunk_interior<M>(a, c, F.inv, y);
#pragma unroll
        for (int r = 0; r < M - 1; ++r) x[r] = y[r];
        x[M - 1] = z;
    }
}

// Factor and solve at once, for an operator used with one right-hand side
// (nothing is kept): the reduced coefficients and the reduced right-hand side
// are published together, so a work-group tile needs a single barrier.  LDS
// use (work-group tiles): the solve buffers sh[5W, 9W) selected by `ph`.
// (Lo, Up of the thread's row r at position base + r * rs; by default the
// tile's position order, base = the thread's tile index, rs = W.)
template <int W, int M>
__device__ __forceinline__ void tri_factor_solve(double s, const double *Lo, const double *Up,
                                                 const double (&b)[M], const double (&d)[M], double (&x)[M],
                                                 double *sh, int &ph, int base = -1, int rs = W)
{
    const int k = tile_lane<W>();
    if (base < 0) base = k;
    auto a = [&](int r) { return s * Lo[base + r * rs]; };
    auto c = [&](int r) { return s * Up[base + r * rs]; };
    if constexpr (W == 64) {
        WaveFac<M> F;
        wave_factor<M>(a, c, b, F);
        wave_solve<M>(a, c, F, d, x);
    } else {
        double inv[M - 1], Q[M - 1], R[M - 1], y[M - 1];
        chunk_factor<M>(a, c, b, inv, Q, R);
#pragma unroll
        for (int r = 0; r < M - 1; ++r) y[r] = d[r];
        chunk_interior<M>(a, c, inv, y);
        // one exchange: A, B-part, c_e, Q[0], R[0], D-part, y[0] of every chunk
        double *rg = sh + 7 * W * ph;
        ph ^= 1;
        const double ae = a(M - 1), ce = c(M - 1);
        rg[k] = ae * Q[M - 2];
        rg[W + k] = ae * R[M - 2] + b[M - 1];
        rg[2 * W + k] = ce;
        rg[3 * W + k] = Q[0];
        rg[4 * W + k] = R[0];
        rg[5 * W + k] = d[M - 1] - ae * y[M - 2];
        rg[6 * W + k] = y[0];
        __syncthreads();
        const int l = threadIdx.x & 63;
        double ra[4], rb[4], rc[4], Dr[4], zr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = 4 * l + i;
            const bool nx = kk + 1 < W;
            const double cek = rg[2 * W + kk];
            ra[i] = rg[kk];
            rb[i] = rg[W + kk] + cek * (nx ? rg[3 * W + kk + 1] : 0.0);
            rc[i] = cek * (nx ? rg[4 * W + kk + 1] : 0.0);
            Dr[i] = rg[5 * W + kk] - cek * (nx ? rg[6 * W + kk + 1] : 0.0);
        }
        WaveFac<4> RF;
        wave_factor<4>([&](int r) { return ra[r]; }, [&](int r) { return rc[r]; }, rb, RF);
        wave_solve<4>([&](int r) { return ra[r]; }, [&](int r) { return rc[r]; }, RF, Dr, zr);
        const int src = k >> 2, sub = k & 3;
        const double z0 = __shfl(zr[0], src, 64), z1 = __shfl(zr[1], src, 64);
        const double z2 = __shfl(zr[2], src, 64), z3 = __shfl(zr[3], src, 64);
        const double zp = __shfl(zr[3], src > 0 ? src - 1 : 0, 64);
        const double z = sub == 0 ? z0 : sub == 1 ? z1 : sub == 2 ? z2 : z3;
        const double zl = sub == 0 ? (k > 0 ? zp : 0.0) : sub == 1 ? z0 : sub == 2 ? z1 : z2;
#pragma unroll
        for (int r = 0; r < M - 1; ++r) y[r] = d[r];
        y[0] -= a(0) * zl;
        y[M - 2] -= c(M - 2) * z;
        chunk_interior<M>(a, c, inv, y);
#pragma unroll
        for (int r = 0; r < M - 1; ++r) x[r] = y[r];
        x[M - 1] = z;
    }
}

// -------------------------------------------------------------------------
// wavefront solver with many rows per lane and O(M) registers
// -------------------------------------------------------------------------
// One wavefront solves a tridiagonal system of 64 M rows on its own (row
// j = lane M + i of the lane's chunk i = 0..M-1, LDS position i * 64 + lane),
// so the four wavefronts of a work-group can take four different systems at
// once: four dependent elimination chains in flight per work-group instead of
// the one a work-group-wide solve gives.  The interior rows 0..M-2 of a chunk
// are eliminated twice, top-down (LU: the pivots are kept for the final
// substitution; the last interior row's responses to the right-hand side and
// to the two separators) and bottom-up (UL: the first interior row's
// responses), two recurrences independent of each other; the separators (row
// M-1 of every lane) then form a 64-row tridiagonal system, solved by parallel
// cyclic reduction over lane shuffles with the right-hand side carried along;
// a last top-down substitution with the separators known gives the interior
// rows.  a(i), b(i), c(i) return the sub-, main and super-diagonal of the
// lane's row i (a = 0 in row 0 of the system, c = 0 in its last row); x holds
// the right-hand side on entry and the solution on return.  Reciprocals are
// v_rcp_f64 refined by two Newton steps, within about an ulp of the quotient
// (the pivots of these diagonally dominant systems are finite, normal, and
// far from zero).

constexpr int LCS_WIN = 4;       // rows of coefficient loads in flight ahead of a recurrence
constexpr int LCS_IL_MAX = 32;   // chunks up to this size run their two recurrences interleaved

__device__ __forceinline__ double rcp64(double v)
{
    double r = __builtin_amdgcn_rcp(v);
    double e = fma(-v, r, 1.0);
    r = fma(r, e, r);
    e = fma(-v, r, 1.0);
    return fma(r, e, r);
}

template <int M, class GA, class GB, class GC>
__device__ __forceinline__ void lane_chunk_solve(GA a, GB b, GC c, double (&x)[M])
{
    static_assert(M >= 2, "at least two rows per lane");
    double inv[M - 1];
    double yf = 0.0, qf = 0.0, cp = 0.0;       // LU: y and the response to the left separator
    double ei = rcp64(b(M - 2)), w = x[M - 2], pr = 1.0;   // UL: 1/e, w, prod(-c_i / e_{i+1})
    auto lu_row = [&](int i) {
        const double ai = a(i);
        inv[i] = rcp64(i > 0 ? b(i) - ai * cp : b(i));
        yf = (i > 0 ? x[i] - ai * yf : x[i]) * inv[i];
        qf = (i > 0 ? -ai * qf : -ai) * inv[i];
        cp = c(i) * inv[i];
    };
    auto ul_row = [&](int i) {
        const double f = c(i) * ei;
        w = x[i] - f * w;
        pr *= -f;
        ei = rcp64(b(i) - f * a(i + 1));
    };
    if constexpr (M <= LCS_IL_MAX) {
        // the two recurrences interleaved (two chains in flight); the
        // coefficient loads may run at most LCS_WIN rows ahead (registers)
#pragma unroll
        for (int s = 0; s < M - 1; ++s) {
            lu_row(s);
            if (s < M - 2) ul_row(M - 3 - s);
            if (s % LCS_WIN == LCS_WIN - 1) __asm__ volatile("" ::: "memory");
        }
    } else {
#pragma unroll
        for (int s = 0; s < M - 1; ++s) {
            lu_row(s);
            if (s % LCS_WIN == LCS_WIN - 1) __asm__ volatile("" ::: "memory");
        }
#pragma unroll
        for (int s = 0; s < M - 2; ++s) {
            ul_row(M - 3 - s);
            if (s % LCS_WIN == LCS_WIN - 1) __asm__ volatile("" ::: "memory");
        }
    }
    // Chunk k's interior rows in terms of the separators z_{k-1} (left) and z_k:
    //   x_0 = W0 + A0 z_{k-1} + C0 z_k,  x_{M-2} = yf + qf z_{k-1} + Dk z_k.
    __asm__ volatile("" ::: "memory");
    const double cm2 = c(M - 2);
    const double W0 = w * ei, A0 = -a(0) * ei, C0 = -cm2 * pr * ei;
    const double Dk = -cm2 * inv[M - 2];
    const double W0n = wave_nb(W0, 1, 0.0), A0n = wave_nb(A0, 1, 0.0), C0n = wave_nb(C0, 1, 0.0);
    const double as = a(M - 1), cs = c(M - 1);
    double PA = as * qf, PB = b(M - 1) + as * Dk + cs * A0n, PC = cs * C0n;
    double PD = x[M - 1] - as * yf - cs * W0n;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const int st = 1 << l;
        const double Am = wave_nb(PA, -st, 0.0), Bm = wave_nb(PB, -st, 1.0), Cm = wave_nb(PC, -st, 0.0),
                     Dm = wave_nb(PD, -st, 0.0);
        const double Ap = wave_nb(PA, st, 0.0), Bp = wave_nb(PB, st, 1.0), Cp = wave_nb(PC, st, 0.0),
                     Dp = wave_nb(PD, st, 0.0);
        const double k1 = PA * rcp64(Bm), k2 = PC * rcp64(Bp);
        PA = -Am * k1;
        PC = -Cp * k2;
        PB = PB - Cm * k1 - Ap * k2;
        PD = PD - Dm * k1 - Dp * k2;
    }
    const double z = PD * rcp64(PB);
    const double zl = wave_nb(z, -1, 0.0);
    // (the compiler barriers make the coefficients be re-read from LDS rather
    // than kept live in registers across the phases)
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < M - 1; ++i) {
        double di = x[i];
        if (i == 0) di -= a(0) * zl;
        if (i == M - 2) di -= cm2 * z;
        x[i] = (i > 0 ? di - a(i) * x[i - 1] : di) * inv[i];
    }
#pragma unroll
    for (int i = M - 3; i >= 0; --i) x[i] -= c(i) * inv[i] * x[i + 1];
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
        double *m2 = sh + 14 * W;
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            m2[w] = a;
            m2[8 + w] = b;
        }
        __syncthreads();
        a = m2[0];
        b = m2[8];
#pragma unroll
        for (int q = 1; q < W / 64; ++q) {
            a = fmax(a, m2[q]);
            b = fmax(b, m2[8 + q]);
        }
        __syncthreads();
    }
}

// sum over the tile of two values at once (fixed order: a butterfly within
// each wavefront, then the wavefronts' sums in wave order; result in every
// tile thread), exchanging through the 16 doubles at m2 (work-group tiles)
template <int W>
__device__ __forceinline__ void tile_sum2_at(double &a, double &b, double *m2)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if constexpr (W == 256) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            m2[w] = a;
            m2[8 + w] = b;
        }
        __syncthreads();
        a = m2[0];
        b = m2[8];
#pragma unroll
        for (int q = 1; q < W / 64; ++q) {
            a += m2[q];
            b += m2[8 + q];
        }
        __syncthreads();
    }
}

// the same with the 16-double exchange area at sh + 14 W (the solver scratch)
template <int W>
__device__ __forceinline__ void tile_sum2(double &a, double &b, double *sh)
{
    tile_sum2_at<W>(a, b, sh + 14 * W);
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
// barrier over a set of co-resident work-groups of a cooperative launch
// -------------------------------------------------------------------------
// The set is `nblk` work-groups whose member index is `bid` (0..nblk-1), with
// their own flag array.  Every work-group publishes the generation number in
// its own flag (no contended counter); lanes of wave 0 watch one flag each.  Each thread makes
// its own global writes visible at agent scope before the work-group
// barrier, and the flag store is a release, so the writes are visible on every
// XCD to a work-group that has observed the flag and executed the acquire.
// The wait is bounded: on a timeout, or when another work-group has already
// reported one, the error flag is raised and false is returned so that every
// work-group leaves the iteration instead of hanging the device.
__device__ __forceinline__ bool grid_barrier(unsigned long long *flags, unsigned long long gen, int *err,
                                             int bid, int nblk)
{
    __shared__ int s_fail;
    // The work-group barrier orders every wave's prior stores before thread 0's
    // agent-scope release, whose write-back covers the work-group's data (one
    // write-back per work-group rather than one per wave).
    __syncthreads();
    if (threadIdx.x == 0) {
        s_fail = 0;
        __hip_atomic_store(&flags[(size_t)bid * BAR_STRIDE], gen, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x < 64) {
        bool fail = false;
        for (int b = threadIdx.x; b < nblk; b += 64) {
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

// O^n may be stored in binary64 or binary32 (OT); arithmetic is binary64
template <class OT>
__device__ __forceinline__ double node_flux(const double *Eall, const OT *O, const double *Aw,
                                            const double *Bc, double mu, int N, int P, int i, int p)
{
    // interior node i (1..N-1): O_i = Aw_i O^n_i - Bc_i mu (E_i - E_{i-1})
    return Aw[i] * (double)O[(size_t)i * P + p] -
           Bc[i] * mu * (Eall[(size_t)i * P + p] - Eall[(size_t)(i - 1) * P + p]);
}

template <class OT>
__device__ __forceinline__ double node_any(const double *Eall, const OT *O, const double *Aw,
                                           const double *Bc, double mu, double bl, double br, double eps,
                                           int N, int P, int i, int p)
{
    if (i >= 1 && i <= N - 1) return node_flux(Eall, O, Aw, Bc, mu, N, P, i, p);
    if (i == 0)   // inflow relation (4.7) at x = 0
        return 2.0 / eps * (bl - Eall[p]) - node_flux(Eall, O, Aw, Bc, mu, N, P, 1, p);
    // i == N, (4.7) at x = L
    return 2.0 / eps * (Eall[(size_t)(N - 1) * P + p] - br) - node_flux(Eall, O, Aw, Bc, mu, N, P, N - 1, p);
}

// -------------------------------------------------------------------------
// prediction iteration: acceleration and stopping test
// -------------------------------------------------------------------------
// Adaptive Chebyshev semi-iteration on top of the preconditioned Richardson
// update z = res + D^-1 (G res).  The iteration matrix I - (I + D^-1 G) S has a
// real spectrum in [0, b] with b < 1 (b ~ 0.1-0.3 on optically thick slabs), so
// the three-term Chebyshev recurrence for that interval needs no inner
// products; it replaces the plain updates by d_k = alpha_k d_{k-1} + beta_k z_k
// once the plain contraction ratio r = |z_k| / |z_{k-1}| (max norms relative
// to max|rho|) has settled: two consecutive ratios within CHEB_STAB of each
// other, r <= CHEB_RMAX (larger ratios belong to the transient of the first
// updates from a poor start, not to the spectrum), and the update norm still
// above CHEB_MARGIN times the tolerance (close to it the norms approach the
// rounding level).  The interval is [0, CHEB_KAPPA r].  The solve falls back to
// plain updates for good if, CHEB_PROG or more recurrence steps in, the update
// norm is above what plain updates at ratio r would have reached, or at any
// point above the norm at which the recurrence began.  The state is a function
// of the reduced norms only, so every thread of a tile, and every work-group of
// a cooperative solve, takes the same decisions.  Convergence is tested on
// max|z| as for the plain iteration.
struct ChebState {
    int nr = 0;                 // plain updates taken
    int on = 0;                 // recurrence running
    int off = 0;                // fell back to plain updates
    int j = 0;                  // recurrence steps taken
    // relative update norms max|z| / max|rho|, newest first (binary32: they
    // only steer the recurrence and the decisions around it)
    float q1 = 0.0f, q2 = 0.0f, q3 = 0.0f;
    float q0 = 0.0f, r0 = 0.0f, rj = 1.0f;   // at the start: norm, ratio; r0^j
    float s1 = 0.0f, rp = 0.0f, de = 1.0f;   // recurrence parameters
};
constexpr int CHEB_K0 = 3, CHEB_PROG = 4;
constexpr float CHEB_KAPPA = 1.2f, CHEB_STAB = 0.15f, CHEB_RMAX = 0.5f, CHEB_BMIN = 0.02f, CHEB_MARGIN = 100.0f;

// coefficients (alpha, beta) of this update
__device__ __forceinline__ void cheb_coeffs(ChebState &C, int accel, double tol, double &alpha, double &beta)
{
    alpha = 0.0;
    beta = 1.0;
    if (!accel || C.off || C.nr < CHEB_K0) return;
    if (!C.on) {
        if (!(C.q1 > CHEB_MARGIN * (float)tol) || !(C.q2 > 0.0f) || !(C.q3 > 0.0f)) return;
        const float r = C.q1 / C.q2, r2 = C.q2 / C.q3;
        if (!(r <= CHEB_RMAX) || !(fabsf(r - r2) <= CHEB_STAB * r)) return;
        const float b = fmaxf(CHEB_BMIN, CHEB_KAPPA * r);
        const float th = 1.0f - 0.5f * b;
        C.de = 0.5f * b;
        C.s1 = th / C.de;
        C.rp = 1.0f / C.s1;
        C.q0 = C.q1;
        C.r0 = r;
        C.rj = 1.0f;
        C.j = 0;
        C.on = 1;
        beta = 1.0 / (double)th;
        return;
    }
    const float rn = 1.0f / (2.0f * C.s1 - C.rp);
    alpha = (double)(rn * C.rp);
    beta = (double)(2.0f * rn / C.de);
    C.rp = rn;
}

// record this update's relative norm q
__device__ __forceinline__ void cheb_record(ChebState &C, float q)
{
    if (C.on) {
        ++C.j;
        C.rj *= C.r0;
        if (q > C.q0 || (C.j >= CHEB_PROG && q > C.q0 * C.rj)) {
            C.on = 0;
            C.off = 1;
        }
    } else {
        ++C.nr;
    }
    C.q3 = C.q2;
    C.q2 = C.q1;
    C.q1 = q;
}

// Stopping test of the prediction iteration for update norm md and iterate
// norm mr, with the relative update norms q = md / mr of this update and
// qprev, qprev2, qprev3 of the three before: 1 if md <= tol mr; 2 (a
// safeguard) when the updates have reached the rounding level of the residual,
// where they only fluctuate and further updates do not improve the iterate:
// either md <= PRED_FLOOR tol mr and the relative update norm has not
// decreased over the last two updates, or md <= PRED_STALL tol mr and it is
// still above 0.9 of what it was three updates earlier (no progress; a
// converging iteration shrinks it by the contraction ratio every update, well
// below 0.9^(1/3) here).  0 otherwise.
constexpr double PRED_FLOOR = 16.0, PRED_STALL = 64.0;
__device__ __forceinline__ int pred_stop(double md, double mr, float q, float qprev, float qprev2, float qprev3,
                                         int it, double tol)
{
    if (md <= tol * mr) return 1;
    if (it > 2 && md <= PRED_FLOOR * tol * mr && q >= qprev && qprev >= qprev2) return 2;
    if (it > 3 && md <= PRED_STALL * tol * mr && q >= 0.9f * qprev3) return 2;
    return 0;
}


// -------------------------------------------------------------------------
// scalar temperature equation (4.13): Newton with an upper bound of the root
// -------------------------------------------------------------------------
// g is convex and increasing for T >= 0, and its root lies below both
// single-term roots (C/q4)^{1/4} and C/lin, C = rhs + lin Tn (each term alone
// is non-negative), and above half the smaller of them; iterates are clamped to
// that bound, so a start far below the root (a cold cell heated by the inflow)
// does not overshoot by orders of magnitude and then creep back by 3/4 per
// step.  The root and the stopping test are those of the plain iteration.
__device__ __forceinline__ double newton_cap(double q4, double lin, double rhs, double Tn)
{
    const double C = rhs + lin * Tn;
    // no positive root, or a linear equation (Newton exact in one step): no bound
    if (!(C > 0.0) || !(q4 > 0.0)) return INFINITY;
    // widened by 2^-50 so that rounding never puts the bound below the root
    return fmin(sqrt(sqrt(C / q4)), C / lin) * (1.0 + 0x1p-50);
}

__device__ __forceinline__ bool newton_quartic(double T0, double Tn, double q4, double lin, double rhs, int maxit,
                                               double &T, int &its)
{
    const double cap = newton_cap(q4, lin, rhs, Tn);
    T = T0;
    for (int k = 0; k < maxit; ++k) {
        const double T2 = T * T;
        const double g = q4 * T2 * T2 + lin * (T - Tn) - rhs;
        const double dg = 4.0 * q4 * T2 * T + lin;
        const double Tp = T;
        T = fmin(T - g / dg, cap);
        const double step = Tp - T;
        ++its;
        if (fabs(step) <= 0x1p-50 * fmax(fabs(T), fabs(Tn))) return true;
    }
    return false;
}

}  // namespace
