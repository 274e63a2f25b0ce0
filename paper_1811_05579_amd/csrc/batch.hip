// batch.hip -- batched form of the AP step: many independent 1-D slabs of
// different size, ordinate count, eps, dt and opacity advanced together, one
// graph of eight launches per step (the grte_batch_* calls of include/grte.h):
// the per-cell phases (coefficients and right-hand sides, moments and Newton,
// the correction's right-hand sides, the projection) as flat kernels over all
// cells, the two per-slab solves (prediction, correction) as persistent tile
// kernels.
//
// In the solve kernels every instance is advanced by one "tile": a whole
// work-group (W = 256 threads) or, for small slabs, one wavefront (W = 64; four
// independent instances per work-group).  In a work-group tile the per-pair
// tridiagonal solves are split over its four wavefronts (pairs p = w, w + 4,
// ... on wavefront w), each solving its pair alone with 4 M rows per lane:
// four independent elimination chains in flight per work-group.  The step is
// the algebra of the
// single-instance path (Algorithm 2 and Section 5 of Tang, Wang & Zhang):
// the per-pair tridiagonal operators T_p = Lam + mu_p^2 L + mu_p B with U*
// eliminated through (4.5c), the angular coupling of the prediction solved by
// the DSA-preconditioned residual-form iteration with adaptive Chebyshev
// updates (warm-started from the previous step's rho*),
// Newton on (4.13)/(5.5), the per-pair correction (4.11) and the projection
// (4.14).  One tile owns all parity pairs of its instance, so the angular sum
// is accumulated in registers (and, across the wavefronts of a work-group,
// summed through LDS in a fixed order) and no grid-wide synchronisation
// exists.
// Instances are taken from two work queues -- work-group tiles first, then
// wavefront tiles -- in an order chosen by the host (longest expected work
// first), so that work-groups that finish their large slabs early drain the
// small ones.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/grte.h"
#include "solver_common.hpp"

namespace {

constexpr int BNT = 256;              // threads per work-group
constexpr int WAVE = 64;
constexpr int BMAX_N = 2048;          // largest slab of the batched path (8 rows per thread)
constexpr int BMAX_P = 64;
constexpr int WAVE_MAX_N = 256;       // largest slab a wavefront tile can take (4 rows per lane)

// per-instance cell scratch: NCA arrays of N+1 entries
enum {
    C_AW, C_BC, C_LL, C_LU, C_LAM, C_LMG, C_BD, C_BETA, C_RHON, C_TNEW,
    C_FLUX,     // [0], [1]: sum_p omega_p mu_p O*_{0,p} and O*_{N,p} (energy balance)
    NCA
};

// LDS of one tile (doubles).  A work-group tile (NP = 256 M padded rows, in
// the layout of the wavefront solver: 64 lanes of 4 M rows) holds rho, Ll, Lu,
// Lam and Lam - G, the angular sums of its four wavefronts (4 NP), the last
// Chebyshev update of every row (NP binary32) and a 32-double reduction area;
// a wavefront tile holds rho, Ll, Lu in its position order and its solver's
// scratch.
constexpr int LDS_WG = 9 * BMAX_N + BMAX_N / 2 + 32;
constexpr int LDS_WAVE = 3 * WAVE_MAX_N + tile_scratch<WAVE>();
static_assert(4 * LDS_WAVE <= LDS_WG, "four wavefront tiles fit in the work-group LDS");

struct BInst {
    int N, P, m, W, M;                 // tile of W threads, M rows each
    int cb0, ncb;                      // the instance's blocks of the per-cell kernels (cblk)
    int pad;
    double dx, a, c, cv, eps, dt;
    double one_minus_W, mu1, mu2;      // 1 - sum omega (exact), sum omega mu, sum omega mu^2
    long long oE, oO, oT, oP;          // offsets of E (N P), O ((N+1) P), cells (N), pairs (P)
    long long oC, oR, NPa;             // cell scratch, pair scratch (2 P NPa), padded rows allocated
};

struct BatchArgs {
    int n_wg, n_wave;
    const BInst *inst;
    const int *order;                  // n_wg work-group instances, then n_wave wavefront instances
    int *queue;                        // per solve kernel: [0] work-group queue head, [1] wavefront queue head
    const int2 *cblk;                  // blocks of the per-cell kernels: (instance, first cell)
    double *epart;                     // 2 per block of the projection: the energy partial sums
    int n_inst;
    const double *E, *O, *T, *sigma0;
    double *E2, *O2, *T2;
    // binary32 storage (f32 != 0): E^n = a c (T^n)^4 + E32, O^n = O32 in;
    // E32o = E^{n+1} - a c (T^{n+1})^4, O32o = O^{n+1} out (E, O, E2, O2 unused)
    const float *E32, *O32;
    float *E32o, *O32o;
    int f32;                    // (the kernel variant is chosen by the host)
    const double *mu, *omega, *bL, *bR;
    double *cells, *pairs;
    int *istat;                        // 8 per instance
    double tol;
    int maxit, newton_maxit;
    int accel;                  // prediction acceleration (GRTE_ACCEL_*)
    double *rprev;              // per cell: the last prediction's rho* (written every step)
    int warm;                   // start the prediction from rprev instead of rho^n
    double *ienergy;            // per instance: E_tot^n, E_tot^{n+1}, outflow dt, defect
    int *sticky;                // error flags OR-ed over steps (GRTE_ERRF_*), not cleared by a step
};

// make the tile's LDS and global writes visible to the whole tile
template <int W>
__device__ __forceinline__ void tsync()
{
    if constexpr (W == BNT) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// v through an empty asm: the compiler cannot hoist what is derived from the
// result out of the enclosing loop (keeps per-row addresses out of registers)
__device__ __forceinline__ int opaque(int v)
{
    __asm__ volatile("" : "+v"(v));
    return v;
}

// interior node i (1..N-1): harmonic-mean sigma, arithmetic-mean K
__device__ __forceinline__ void b_node(const BInst &I, const double *Tk, const double *sg, int i,
                                       double &aw, double &bc)
{
    const double Kn = 0.5 * (kpow(Tk[i - 1], I.m) + kpow(Tk[i], I.m));
    const double sl = sg[i - 1], sr = sg[i];
    const double ss = sl + sr;
    const double sn = ss > 0.0 ? 2.0 * sl * sr / ss : 0.0;
    const double den = Kn * I.eps * I.eps + sn * I.c * I.dt;
    if (den > 0.0) {
        aw = Kn * I.eps * I.eps / den;
        bc = Kn * I.c * I.dt / (I.dx * den);
    } else {
        aw = 0.0;
        bc = 0.0;
    }
}

// the coefficients of cell j's right-hand sides (used by the thread that
// formed them, not stored): h = K eps^2 c dt / dx, K eps^2, the source term,
// and the two face weights of the node relations (doubled at the ends)
struct CellRhs {
    double h, keps, src, awr, awl;
};

// per-cell coefficients of cell j; mode 0: prediction (K from T^n, with the
// U* elimination of (4.5c)), 1: correction (K from T^{n+1})
__device__ CellRhs b_cell(const BInst &I, int mode, const double *Tk, const double *Tn, const double *sg,
                          int j, double *C, int N1)
{
    CellRhs R;
    const int N = I.N;
    const double eps = I.eps, c = I.c, dt = I.dt;
    double awl = 0.0, bcl = 0.0, awr = 0.0, bcr = 0.0;
    if (j >= 1) b_node(I, Tk, sg, j, awl, bcl);
    if (j <= N - 2) b_node(I, Tk, sg, j + 1, awr, bcr);
    C[C_AW * N1 + j] = awl;
    C[C_BC * N1 + j] = bcl;
    if (j == N - 1) {
        C[C_AW * N1 + N] = 0.0;
        C[C_BC * N1 + N] = 0.0;
    }
    const double Kc = kpow(Tk[j], I.m);
    const double s0 = sg[j];
    const double h = Kc * eps * eps * c * dt / I.dx;
    const double fr = (j <= N - 2) ? h * bcr * (j == 0 ? 2.0 : 1.0) : 0.0;
    const double fl = (j >= 1) ? h * bcl * (j == N - 1 ? 2.0 : 1.0) : 0.0;
    const double bd = (j == 0 || j == N - 1) ? 2.0 * h / eps : 0.0;
    C[C_LL * N1 + j] = -fl;
    C[C_LU * N1 + j] = -fr;
    C[C_BD * N1 + j] = bd;
    C[C_LAM * N1 + j] = Kc * eps * eps + s0 * c * dt;
    R.h = h;
    R.awr = (j <= N - 2) ? awr * (j == 0 ? 2.0 : 1.0) : 0.0;
    R.awl = (j >= 1) ? awl * (j == N - 1 ? 2.0 : 1.0) : 0.0;
    R.keps = Kc * eps * eps;
    const double ac = I.a * c;
    if (mode == 0) {
        const double t = Tn[j];
        const double Un = t * t * t * t;
        const double t3m = (I.m == 0) ? t * t * t : 1.0;
        const double beta = 4.0 * s0 * dt * t3m / (eps * eps * I.cv);
        const double opb = 1.0 + ac * beta;
        const double lmg = Kc * eps * eps + s0 * c * dt / opb;
        C[C_BETA * N1 + j] = beta;
        C[C_LMG * N1 + j] = lmg;
        R.src = s0 * c * dt * ac * Un / opb;
    } else {
        const double t1 = Tk[j];
        R.src = s0 * c * dt * ac * (t1 * t1 * t1 * t1);
    }
    return R;
}

// The state E^n, O^n of one instance: binary64 arrays in the caller's
// cell-major layout (E[j P + p], O[i P + p]), or the binary32 storage
// E32 = E^n - a c (T^n)^4, O32 = O^n (f32 != 0), kept pair-major
// (E32[p N + j], O32[p (N + 1) + i]): the per-cell kernels take consecutive
// cells on consecutive lanes, so their loads and stores of one pair are
// contiguous (set_state / get_state transpose, batch_convert).
template <bool F32>
struct BState {
    static constexpr bool f32 = F32;
    const double *E, *O, *Tn;
    const float *E32, *O32;
    double ac;
    int P, N;
    __device__ __forceinline__ size_t ei(int j, int p) const
    {
        return F32 ? (size_t)p * N + j : (size_t)j * P + p;
    }
    __device__ __forceinline__ size_t oi(int i, int p) const
    {
        return F32 ? (size_t)p * (N + 1) + i : (size_t)i * P + p;
    }
    __device__ __forceinline__ double e(int j, int p) const
    {
        if constexpr (!F32) return E[ei(j, p)];
        const double t = Tn[j];
        return ac * (t * t) * (t * t) + (double)E32[ei(j, p)];
    }
    __device__ __forceinline__ double o(int i, int p) const
    {
        if constexpr (F32) return (double)O32[oi(i, p)];
        else return O[oi(i, p)];
    }
};

// O at node i of pair p from cell values ec[] of that pair (cell order) and
// the stored O^n: the node relation at interior nodes, the inflow relations
// (4.7) at the two ends
template <bool F32>
__device__ __forceinline__ double node_pc(const double *ec, const BState<F32> &S, const double *Aw,
                                          const double *Bc, double mu, double bl, double br, double eps, int N,
                                          int i, int p)
{
    auto inner = [&](int ii) { return Aw[ii] * S.o(ii, p) - Bc[ii] * mu * (ec[ii] - ec[ii - 1]); };
    if (i >= 1 && i <= N - 1) return inner(i);
    if (i == 0) return 2.0 / eps * (bl - ec[0]) - inner(1);
    return 2.0 / eps * (ec[N - 1] - br) - inner(N - 1);
}

// The per-cell phases take the pairs of their cell in groups of RHS_U: the
// group's state loads are all issued before its arithmetic (RHS_U memory round
// trips in flight per thread), and the cell's coefficients are read once.
constexpr int RHS_U = 4;

// ---------------------------------------------------------------------------
// The per-cell phases run as flat kernels over every cell of every slab (one
// thread per cell, blocks of CB cells of one slab, cblk): they stream the
// state and the pair scratch, and at the occupancy of a small kernel many more
// of their memory round trips are in flight than inside the solve kernels,
// which hold one work-group per CU for their LDS and registers.

// one instance's arrays, as the phases see them
template <bool F32>
struct IView {
    BInst I;
    int N, P, N1, NP;               // NP: pair stride of the pair scratch (the instance's tile, W M)
    const double *Tn, *sg, *mu, *om, *bL, *bR;
    double *T2, *C, *Rt, *Et;
    int *st;
    BState<F32> S;
};

template <bool F32>
__device__ __forceinline__ IView<F32> iview(const BatchArgs &A, int i)
{
    IView<F32> V;
    V.I = A.inst[i];
    const BInst &I = V.I;
    V.N = I.N;
    V.P = I.P;
    V.N1 = I.N + 1;
    V.NP = 64 * I.M;                           // rows per lane: wavefront M, work-group LMW
    V.Tn = A.T + I.oT;
    V.sg = A.sigma0 + I.oT;
    V.mu = A.mu + I.oP;
    V.om = A.omega + I.oP;
    V.bL = A.bL + I.oP;
    V.bR = A.bR + I.oP;
    V.T2 = A.T2 + I.oT;
    V.C = A.cells + I.oC;
    V.Rt = A.pairs + I.oR;
    V.Et = V.Rt + (size_t)I.P * I.NPa;
    V.st = A.istat + 8 * i;
    V.S.P = I.P;
    V.S.N = I.N;
    V.S.ac = I.a * I.c;
    V.S.Tn = V.Tn;
    V.S.E = F32 ? nullptr : A.E + I.oE;
    V.S.O = F32 ? nullptr : A.O + I.oO;
    V.S.E32 = F32 ? A.E32 + I.oE : nullptr;
    V.S.O32 = F32 ? A.O32 + I.oO : nullptr;
    return V;
}

// right-hand sides of cell j's per-pair systems into Rt (pair-major, cell order)
template <bool F32>
__device__ __forceinline__ void rhs_cell(const IView<F32> &V, int j, const CellRhs &R)
{
    const BInst &I = V.I;
    const int N = V.N, P = V.P, NP = V.NP;
    const double *mu = V.mu, *bL = V.bL, *bR = V.bR;
    double *Rt = V.Rt;
    const BState<F32> &S = V.S;
    const double h = R.h, keps = R.keps, src = R.src, awr = R.awr, awl = R.awl;
    const bool has_r = j <= N - 2, has_l = j >= 1;
    for (int p0 = 0; p0 < P; p0 += RHS_U) {
        double e[RHS_U], orr[RHS_U], ol[RHS_U];
#pragma unroll
        for (int u = 0; u < RHS_U; ++u) {
            const int p = p0 + u < P ? p0 + u : P - 1;   // tail: a valid index, result unused
            e[u] = S.e(j, p);
            orr[u] = has_r ? S.o(j + 1, p) : 0.0;
            ol[u] = has_l ? S.o(j, p) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RHS_U; ++u) {
            const int p = p0 + u;
            if (p >= P) break;
            double rv = keps * e[u] + src - h * mu[p] * (awr * orr[u] - awl * ol[u]);
            if (j == 0) rv += 2.0 * h * mu[p] * bL[p] / I.eps;
            if (j == N - 1) rv += 2.0 * h * mu[p] * bR[p] / I.eps;
            Rt[(size_t)p * NP + j] = rv;
        }
    }
}

// prediction set-up of cell j: coefficients (K from T^n), rho^n, the pairs'
// right-hand sides
template <bool F32>
__device__ __forceinline__ void cell_pred_setup(const IView<F32> &V, int j)
{
    const BInst &I = V.I;
    const int P = V.P, N1 = V.N1;
    double *C = V.C;
    const CellRhs R = b_cell(I, 0, V.Tn, V.Tn, V.sg, j, C, N1);
    double rn = 0.0;
#pragma unroll 4
    for (int p = 0; p < P; ++p) rn += V.om[p] * V.S.e(j, p);
    C[C_RHON * N1 + j] = rn;
    rhs_cell(V, j, R);
}

// correction set-up of cell j: coefficients with K from T^{n+1}, right-hand sides
template <bool F32>
__device__ __forceinline__ void cell_corr_setup(const IView<F32> &V, int j)
{
    const CellRhs R = b_cell(V.I, 1, V.C + C_TNEW * V.N1, V.Tn, V.sg, j, V.C, V.N1);
    rhs_cell(V, j, R);
}

// correction substep 1 of cell j: moments of E*, D from the prediction's node
// fluxes, U*, K*, Newton on (4.13)/(5.5); step counters accumulated in the caller's
template <bool F32>
__device__ __forceinline__ void cell_newton(const BatchArgs &A, const IView<F32> &V, int j, int &n_its,
                                            int &n_fail, int &n_clamp, int &n_neg)
{
    const BInst &I = V.I;
    const int N = V.N, P = V.P, N1 = V.N1, NP = V.NP;
    const double eps = I.eps;
    const double *Tn = V.Tn, *sg = V.sg, *mu = V.mu, *om = V.om, *bL = V.bL, *bR = V.bR;
    double *C = V.C, *T2 = V.T2;
    const double *Et = V.Et;
    const BState<F32> &S = V.S;
    double rs = 0.0, D = 0.0, f0 = 0.0, fN = 0.0;
    // O* at nodes j and j+1 from the node relation (inline for interior
    // nodes) and the inflow relations (4.7) at the two ends (node_pc); the
    // pairs in groups of RHS_U whose loads are issued first
    const bool inner_l = j >= 1, inner_r = j + 1 <= N - 1;
    const double awl = C[C_AW * N1 + j], bcl = C[C_BC * N1 + j];
    const double awr = inner_r ? C[C_AW * N1 + j + 1] : 0.0, bcr = inner_r ? C[C_BC * N1 + j + 1] : 0.0;
    for (int p0 = 0; p0 < P; p0 += RHS_U) {
        double em[RHS_U], ej[RHS_U], ep1[RHS_U], onl[RHS_U], onr[RHS_U];
#pragma unroll
        for (int u = 0; u < RHS_U; ++u) {
            const int p = p0 + u < P ? p0 + u : P - 1;   // tail: a valid index, result unused
            const double *ep = Et + (size_t)p * NP;
            ej[u] = ep[j];
            em[u] = inner_l ? ep[j - 1] : 0.0;
            ep1[u] = inner_r ? ep[j + 1] : 0.0;
            onl[u] = inner_l ? S.o(j, p) : 0.0;
            onr[u] = inner_r ? S.o(j + 1, p) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RHS_U; ++u) {
            const int p = p0 + u;
            if (p >= P) break;
            const double *ep = Et + (size_t)p * NP;
            const double m1 = mu[p];
            double ol, orr;
            if (inner_l) {
                ol = awl * onl[u] - bcl * m1 * (ej[u] - em[u]);
            } else {
                ol = node_pc(ep, S, C + C_AW * N1, C + C_BC * N1, m1, bL[p], bR[p], eps, N, j, p);
            }
            if (inner_r) {
                orr = awr * onr[u] - bcr * m1 * (ep1[u] - ej[u]);
            } else {
                orr = node_pc(ep, S, C + C_AW * N1, C + C_BC * N1, m1, bL[p], bR[p], eps, N, j + 1, p);
            }
            rs += om[p] * ej[u];
            D += om[p] * m1 * (orr - ol);
            f0 += om[p] * m1 * ol;
            fN += om[p] * m1 * orr;
        }
    }
    if (j == 0) C[C_FLUX * N1] = f0;
    if (j == N - 1) C[C_FLUX * N1 + 1] = fN;
    D /= I.dx;
    const double ac = I.a * I.c;
    const double t = Tn[j];
    const double Un = t * t * t * t;
    const double beta = C[C_BETA * N1 + j];
    const double us = (Un + beta * rs) / (1.0 + ac * beta);
    double Ks = 1.0;
    if (I.m == 3) {
        if (us < 0.0) {
            Ks = 0.0;
            ++n_clamp;
        } else {
            Ks = pow(us, 0.75);
        }
    }
    const double s0 = sg[j];
    const double lin = I.cv * (eps * eps * Ks + I.c * s0 * I.dt);
    const double q4 = ac * s0 * I.dt;
    const double rhs = s0 * I.dt * (C[C_RHON * N1 + j] - I.c * I.dt * D);
    double T = t;
    int its = 0;
    if (!(s0 == 0.0 && Ks == 0.0)) {
        if (t + rhs / lin < 0.0) ++n_neg;
        bool ok = false;
        // Newton from T^n, iterates clamped to the upper bound of the root
        // (the smaller single-term root of q4 T^4 + lin T = rhs + lin T^n)
        const double Cq = rhs + lin * t;
        const double cap = (Cq > 0.0 && q4 > 0.0)
                               ? fmin(sqrt(sqrt(Cq / q4)), Cq / lin) * (1.0 + 0x1p-50) : INFINITY;
        for (its = 0; its < A.newton_maxit;) {
            const double T2v = T * T;
            const double g = q4 * T2v * T2v + lin * (T - t) - rhs;
            const double dg = 4.0 * q4 * T2v * T + lin;
            const double Tp = T;
            T = fmin(T - g / dg, cap);
            const double step = Tp - T;
            ++its;
            if (fabs(step) <= 0x1p-50 * fmax(fabs(T), fabs(t))) { ok = true; break; }
        }
        if (!ok) ++n_fail;
    }
    C[C_TNEW * N1 + j] = T;
    T2[j] = T;
    n_its = max(n_its, its);
}

// projection (4.14) of cell j: E^{n+1} and O^{n+1} (node relation with K^{n+1})
// into the state, and cell j's terms of the energy balance ((3.12)-(3.13)):
// E_tot = sum_j dx (rho_j / c + Cv T_j) before (eb) and after (ea) the step
template <bool F32>
__device__ __forceinline__ void cell_project(const BatchArgs &A, const IView<F32> &V, int j, double &eb,
                                             double &ea)
{
    const BInst &I = V.I;
    const int N = V.N, P = V.P, N1 = V.N1, NP = V.NP;
    const double eps = I.eps;
    const double *Tn = V.Tn, *mu = V.mu, *om = V.om, *bL = V.bL, *bR = V.bR;
    const double *C = V.C, *T2 = V.T2, *Et = V.Et;
    const BState<F32> &S = V.S;
    const double *Aw = C + C_AW * N1, *Bc = C + C_BC * N1;
    // the pairs in groups of RHS_U: the group's loads are issued before its
    // stores (O at node j from the node relation, the interior case inline;
    // the two end nodes by node_pc)
    float *E32o = F32 ? A.E32o + I.oE : nullptr, *O32o = F32 ? A.O32o + I.oO : nullptr;
    double *E2 = F32 ? nullptr : A.E2 + I.oE, *O2 = F32 ? nullptr : A.O2 + I.oO;
    const double t1 = T2[j];
    const double base = S.ac * (t1 * t1) * (t1 * t1);
    const double awj = Aw[j], bcj = Bc[j];
    double r1 = 0.0;
    for (int p0 = 0; p0 < P; p0 += RHS_U) {
        double ej[RHS_U], em[RHS_U], on[RHS_U];
#pragma unroll
        for (int u = 0; u < RHS_U; ++u) {
            const int p = p0 + u < P ? p0 + u : P - 1;   // tail: a valid index, result unused
            const double *ep = Et + (size_t)p * NP;
            ej[u] = ep[j];
            em[u] = j >= 1 ? ep[j - 1] : 0.0;
            on[u] = j >= 1 ? S.o(j, p) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RHS_U; ++u) {
            const int p = p0 + u;
            if (p >= P) break;
            const double *ep = Et + (size_t)p * NP;
            r1 += om[p] * ej[u];
            double oj;
            if (j >= 1) {
                oj = awj * on[u] - bcj * mu[p] * (ej[u] - em[u]);
            } else {
                oj = node_pc(ep, S, Aw, Bc, mu[p], bL[p], bR[p], eps, N, 0, p);
            }
            // the new state in the layout of the stored one (S.ei, S.oi)
            if constexpr (F32) {
                E32o[S.ei(j, p)] = (float)(ej[u] - base);
                O32o[S.oi(j, p)] = (float)oj;
                if (j == N - 1) O32o[S.oi(N, p)] = (float)node_pc(ep, S, Aw, Bc, mu[p], bL[p], bR[p], eps, N, N, p);
            } else {
                E2[S.ei(j, p)] = ej[u];
                O2[S.oi(j, p)] = oj;
                if (j == N - 1) O2[S.oi(N, p)] = node_pc(ep, S, Aw, Bc, mu[p], bL[p], bR[p], eps, N, N, p);
            }
        }
    }
    eb = I.dx * (C[C_RHON * N1 + j] / I.c + I.cv * Tn[j]);
    ea = I.dx * (r1 / I.c + I.cv * t1);
}

// W = BNT: a work-group tile of LMW rows per lane (NP = 64 LMW; M = LMW / 4 rows per
// thread of the work-group-wide diffusion solve where LMW is a multiple of 4 and at
// least 8); W = 64: a wavefront tile of M rows per lane
template <int W, int M, bool F32, int LMW = 4 * M>
__device__ __forceinline__ void pred_solve(const BatchArgs &A, int i, double *sm)
{
    constexpr int NP = 64 * (W == BNT ? LMW : M);
    const BInst I = A.inst[i];
    const int N = I.N, P = I.P, N1 = N + 1;
    const int k = opaque(tile_lane<W>());   // opaque: per-thread addresses are formed per instance, not held across the queue loop
    const int j0 = k * M;
    const double *Tn = A.T + I.oT;
    BState<F32> S;
    S.P = I.P;
    S.N = I.N;
    S.ac = I.a * I.c;
    S.Tn = Tn;
    S.E = F32 ? nullptr : A.E + I.oE;
    S.O = F32 ? nullptr : A.O + I.oO;
    S.E32 = F32 ? A.E32 + I.oE : nullptr;
    S.O32 = F32 ? A.O32 + I.oO : nullptr;
    const double *mu = A.mu + I.oP, *om = A.omega + I.oP;
    double *C = A.cells + I.oC;
    // Per-pair global arrays are pair-major in cell order: thread k's rows
    // j0 .. j0+M-1 are contiguous, so its loads and stores are wide and the
    // later per-cell phases read along cells.
    double *Rt = A.pairs + I.oR;                  // right-hand sides
    double *Et = Rt + (size_t)P * I.NPa;          // E* (prediction), then E^{n+1} (correction)
    int *st = A.istat + 8 * i;
    // Work-group tiles keep the per-row arrays in the layout of the wavefront
    // solver (LM = 4 M rows per lane, row j at LDS position (j % LM) 64 + j / LM);
    // wavefront tiles in their own position order (LM = M, the same formula).
    constexpr bool WG = (W == BNT);
    constexpr int LM = WG ? LMW : M;
    auto lpos = [](int j) { return (j % LM) * 64 + j / LM; };
    double *rho = sm, *sLl = sm + NP, *sLu = sm + 2 * NP, *sh = sm + 3 * NP;
    double *slam = nullptr, *slmg = nullptr, *accw = nullptr, *red = nullptr;
    float *sdch = nullptr;
    if constexpr (WG) {
        slam = sm + 3 * NP;
        slmg = sm + 4 * NP;
        accw = sm + 5 * NP;
        sdch = reinterpret_cast<float *>(sm + 9 * NP);
        red = sm + 9 * NP + NP / 2;
    }

    double *rp = A.rprev + I.oT;
    for (int j = k; j < NP; j += W) {
        const int t = lpos(j);
        const bool in = j < N;
        rho[t] = in ? (A.warm ? rp[j] : C[C_RHON * N1 + j]) : 0.0;
        sLl[t] = in ? C[C_LL * N1 + j] : 0.0;
        sLu[t] = in ? C[C_LU * N1 + j] : 0.0;
        if constexpr (WG) {
            slam[t] = in ? C[C_LAM * N1 + j] : 1.0;   // padding rows: T_p = D = 1, no coupling
            slmg[t] = in ? C[C_LMG * N1 + j] : 1.0;
            sdch[t] = 0.0f;
        }
    }
    tsync<W>();
    const double bd0 = C[C_BD * N1 + 0], bdN = C[C_BD * N1 + N - 1];

    // ---------------- prediction: DSA-preconditioned iteration (plain or Chebyshev updates)
    int it = 0, converged = 0, ph = 0;
    ChebState Cs;
    if constexpr (WG) {
        const int w = threadIdx.x >> 6;
        // Per lane: jq = first row, nv = rows inside the slab, rl1 = lane row of
        // the slab's last row.  The lane index is re-derived through opaque() in
        // every pair step, so each array costs one base register there and the
        // rows are immediate offsets r * 64 doubles.
        // Padding rows (j >= N) need no tests: their right-hand sides are zero,
        // Lam = Lam - G = 1 and Ll = Lu = 0 there, so every solve and update
        // below yields exact zeros in them.
        auto load_r = [&](int p, double (&v)[LM]) {
            const double *src = Rt + (size_t)p * NP + opaque(threadIdx.x & 63) * LM;
#pragma unroll
            for (int r = 0; r < LM; ++r) v[r] = src[r];
        };
        // One sweep of this wavefront's pairs from the current rho: v_p = T_p^{-1}
        // [r_p - (Lam - G + mu^2 L + mu B) rho], summed as omega_p v_p into the
        // wavefront's LDS row sums, or (final) E*_p = rho + v_p written.  rnext
        // holds pair w's right-hand side on entry and again on return (loaded
        // while the tile waits).
        double rnext[LM];
        if (w < P) load_r(w, rnext);
        auto sweep = [&](bool final_sweep) {
            if (!final_sweep) {
                double *acc = accw + w * NP + opaque(threadIdx.x & 63);
#pragma unroll
                for (int r = 0; r < LM; ++r) acc[r * 64] = 0.0;
            }
            for (int p = w; p < P; p += 4) {
                const double m1 = mu[p], m2 = m1 * m1, wp = om[p];
                double x[LM];
#pragma unroll
                for (int r = 0; r < LM; ++r) x[r] = rnext[r];
                load_r(p + 4 < P ? p + 4 : w, rnext);
                const int lq = opaque(threadIdx.x & 63), jq = lq * LM, rl1 = N - 1 - jq;
                const double *rh = rho + lq, *ll = sLl + lq, *lu = sLu + lq, *la = slam + lq, *lg = slmg + lq;
                const double b0 = jq == 0 ? bd0 : 0.0;
                auto bdr = [&](int r) { return (r == 0 ? b0 : 0.0) + (r == rl1 ? bdN : 0.0); };
#pragma unroll
                for (int r = 0; r < LM; ++r) {
                    // the neighbours' rho (an in-bounds dummy where there is none: its
                    // coefficient ll or lu is 0 there)
                    const double rj = rh[r * 64];
                    const double rl = (r > 0) ? rh[(r - 1) * 64] : (jq > 0 ? rh[(LM - 1) * 64 - 1] : rj);
                    const double rn = (r < LM - 1) ? rh[(r + 1) * 64] : (lq < 63 ? rh[1] : rj);
                    const double q = ll[r * 64] * (rl - rj) + lu[r * 64] * (rn - rj);   // difference form
                    x[r] = x[r] - lg[r * 64] * rj - m2 * q - m1 * bdr(r) * rj;
                }
                lane_chunk_solve<LM>(
                    [&](int r) { return m2 * ll[r * 64]; },
                    [&](int r) { return la[r * 64] + m2 * (-(ll[r * 64] + lu[r * 64])) + m1 * bdr(r); },
                    [&](int r) { return m2 * lu[r * 64]; }, x);
                if (final_sweep) {
                    double *ep = Et + (size_t)p * NP + jq;
#pragma unroll
                    for (int r = 0; r < LM; ++r) ep[r] = rh[r * 64] + x[r];
                } else {
                    double *acc = accw + w * NP + lq;
#pragma unroll
                    for (int r = 0; r < LM; ++r) acc[r * 64] += wp * x[r];
                }
            }
        };
        while (true) {
            {
                sweep(false);
                __syncthreads();
                double alpha, beta;
                cheb_coeffs(Cs, A.accel, A.tol, alpha, beta);   // every wavefront: the same state
                if constexpr (LM % 4 == 0 && LM >= 8) {
                    // res = sum_p omega_p v_p - (1 - W) rho (the four wavefronts' sums in
                    // a fixed order);  rho += res + D^{-1} (G res), G = Lam - (Lam - G),
                    // D = Lam - G + <mu^2> L + <mu> B (the diffusion operator of the DSA),
                    // solved by the whole work-group (tri_factor_solve): thread k takes the
                    // M rows j = k M + r, which lie in lane k / 4 of the wavefront layout
                    // at rows (k % 4) M + r, i.e. at LDS position base + 64 r
                    const int kk = opaque((int)threadIdx.x);
                    const int base = (kk & 3) * M * 64 + (kk >> 2), jk = kk * M;
                    double rl[M], d[M], bb[M], f[M];
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const int t = base + r * 64, j = jk + r;
                        const double tot = ((accw[t] + accw[NP + t]) + accw[2 * NP + t]) + accw[3 * NP + t];
                        rl[r] = tot - I.one_minus_W * rho[t];
                        d[r] = (slam[t] - slmg[t]) * rl[r];
                        const double bdj = (j == 0 ? bd0 : 0.0) + (j == N - 1 ? bdN : 0.0);
                        bb[r] = slmg[t] + I.mu2 * (-(sLl[t] + sLu[t])) + I.mu1 * bdj;
                    }
                    __syncthreads();                  // every angular sum read: accw is the solver's scratch now
                    int ph0 = 0;
                    tri_factor_solve<BNT, M>(I.mu2, sLl, sLu, bb, d, f, accw, ph0, base, 64);
                    double md = 0.0, mr = 0.0;
#pragma unroll
                    for (int r = 0; r < M; ++r) {
                        const int t = base + r * 64;
                        const double z = rl[r] + f[r];
                        const double upd = alpha * (double)sdch[t] + beta * z;
                        sdch[t] = (float)upd;
                        const double nw = rho[t] + upd;
                        rho[t] = nw;
                        md = fmax(md, fabs(z));
                        mr = fmax(mr, fabs(nw));
                    }
                    // maxima over the tile: a butterfly per wavefront, then the four in order
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        md = fmax(md, __shfl_xor(md, o, 64));
                        mr = fmax(mr, __shfl_xor(mr, o, 64));
                    }
                    if ((threadIdx.x & 63) == 0) {
                        red[w] = md;
                        red[8 + w] = mr;
                    }
                } else {
                    // the same correction where the tile's rows per lane are not 4 M
                    // (M >= 2): every wavefront solves the whole diffusion system in the
                    // wavefront layout (lane_chunk_solve, LM rows per lane), the same in
                    // all four; wavefront w then updates the rows r = w (mod 4) of its lanes
                    const int lq = opaque(threadIdx.x & 63), jq = lq * LM, rl1 = N - 1 - jq;
                    const double *ll = sLl + lq, *lu = sLu + lq, *lg = slmg + lq;
                    auto res_at = [&](int r) {
                        const int t = r * 64 + lq;
                        const double tot = ((accw[t] + accw[NP + t]) + accw[2 * NP + t]) + accw[3 * NP + t];
                        return tot - I.one_minus_W * rho[t];
                    };
                    double f[LM];
#pragma unroll
                    for (int r = 0; r < LM; ++r) f[r] = (slam[r * 64 + lq] - slmg[r * 64 + lq]) * res_at(r);
                    __syncthreads();                  // every wavefront has read rho before any update
                    const double b0 = jq == 0 ? bd0 : 0.0;
                    auto bdr = [&](int r) { return (r == 0 ? b0 : 0.0) + (r == rl1 ? bdN : 0.0); };
                    lane_chunk_solve<LM>(
                        [&](int r) { return I.mu2 * ll[r * 64]; },
                        [&](int r) { return lg[r * 64] + I.mu2 * (-(ll[r * 64] + lu[r * 64])) + I.mu1 * bdr(r); },
                        [&](int r) { return I.mu2 * lu[r * 64]; }, f);
                    double md = 0.0, mr = 0.0;
#pragma unroll
                    for (int r = 0; r < LM; ++r) {
                        if ((r & 3) != w) continue;
                        const int t = r * 64 + lq;
                        const double z = res_at(r) + f[r];
                        const double upd = alpha * (double)sdch[t] + beta * z;
                        sdch[t] = (float)upd;
                        const double nw = rho[t] + upd;
                        rho[t] = nw;
                        md = fmax(md, fabs(z));
                        mr = fmax(mr, fabs(nw));
                    }
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        md = fmax(md, __shfl_xor(md, o, 64));
                        mr = fmax(mr, __shfl_xor(mr, o, 64));
                    }
                    if ((threadIdx.x & 63) == 0) {
                        red[w] = md;
                        red[8 + w] = mr;
                    }
                }
                __syncthreads();                      // the rho update and its norms visible to the tile
            }
            const double md = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            const double mr = fmax(fmax(red[8], red[9]), fmax(red[10], red[11]));
            ++it;
            const float qprev = Cs.q1, qprev2 = Cs.q2, qprev3 = Cs.q3;
            const float q = (float)(mr > 0.0 ? md / mr : md);
            cheb_record(Cs, q);
            converged = pred_stop(md, mr, q, qprev, qprev2, qprev3, it, A.tol);
            if (converged || it >= A.maxit) break;
        }
        sweep(true);                                  // E* of the final iterate
    } else {
        double lam[M], lmg[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const int j = j0 + r;
            const bool in = j < N;
            lam[r] = in ? C[C_LAM * N1 + j] : 1.0;
            lmg[r] = in ? C[C_LMG * N1 + j] : 0.0;
        }
        float dch[M];                             // previous update (steers the next one only)
#pragma unroll
        for (int r = 0; r < M; ++r) dch[r] = 0.0f;
        // One sweep over the pairs from the current rho, v_p = T_p^{-1} [r_p -
        // (Lam - G + mu^2 L + mu B) rho]: accumulates sum_p omega_p v_p into acc,
        // or (final) writes E*_p = rho + v_p of the final iterate.
        auto sweep = [&](double (&acc)[M], bool final_sweep) {
            double rnext[M];
#pragma unroll
            for (int r = 0; r < M; ++r) {
                acc[r] = 0.0;
                rnext[r] = Rt[j0 + r];              // right-hand side of pair 0
            }
            for (int p = 0; p < P; ++p) {
                const double m1 = mu[p], m2 = m1 * m1, wp = om[p];
                double rcur[M];
#pragma unroll
                for (int r = 0; r < M; ++r) {       // this pair's right-hand side; fetch the next one
                    rcur[r] = rnext[r];
                    if (p + 1 < P) rnext[r] = Rt[(size_t)(p + 1) * NP + j0 + r];
                }
                double b[M], y[M], v[M];
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const int j = j0 + r;
                    const int t = r * W + k;
                    if (j < N) {
                        const double ll = sLl[t], lu = sLu[t];
                        const double bdj = (j == 0 ? bd0 : 0.0) + (j == N - 1 ? bdN : 0.0);
                        b[r] = lam[r] + m2 * (-(ll + lu)) + m1 * bdj;
                        const double rj = rho[t];
                        double rl = rj, rn = rj;   // boundary rows: ll or lu is 0
                        if (j > 0) rl = (r > 0) ? rho[t - W] : rho[(M - 1) * W + k - 1];
                        if (j < N - 1) rn = (r < M - 1) ? rho[t + W] : rho[k + 1];
                        const double q = ll * (rl - rj) + lu * (rn - rj);   // difference form (low rounding floor)
                        y[r] = rcur[r] - lmg[r] * rj - m2 * q - m1 * bdj * rj;
                    } else {
                        b[r] = 1.0;
                        y[r] = 0.0;
                    }
                }
                tri_factor_solve<W, M>(m2, sLl, sLu, b, y, v, sh, ph);
                if (final_sweep) {
                    double *ep = Et + (size_t)p * NP;
#pragma unroll
                    for (int r = 0; r < M; ++r) ep[j0 + r] = rho[r * W + k] + v[r];
                } else {
#pragma unroll
                    for (int r = 0; r < M; ++r) acc[r] += wp * v[r];
                }
            }
        };
        while (true) {
            double acc[M];
            sweep(acc, false);
            // res = sum_p omega_p v_p - (1 - W) rho;  rho += res + D^{-1} (G res).
            // Every operator is factored and solved in one call (one barrier); the
            // diffusion operator is factored again each iteration rather than held
            // in registers across the pair loop (one factorisation per P solves).
            double rl[M], d[M], f[M];
            {
                double b[M];
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const int j = j0 + r;
                    const bool in = j < N;
                    rl[r] = in ? acc[r] - I.one_minus_W * rho[r * W + k] : 0.0;
                    const int t = r * W + k;
                    const double bdj = (j == 0 ? bd0 : 0.0) + (j == N - 1 ? bdN : 0.0);
                    d[r] = in ? (lam[r] - lmg[r]) * rl[r] : 0.0;                 // G res
                    b[r] = in ? lmg[r] + I.mu2 * (-(sLl[t] + sLu[t])) + I.mu1 * bdj : 1.0;
                }
                tri_factor_solve<W, M>(I.mu2, sLl, sLu, b, d, f, sh, ph);
            }
            double alpha, beta;
            cheb_coeffs(Cs, A.accel, A.tol, alpha, beta);
            double md = 0.0, mr = 0.0;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                if (j0 + r < N) {
                    const int t = r * W + k;
                    const double z = rl[r] + f[r];
                    const double upd = alpha * (double)dch[r] + beta * z;
                    dch[r] = (float)upd;
                    const double nw = rho[t] + upd;
                    rho[t] = nw;
                    md = fmax(md, fabs(z));
                    mr = fmax(mr, fabs(nw));
                }
            }
            tile_max2<W>(md, mr, sh);
            tsync<W>();                               // rho update visible to the tile
            ++it;
            const float qprev = Cs.q1, qprev2 = Cs.q2, qprev3 = Cs.q3;
            const float q = (float)(mr > 0.0 ? md / mr : md);
            cheb_record(Cs, q);
            converged = pred_stop(md, mr, q, qprev, qprev2, qprev3, it, A.tol);
            if (converged || it >= A.maxit) break;
        }
        {
            double acc[M];
            sweep(acc, true);                         // E* of the final iterate
        }
    }
    for (int j = k; j < N; j += W) rp[j] = rho[lpos(j)];   // next step's starting iterate
    tsync<W>();                                   // E* visible to the tile
    if (k == 0) {
        st[0] = it;
        st[1] = converged;
    }

    if (k == 0 && !converged) atomicOr(A.sticky, GRTE_ERRF_PRED_NOCONV);
}

template <int W, int M, bool F32, int LMW = 4 * M>
__device__ __forceinline__ void corr_solve(const BatchArgs &A, int i, double *sm)
{
    constexpr int NP = 64 * (W == BNT ? LMW : M);
    const BInst I = A.inst[i];
    const int N = I.N, P = I.P, N1 = N + 1;
    const int k = opaque(tile_lane<W>());   // opaque: per-thread addresses are formed per instance, not held across the queue loop
    const int j0 = k * M;
    const double *Tn = A.T + I.oT;
    BState<F32> S;
    S.P = I.P;
    S.N = I.N;
    S.ac = I.a * I.c;
    S.Tn = Tn;
    S.E = F32 ? nullptr : A.E + I.oE;
    S.O = F32 ? nullptr : A.O + I.oO;
    S.E32 = F32 ? A.E32 + I.oE : nullptr;
    S.O32 = F32 ? A.O32 + I.oO : nullptr;
    const double *mu = A.mu + I.oP;
    double *C = A.cells + I.oC;
    // Per-pair global arrays are pair-major in cell order: thread k's rows
    // j0 .. j0+M-1 are contiguous, so its loads and stores are wide and the
    // later per-cell phases read along cells.
    double *Rt = A.pairs + I.oR;                  // right-hand sides
    double *Et = Rt + (size_t)P * I.NPa;          // E* (prediction), then E^{n+1} (correction)
    constexpr bool WG = (W == BNT);
    constexpr int LM = WG ? LMW : M;
    auto lpos = [](int j) { return (j % LM) * 64 + j / LM; };
    double *sLl = sm + NP, *sLu = sm + 2 * NP, *sh = sm + 3 * NP;
    double *slam = WG ? sm + 3 * NP : nullptr;
    int ph = 0;
    for (int j = k; j < NP; j += W) {
        const int t = lpos(j);
        const bool in = j < N;
        sLl[t] = in ? C[C_LL * N1 + j] : 0.0;
        sLu[t] = in ? C[C_LU * N1 + j] : 0.0;
        if constexpr (WG) slam[t] = in ? C[C_LAM * N1 + j] : 1.0;
    }
    tsync<W>();
    const double cb0 = C[C_BD * N1 + 0], cbN = C[C_BD * N1 + N - 1];
    if constexpr (WG) {
        // wavefront w solves pairs w, w + 4, ... alone; E*, no longer needed, takes E^{n+1}
        const int w = threadIdx.x >> 6;
        auto load_r = [&](int p, double (&v)[LM]) {   // padding rows hold zeros
            const double *src = Rt + (size_t)p * NP + opaque(threadIdx.x & 63) * LM;
#pragma unroll
            for (int r = 0; r < LM; ++r) v[r] = src[r];
        };
        double rnext[LM];
        if (w < P) load_r(w, rnext);
        for (int p = w; p < P; p += 4) {
            const double m1 = mu[p], m2 = m1 * m1;
            double x[LM];
#pragma unroll
            for (int r = 0; r < LM; ++r) x[r] = rnext[r];
            if (p + 4 < P) load_r(p + 4, rnext);
            const int lq = opaque(threadIdx.x & 63), jq = lq * LM, rl1 = N - 1 - jq;
            const double *ll = sLl + lq, *lu = sLu + lq, *la = slam + lq;
            const double c0 = jq == 0 ? cb0 : 0.0;
            auto bdc = [&](int r) { return (r == 0 ? c0 : 0.0) + (r == rl1 ? cbN : 0.0); };
            lane_chunk_solve<LM>(
                [&](int r) { return m2 * ll[r * 64]; },
                [&](int r) { return la[r * 64] + m2 * (-(ll[r * 64] + lu[r * 64])) + m1 * bdc(r); },
                [&](int r) { return m2 * lu[r * 64]; }, x);
            double *ep = Et + (size_t)p * NP + jq;
#pragma unroll
            for (int r = 0; r < LM; ++r) ep[r] = x[r];
        }
    } else {
        double lam[M];
#pragma unroll
        for (int r = 0; r < M; ++r) lam[r] = (j0 + r < N) ? C[C_LAM * N1 + j0 + r] : 1.0;
        for (int p = 0; p < P; ++p) {
            const double m1 = mu[p], m2 = m1 * m1;
            const double *rp = Rt + (size_t)p * NP;
            double b[M], d[M], x[M];
#pragma unroll
            for (int r = 0; r < M; ++r) {
                const int j = j0 + r;
                const int t = r * W + k;
                if (j < N) {
                    const double bdj = (j == 0 ? cb0 : 0.0) + (j == N - 1 ? cbN : 0.0);
                    b[r] = lam[r] + m2 * (-(sLl[t] + sLu[t])) + m1 * bdj;
                    d[r] = rp[j];
                } else {
                    b[r] = 1.0;
                    d[r] = 0.0;
                }
            }
            tri_factor_solve<W, M>(m2, sLl, sLu, b, d, x, sh, ph);
            double *ep = Et + (size_t)p * NP;   // E*, no longer needed, takes E^{n+1}
#pragma unroll
            for (int r = 0; r < M; ++r) ep[j0 + r] = x[r];
        }
    }
    tsync<W>();

}

// binary64 state <-> binary32 storage of every instance (one block per
// instance): E32 = E - a c T^4, O32 = O (to32), or back; the binary32 arrays
// are pair-major (see BState)
__global__ void __launch_bounds__(256) batch_convert(const BInst *inst, const double *T, double *E, double *O,
                                                    float *E32, float *O32, int to32)
{
    const BInst I = inst[blockIdx.x];
    const int N = I.N, P = I.P;
    const int ne = N * P, no = (N + 1) * P;     // per instance: well below 2^31
    const double ac = I.a * I.c;
    // t runs over the binary64 (cell-major) index j P + p; the binary32 state is
    // pair-major, p N + j (cells) and p (N + 1) + i (nodes)
    for (int t = threadIdx.x; t < ne; t += blockDim.x) {
        const int j = t / P, p = t - j * P;
        const double tj = T[I.oT + j];
        const double base = ac * (tj * tj) * (tj * tj);
        const size_t q = I.oE + (size_t)p * N + j;
        if (to32) E32[q] = (float)(E[I.oE + t] - base);
        else E[I.oE + t] = base + (double)E32[q];
    }
    for (int t = threadIdx.x; t < no; t += blockDim.x) {
        const int i = t / P, p = t - i * P;
        const size_t q = I.oO + (size_t)p * (N + 1) + i;
        if (to32) O32[q] = (float)O[I.oO + t];
        else O[I.oO + t] = (double)O32[q];
    }
}


// The step's kernels, in stream order (one graph per state-buffer parity):
//   batch_reset, cells_kernel<CP_PRED>, solve_kernel<0>, cells_kernel<CP_NEWTON>,
//   cells_kernel<CP_CORR>, solve_kernel<1>, cells_kernel<CP_PROJECT>, batch_energy.
enum { CP_PRED = 0, CP_NEWTON = 1, CP_CORR = 2, CP_PROJECT = 3 };
constexpr int CB = 128;   // cells per block of the per-cell kernels (a multiple of 64, at most 512)

template <int PH, bool F32>
__global__ void __launch_bounds__(CB) cells_kernel(BatchArgs A)
{
    const int2 cb = A.cblk[blockIdx.x];          // (instance, first cell)
    const IView<F32> V = iview<F32>(A, cb.x);
    const int j = cb.y + (int)threadIdx.x;
    const bool in = j < V.N;
    if constexpr (PH == CP_PRED) {
        if (in) cell_pred_setup(V, j);
    } else if constexpr (PH == CP_CORR) {
        if (in) cell_corr_setup(V, j);
    } else if constexpr (PH == CP_NEWTON) {
        int n_its = 0, n_fail = 0, n_clamp = 0, n_neg = 0;
        if (in) cell_newton(A, V, j, n_its, n_fail, n_clamp, n_neg);
        // one atomic per wavefront for the step counters
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            n_its = max(n_its, __shfl_xor(n_its, o, 64));
            n_fail += __shfl_xor(n_fail, o, 64);
            n_clamp += __shfl_xor(n_clamp, o, 64);
            n_neg += __shfl_xor(n_neg, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            int *st = V.st;
            atomicMax(&st[2], n_its);
            if (n_fail) atomicAdd(&st[3], n_fail);
            if (n_clamp) atomicAdd(&st[4], n_clamp);
            if (n_neg) atomicAdd(&st[5], n_neg);
            const int ef = (n_fail ? GRTE_ERRF_NEWTON : 0) | (n_neg ? GRTE_ERRF_NEGATIVE_ROOT : 0);
            if (ef) atomicOr(A.sticky, ef);
        }
    } else {
        __shared__ double s_red[16];
        double eb = 0.0, ea = 0.0;
        if (in) cell_project(A, V, j, eb, ea);
        // the block's sums (fixed order: a butterfly per wavefront, then the
        // wavefronts in order); batch_energy adds the slab's blocks in order
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            eb += __shfl_xor(eb, o, 64);
            ea += __shfl_xor(ea, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            s_red[threadIdx.x >> 6] = eb;
            s_red[8 + (threadIdx.x >> 6)] = ea;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            eb = s_red[0];
            ea = s_red[8];
#pragma unroll
            for (int q = 1; q < CB / 64; ++q) {
                eb += s_red[q];
                ea += s_red[8 + q];
            }
            A.epart[2 * blockIdx.x] = eb;
            A.epart[2 * blockIdx.x + 1] = ea;
        }
    }
}
static_assert(CB % 64 == 0 && CB <= 512, "per-cell blocks: whole wavefronts, at most eight");

// the two per-slab solves: work-group tiles first (largest work first), then
// wavefront tiles; PH 0: the prediction, 1: the correction
template <int PH, bool F32>
__global__ void __launch_bounds__(BNT) solve_kernel(BatchArgs A)
{
    extern __shared__ double smem[];
    __shared__ int s_q;
    int *queue = A.queue + 2 * PH;
    while (true) {
        if (threadIdx.x == 0) s_q = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int q = __builtin_amdgcn_readfirstlane(s_q);   // uniform: instance data in SGPRs
        __syncthreads();
        if (q >= A.n_wg) break;
        const int i = A.order[q];
        if constexpr (PH == 0) {
            switch (A.inst[i].M) {   // rows per lane
            case 4: pred_solve<BNT, 1, F32, 4>(A, i, smem); break;
            case 6: pred_solve<BNT, 1, F32, 6>(A, i, smem); break;
            case 8: pred_solve<BNT, 2, F32, 8>(A, i, smem); break;
            case 10: pred_solve<BNT, 1, F32, 10>(A, i, smem); break;
            case 12: pred_solve<BNT, 3, F32, 12>(A, i, smem); break;
            case 14: pred_solve<BNT, 1, F32, 14>(A, i, smem); break;
            case 16: pred_solve<BNT, 4, F32, 16>(A, i, smem); break;
            case 18: pred_solve<BNT, 1, F32, 18>(A, i, smem); break;
            case 20: pred_solve<BNT, 5, F32, 20>(A, i, smem); break;
            case 22: pred_solve<BNT, 1, F32, 22>(A, i, smem); break;
            case 24: pred_solve<BNT, 6, F32, 24>(A, i, smem); break;
            case 26: pred_solve<BNT, 1, F32, 26>(A, i, smem); break;
            case 28: pred_solve<BNT, 7, F32, 28>(A, i, smem); break;
            case 30: pred_solve<BNT, 1, F32, 30>(A, i, smem); break;
            case 32: pred_solve<BNT, 8, F32, 32>(A, i, smem); break;
            }
        } else {
            switch (A.inst[i].M) {
            case 4: corr_solve<BNT, 1, F32, 4>(A, i, smem); break;
            case 6: corr_solve<BNT, 1, F32, 6>(A, i, smem); break;
            case 8: corr_solve<BNT, 2, F32, 8>(A, i, smem); break;
            case 10: corr_solve<BNT, 1, F32, 10>(A, i, smem); break;
            case 12: corr_solve<BNT, 3, F32, 12>(A, i, smem); break;
            case 14: corr_solve<BNT, 1, F32, 14>(A, i, smem); break;
            case 16: corr_solve<BNT, 4, F32, 16>(A, i, smem); break;
            case 18: corr_solve<BNT, 1, F32, 18>(A, i, smem); break;
            case 20: corr_solve<BNT, 5, F32, 20>(A, i, smem); break;
            case 22: corr_solve<BNT, 1, F32, 22>(A, i, smem); break;
            case 24: corr_solve<BNT, 6, F32, 24>(A, i, smem); break;
            case 26: corr_solve<BNT, 1, F32, 26>(A, i, smem); break;
            case 28: corr_solve<BNT, 7, F32, 28>(A, i, smem); break;
            case 30: corr_solve<BNT, 1, F32, 30>(A, i, smem); break;
            case 32: corr_solve<BNT, 8, F32, 32>(A, i, smem); break;
            }
        }
    }
    double *wsm = smem + (threadIdx.x >> 6) * LDS_WAVE;
    while (true) {
        int q = 0;
        if ((threadIdx.x & 63) == 0) q = atomicAdd(&queue[1], 1);
        q = __builtin_amdgcn_readfirstlane(q);
        if (q >= A.n_wave) break;
        const int i = A.order[A.n_wg + q];
        if constexpr (PH == 0) {
            if (A.inst[i].M == 2) pred_solve<WAVE, 2, F32>(A, i, wsm);
            else pred_solve<WAVE, 4, F32>(A, i, wsm);
        } else {
            if (A.inst[i].M == 2) corr_solve<WAVE, 2, F32>(A, i, wsm);
            else corr_solve<WAVE, 4, F32>(A, i, wsm);
        }
    }
}

// the energy balance of every slab: its blocks' partial sums in block order,
// the outflow of the prediction's fluxes over the step, the defect
__global__ void __launch_bounds__(256) batch_energy(BatchArgs A)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n_inst) return;
    const BInst I = A.inst[i];
    double eb = 0.0, ea = 0.0;
    for (int q = 0; q < I.ncb; ++q) {
        eb += A.epart[2 * (I.cb0 + q)];
        ea += A.epart[2 * (I.cb0 + q) + 1];
    }
    const double *C = A.cells + I.oC;
    const int N1 = I.N + 1;
    const double fdt = I.dt * (C[C_FLUX * N1 + 1] - C[C_FLUX * N1]);
    double *en = A.ienergy + 4 * (size_t)i;
    en[0] = eb;
    en[1] = ea;
    en[2] = fdt;
    en[3] = (ea - eb) + fdt;
}

// queue heads and per-instance counters cleared by a kernel (not a memset node)
__global__ void batch_reset(int *queue, int *istat, int n8)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 4) queue[t] = 0;
    if (t < n8) istat[t] = 0;
}

// one int cleared (the sticky error flags)
__global__ void iclear1(int *x)
{
    if (threadIdx.x == 0) x[0] = 0;
}

__global__ void bfill(double *x, size_t n, double v)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

int pow2_rows(int N, int W)
{
    int M = 2;
    while (W * M < N) M *= 2;
    return M;
}

// rows per lane of a slab's tile (the tile holds 64 x that many rows): a
// wavefront tile takes 2 or 4 (powers of two), a work-group tile the smallest
// even LM = 4 .. 32 that holds the slab -- the padding rows cost as much as
// real ones, and with 256-row steps 12 % of the solves' rows were padding on
// slabs of N ~ U{64..2048}
int tile_rows(int N, int W)
{
    if (W != BNT) return pow2_rows(N, W);
    int LM = 4;
    while (64 * LM < N) LM += 2;
    return LM;
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct grte_batch {
    int n = 0, dev = 0, ncu = 0;
    int wave_max_n = 256, grid = 0, tuned = 0;
    double tol = 1e-15;
    int maxit = 200, newton_maxit = 100;
    int accel = GRTE_ACCEL_CHEBYSHEV;
    long long tot_cells = 0, tot_E = 0, tot_O = 0, tot_pairs = 0;
    std::vector<BInst> h_inst;
    std::vector<int> h_order;
    std::vector<double> cost;                  // expected work per instance (scheduling)
    int n_wg = 0, n_wave = 0;
    hipStream_t stream = nullptr;
    std::vector<void *> allocs;
    BInst *d_inst = nullptr;
    int *d_order = nullptr, *d_queue = nullptr, *d_istat = nullptr;
    int2 *d_cblk = nullptr;                    // blocks of the per-cell kernels
    double *d_epart = nullptr;                 // their energy partial sums (2 per block)
    int n_cblk = 0;
    double *E[2] = {nullptr, nullptr}, *O[2] = {nullptr, nullptr}, *T[2] = {nullptr, nullptr};
    int cur = 0;                               // state buffers in use: E[cur], O[cur], T[cur]
    // binary32 storage (f32 != 0): the state is E32[cur], O32[cur] with T[cur];
    // E[cur], O[cur] then only stage set_state / get_state
    float *E32[2] = {nullptr, nullptr}, *O32[2] = {nullptr, nullptr};
    int f32 = 0;
    double *sigma0 = nullptr, *mu = nullptr, *omega = nullptr, *bL = nullptr, *bR = nullptr;
    double *cells = nullptr, *pairs = nullptr;
    long long pairs_doubles = 0;               // size of the pair scratch
    double *rprev = nullptr;                   // per cell: the last prediction's rho*
    double *d_energy = nullptr;                // per instance: energy balance of the last step (4)
    int *d_sticky = nullptr;                   // error flags OR-ed over steps (GRTE_ERRF_*)
    int warm = 0;                              // rprev belongs to the step that produced the state
    // graphs, one per buffer parity; rebuilt when the launch changes
    int use_graph = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;
    // timing
    int profiling = 0;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
};

namespace {

grte_status bhip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GRTE_OK;
    fprintf(stderr, "grte_batch: %s failed: %s\n", what, hipGetErrorString(e));
    return GRTE_E_HIP;
}

#define BCHK(x)                                                 \
    do {                                                        \
        grte_status _s = bhip((x), #x);                         \
        if (_s != GRTE_OK) return _s;                           \
    } while (0)

template <class Tp>
grte_status balloc(grte_batch *b, Tp **p, size_t n)
{
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(Tp)) != hipSuccess) return GRTE_E_NOMEM;
    b->allocs.push_back(q);
    *p = (Tp *)q;
    return GRTE_OK;
}

void drop_graphs(grte_batch *b)
{
    for (int q = 0; q < 2; ++q) {
        if (b->gexec[q]) (void)hipGraphExecDestroy(b->gexec[q]);
        b->gexec[q] = nullptr;
    }
}

// tiles for the current wave_max_n; processing order: largest expected work first
grte_status assign_tiles(grte_batch *b)
{
    std::vector<int> wg, wv;
    for (int i = 0; i < b->n; ++i) {
        BInst &I = b->h_inst[i];
        if (I.N <= b->wave_max_n && I.N <= WAVE_MAX_N) {
            I.W = WAVE;
            wv.push_back(i);
        } else {
            I.W = BNT;
            wg.push_back(i);
        }
        I.M = tile_rows(I.N, I.W);
    }
    auto by_cost = [&](int x, int y) { return b->cost[x] > b->cost[y] || (b->cost[x] == b->cost[y] && x < y); };
    std::sort(wg.begin(), wg.end(), by_cost);
    std::sort(wv.begin(), wv.end(), by_cost);
    b->h_order = wg;
    b->h_order.insert(b->h_order.end(), wv.begin(), wv.end());
    b->n_wg = (int)wg.size();
    b->n_wave = (int)wv.size();
    // The work-group tiles read the padding rows (N..NP-1) of every pair of the
    // pair scratch as decoupled rows with a zero right-hand side; no step writes
    // them, but a slab run by a wavefront tile uses a smaller pair stride whose
    // rows fall into another layout's padding.  The scratch is cleared whenever
    // the tiles are (re)assigned (never inside a captured step).
    BCHK(hipMemsetAsync(b->pairs, 0, (size_t)b->pairs_doubles * sizeof(double), b->stream));
    BCHK(hipMemcpyAsync(b->d_inst, b->h_inst.data(), b->n * sizeof(BInst), hipMemcpyHostToDevice, b->stream));
    BCHK(hipMemcpyAsync(b->d_order, b->h_order.data(), b->n * sizeof(int), hipMemcpyHostToDevice, b->stream));
    BCHK(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    return GRTE_OK;
}

BatchArgs make_args(const grte_batch *b, int src)
{
    BatchArgs A{};
    A.n_wg = b->n_wg;
    A.n_wave = b->n_wave;
    A.inst = b->d_inst;
    A.order = b->d_order;
    A.queue = b->d_queue;
    A.cblk = b->d_cblk;
    A.epart = b->d_epart;
    A.n_inst = b->n;
    A.E = b->E[src]; A.O = b->O[src]; A.T = b->T[src];
    A.E2 = b->E[1 - src]; A.O2 = b->O[1 - src]; A.T2 = b->T[1 - src];
    A.sigma0 = b->sigma0; A.mu = b->mu; A.omega = b->omega; A.bL = b->bL; A.bR = b->bR;
    A.cells = b->cells; A.pairs = b->pairs; A.istat = b->d_istat;
    A.tol = b->tol; A.maxit = b->maxit; A.newton_maxit = b->newton_maxit; A.accel = b->accel;
    A.f32 = b->f32;
    A.rprev = b->rprev;
    A.warm = b->warm;
    A.E32 = b->E32[src]; A.O32 = b->O32[src];
    A.E32o = b->E32[1 - src]; A.O32o = b->O32[1 - src];
    A.ienergy = b->d_energy;
    A.sticky = b->d_sticky;
    return A;
}

constexpr size_t BATCH_LDS = (size_t)LDS_WG * sizeof(double);

// kev: if given, an event pair recorded around the prediction-solve kernel
grte_status enqueue_step(grte_batch *b, hipStream_t s, int src, const hipEvent_t *kev = nullptr)
{
    BatchArgs A = make_args(b, src);
    const int n8 = 8 * b->n;
    hipLaunchKernelGGL(batch_reset, dim3((unsigned)((std::max(n8, 4) + 255) / 256)), dim3(256), 0, s,
                       b->d_queue, b->d_istat, n8);
    BCHK(hipGetLastError());
    const dim3 cg((unsigned)b->n_cblk), sg((unsigned)b->grid), eg((unsigned)((b->n + 255) / 256));
    if (b->f32) {
        hipLaunchKernelGGL((cells_kernel<CP_PRED, true>), cg, dim3(CB), 0, s, A);
        if (kev) BCHK(hipEventRecord(kev[0], s));
        hipLaunchKernelGGL((solve_kernel<0, true>), sg, dim3(BNT), BATCH_LDS, s, A);
        if (kev) BCHK(hipEventRecord(kev[1], s));
        hipLaunchKernelGGL((cells_kernel<CP_NEWTON, true>), cg, dim3(CB), 0, s, A);
        hipLaunchKernelGGL((cells_kernel<CP_CORR, true>), cg, dim3(CB), 0, s, A);
        hipLaunchKernelGGL((solve_kernel<1, true>), sg, dim3(BNT), BATCH_LDS, s, A);
        hipLaunchKernelGGL((cells_kernel<CP_PROJECT, true>), cg, dim3(CB), 0, s, A);
    } else {
        hipLaunchKernelGGL((cells_kernel<CP_PRED, false>), cg, dim3(CB), 0, s, A);
        if (kev) BCHK(hipEventRecord(kev[0], s));
        hipLaunchKernelGGL((solve_kernel<0, false>), sg, dim3(BNT), BATCH_LDS, s, A);
        if (kev) BCHK(hipEventRecord(kev[1], s));
        hipLaunchKernelGGL((cells_kernel<CP_NEWTON, false>), cg, dim3(CB), 0, s, A);
        hipLaunchKernelGGL((cells_kernel<CP_CORR, false>), cg, dim3(CB), 0, s, A);
        hipLaunchKernelGGL((solve_kernel<1, false>), sg, dim3(BNT), BATCH_LDS, s, A);
        hipLaunchKernelGGL((cells_kernel<CP_PROJECT, false>), cg, dim3(CB), 0, s, A);
    }
    BCHK(hipGetLastError());
    hipLaunchKernelGGL(batch_energy, eg, dim3(256), 0, s, A);
    BCHK(hipGetLastError());
    return GRTE_OK;
}

grte_status capture(grte_batch *b, int src)
{
    if (!b->cap_stream) BCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    BCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    grte_status st = enqueue_step(b, b->cap_stream, src);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st != GRTE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    BCHK(e);
    e = hipGraphInstantiate(&b->gexec[src], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BCHK(e);
    return GRTE_OK;
}

// one step from buffers `src` into 1 - src, as a graph replay or a direct launch
grte_status run_step(grte_batch *b, int src)
{
    if (b->use_graph) {
        if (!b->gexec[src]) {
            grte_status st = capture(b, src);
            if (st != GRTE_OK) return st;
        }
        BCHK(hipGraphLaunch(b->gexec[src], b->stream));
        return GRTE_OK;
    }
    return enqueue_step(b, b->stream, src);
}

grte_status read_stats(grte_batch *b, std::vector<int> &h)
{
    h.resize((size_t)8 * b->n);
    BCHK(hipMemcpyAsync(h.data(), b->d_istat, h.size() * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BCHK(hipStreamSynchronize(b->stream));
    return GRTE_OK;
}

// expected work of each instance from the iteration counts of a step
void update_cost(grte_batch *b, const std::vector<int> &h)
{
    for (int i = 0; i < b->n; ++i) {
        const BInst &I = b->h_inst[i];
        b->cost[i] = (double)I.N * I.P * std::max(1, h[8 * i]);
    }
}

grte_status copy_dev(grte_batch *b, void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    BCHK(hipMemcpyAsync(dst, src, bytes, kind, b->stream));
    if (kind != hipMemcpyDeviceToDevice) BCHK(hipStreamSynchronize(b->stream));
    return GRTE_OK;
}

}  // namespace

extern "C" {

grte_status grte_batch_destroy(grte_batch *b)
{
    if (!b) return GRTE_OK;
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    for (void *p : b->allocs) (void)hipFree(p);
    delete b;
    return GRTE_OK;
}

grte_status grte_batch_create(int n, const grte_instance *inst, const double *mu, const double *omega,
                              grte_batch **out)
{
    if (!out) return GRTE_E_INVAL;
    *out = nullptr;
    if (n < 1 || !inst || !mu || !omega) return GRTE_E_INVAL;
    long long tp = 0;
    for (int i = 0; i < n; ++i) {
        const grte_instance &d = inst[i];
        if (d.nx < 2 || d.npairs < 1 || !(d.length > 0) || !(d.a > 0) || !(d.c > 0) || !(d.cv > 0) ||
            (d.opacity_law != 0 && d.opacity_law != 3) || !(d.dt > 0) || !(d.eps > 0) ||
            !std::isfinite(d.dt) || !std::isfinite(d.eps) || !std::isfinite(d.length))
            return GRTE_E_INVAL;
        if (d.nx > BMAX_N || d.npairs > BMAX_P) return GRTE_E_UNSUPPORTED;
        tp += d.npairs;
    }
    for (long long q = 0; q < tp; ++q)
        if (!(mu[q] > 0) || !(omega[q] > 0) || !std::isfinite(mu[q]) || !std::isfinite(omega[q]))
            return GRTE_E_INVAL;
    grte_batch *b = new (std::nothrow) grte_batch();
    if (!b) return GRTE_E_NOMEM;
    b->n = n;
    if (hipGetDevice(&b->dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->dev) != hipSuccess) {
        delete b;
        return GRTE_E_HIP;
    }
    b->h_inst.resize(n);
    b->cost.resize(n);
    long long oE = 0, oO = 0, oT = 0, oP = 0, oC = 0, oR = 0;
    for (int i = 0; i < n; ++i) {
        const grte_instance &d = inst[i];
        BInst &I = b->h_inst[i];
        I.N = d.nx; I.P = d.npairs; I.m = d.opacity_law;
        I.dx = d.length / d.nx; I.a = d.a; I.c = d.c; I.cv = d.cv; I.eps = d.eps; I.dt = d.dt;
        // 1 - sum(omega) exactly rounded (two-sum), first and second moments
        double s = 0.0, e = 0.0, m1 = 0.0, m2 = 0.0;
        for (int p = 0; p < I.P; ++p) {
            const double x = omega[oP + p];
            const double t = s + x;
            const double bp = t - s;
            e += (s - (t - bp)) + (x - bp);
            s = t;
            m1 += omega[oP + p] * mu[oP + p];
            m2 += omega[oP + p] * mu[oP + p] * mu[oP + p];
        }
        I.one_minus_W = (1.0 - s) - e;
        I.mu1 = m1;
        I.mu2 = m2;
        I.oE = oE; I.oO = oO; I.oT = oT; I.oP = oP; I.oC = oC; I.oR = oR;
        I.NPa = 64LL * tile_rows(I.N, BNT);   // also covers every wavefront tile (N <= 256)
        oE += (long long)I.N * I.P;
        oO += (long long)(I.N + 1) * I.P;
        oT += I.N;
        oP += I.P;
        oC += (long long)NCA * (I.N + 1);
        oR += 2LL * I.P * I.NPa;
        b->cost[i] = (double)I.N * I.P;
    }
    b->tot_E = oE; b->tot_O = oO; b->tot_cells = oT; b->tot_pairs = oP;
    // blocks of the per-cell kernels: 256 consecutive cells of one instance each,
    // the instances' blocks contiguous and in instance order
    std::vector<int2> cblk;
    for (int i = 0; i < n; ++i) {
        BInst &I = b->h_inst[i];
        I.cb0 = (int)cblk.size();
        for (int c0 = 0; c0 < I.N; c0 += CB) cblk.push_back(make_int2(i, c0));
        I.ncb = (int)cblk.size() - I.cb0;
    }
    b->n_cblk = (int)cblk.size();
    grte_status st = GRTE_OK;
    if (st == GRTE_OK) st = balloc(b, &b->d_cblk, cblk.size());
    if (st == GRTE_OK) st = balloc(b, &b->d_epart, 2 * cblk.size());
    if (st == GRTE_OK &&
        hipMemcpy(b->d_cblk, cblk.data(), cblk.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        st = GRTE_E_HIP;
    if (st == GRTE_OK) st = balloc(b, &b->d_inst, n);
    if (st == GRTE_OK) st = balloc(b, &b->d_order, n);
    if (st == GRTE_OK) st = balloc(b, &b->d_queue, 4);
    if (st == GRTE_OK) st = balloc(b, &b->d_istat, (size_t)8 * n);
    for (int q = 0; q < 2 && st == GRTE_OK; ++q) {
        st = balloc(b, &b->E[q], oE);
        if (st == GRTE_OK) st = balloc(b, &b->O[q], oO);
        if (st == GRTE_OK) st = balloc(b, &b->T[q], oT);
    }
    if (st == GRTE_OK) st = balloc(b, &b->sigma0, oT);
    if (st == GRTE_OK) st = balloc(b, &b->mu, oP);
    if (st == GRTE_OK) st = balloc(b, &b->omega, oP);
    if (st == GRTE_OK) st = balloc(b, &b->bL, oP);
    if (st == GRTE_OK) st = balloc(b, &b->bR, oP);
    if (st == GRTE_OK) st = balloc(b, &b->cells, oC);
    if (st == GRTE_OK) st = balloc(b, &b->pairs, oR);
    b->pairs_doubles = oR;
    if (st == GRTE_OK) st = balloc(b, &b->rprev, oT);
    if (st == GRTE_OK) st = balloc(b, &b->d_energy, (size_t)4 * n);
    if (st == GRTE_OK) st = balloc(b, &b->d_sticky, 1);
    if (st == GRTE_OK && (hipMemset(b->d_sticky, 0, sizeof(int)) != hipSuccess ||
                          hipMemset(b->d_energy, 0, (size_t)4 * n * sizeof(double)) != hipSuccess))
        st = GRTE_E_HIP;
    if (st != GRTE_OK) { grte_batch_destroy(b); return st; }
    const void *solvers[] = {(const void *)solve_kernel<0, false>, (const void *)solve_kernel<1, false>,
                             (const void *)solve_kernel<0, true>, (const void *)solve_kernel<1, true>};
    int nbmin = 1 << 30;
    for (const void *f : solvers) {
        int nb = 0;
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BATCH_LDS) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, BNT, BATCH_LDS) != hipSuccess || nb < 1) {
            grte_batch_destroy(b);
            return GRTE_E_HIP;
        }
        nbmin = std::min(nbmin, nb);
    }
    b->grid = nbmin * b->ncu;
    if (hipMemcpy(b->mu, mu, oP * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->omega, omega, oP * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        grte_batch_destroy(b);
        return GRTE_E_HIP;
    }
    // defaults: zero state and inflow, unit opacity
    const unsigned t = 256;
    auto fill = [&](double *x, long long cnt, double v) {
        hipLaunchKernelGGL(bfill, dim3((unsigned)((cnt + t - 1) / t)), dim3(t), 0, nullptr, x, (size_t)cnt, v);
    };
    fill(b->E[0], oE, 0.0);
    fill(b->O[0], oO, 0.0);
    fill(b->T[0], oT, 0.0);
    fill(b->sigma0, oT, 1.0);
    fill(b->bL, oP, 0.0);
    fill(b->bR, oP, 0.0);
    if (hipDeviceSynchronize() != hipSuccess || assign_tiles(b) != GRTE_OK) {
        grte_batch_destroy(b);
        return GRTE_E_HIP;
    }
    *out = b;
    return GRTE_OK;
}

grte_status grte_batch_sizes(const grte_batch *b, long long *cells, long long *e_len, long long *o_len,
                             long long *pairs)
{
    if (!b) return GRTE_E_INVAL;
    if (cells) *cells = b->tot_cells;
    if (e_len) *e_len = b->tot_E;
    if (o_len) *o_len = b->tot_O;
    if (pairs) *pairs = b->tot_pairs;
    return GRTE_OK;
}

grte_status grte_batch_set_stream(grte_batch *b, void *hip_stream)
{
    if (!b) return GRTE_E_INVAL;
    b->stream = (hipStream_t)hip_stream;
    return GRTE_OK;
}

grte_status grte_batch_set_solver(grte_batch *b, double pred_tol, int pred_maxit, int newton_maxit)
{
    if (!b || !(pred_tol > 0) || pred_maxit < 1 || newton_maxit < 1) return GRTE_E_INVAL;
    b->tol = pred_tol;
    b->maxit = pred_maxit;
    b->newton_maxit = newton_maxit;
    drop_graphs(b);
    return GRTE_OK;
}

grte_status grte_batch_set_acceleration(grte_batch *b, int mode)
{
    if (!b || (mode != GRTE_ACCEL_RICHARDSON && mode != GRTE_ACCEL_CHEBYSHEV)) return GRTE_E_INVAL;
    b->accel = mode;
    drop_graphs(b);
    return GRTE_OK;
}

grte_status grte_batch_set_opacity(grte_batch *b, const double *sigma0, int on_device)
{
    if (!b || !sigma0) return GRTE_E_INVAL;
    if (!on_device)
        for (long long j = 0; j < b->tot_cells; ++j)
            if (!(sigma0[j] >= 0) || !std::isfinite(sigma0[j])) return GRTE_E_INVAL;
    return copy_dev(b, b->sigma0, sigma0, b->tot_cells * sizeof(double),
                    on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
}

grte_status grte_batch_set_inflow(grte_batch *b, const double *b_left, const double *b_right)
{
    if (!b || !b_left || !b_right) return GRTE_E_INVAL;
    grte_status s = copy_dev(b, b->bL, b_left, b->tot_pairs * sizeof(double), hipMemcpyHostToDevice);
    if (s != GRTE_OK) return s;
    return copy_dev(b, b->bR, b_right, b->tot_pairs * sizeof(double), hipMemcpyHostToDevice);
}

namespace {
grte_status convert_state(grte_batch *b, int to32)
{
    hipLaunchKernelGGL(batch_convert, dim3((unsigned)b->n), dim3(256), 0, b->stream, b->d_inst, b->T[b->cur],
                       b->E[b->cur], b->O[b->cur], b->E32[b->cur], b->O32[b->cur], to32);
    BCHK(hipGetLastError());
    return GRTE_OK;
}
}  // namespace

grte_status grte_batch_set_storage(grte_batch *b, int fp32)
{
    if (!b || (fp32 != 0 && fp32 != 1)) return GRTE_E_INVAL;
    if (fp32 == b->f32) return GRTE_OK;
    if (fp32 && !b->E32[0]) {
        for (int q = 0; q < 2; ++q) {
            void *pe = nullptr, *po = nullptr;
            if (hipMalloc(&pe, std::max<long long>(b->tot_E, 1) * sizeof(float)) != hipSuccess) return GRTE_E_NOMEM;
            b->allocs.push_back(pe);
            if (hipMalloc(&po, std::max<long long>(b->tot_O, 1) * sizeof(float)) != hipSuccess) return GRTE_E_NOMEM;
            b->allocs.push_back(po);
            b->E32[q] = (float *)pe;
            b->O32[q] = (float *)po;
        }
    }
    grte_status s = convert_state(b, fp32);
    if (s != GRTE_OK) return s;
    BCHK(hipStreamSynchronize(b->stream));
    b->f32 = fp32;
    b->warm = 0;
    drop_graphs(b);
    return GRTE_OK;
}

grte_status grte_batch_set_state(grte_batch *b, const double *E, const double *O, const double *T, int on_device)
{
    if (!b || !E || !O || !T) return GRTE_E_INVAL;
    if (!on_device)
        for (long long j = 0; j < b->tot_cells; ++j)
            if (!(T[j] >= 0) || !std::isfinite(T[j])) return GRTE_E_INVAL;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (b->warm) {           // the next prediction starts from rho^n again
        b->warm = 0;
        drop_graphs(b);
    }
    grte_status s = copy_dev(b, b->E[b->cur], E, b->tot_E * sizeof(double), k);
    if (s == GRTE_OK) s = copy_dev(b, b->O[b->cur], O, b->tot_O * sizeof(double), k);
    if (s == GRTE_OK) s = copy_dev(b, b->T[b->cur], T, b->tot_cells * sizeof(double), k);
    if (s == GRTE_OK && b->f32) s = convert_state(b, 1);
    return s;
}

grte_status grte_batch_get_state(grte_batch *b, double *E, double *O, double *T, int on_device)
{
    if (!b) return GRTE_E_INVAL;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    grte_status s = GRTE_OK;
    if (b->f32 && (E || O)) s = convert_state(b, 0);   // binary64 values of the stored state
    if (s == GRTE_OK && E) s = copy_dev(b, E, b->E[b->cur], b->tot_E * sizeof(double), k);
    if (s == GRTE_OK && O) s = copy_dev(b, O, b->O[b->cur], b->tot_O * sizeof(double), k);
    if (s == GRTE_OK && T) s = copy_dev(b, T, b->T[b->cur], b->tot_cells * sizeof(double), k);
    return s;
}

grte_status grte_batch_set_tuning(grte_batch *b, const grte_batch_tuning *t)
{
    if (!b || !t) return GRTE_E_INVAL;
    if (t->wave_max_n < 0 || t->grid < 1 || t->grid > 65535) return GRTE_E_INVAL;
    b->wave_max_n = t->wave_max_n;
    b->grid = t->grid;
    return assign_tiles(b);
}

grte_status grte_batch_get_tuning(const grte_batch *b, grte_batch_tuning *t)
{
    if (!b || !t) return GRTE_E_INVAL;
    t->wave_max_n = b->wave_max_n;
    t->grid = b->grid;
    t->step_ms = 0.0;
    return GRTE_OK;
}

grte_status grte_batch_use_graph(grte_batch *b, int on)
{
    if (!b) return GRTE_E_INVAL;
    b->use_graph = on ? 1 : 0;
    return GRTE_OK;
}

grte_status grte_batch_step(grte_batch *b, grte_batch_info *info)
{
    if (!b) return GRTE_E_INVAL;
    int k = -1;
    grte_status st;
    if (b->profiling) {
        // a profiled step runs its kernels as direct launches (an event pair
        // can then bracket the prediction-solve kernel): events 4k, 4k+3 around
        // the step, 4k+1, 4k+2 around that kernel
        while (b->ev_used * 4 + 4 > b->ev.size()) {
            hipEvent_t e;
            BCHK(hipEventCreate(&e));
            b->ev.push_back(e);
        }
        k = (int)b->ev_used++;
        BCHK(hipEventRecord(b->ev[4 * k], b->stream));
        st = enqueue_step(b, b->stream, b->cur, &b->ev[4 * k + 1]);
        if (st != GRTE_OK) return st;
        BCHK(hipEventRecord(b->ev[4 * k + 3], b->stream));
    } else {
        st = run_step(b, b->cur);
        if (st != GRTE_OK) return st;
    }
    b->cur = 1 - b->cur;
    if (!b->warm) {          // rprev now belongs to the current state; the launch changes
        b->warm = 1;
        drop_graphs(b);
    }
    if (!info) return GRTE_OK;
    std::vector<int> h;
    std::vector<double> en((size_t)4 * b->n);
    BCHK(hipMemcpyAsync(en.data(), b->d_energy, en.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if ((st = read_stats(b, h)) != GRTE_OK) return st;   // (synchronises the stream)
    int bad = 0;
    for (int i = 0; i < b->n; ++i) {
        grte_batch_info &f = info[i];
        f.energy_before = en[4 * i];
        f.energy_after = en[4 * i + 1];
        f.boundary_flux_dt = en[4 * i + 2];
        f.energy_defect = en[4 * i + 3];
        f.pred_iters = h[8 * i + 0];
        f.pred_converged = h[8 * i + 1] ? 1 : 0;
        f.pred_floor_stop = h[8 * i + 1] == 2 ? 1 : 0;
        f.newton_max_iters = h[8 * i + 2];
        f.newton_failed = h[8 * i + 3];
        f.kstar_clamped = h[8 * i + 4];
        f.negative_root = h[8 * i + 5];
        if (!f.pred_converged || f.newton_failed) bad = 1;
    }
    return bad ? GRTE_E_NOCONV : GRTE_OK;
}

grte_status grte_batch_get_error_flags(grte_batch *b, int *flags, int clear)
{
    if (!b || !flags) return GRTE_E_INVAL;
    BCHK(hipMemcpyAsync(flags, b->d_sticky, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BCHK(hipStreamSynchronize(b->stream));
    if (clear) {
        hipLaunchKernelGGL(iclear1, dim3(1), dim3(64), 0, b->stream, b->d_sticky);
        BCHK(hipGetLastError());
        BCHK(hipStreamSynchronize(b->stream));
    }
    return GRTE_OK;
}

grte_status grte_batch_tune(grte_batch *b, int trials, grte_batch_tuning *best)
{
    if (!b || trials < 1) return GRTE_E_INVAL;
    // every candidate step starts from the current state and writes the other
    // buffers, so the state is left unchanged
    const int save_graph = b->use_graph;
    b->use_graph = 0;
    // every candidate step also starts its prediction from the same iterate: the
    // warm start (the previous step's rho*) is saved and put back before each,
    // else all but the first would start from the answer of this very step
    double *rsave = nullptr;
    if (b->warm) {
        if (hipMalloc((void **)&rsave, std::max<long long>(b->tot_cells, 1) * sizeof(double)) != hipSuccess) {
            b->use_graph = save_graph;
            return GRTE_E_NOMEM;
        }
        if (hipMemcpyAsync(rsave, b->rprev, b->tot_cells * sizeof(double), hipMemcpyDeviceToDevice, b->stream) !=
            hipSuccess) {
            (void)hipFree(rsave);
            b->use_graph = save_graph;
            return GRTE_E_HIP;
        }
    }
    auto restore = [&]() -> grte_status {
        if (rsave && hipMemcpyAsync(b->rprev, rsave, b->tot_cells * sizeof(double), hipMemcpyDeviceToDevice,
                                    b->stream) != hipSuccess)
            return GRTE_E_HIP;
        return GRTE_OK;
    };
    std::vector<int> h;
    grte_status st = assign_tiles(b);
    if (st == GRTE_OK) st = restore();
    if (st == GRTE_OK) st = enqueue_step(b, b->stream, b->cur);
    if (st == GRTE_OK) st = read_stats(b, h);
    if (st != GRTE_OK) {
        if (rsave) (void)hipFree(rsave);
        b->use_graph = save_graph;
        return st;
    }
    update_cost(b, h);
    int nb = 0;
    const void *kfn = b->f32 ? (const void *)solve_kernel<0, true> : (const void *)solve_kernel<0, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kfn, BNT, BATCH_LDS) != hipSuccess) nb = 1;
    const int waves[] = {0, 128, 256};
    std::vector<int> grids;
    for (int f = 1; f <= std::max(1, nb); f *= 2) grids.push_back(f * b->ncu);
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    double best_ms = 1e300;
    int bw = b->wave_max_n, bg = b->grid;
    for (int wv : waves) {
        for (int g : grids) {
            b->wave_max_n = wv;
            b->grid = g;
            if ((st = assign_tiles(b)) != GRTE_OK) break;
            if ((st = restore()) != GRTE_OK) break;
            if ((st = enqueue_step(b, b->stream, b->cur)) != GRTE_OK) break;   // warm-up
            if ((st = restore()) != GRTE_OK) break;
            if (hipEventRecord(e0, b->stream) != hipSuccess) { st = GRTE_E_HIP; break; }
            for (int r = 0; r < trials && st == GRTE_OK; ++r) {
                if (r > 0) st = restore();
                if (st == GRTE_OK) st = enqueue_step(b, b->stream, b->cur);
            }
            if (st != GRTE_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = GRTE_E_HIP;
                break;
            }
            const double per = ms / trials;
            if (per < best_ms) {
                best_ms = per;
                bw = wv;
                bg = g;
            }
        }
        if (st != GRTE_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == GRTE_OK) st = restore();   // the next step starts as it would have without tuning
    if (rsave) {
        if (hipStreamSynchronize(b->stream) != hipSuccess && st == GRTE_OK) st = GRTE_E_HIP;
        (void)hipFree(rsave);
    }
    b->use_graph = save_graph;
    if (st != GRTE_OK) return st;
    b->wave_max_n = bw;
    b->grid = bg;
    b->tuned = 1;
    if ((st = assign_tiles(b)) != GRTE_OK) return st;
    if (best) {
        best->wave_max_n = bw;
        best->grid = bg;
        best->step_ms = best_ms;
    }
    return GRTE_OK;
}

grte_status grte_batch_set_profiling(grte_batch *b, int on)
{
    if (!b) return GRTE_E_INVAL;
    b->profiling = on ? 1 : 0;
    b->ev_used = 0;
    return GRTE_OK;
}

grte_status grte_batch_read_timing(grte_batch *b, double *total_ms, int *count)
{
    if (!b || !total_ms || !count) return GRTE_E_INVAL;
    double solve_ms = 0.0;
    return grte_batch_read_timing2(b, total_ms, &solve_ms, count);
}

grte_status grte_batch_read_timing2(grte_batch *b, double *step_ms, double *solve_ms, int *count)
{
    if (!b || !step_ms || !solve_ms || !count) return GRTE_E_INVAL;
    *step_ms = 0.0;
    *solve_ms = 0.0;
    *count = 0;
    BCHK(hipStreamSynchronize(b->stream));
    for (size_t k = 0; k < b->ev_used; ++k) {
        float ms = 0.0f, ks = 0.0f;
        BCHK(hipEventElapsedTime(&ms, b->ev[4 * k], b->ev[4 * k + 3]));
        BCHK(hipEventElapsedTime(&ks, b->ev[4 * k + 1], b->ev[4 * k + 2]));
        *step_ms += ms;
        *solve_ms += ks;
        *count += 1;
    }
    b->ev_used = 0;
    return GRTE_OK;
}

}  // extern "C"
