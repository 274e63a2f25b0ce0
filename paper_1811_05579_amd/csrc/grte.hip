// grte.hip -- MI355X (gfx950) implementation of the AP step of Tang, Wang &
// Zhang (arXiv 1811.05579) for the 1-D gray radiative transfer equation, and
// the C ABI declared in include/grte.h.
//
// Formulation (exact algebra of Section 4/5, arranged for the GPU)
// ----------------------------------------------------------------
// Every equation is multiplied by eps^2 c dt.  The node equation (4.5a)/(5.2a)
// gives O at interior nodes explicitly in E:
//     O_i = Aw_i O^n_i - Bc_i mu (E_i - E_{i-1}),
//     Aw_i = K_i eps^2 / den_i,  Bc_i = K_i c dt / (dx den_i),
//     den_i = K_i eps^2 + sigma_i c dt,
// and the inflow relations (4.6) give the two boundary nodes.  Substituting in
// the cell equation (4.5b)/(5.2b) leaves, for every parity pair p, a
// tridiagonal system in the cell values
//     T_p E_p - G rho = r_p ,    T_p = Lam + mu_p^2 L + mu_p B ,
// where Lam = K eps^2 + sigma0 c dt (diagonal), L is a p-independent
// tridiagonal diffusion operator (face weights h_j Bc_i, h_j = K_j eps^2 c dt/dx,
// doubled at the two boundary faces), B is diagonal with 2 h/eps in the two
// boundary cells, and G = sigma0 c dt ac beta/(1 + ac beta) is the material
// coupling left after U* is eliminated with (4.5c).
//
// Prediction (hot loop).  With W = sum_p omega_p (not exactly one in binary64)
// the angular moment rho = sum_p omega_p E_p satisfies
//     S rho = s ,  S x = (1 - W) x + sum_p omega_p T_p^{-1} [(Lam - G) x + mu_p^2 L x + mu_p B x],
// where Lam - G = K eps^2 + sigma0 c dt/(1 + ac beta) is formed directly, so
// the small isotropic coefficient of optically thick cells carries no
// cancellation.  The update is preconditioned with the diffusion operator
// D = (Lam - G) + <mu^2> L + <mu> B (a consistent diffusion-synthetic
// acceleration):
//     res = s - S rho^k = sum_p omega_p T_p^{-1}[r_p - (T_p - G) rho^k] - (1 - W) rho^k,
//     z^k = res + D^{-1}(G res),
// applied as rho^{k+1} = rho^k + z^k (plain) or through an adaptive Chebyshev
// recurrence (solver_common.hpp), starting from the previous step's rho* when
// the state is the one that step produced; E*_p = rho + T_p^{-1}[r_p - (T_p - G) rho]
// from a final sweep of the converged iterate.
// One cooperative kernel runs the whole iteration: one work-group per
// parity pair solves its tridiagonal system in registers/LDS, a grid barrier
// separates the angular reduction, and every work-group then performs the
// (cheap, N-sized) DSA solve redundantly so that all groups hold the same
// iterate and take the same convergence decision.
//
// Correction substep 1: D_j from O* (text after (4.13)), K* = max(U*,0)^{3/4}
// for sigma/T^3, and the scalar equation (4.13)/(5.5) multiplied by
// c sigma0 dt^2:  a c sigma0 dt T^4 + Cv (eps^2 K* + c sigma0 dt)(T - T^n)
//                 - sigma0 dt (rho^n - c dt D) = 0,  Newton from T^n.
// Correction substep 2 + projection: with E = ac U^{n+1} + eps E_J and
// O = O_J, (4.11a,b) + (4.12) and the inflow relations are the same operator
// T_p (with K^{n+1}) without angular coupling, so E^{n+1} solves one
// tridiagonal system per pair and O^{n+1} follows from the node relation.
//
// Tridiagonal systems are solved inside one work-group by a partitioned
// method: each thread owns M consecutive rows, eliminates its interior rows
// (Thomas), the chunk-boundary rows form a tridiagonal system of size NT that
// every wavefront solves redundantly (published once in LDS; parallel cyclic
// reduction across the lanes), and each thread back-substitutes.  All systems are M-matrices (diagonally
// dominant), so no pivoting is needed.  All reductions have a fixed order:
// results are bitwise reproducible.

#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/grte.h"

#include "solver_common.hpp"
#include "mlp_common.hpp"

namespace {

// Several contexts (independent slabs of the same tile shape) can be advanced
// by one launch of each kernel: blockIdx.y selects the context of the
// per-cell and per-pair kernels, and the cooperative prediction kernel maps
// its work-groups to contexts through `first` (one work-group per pair of
// every context, each context synchronising only its own work-groups).
constexpr int GMAX = 4;
constexpr int NSTAT = 16;    // per-step counters of a context
constexpr int STAT_STICKY = NSTAT - 1;   // error flags OR-ed over steps (GRTE_ERRF_*), cleared on request

template <class Args>
struct Group {
    int n;
    int first[GMAX + 1];    // prediction: first work-group of each context
    Args a[GMAX];
};

// -------------------------------------------------------------------------
// coefficients: one work-group per group of cells, all pairs of those cells
// -------------------------------------------------------------------------
struct CoefArgs {
    int N, P, m, mode, cpb;      // mode 0: prediction (K from T^n), 1: correction (K from T^{n+1})
    double a, c, cv, eps, dt, dx;
    const double *T;             // temperature defining K (T^n or T^{n+1})
    const double *Tn;            // T^n (U^n and beta)
    const double *sigma0, *mu, *omega, *bL, *bR;
    const double *E, *O;         // E^n, O^n, cell-major (binary64 storage)
    const float *E32, *O32;      // binary32 storage: E^n = a c (T^n)^4 + E32, O^n = O32
    int f32;
    double mu1, mu2;             // sum omega mu, sum omega mu^2 (diffusion operator)
    double *Ll, *Lu, *Lam, *LmG, *Gt, *Bd, *Aw, *Bc, *beta;   // Gt: position order (row_pos)
    int M;                       // rows per thread of the prediction kernel (for Gt)
    double *Dl, *Dd, *Du;        // diffusion operator (prediction only)
    double *rho_n;               // sum_p omega_p E^n_p (prediction only)
    double *r;                   // right-hand sides, pair-major position order [p*NT*M + row_pos(j)]
    int *stat;                   // cleared by the prediction pass
};

__device__ __forceinline__ void node_coef(const CoefArgs &A, int i, double &aw, double &bc)
{
    // interior node i (1..N-1) between cells i-1 and i
    const double Kn = 0.5 * (kpow(A.T[i - 1], A.m) + kpow(A.T[i], A.m));
    const double sl = A.sigma0[i - 1], sr = A.sigma0[i];
    const double ss = sl + sr;
    const double sn = ss > 0.0 ? 2.0 * sl * sr / ss : 0.0;      // harmonic mean
    const double den = Kn * A.eps * A.eps + sn * A.c * A.dt;
    if (den > 0.0) {
        aw = Kn * A.eps * A.eps / den;
        bc = Kn * A.c * A.dt / (A.dx * den);
    } else {
        aw = 0.0;
        bc = 0.0;
    }
}

__device__ __forceinline__ void coef_body(const CoefArgs &A)
{
    __shared__ double s_h[256], s_awr[256], s_awl[256], s_src[256], s_keps[256], s_w[256];
    const int N = A.N, P = A.P, cpb = A.cpb;
    const int c0 = blockIdx.x * cpb;
    const int t = threadIdx.x;
    if (A.mode == 0 && blockIdx.x == 0 && t < STAT_STICKY) A.stat[t] = 0;   // the sticky word survives
    // ---- per cell
    if (t < cpb && c0 + t < N) {
        const int j = c0 + t;
        const double eps = A.eps, c = A.c, dt = A.dt;
        double awl = 0.0, bcl = 0.0, awr = 0.0, bcr = 0.0;
        if (j >= 1) node_coef(A, j, awl, bcl);
        if (j <= N - 2) node_coef(A, j + 1, awr, bcr);
        A.Aw[j] = awl;
        A.Bc[j] = bcl;
        if (j == N - 1) {
            A.Aw[N] = 0.0;
            A.Bc[N] = 0.0;
        }
        const double Kc = kpow(A.T[j], A.m);
        const double s0 = A.sigma0[j];
        const double h = Kc * eps * eps * c * dt / A.dx;
        const double fr = (j <= N - 2) ? h * bcr * (j == 0 ? 2.0 : 1.0) : 0.0;
        const double fl = (j >= 1) ? h * bcl * (j == N - 1 ? 2.0 : 1.0) : 0.0;
        const double bd = (j == 0 || j == N - 1) ? 2.0 * h / eps : 0.0;
        const double lam = Kc * eps * eps + s0 * c * dt;
        A.Ll[j] = -fl;
        A.Lu[j] = -fr;
        A.Bd[j] = bd;
        A.Lam[j] = lam;
        const double ac = A.a * c;
        double src;
        if (A.mode == 0) {
            const double Tn = A.Tn[j];
            const double Un = Tn * Tn * Tn * Tn;
            // (4.5c): beta = 4 sigma0 dt (T^n)^(3-m) / (eps^2 Cv)
            const double t3m = (A.m == 0) ? Tn * Tn * Tn : 1.0;
            const double beta = 4.0 * s0 * dt * t3m / (eps * eps * A.cv);
            const double opb = 1.0 + ac * beta;
            const double lmg = Kc * eps * eps + s0 * c * dt / opb;
            A.beta[j] = beta;
            A.LmG[j] = lmg;
            A.Gt[(j % A.M) * NT + j / A.M] = s0 * c * dt * (ac * beta) / opb;
            A.Dl[j] = A.mu2 * (-fl);
            A.Du[j] = A.mu2 * (-fr);
            A.Dd[j] = lmg + A.mu2 * (fl + fr) + A.mu1 * bd;
            src = s0 * c * dt * ac * Un / opb;
        } else {
            const double T1 = A.T[j];
            src = s0 * c * dt * ac * (T1 * T1 * T1 * T1);
        }
        s_h[t] = h;
        s_awr[t] = (j <= N - 2) ? awr * (j == 0 ? 2.0 : 1.0) : 0.0;
        s_awl[t] = (j >= 1) ? awl * (j == N - 1 ? 2.0 : 1.0) : 0.0;
        s_src[t] = src;
        s_keps[t] = Kc * eps * eps;
    }
    __syncthreads();
    // ---- per (cell, pair): right-hand sides of the per-pair systems
    const int cl = t / P, p = t - (t / P) * P;
    const int j = c0 + cl;
    if (cl < cpb && j < N) {
        const double mu = A.mu[p];
        const double h = s_h[cl];
        double On_r = 0.0, On_l = 0.0, En;
        if (A.f32) {
            if (j <= N - 2) On_r = (double)A.O32[(size_t)(j + 1) * P + p];
            if (j >= 1) On_l = (double)A.O32[(size_t)j * P + p];
            const double tn = A.Tn[j];
            En = A.a * A.c * (tn * tn) * (tn * tn) + (double)A.E32[(size_t)j * P + p];
        } else {
            if (j <= N - 2) On_r = A.O[(size_t)(j + 1) * P + p];
            if (j >= 1) On_l = A.O[(size_t)j * P + p];
            En = A.E[(size_t)j * P + p];
        }
        double rv = s_keps[cl] * En + s_src[cl] - h * mu * (s_awr[cl] * On_r - s_awl[cl] * On_l);
        if (j == 0) rv += 2.0 * h * mu * A.bL[p] / A.eps;
        if (j == N - 1) rv += 2.0 * h * mu * A.bR[p] / A.eps;
        A.r[(size_t)p * NT * A.M + (j % A.M) * NT + j / A.M] = rv;   // pair-major, position order
        if (A.mode == 0) s_w[t] = A.omega[p] * En;
    }
    if (A.mode == 0) {
        __syncthreads();
        if (t < cpb && c0 + t < N) {
            double rho = 0.0;
            for (int q = 0; q < P; ++q) rho += s_w[t * P + q];
            A.rho_n[c0 + t] = rho;
        }
    }
}

__global__ void __launch_bounds__(256) coef_kernel(Group<CoefArgs> G)
{
    const CoefArgs A = G.a[blockIdx.y];
    coef_body(A);
}

// -------------------------------------------------------------------------
// prediction: cooperative DSA-preconditioned iteration (plain or Chebyshev updates)
// -------------------------------------------------------------------------
// Row j of a system is owned by thread k = j / M as its row r = j % M.  Every
// per-row array the iteration touches is kept in "position" order
// t = r * NT + k, so that consecutive threads touch consecutive words (no LDS
// bank conflicts, coalesced global traffic).
struct PredArgs {
    int N, P, maxit;
    int accel;                         // 0 Richardson, 1 adaptive Chebyshev (see cheb_coeffs)
    double tol, one_minus_W, mu2avg;   // mu2avg = sum_p omega_p mu_p^2 (diffusion operator)
    const double *Ll, *Lu, *Lam, *LmG, *Bd, *Dd;   // cell order; diffusion off-diagonals are mu2avg * L
    const double *Gt;                  // G in position order (padded entries zero)
    const double *r, *mu, *omega, *rho0;
    double *part;                      // omega_p v_p, pair-major, position order [p*NP + t]
    double *res;                       // position order
    double *estar;                     // E* of the final iterate, cell-major [j*P + p]
    double *rho_out;                   // cell order
    int *stat;                         // [0] iterations, [1] converged, [6] barrier error
    double *hist;                      // max|z| / max|rho| of each update (first HIST_CAP)
    unsigned long long *flags;
    unsigned long long gen0;
};

constexpr int HIST_CAP = GRTE_HIST_CAP;

// One sweep of a pair from the iterate rho (position order, LDS):
// v = T_p^{-1} [r_p - (Lam - G + mu^2 L + mu B) rho] for this thread's rows.
template <int M>
__device__ __forceinline__ void pred_sweep(const double *rho, const double *sLl, const double *sLu,
                                           const double (&rr)[M], const double (&lmg)[M], double mu, double mu2,
                                           double bd0, double bdN, int N, const TriFac<NT, M> &Ft, double (&v)[M],
                                           double *sh, int &ph)
{
    const int k = threadIdx.x, j0 = k * M;
    double y[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int j = j0 + r;
        if (j < N) {
            const int t = r * NT + k;
            const double rj = rho[t];
            double rl = rj, rn = rj;   // boundary rows have no coupling (ll or lu is 0)
            if (j > 0) rl = (r > 0) ? rho[t - NT] : rho[(M - 1) * NT + k - 1];
            if (j < N - 1) rn = (r < M - 1) ? rho[t + NT] : rho[k + 1];
            const double ll = sLl[t], lu = sLu[t];
            // L rho from neighbour differences: near convergence the products
            // ll rho_j and ll rho_{j-1} nearly cancel, and the rounding of that
            // form sets a floor of ~1e-14 on the relative update; the
            // differences are formed almost exactly
            const double q = ll * (rl - rj) + lu * (rn - rj);
            const double bdj = (j == 0 ? bd0 : 0.0) + (j == N - 1 ? bdN : 0.0);
            y[r] = rr[r] - lmg[r] * rj - mu2 * q - mu * bdj * rj;
        } else {
            y[r] = 0.0;
        }
    }
    tri_solve<NT, M>(mu2, sLl, sLu, Ft, y, v, sh, ph);
}

template <int M>
__device__ __forceinline__ void pred_body(const PredArgs &A, const int bid, const int nblk)
{
    extern __shared__ double smem[];
    constexpr int NP = NT * M;           // padded rows
    // Everything an iteration reads besides the other work-groups' partial sums
    // stays in LDS or registers: the grid barrier's device-scope release and
    // acquire write back and invalidate the L2, so global data would be
    // fetched again from memory in every iteration.
    double *rho = smem;                  // current iterate (position order)
    double *sLl = smem + NP;             // operator coefficients (position order)
    double *sLu = smem + 2 * NP;
    double *sh = smem + 3 * NP;          // solver scratch (tile_scratch<NT>())
    double *redT = sh + tile_scratch<NT>();   // reduced systems of the two factorisations
    double *redD = redT + red_doubles();
    const int k = threadIdx.x;
    const int N = A.N, P = A.P;
    const int j0 = k * M;
    for (int j = k; j < NP; j += NT) {
        const bool in = j < N;
        const int t = row_pos(j, M);
        rho[t] = in ? A.rho0[j] : 0.0;
        sLl[t] = in ? A.Ll[j] : 0.0;
        sLu[t] = in ? A.Lu[j] : 0.0;
    }
    const double bd0 = A.Bd[0], bdN = A.Bd[N - 1];
    __syncthreads();
    const int p = bid;                   // one parity pair per work-group
    const double mu = A.mu[p], mu2 = mu * mu, wp = A.omega[p];

    TriFac<NT, M> Ft, Fd;
    double rr[M], gg[M], lmg[M];         // r_p, G and Lam - G of this thread's rows
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int j = j0 + r;
        rr[r] = A.r[(size_t)p * NP + r * NT + k];
        gg[r] = A.Gt[r * NT + k];
        lmg[r] = (j < N) ? A.LmG[j] : 0.0;
    }
    {
        double b[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const int j = j0 + r;
            if (j < N) {
                const double ll = sLl[r * NT + k], lu = sLu[r * NT + k];
                const double bdj = (j == 0 ? bd0 : 0.0) + (j == N - 1 ? bdN : 0.0);
                b[r] = A.Lam[j] + mu2 * (-(ll + lu)) + mu * bdj;
            } else {
                b[r] = 1.0;
            }
        }
        tri_factor<NT, M>(mu2, sLl, sLu, b, Ft, sh, redT);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const int j = j0 + r;
            b[r] = (j < N) ? A.Dd[j] : 1.0;
        }
        __syncthreads();   // the two factorisations share their LDS exchange area
        tri_factor<NT, M>(A.mu2avg, sLl, sLu, b, Fd, sh, redD);
    }

    // positions whose angular sum this work-group forms
    const int chunk = (NP + nblk - 1) / nblk;
    const int tb = bid * chunk;
    const int te = min(NP, tb + chunk);
    double *part_p = A.part + (size_t)p * NP;
    unsigned long long gen = A.gen0;
    int it = 0, converged = 0, ph = 0;
    ChebState C;
    // previous update of this thread's rows, kept in binary32: it only steers
    // the next update (the residual is formed from rho in full precision), and
    // near convergence it is below tol relative to rho
    float dch[M];
#pragma unroll
    for (int r = 0; r < M; ++r) dch[r] = 0.0f;
    while (true) {
        // ---- sweep: v_p = T_p^{-1} [r_p - (Lam - G + mu^2 L + mu B) rho]
        double v[M];
        pred_sweep<M>(rho, sLl, sLu, rr, lmg, mu, mu2, bd0, bdN, N, Ft, v, sh, ph);
#pragma unroll
        for (int r = 0; r < M; ++r) part_p[r * NT + k] = wp * v[r];   // padded rows give v = 0
        if (!grid_barrier(A.flags, ++gen, A.stat + 6, bid, nblk)) break;
        // ---- angular sum for my positions: res = sum_p omega_p v_p - (1 - W) rho.
        // Two adjacent lanes share a position, each summing half of the pairs
        // (half the dependent load round trips), combined in a fixed order.
        {
            const int h = k & 1, Ph = (P + 1) >> 1;
            const int q0 = h ? Ph : 0, q1 = h ? P : Ph;
            // lanes k and k^1 have the same position, so they iterate together
            for (int t = tb + (k >> 1); t < te; t += NT / 2) {
                double s = 0.0;
                int q = q0;
                for (; q + 8 <= q1; q += 8) {
                    double t8[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) t8[u] = A.part[(size_t)(q + u) * NP + t];
#pragma unroll
                    for (int u = 0; u < 8; ++u) s += t8[u];
                }
                for (; q < q1; ++q) s += A.part[(size_t)q * NP + t];
                const double other = __shfl_xor(s, 1);
                if (h == 0) A.res[t] = (s + other) - A.one_minus_W * rho[t];
            }
        }
        if (!grid_barrier(A.flags, ++gen, A.stat + 6, bid, nblk)) break;
        // ---- diffusion acceleration, identical in every work-group
        double rl[M], d[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const int t = r * NT + k;
            rl[r] = A.res[t];
            d[r] = gg[r] * rl[r];
        }
        tri_solve<NT, M>(A.mu2avg, sLl, sLu, Fd, d, f, sh, ph);
        double alpha, beta;
        cheb_coeffs(C, A.accel, A.tol, alpha, beta);
        double md = 0.0, mr = 0.0;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            if (j0 + r < N) {
                const int t = r * NT + k;
                const double z = rl[r] + f[r];
                const double upd = alpha * (double)dch[r] + beta * z;
                dch[r] = (float)upd;
                const double nw = rho[t] + upd;
                rho[t] = nw;
                md = fmax(md, fabs(z));
                mr = fmax(mr, fabs(nw));
            }
        }
        tile_max2<NT>(md, mr, sh);   // its barriers also publish the rho update
        ++it;
        if (bid == 0 && k == 0 && it <= HIST_CAP) A.hist[it - 1] = mr > 0.0 ? md / mr : md;
        const float qprev = C.q1, qprev2 = C.q2, qprev3 = C.q3;
        const float q = (float)(mr > 0.0 ? md / mr : md);
        cheb_record(C, q);
        converged = pred_stop(md, mr, q, qprev, qprev2, qprev3, it, A.tol);
        if (converged || it >= A.maxit) break;
    }
    {
        // E*_p = rho + T_p^{-1} [r_p - (T_p - G) rho] from the final iterate
        // (no grid barrier: each work-group sweeps its own pair once more)
        double v[M];
        pred_sweep<M>(rho, sLl, sLu, rr, lmg, mu, mu2, bd0, bdN, N, Ft, v, sh, ph);
#pragma unroll
        for (int r = 0; r < M; ++r)
            if (j0 + r < N) A.estar[(size_t)(j0 + r) * P + p] = rho[r * NT + k] + v[r];
    }
    if (bid == 0) {
        for (int j = k; j < N; j += NT) A.rho_out[j] = rho[row_pos(j, M)];
        if (k == 0) {
            A.stat[0] = it;
            A.stat[1] = converged;
        }
    }
}

template <int M>
__global__ void __launch_bounds__(NT) pred_kernel(Group<PredArgs> G)
{
    int g = 0;
    while (g + 1 < G.n && (int)blockIdx.x >= G.first[g + 1]) ++g;
    const PredArgs A = G.a[g];
    pred_body<M>(A, (int)blockIdx.x - G.first[g], G.first[g + 1] - G.first[g]);
}

// -------------------------------------------------------------------------
// correction substep 1: moments, D, K*, scalar Newton
// -------------------------------------------------------------------------
struct NewtonArgs {
    int N, P, m, maxit, keep, cpb;
    double a, c, cv, eps, dt, dx;
    const double *O, *Aw, *Bc, *beta, *rho_n, *Tn, *sigma0, *mu, *omega, *bL, *bR;
    double *Ecm;             // E* in cell-major order, as the prediction writes it
    double *Tnew, *ustar, *Dv, *ostar, *rstar;
    double *obnd;            // O* at the two end nodes, [p] (node 0) and [P + p] (node N)
    int moments_only;        // 1: rho*, U*, D and O* only, T^{n+1} = T^n (the alternative correction)
    const float *O32;        // binary32 storage of O^n (f32 != 0)
    int f32;
    const uint16_t *gw;      // learned initial guess: bfloat16 weights (null: Newton from T^n)
    const float *gnorm;      // and its normalisation
    double gtol;             // residual below which the guess is taken as the root
    int *stat;   // [2] max its, [3] failed, [4] K* clamped, [5] negative root,
                 // [7] guesses accepted, [8] guesses not used (Newton from T^n), [9] sum of Newton its,
                 // [10] Newton started from the guess
};

// Newton on g(T) = q4 T^4 + lin (T - Tn) - rhs from T0; false if the cap is hit.
template <bool GUESS>
__device__ __forceinline__ void newton_body(const NewtonArgs &A, const uint16_t *sW, const float *sN)
{
    __shared__ double s_w[256], s_f[256];
    const int N = A.N, P = A.P, cpb = A.cpb;
    const int c0 = blockIdx.x * cpb, t = threadIdx.x;
    const int cl = t / P, p = t - (t / P) * P;
    const int jj = c0 + cl;
    if (cl < cpb && jj < N) {
        const double mu = A.mu[p], w = A.omega[p];
        double ol, orr;
        if (A.f32) {
            ol = node_any(A.Ecm, A.O32, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, jj, p);
            orr = node_any(A.Ecm, A.O32, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, jj + 1, p);
        } else {
            ol = node_any(A.Ecm, A.O, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, jj, p);
            orr = node_any(A.Ecm, A.O, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, jj + 1, p);
        }
        s_w[t] = w * A.Ecm[(size_t)jj * P + p];
        s_f[t] = w * mu * (orr - ol);
        if (A.keep) {
            A.ostar[(size_t)jj * P + p] = ol;
            if (jj == N - 1) A.ostar[(size_t)N * P + p] = orr;
        }
        if (jj == 0) A.obnd[p] = ol;
        if (jj == N - 1) A.obnd[P + p] = orr;
    }
    __syncthreads();
    if (t >= cpb || c0 + t >= N) return;
    const int j = c0 + t;
    double rho = 0.0, D = 0.0;
    for (int q = 0; q < P; ++q) {
        rho += s_w[t * P + q];
        D += s_f[t * P + q];
    }
    D /= A.dx;
    const double ac = A.a * A.c;
    const double Tn = A.Tn[j];
    const double Un = Tn * Tn * Tn * Tn;
    const double beta = A.beta[j];
    const double us = (Un + beta * rho) / (1.0 + ac * beta);
    A.ustar[j] = us;
    A.Dv[j] = D;
    double Ks = 1.0;
    if (A.m == 3) {
        if (us < 0.0) {
            Ks = 0.0;
            atomicAdd(&A.stat[4], 1);
        } else {
            Ks = pow(us, 0.75);
        }
    }
    // (4.13) times c sigma0 dt^2:
    //   a c sigma0 dt T^4 + Cv (eps^2 K* + c sigma0 dt)(T - T^n) - sigma0 dt (rho^n - c dt D) = 0
    const double s0 = A.sigma0[j];
    const double lin = A.cv * (A.eps * A.eps * Ks + A.c * s0 * A.dt);
    const double q4 = ac * s0 * A.dt;
    const double rhs = s0 * A.dt * (A.rho_n[j] - A.c * A.dt * D);
    A.rstar[j] = rho;
    if (A.moments_only) {
        A.Tnew[j] = Tn;
        return;
    }
    double T = Tn;
    int its = 0;
    if (!(s0 == 0.0 && Ks == 0.0)) {
        if (Tn + rhs / lin < 0.0) atomicAdd(&A.stat[5], 1);   // no root >= 0
        bool ok = false, done = false;
        if (GUESS && s0 > 0.0 && Tn > 0.0) {
            // learned starting value; judged by the normalised residual of (4.13)
            float f[MLP_IN];
            mlp_features(rho, Tn, s0, A.m, A.eps, A.dt, f);
            const float y = mlp_eval(sW, sN, f);
            const double Tg = Tn * exp((double)sN[10] + (double)sN[11] * (double)y);
            if (isfinite(Tg) && Tg > 0.0) {
                // normalised residuals of the guess and of T^n
                const double T2 = Tg * Tg;
                const double rg = fabs(q4 * T2 * T2 + lin * (Tg - Tn) - rhs) / lin;
                const double Tn2 = Tn * Tn;
                const double rn = fabs(q4 * Tn2 * Tn2 - rhs) / lin;
                if (rg <= A.gtol * fmax(fabs(Tn + rhs / lin), 1e-300)) {
                    T = Tg;
                    ok = done = true;
                    atomicAdd(&A.stat[7], 1);
                } else if (rg < rn) {
                    ok = done = newton_quartic(Tg, Tn, q4, lin, rhs, A.maxit, T, its);
                    if (done) atomicAdd(&A.stat[10], 1);
                }
            }
            if (!done) atomicAdd(&A.stat[8], 1);
        }
        if (!done) ok = newton_quartic(Tn, Tn, q4, lin, rhs, A.maxit, T, its);   // plain: from T^n
        if (!ok) atomicAdd(&A.stat[3], 1);
    }
    A.Tnew[j] = T;
    atomicMax(&A.stat[2], its);
    atomicAdd(&A.stat[9], its);
}

// GUESS: some context of the launch carries a learned guess (its weights are
// staged in LDS); the plain kernel pays for none of it
template <bool GUESS>
__global__ void __launch_bounds__(256) newton_kernel(Group<NewtonArgs> G)
{
    const NewtonArgs A = G.a[blockIdx.y];
    if constexpr (GUESS) {
        __shared__ uint16_t sW[MLP_NPARAM + 3];
        __shared__ float sN[MLP_NNORM];
        if (A.gw) {
            for (int e = threadIdx.x; e < MLP_NPARAM; e += 256) sW[e] = A.gw[e];
            if (threadIdx.x < MLP_NNORM) sN[threadIdx.x] = A.gnorm[threadIdx.x];
            __syncthreads();
            newton_body<true>(A, sW, sN);
            return;
        }
    }
    newton_body<false>(A, nullptr, nullptr);
}

// training rows (f_0..f_4, log(T^{n+1}/T^n)) of the last step, binary32;
// cells without a defined input (sigma0 = 0 or T <= 0) give a zero row
__global__ void log_pairs_kernel(int N, int m, double eps, double dt, const double *rstar, const double *Told,
                                 const double *Tnew, const double *sigma0, float *out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const double t0 = Told[j], t1 = Tnew[j], s0 = sigma0[j];
    float f[MLP_IN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    float tg = 0.0f;
    if (s0 > 0.0 && t0 > 0.0 && t1 > 0.0) {
        mlp_features(rstar[j], t0, s0, m, eps, dt, f);
        tg = (float)log(t1 / t0);
    }
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) out[(size_t)j * 6 + q] = f[q];
    out[(size_t)j * 6 + 5] = tg;
}

// -------------------------------------------------------------------------
// correction substep 2: E^{n+1} per pair (one work-group per pair)
// -------------------------------------------------------------------------
struct CorrArgs {
    int N, P;
    const double *Ll, *Lu, *Lam, *Bd, *r, *mu;
    double *Enew;   // cell-major E^{n+1} (binary64)
    float *E32new;  // binary32 storage: E^{n+1} - a c (T^{n+1})^4 (f32 != 0)
    const double *Tnew;
    double ac;
    int f32;
};

template <int M>
__global__ void __launch_bounds__(NT) corr_kernel(Group<CorrArgs> G)
{
    extern __shared__ double smem[];
    constexpr int NP = NT * M;
    const CorrArgs A = G.a[blockIdx.y];
    double *sLl = smem, *sLu = smem + NP, *sh = smem + 2 * NP;
    const int p = blockIdx.x;
    if (p >= A.P) return;                // contexts of the group may have fewer pairs
    const int N = A.N, P = A.P, k = threadIdx.x;
    const int j0 = k * M;
    for (int j = k; j < NP; j += NT) {
        const int t = row_pos(j, M);
        sLl[t] = (j < N) ? A.Ll[j] : 0.0;
        sLu[t] = (j < N) ? A.Lu[j] : 0.0;
    }
    __syncthreads();
    const double mu = A.mu[p], mu2 = mu * mu;
    double b[M], d[M], x[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int j = j0 + r;
        if (j < N) {
            const double ll = sLl[r * NT + k], lu = sLu[r * NT + k];
            b[r] = A.Lam[j] + mu2 * (-(ll + lu)) + mu * A.Bd[j];
            d[r] = A.r[(size_t)p * NP + r * NT + k];
        } else {
            b[r] = 1.0;
            d[r] = 0.0;
        }
    }
    int ph = 0;
    tri_factor_solve<NT, M>(mu2, sLl, sLu, b, d, x, sh, ph);
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const int j = j0 + r;
        if (j < N) {
            A.Enew[(size_t)j * P + p] = x[r];
            if (A.f32) {
                const double t1 = A.Tnew[j];
                A.E32new[(size_t)j * P + p] = (float)(x[r] - A.ac * (t1 * t1) * (t1 * t1));
            }
        }
    }
}

// -------------------------------------------------------------------------
// projection (4.14): O^{n+1} at the nodes (E^{n+1} is already in place),
// rho^{n+1}, and the energy balance of the step ((3.12)-(3.13)):
//   E_tot = sum_j dx (rho_j / c + Cv T_j) before and after the step, the
//   outflow dt sum_p omega_p mu_p (O*_{N,p} - O*_{0,p}) of the prediction's
//   fluxes (the correction's moment equation uses D from O*), and the defect
//   E_tot^{n+1} - E_tot^n + outflow.
// Binary64 sums in a fixed order: a tree over each block's cells, per-block
// partials, and a one-block-per-context kernel that sums the partials by index.
// -------------------------------------------------------------------------
struct ProjArgs {
    int N, P, keep, cpb;
    double eps;
    const double *Enew, *O, *Aw, *Bc, *mu, *omega, *bL, *bR;
    double *Oout, *rho_out;
    const float *O32;       // binary32 storage (f32 != 0): O^n in, O^{n+1} out
    float *O32out;
    int f32;
    // energy balance
    double dx, c, cv, dt;
    const double *Tn, *Tnew, *rho_n, *obnd;
    double *epart;          // 2 per block
    double *energy;         // E_before, E_after, outflow dt, defect
    int *stat;              // per-step counters; the sticky word collects their error flags
};

// Energy balance, first level: the block's sum of e0 and e1 (fixed order, a
// tree in LDS) written to epart[2 b], epart[2 b + 1].  The sums over the
// blocks are formed by the next kernel on the stream (energy_final_kernel),
// whose launch makes every block's partials visible without a device-scope
// fence per block (on this chip such a fence writes back the XCD's L2).
__device__ void energy_partial(double e0, double e1, double *epart)
{
    __shared__ double s_e0[256], s_e1[256];
    const int t = threadIdx.x;
    s_e0[t] = e0;
    s_e1[t] = e1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            s_e0[t] += s_e0[t + o];
            s_e1[t] += s_e1[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        epart[2 * blockIdx.x] = s_e0[0];
        epart[2 * blockIdx.x + 1] = s_e1[0];
    }
}

// Second level: the nb partials of one context summed in a fixed order (each
// thread its strided share, then a tree), result in every thread's E0, E1.
__device__ void energy_total(const double *epart, int nb, double &E0, double &E1)
{
    __shared__ double s_e0[256], s_e1[256];
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0;
    for (int b = t; b < nb; b += 256) {
        a0 += epart[2 * b];
        a1 += epart[2 * b + 1];
    }
    s_e0[t] = a0;
    s_e1[t] = a1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            s_e0[t] += s_e0[t + o];
            s_e1[t] += s_e1[t + o];
        }
        __syncthreads();
    }
    E0 = s_e0[0];
    E1 = s_e1[0];
}

__global__ void __launch_bounds__(256) project_kernel(Group<ProjArgs> G)
{
    const ProjArgs A = G.a[blockIdx.y];
    __shared__ double s_w[256];
    const int N = A.N, P = A.P, cpb = A.cpb;
    const int nb = (N + cpb - 1) / cpb;
    if ((int)blockIdx.x >= nb) return;          // whole block: contexts of the group differ in size
    const int c0 = blockIdx.x * cpb, t = threadIdx.x;
    const int cl = t / P, p = t - (t / P) * P;
    const int j = c0 + cl;
    double wE = 0.0;
    if (cl < cpb && j < N) {
        const double mu = A.mu[p];
        if (A.f32) {
            A.O32out[(size_t)j * P + p] =
                (float)node_any(A.Enew, A.O32, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, j, p);
            if (j == N - 1)
                A.O32out[(size_t)N * P + p] =
                    (float)node_any(A.Enew, A.O32, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, N, p);
        } else {
            A.Oout[(size_t)j * P + p] = node_any(A.Enew, A.O, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, j, p);
            if (j == N - 1)
                A.Oout[(size_t)N * P + p] =
                    node_any(A.Enew, A.O, A.Aw, A.Bc, mu, A.bL[p], A.bR[p], A.eps, N, P, N, p);
        }
        wE = A.omega[p] * A.Enew[(size_t)j * P + p];
    }
    s_w[t] = wE;
    __syncthreads();
    double e0 = 0.0, e1 = 0.0;
    if (t < cpb && c0 + t < N) {
        const int jc = c0 + t;
        double s = 0.0;
        for (int q = 0; q < P; ++q) s += s_w[t * P + q];
        if (A.keep) A.rho_out[jc] = s;
        e0 = A.dx * (A.rho_n[jc] / A.c + A.cv * A.Tn[jc]);
        e1 = A.dx * (s / A.c + A.cv * A.Tnew[jc]);
    }
    energy_partial(e0, e1, A.epart);
}

// the energy balance of each context (one block per context) and the step's
// error flags, after project_kernel
__global__ void __launch_bounds__(256) energy_final_kernel(Group<ProjArgs> G)
{
    const ProjArgs A = G.a[blockIdx.x];
    const int nb = (A.N + A.cpb - 1) / A.cpb;
    double eb, ea;
    energy_total(A.epart, nb, eb, ea);
    if (threadIdx.x == 0) {
        const int P = A.P;
        double fl = 0.0;
        for (int q = 0; q < P; ++q) fl += A.omega[q] * A.mu[q] * (A.obnd[P + q] - A.obnd[q]);
        const double fdt = A.dt * fl;
        A.energy[0] = eb;
        A.energy[1] = ea;
        A.energy[2] = fdt;
        A.energy[3] = (ea - eb) + fdt;
        // error flags of this step, kept until read (the counters are cleared next step)
        int f = 0;
        if (A.stat[6]) f |= GRTE_ERRF_SYNC;
        if (!A.stat[1]) f |= GRTE_ERRF_PRED_NOCONV;
        if (A.stat[3]) f |= GRTE_ERRF_NEWTON;
        if (A.stat[5]) f |= GRTE_ERRF_NEGATIVE_ROOT;
        if (f) A.stat[STAT_STICKY] |= f;
    }
}

// -------------------------------------------------------------------------
// The alternative correction of the remark closing Section 3, (3.14): the time
// derivative taken from the prediction's update, the emission at U*, no
// nonlinear solve.  For the state a c U* + eps Jh its per-direction equations
// are (4.11a,b) with U^{n+1} -> U* and the time-derivative terms known:
//   nodes: K_i [(O*_i - O^n_i)/(c dt) + ac mu (U*_i - U*_{i-1})/(eps^2 dx)
//               + mu (E_J,i - E_J,i-1)/(eps dx)] = -sigma_i O_J,i / eps^2
//   cells: K_j [(E*_j - E^n_j)/(c dt) + mu (O_J,j+1 - O_J,j)/dx] = -sigma0_j E_J,j / eps
// with the inflow relations (4.6) for a c U* + eps E_J, K = (T^n)^m (the
// prediction's).  The node rows give O_J,i = alpha_i - mu beta_i (E_J,i - E_J,i-1),
// beta_i = K_i eps / (sigma_i dx), so each direction is tridiagonal in E_J (the
// operator form of the correction kernel: Lam = sigma0 c dt, face weights
// -h beta, doubled at the two ends, and 2h in the boundary cells, h = K eps c dt
// / dx; rows scaled by eps c dt).  Then (3.14b), T^{n+1} = T^n + dt sigma0
// rho_J / (eps K Cv), and the projection (4.14).  Needs sigma0 > 0.
// -------------------------------------------------------------------------
struct AltArgs {
    int N, P, m, cpb, M;
    double a, c, cv, eps, dt, dx;
    const double *Tn, *sigma0, *mu, *omega, *bL, *bR;
    const double *En, *On, *Es, *Os, *Us;   // E^n, O^n, E*, O* (cell-major), U*
    double *Ll, *Lu, *Lam, *Bd, *r;         // the per-direction operators and right-hand sides
    const double *EJ;                       // E_J, cell-major (projection)
    double *Enew, *Onew, *Tnew, *rho_out;
    const double *rho_n;
    double *epart, *energy;
    int *stat;
};

// node quantities of interior node i (1..N-1): K_i / sigma_i and K_i (the node
// opacity is the harmonic mean of the two cells', K the mean of theirs)
__device__ __forceinline__ void alt_node_coef(const AltArgs &A, int i, double &Ki, double &ksig)
{
    Ki = 0.5 * (kpow(A.Tn[i - 1], A.m) + kpow(A.Tn[i], A.m));
    const double sl = A.sigma0[i - 1], sr = A.sigma0[i];
    const double sn = 2.0 * sl * sr / (sl + sr);
    ksig = Ki / sn;
}

// alpha_i of interior node i for direction p
__device__ __forceinline__ double alt_alpha(const AltArgs &A, int i, int p, double Ki, double ksig)
{
    const int P = A.P;
    const double mu = A.mu[p];
    const double dO = A.Os[(size_t)i * P + p] - A.On[(size_t)i * P + p];
    const double dU = A.Us[i] - A.Us[i - 1];
    return -(ksig / (A.c * A.dt)) * (A.eps * A.eps * dO + A.a * A.c * mu * A.c * A.dt * dU / A.dx);
}

__global__ void __launch_bounds__(256) alt_coef_kernel(Group<AltArgs> G)
{
    const AltArgs A = G.a[blockIdx.y];
    __shared__ double s_h[256], s_bl[256], s_br[256], s_kl[256], s_kr[256], s_nl[256], s_nr[256], s_K[256];
    const int N = A.N, P = A.P, cpb = A.cpb;
    const int c0 = blockIdx.x * cpb, t = threadIdx.x;
    if (c0 >= N) return;
    if (t < cpb && c0 + t < N) {
        const int j = c0 + t;
        const double K = kpow(A.Tn[j], A.m);
        const double h = K * A.eps * A.c * A.dt / A.dx;
        double Kl = 0.0, kl = 0.0, Kr = 0.0, kr = 0.0;
        if (j >= 1) alt_node_coef(A, j, Kl, kl);
        if (j <= N - 2) alt_node_coef(A, j + 1, Kr, kr);
        const double bl = (j >= 1) ? kl * A.eps / A.dx : 0.0;      // beta at node j
        const double br = (j <= N - 2) ? kr * A.eps / A.dx : 0.0;  // beta at node j + 1
        A.Lam[j] = A.sigma0[j] * A.c * A.dt;
        A.Ll[j] = (j >= 1) ? -h * bl * (j == N - 1 ? 2.0 : 1.0) : 0.0;
        A.Lu[j] = (j <= N - 2) ? -h * br * (j == 0 ? 2.0 : 1.0) : 0.0;
        A.Bd[j] = (j == 0 || j == N - 1) ? 2.0 * h : 0.0;
        s_h[t] = h;
        s_K[t] = K;
        s_kl[t] = Kl;
        s_nl[t] = kl;
        s_kr[t] = Kr;
        s_nr[t] = kr;
        s_bl[t] = bl;
        s_br[t] = br;
    }
    __syncthreads();
    const int cl = t / P, p = t - (t / P) * P;
    const int j = c0 + cl;
    if (cl < cpb && j < N) {
        const double mu = A.mu[p], h = s_h[cl], eps = A.eps;
        double rv = -s_K[cl] * eps * (A.Es[(size_t)j * P + p] - A.En[(size_t)j * P + p]);
        const double al = (j >= 1) ? alt_alpha(A, j, p, s_kl[cl], s_nl[cl]) : 0.0;
        const double ar = (j <= N - 2) ? alt_alpha(A, j + 1, p, s_kr[cl], s_nr[cl]) : 0.0;
        if (j == 0) {
            rv += -2.0 * h * mu * ar + 2.0 * h * mu / eps * (A.bL[p] - A.a * A.c * A.Us[0]);
        } else if (j == N - 1) {
            rv += -2.0 * h * mu / eps * (A.a * A.c * A.Us[N - 1] - A.bR[p]) + 2.0 * h * mu * al;
        } else {
            rv += -h * mu * (ar - al);
        }
        A.r[(size_t)p * NT * A.M + (j % A.M) * NT + j / A.M] = rv;   // pair-major, position order
    }
}

// O_J at node i of direction p from E_J (interior: the node row; ends: the
// inflow relations for a c U* + eps E_J)
__device__ __forceinline__ double alt_oj(const AltArgs &A, int i, int p)
{
    const int N = A.N, P = A.P;
    const double mu = A.mu[p];
    auto inner = [&](int ii) {
        double Ki, ks;
        alt_node_coef(A, ii, Ki, ks);
        return alt_alpha(A, ii, p, Ki, ks) -
               mu * (ks * A.eps / A.dx) * (A.EJ[(size_t)ii * P + p] - A.EJ[(size_t)(ii - 1) * P + p]);
    };
    if (i >= 1 && i <= N - 1) return inner(i);
    const double ac = A.a * A.c;
    if (i == 0) return 2.0 / A.eps * (A.bL[p] - ac * A.Us[0] - A.eps * A.EJ[p]) - inner(1);
    return 2.0 / A.eps * (ac * A.Us[N - 1] + A.eps * A.EJ[(size_t)(N - 1) * P + p] - A.bR[p]) - inner(N - 1);
}

__global__ void __launch_bounds__(256) alt_project_kernel(Group<AltArgs> G)
{
    const AltArgs A = G.a[blockIdx.y];
    __shared__ double s_w[256], s_T[256];
    const int N = A.N, P = A.P, cpb = A.cpb;
    const int nb = (N + cpb - 1) / cpb;
    if ((int)blockIdx.x >= nb) return;
    const int c0 = blockIdx.x * cpb, t = threadIdx.x;
    const int cl = t / P, p = t - (t / P) * P;
    const int j = c0 + cl;
    const bool own = cl < cpb && j < N;
    double ej = 0.0;
    if (own) {
        ej = A.EJ[(size_t)j * P + p];
        A.Onew[(size_t)j * P + p] = alt_oj(A, j, p);
        if (j == N - 1) A.Onew[(size_t)N * P + p] = alt_oj(A, N, p);
    }
    s_w[t] = own ? A.omega[p] * ej : 0.0;
    __syncthreads();
    double e0 = 0.0, e1 = 0.0;
    if (t < cpb && c0 + t < N) {
        const int jc = c0 + t;
        double rj = 0.0;
        for (int q = 0; q < P; ++q) rj += s_w[t * P + q];
        // (3.14b): Cv (T^{n+1} - T^n)/dt = sigma rho_J, sigma = sigma0 / K, rho_J = rho(E_J) / eps
        const double tn = A.Tn[jc];
        const double T1 = tn + A.dt * A.sigma0[jc] * rj / (A.eps * kpow(tn, A.m) * A.cv);
        A.Tnew[jc] = T1;
        s_T[t] = T1;
        e0 = A.dx * (A.rho_n[jc] / A.c + A.cv * tn);
    }
    __syncthreads();
    if (own) {
        const double T1 = s_T[cl];
        const double e = A.a * A.c * ((T1 * T1) * (T1 * T1)) + A.eps * ej;
        A.Enew[(size_t)j * P + p] = e;
        s_w[t] = A.omega[p] * e;
    }
    __syncthreads();
    if (t < cpb && c0 + t < N) {
        double r1 = 0.0;
        for (int q = 0; q < P; ++q) r1 += s_w[t * P + q];
        A.rho_out[c0 + t] = r1;
        e1 = A.dx * (r1 / A.c + A.cv * s_T[t]);
    }
    energy_partial(e0, e1, A.epart);
}

// the energy balance of each context after alt_project_kernel (one block per context)
__global__ void __launch_bounds__(256) alt_energy_final_kernel(Group<AltArgs> G)
{
    const AltArgs A = G.a[blockIdx.x];
    const int N = A.N, P = A.P;
    const int nb = (N + A.cpb - 1) / A.cpb;
    double eb, ea;
    energy_total(A.epart, nb, eb, ea);
    if (threadIdx.x == 0) {
        // the outflow of the fluxes the alternative's moment equation uses: O_J
        // at the two end nodes (formed again here from the inputs)
        double fl = 0.0;
        for (int q = 0; q < P; ++q) fl += A.omega[q] * A.mu[q] * (alt_oj(A, N, q) - alt_oj(A, 0, q));
        const double fdt = A.dt * fl;
        A.energy[0] = eb;
        A.energy[1] = ea;
        A.energy[2] = fdt;
        A.energy[3] = (ea - eb) + fdt;
        int f = 0;
        if (A.stat[6]) f |= GRTE_ERRF_SYNC;
        if (!A.stat[1]) f |= GRTE_ERRF_PRED_NOCONV;
        if (f) A.stat[STAT_STICKY] |= f;
    }
}

// ---- iterative implicit reference (6.6): Picard update of the opacity temperature
// U* = (U^n + beta rho*)/(1 + ac beta), T^(k+1) = max(U*, 0)^(1/4); the largest
// change and the largest T^(k+1) (non-negative doubles: their bit patterns
// order like unsigned integers) are reduced with one atomic per work-group
__global__ void __launch_bounds__(256) picard_update_kernel(int N, double ac, const double *Tn, const double *beta,
                                                            const double *rho_star, const double *Tk, double *Tk1,
                                                            double *ustar, unsigned long long *dmax)
{
    __shared__ double s_d[256], s_t[256];
    const int j = blockIdx.x * 256 + threadIdx.x;
    double d = 0.0, tv = 0.0;
    if (j < N) {
        const double t = Tn[j];
        const double us = ((t * t) * (t * t) + beta[j] * rho_star[j]) / (1.0 + ac * beta[j]);
        const double t1 = pow(fmax(us, 0.0), 0.25);
        ustar[j] = us;
        Tk1[j] = t1;
        d = fabs(t1 - Tk[j]);
        tv = t1;
    }
    s_d[threadIdx.x] = d;
    s_t[threadIdx.x] = tv;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s_d[threadIdx.x] = fmax(s_d[threadIdx.x], s_d[threadIdx.x + o]);
            s_t[threadIdx.x] = fmax(s_t[threadIdx.x], s_t[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&dmax[0], (unsigned long long)__double_as_longlong(s_d[0]));
        atomicMax(&dmax[1], (unsigned long long)__double_as_longlong(s_t[0]));
    }
}

__global__ void clear_u64(unsigned long long *x, int n)
{
    if ((int)threadIdx.x < n) x[threadIdx.x] = 0ull;
}

// O at every node from cell values E (cell-major) through the node relation
__global__ void node_all_kernel(int N, int P, double eps, const double *E, const double *O, const double *Aw,
                                const double *Bc, const double *mu, const double *bL, const double *bR, double *Oout)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (N + 1) * P) return;
    const int i = t / P, p = t - (t / P) * P;
    Oout[t] = node_any(E, O, Aw, Bc, mu[p], bL[p], bR[p], eps, N, P, i, p);
}

// cell-centre intensities from the parities (4.2): I(+-mu_p) = E_p +- eps O_p, O
// interpolated to the cell centre as the mean of the cell's two nodes (the
// interpolation of the inflow relations (4.6)); out[j*2P + p] = I(+mu_p),
// out[j*2P + P + p] = I(-mu_p)
__global__ void intensity_kernel(int N, int P, double eps, const double *E, const double *O, double *out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * P) return;
    const int j = t / P, p = t - j * P;
    const double oc = 0.5 * (O[(size_t)j * P + p] + O[(size_t)(j + 1) * P + p]);
    out[(size_t)j * 2 * P + p] = E[t] + eps * oc;
    out[(size_t)j * 2 * P + P + p] = E[t] - eps * oc;
}

// between binary64 state arrays and binary32 storage (E as the deviation from a c T^4)
__global__ void convert_state_kernel(int N, int P, double ac, const double *T, double *E, double *O, float *E32,
                                     float *O32, int to32)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t ne = (size_t)N * P, no = (size_t)(N + 1) * P;
    if (t < ne) {
        const double tj = T[t / P];
        const double base = ac * (tj * tj) * (tj * tj);
        if (to32) E32[t] = (float)(E[t] - base);
        else E[t] = base + (double)E32[t];
    }
    if (t < no) {
        if (to32) O32[t] = (float)O[t];
        else O[t] = (double)O32[t];
    }
}

__global__ void fill_int_kernel(int *x, int n, int v)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

__global__ void fill_kernel(double *x, size_t n, double v)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct grte_ctx {
    int N = 0, P = 0, m = 0, M = 2, dev = 0;
    double L = 1, a = 1, c = 1, cv = 1;
    double one_minus_W = 0, mu1 = 0, mu2 = 0;
    double pred_tol = 1e-15;
    int pred_maxit = 200, newton_maxit = 100;
    int pred_accel = GRTE_ACCEL_CHEBYSHEV;
    double *hist = nullptr;       // convergence history of the last prediction solve
    int coop_capacity = 0;                 // co-resident prediction work-groups on the device
    int coop_launch = 1;                   // 1: cooperative launch of the prediction; 0: ordinary launch
    int keep = 1;
    int corr_kind = GRTE_CORRECTION_CONSERVATIVE;   // grte_set_correction
    hipStream_t stream = nullptr;
    std::vector<double *> allocs;
    double *E = nullptr, *O = nullptr, *T = nullptr;       // current state
    double *E2 = nullptr, *O2 = nullptr, *T2 = nullptr;    // next state
    double *sigma0, *mu, *omega, *bL, *bR;
    double *Ll, *Lu, *Lam, *LmG, *Gt, *Bd, *Aw, *Bc, *beta, *Dl, *Dd, *Du, *rho_n;
    double *r, *part, *res, *estar, *rho;
    double *ustar, *Dv, *ostar, *rho1, *rstar;
    // binary32 storage of the intensity state (f32 != 0): E as E - a c T^4, and O;
    // the binary64 E, O buffers then serve as scratch
    int f32 = 0;
    float *E32 = nullptr, *E32b = nullptr, *O32 = nullptr, *O32b = nullptr;
    double *ibuf = nullptr;                // intensity readout (2 N P), allocated on first use
    // learned initial guess of the temperature solve (borrowed from a grte_mlp)
    const uint16_t *guess_w = nullptr;
    const float *guess_norm = nullptr;
    double guess_tol = 1e-10;
    double last_dt = 0, last_eps = 0;      // of the last step (training-pair log)
    int stepped = 0;
    // warm start: rho (the last prediction's converged rho*, of the step that
    // produced the current state) is the next prediction's starting iterate;
    // cleared whenever the state is set or replaced otherwise
    int warm = 0;
    double *rho_b = nullptr;      // the prediction's output buffer (swapped with rho)
    unsigned long long *flags = nullptr;   // grid-barrier flags of the prediction kernel
    unsigned long long bar_gen = 0;        // generations used so far (strictly increasing)
    int cpb = 1;                           // cells per work-group of the per-cell kernels
    size_t pred_lds = 0;
    int *stat = nullptr;
    // energy balance of the last step (projection kernel): O* at the end nodes,
    // per-block partial sums, and the four results
    double *obnd = nullptr, *epart = nullptr, *energy = nullptr;
    // optional stage timing: event pairs recorded on the context stream
    int profiling = 0;            // 0 off, k: time every k-th step
    long long prof_count = 0;     // steps since profiling was set
    std::vector<hipEvent_t> ev_pool;      // created on demand, reused
    std::vector<int> ev_stage;            // stage index of each recorded pair
    size_t ev_used = 0;                   // pairs recorded since the last read
};

namespace {

grte_status hip_fail(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GRTE_OK;
    fprintf(stderr, "grte: %s failed: %s\n", what, hipGetErrorString(e));
    return GRTE_E_HIP;
}

#define HIPCHK(x)                                               \
    do {                                                        \
        grte_status _s = hip_fail((x), #x);                     \
        if (_s != GRTE_OK) return _s;                           \
    } while (0)

grte_status alloc(grte_ctx *ctx, double **p, size_t n)
{
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(double)) != hipSuccess) return GRTE_E_NOMEM;
    ctx->allocs.push_back((double *)q);
    *p = (double *)q;
    return GRTE_OK;
}

grte_status copy_in(grte_ctx *ctx, double *dst, const double *src, size_t n, int on_device)
{
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(ctx->stream));
    return GRTE_OK;
}

grte_status copy_out(grte_ctx *ctx, double *dst, const double *src, size_t n, int on_device)
{
    HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(ctx->stream));
    return GRTE_OK;
}

// stage timing (profiling only): each pair gets its own index at begin, so
// pairs may nest (the whole step encloses its stages)
grte_status prof_begin(grte_ctx *ctx, int stage, int *idx)
{
    *idx = -1;
    if (!ctx->profiling) return GRTE_OK;
    if (ctx->ev_used * 2 + 2 > ctx->ev_pool.size()) {
        for (int q = 0; q < 2; ++q) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            ctx->ev_pool.push_back(e);
        }
        ctx->ev_stage.push_back(0);
    }
    const int k = (int)ctx->ev_used++;
    ctx->ev_stage[k] = stage;
    HIPCHK(hipEventRecord(ctx->ev_pool[2 * k], ctx->stream));
    *idx = k;
    return GRTE_OK;
}

grte_status prof_end(grte_ctx *ctx, int idx)
{
    if (idx < 0) return GRTE_OK;
    HIPCHK(hipEventRecord(ctx->ev_pool[2 * idx + 1], ctx->stream));
    return GRTE_OK;
}

template <int M>
size_t pred_lds_bytes()
{
    return (size_t)(3 * NT * M + tile_scratch<NT>() + 2 * red_doubles()) * sizeof(double);
}

// The prediction's work-groups wait for each other at grid barriers, so they
// must all be resident at once.  The cooperative launch has the runtime
// guarantee it; the ordinary launch (coop = false) relies on the grid fitting
// the device at once (checked against the occupancy at creation) and on no
// other work occupying it -- when that fails the bounded barrier times out and
// the step reports a sync error (grte_step_info.sync_error, GRTE_E_HIP) instead
// of waiting forever.
template <int M>
grte_status launch_pred(hipStream_t stream, Group<PredArgs> &g, int grid, bool coop)
{
    if (!coop) {
        hipLaunchKernelGGL(pred_kernel<M>, dim3(grid), dim3(NT), pred_lds_bytes<M>(), stream, g);
        HIPCHK(hipGetLastError());
        return GRTE_OK;
    }
    void *args[] = {&g};
    HIPCHK(hipLaunchCooperativeKernel((const void *)pred_kernel<M>, dim3(grid), dim3(NT), args,
                                      (unsigned)pred_lds_bytes<M>(), stream));
    return GRTE_OK;
}

template <int M>
grte_status launch_corr(hipStream_t stream, Group<CorrArgs> &g, int maxP)
{
    const size_t lds = (size_t)(2 * NT * M + tile_scratch<NT>()) * sizeof(double);
    hipLaunchKernelGGL(corr_kernel<M>, dim3(maxP, g.n), dim3(NT), lds, stream, g);
    HIPCHK(hipGetLastError());
    return GRTE_OK;
}

int rows_per_thread(int N)
{
    int M = 2;
    while (NT * M < N) M *= 2;
    return M;
}

// binary64 state buffers <-> binary32 storage, on the context stream
grte_status convert_state(grte_ctx *ctx, int to32)
{
    const size_t no = (size_t)(ctx->N + 1) * ctx->P;
    hipLaunchKernelGGL(convert_state_kernel, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, ctx->stream, ctx->N,
                       ctx->P, ctx->a * ctx->c, ctx->T, ctx->E, ctx->O, ctx->E32, ctx->O32, to32);
    HIPCHK(hipGetLastError());
    return GRTE_OK;
}

template <int M>
int coop_blocks_per_cu()
{
    int nb = 0;
    const size_t lds = pred_lds_bytes<M>();
    if (hipFuncSetAttribute((const void *)pred_kernel<M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)pred_kernel<M>, NT, lds) != hipSuccess)
        return 0;
    return nb;
}

}  // namespace

extern "C" {

const char *grte_status_string(grte_status s)
{
    switch (s) {
    case GRTE_OK: return "ok";
    case GRTE_E_INVAL: return "invalid argument";
    case GRTE_E_NOMEM: return "device allocation failed";
    case GRTE_E_HIP: return "HIP runtime error";
    case GRTE_E_NOCONV: return "a solve stopped at its iteration cap";
    case GRTE_E_UNSUPPORTED: return "size beyond the library's limits";
    }
    return "unknown status";
}

grte_status grte_gauss_legendre(int nv, double *mu, double *omega)
{
    if (nv < 2 || nv > 128 || (nv & 1) || !mu || !omega) return GRTE_E_INVAL;
    const int P = nv / 2;
    // Newton on the Legendre polynomial P_nv (three-term recurrence) in
    // extended precision; weights 2 / ((1 - x^2) P'_nv(x)^2) on [-1, 1].
    for (int q = 0; q < P; ++q) {
        const int k = q + 1;   // k-th largest root
        long double x = cosl(3.14159265358979323846264338327950288L * (k - 0.25L) / (nv + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = x;
            for (int n = 2; n <= nv; ++n) {
                const long double p2 = ((2 * n - 1) * x * p1 - (n - 1) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            dp = nv * (x * p1 - p0) / (x * x - 1.0L);
            const long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) <= 1e-19L * fabsl(x)) break;
        }
        {
            long double p0 = 1.0L, p1 = x;
            for (int n = 2; n <= nv; ++n) {
                const long double p2 = ((2 * n - 1) * x * p1 - (n - 1) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            dp = nv * (x * p1 - p0) / (x * x - 1.0L);
        }
        const long double w = 2.0L / ((1.0L - x * x) * dp * dp);
        // increasing mu: the k-th largest root goes to slot P - k
        mu[P - k] = (double)x;
        omega[P - k] = (double)w;
    }
    return GRTE_OK;
}

grte_status grte_destroy(grte_ctx *ctx)
{
    if (!ctx) return GRTE_OK;
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (double *p : ctx->allocs) (void)hipFree(p);
    if (ctx->stat) (void)hipFree(ctx->stat);
    delete ctx;
    return GRTE_OK;
}

grte_status grte_create(const grte_problem *pb, const double *mu, const double *omega, grte_ctx **out)
{
    if (!pb || !mu || !omega || !out) return GRTE_E_INVAL;
    *out = nullptr;
    if (pb->nx < 2 || pb->npairs < 1 || !(pb->length > 0) || !(pb->a > 0) || !(pb->c > 0) ||
        !(pb->cv > 0) || (pb->opacity_law != 0 && pb->opacity_law != 3))
        return GRTE_E_INVAL;
    if (pb->nx > MAX_N || pb->npairs > MAX_P) return GRTE_E_UNSUPPORTED;
    for (int p = 0; p < pb->npairs; ++p)
        if (!(mu[p] > 0) || !(omega[p] > 0) || !std::isfinite(mu[p]) || !std::isfinite(omega[p]))
            return GRTE_E_INVAL;
    grte_ctx *ctx = new (std::nothrow) grte_ctx();
    if (!ctx) return GRTE_E_NOMEM;
    ctx->N = pb->nx;
    ctx->P = pb->npairs;
    ctx->m = pb->opacity_law;
    ctx->L = pb->length;
    ctx->a = pb->a;
    ctx->c = pb->c;
    ctx->cv = pb->cv;
    ctx->M = rows_per_thread(ctx->N);
    if (hipGetDevice(&ctx->dev) != hipSuccess) { delete ctx; return GRTE_E_HIP; }
    // 1 - sum(omega), exactly rounded: two-sum accumulation, then 1 - hi is exact
    double s = 0.0, e = 0.0;
    ctx->mu1 = 0.0;
    ctx->mu2 = 0.0;
    for (int p = 0; p < ctx->P; ++p) {
        const double x = omega[p];
        const double t = s + x;
        const double bp = t - s;
        e += (s - (t - bp)) + (x - bp);
        s = t;
        ctx->mu1 += omega[p] * mu[p];
        ctx->mu2 += omega[p] * mu[p] * mu[p];
    }
    ctx->one_minus_W = (1.0 - s) - e;

    const size_t N = ctx->N, P = ctx->P;
    grte_status st = GRTE_OK;
    double **cells[] = {&ctx->T, &ctx->T2, &ctx->sigma0, &ctx->Ll, &ctx->Lu, &ctx->Lam,
                        &ctx->LmG, &ctx->Bd, &ctx->beta, &ctx->Dl, &ctx->Dd, &ctx->Du,
                        &ctx->rho_n, &ctx->rho, &ctx->rho_b, &ctx->ustar, &ctx->Dv, &ctx->rho1, &ctx->rstar};
    const size_t NP = (size_t)NT * ctx->M;    // padded rows of the solvers
    double **padded[] = {&ctx->Gt, &ctx->res};
    for (double **q : padded)
        if (st == GRTE_OK) st = alloc(ctx, q, NP);
    double **padded_pairs[] = {&ctx->part, &ctx->r};
    for (double **q : padded_pairs)
        if (st == GRTE_OK) st = alloc(ctx, q, NP * P);
    for (double **q : cells)
        if (st == GRTE_OK) st = alloc(ctx, q, N);
    double **nodes[] = {&ctx->Aw, &ctx->Bc};
    for (double **q : nodes)
        if (st == GRTE_OK) st = alloc(ctx, q, N + 1);
    double **pairs[] = {&ctx->mu, &ctx->omega, &ctx->bL, &ctx->bR};
    for (double **q : pairs)
        if (st == GRTE_OK) st = alloc(ctx, q, P);
    double **cp[] = {&ctx->E, &ctx->E2, &ctx->estar};
    for (double **q : cp)
        if (st == GRTE_OK) st = alloc(ctx, q, N * P);
    double **np[] = {&ctx->O, &ctx->O2, &ctx->ostar};
    for (double **q : np)
        if (st == GRTE_OK) st = alloc(ctx, q, (N + 1) * P);
    if (st == GRTE_OK) st = alloc(ctx, &ctx->hist, HIST_CAP);
    double *flagmem = nullptr;
    if (st == GRTE_OK) st = alloc(ctx, &flagmem, (size_t)MAX_P * BAR_STRIDE);
    ctx->flags = (unsigned long long *)flagmem;
    if (st == GRTE_OK && hipMalloc((void **)&ctx->stat, NSTAT * sizeof(int)) != hipSuccess) st = GRTE_E_NOMEM;
    if (st == GRTE_OK) st = alloc(ctx, &ctx->obnd, 2 * P);
    if (st == GRTE_OK) st = alloc(ctx, &ctx->epart, 2 * N);   // 2 per cell block (at most N blocks)
    if (st == GRTE_OK) st = alloc(ctx, &ctx->energy, 4);
    if (st != GRTE_OK) { grte_destroy(ctx); return st; }

    // co-resident blocks for the cooperative prediction kernel
    int nb = 0;
    switch (ctx->M) {
    case 2: nb = coop_blocks_per_cu<2>(); break;
    case 4: nb = coop_blocks_per_cu<4>(); break;
    case 8: nb = coop_blocks_per_cu<8>(); break;
    default: nb = coop_blocks_per_cu<16>(); break;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->dev) != hipSuccess || nb < 1) {
        grte_destroy(ctx);
        return GRTE_E_HIP;
    }
    // one work-group per parity pair, all co-resident
    if (nb * ncu < ctx->P) {
        grte_destroy(ctx);
        return GRTE_E_UNSUPPORTED;
    }
    ctx->coop_capacity = nb * ncu;
    ctx->cpb = std::max(1, 256 / ctx->P);

    if (hipMemcpy(ctx->mu, mu, P * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->omega, omega, P * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        grte_destroy(ctx);
        return GRTE_E_HIP;
    }
    // defaults: zero state and inflow, unit opacity
    const unsigned b = 256;
    hipLaunchKernelGGL(fill_kernel, dim3((N * P + b - 1) / b), dim3(b), 0, nullptr, ctx->E, N * P, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3(((N + 1) * P + b - 1) / b), dim3(b), 0, nullptr, ctx->O, (N + 1) * P, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3((N + b - 1) / b), dim3(b), 0, nullptr, ctx->T, N, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3((N + b - 1) / b), dim3(b), 0, nullptr, ctx->sigma0, N, 1.0);
    hipLaunchKernelGGL(fill_kernel, dim3((P + b - 1) / b), dim3(b), 0, nullptr, ctx->bL, P, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3((P + b - 1) / b), dim3(b), 0, nullptr, ctx->bR, P, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3((MAX_P * BAR_STRIDE + b - 1) / b), dim3(b), 0, nullptr, flagmem,
                       (size_t)MAX_P * BAR_STRIDE, 0.0);   // all-zero bits: generation 0
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(b), 0, nullptr, ctx->energy, 4, 0.0);
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, nullptr, ctx->stat, NSTAT, 0);
    // padded rows of the position-ordered arrays stay zero
    const size_t npad = (size_t)NT * ctx->M;
    hipLaunchKernelGGL(fill_kernel, dim3((npad + b - 1) / b), dim3(b), 0, nullptr, ctx->Gt, npad, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3((npad + b - 1) / b), dim3(b), 0, nullptr, ctx->res, npad, 0.0);
    if (hipDeviceSynchronize() != hipSuccess) { grte_destroy(ctx); return GRTE_E_HIP; }
    *out = ctx;
    return GRTE_OK;
}

grte_status grte_set_stream(grte_ctx *ctx, void *hip_stream)
{
    if (!ctx) return GRTE_E_INVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return GRTE_OK;
}

grte_status grte_set_solver(grte_ctx *ctx, double pred_tol, int pred_maxit, int newton_maxit)
{
    if (!ctx || !(pred_tol > 0) || pred_maxit < 1 || newton_maxit < 1) return GRTE_E_INVAL;
    ctx->pred_tol = pred_tol;
    ctx->pred_maxit = pred_maxit;
    ctx->newton_maxit = newton_maxit;
    return GRTE_OK;
}

grte_status grte_set_acceleration(grte_ctx *ctx, int mode)
{
    if (!ctx || (mode != GRTE_ACCEL_RICHARDSON && mode != GRTE_ACCEL_CHEBYSHEV)) return GRTE_E_INVAL;
    ctx->pred_accel = mode;
    return GRTE_OK;
}

grte_status grte_set_opacity(grte_ctx *ctx, const double *sigma0, int on_device)
{
    if (!ctx || !sigma0) return GRTE_E_INVAL;
    if (!on_device)
        for (int j = 0; j < ctx->N; ++j)
            if (!(sigma0[j] >= 0) || !std::isfinite(sigma0[j])) return GRTE_E_INVAL;
    return copy_in(ctx, ctx->sigma0, sigma0, ctx->N, on_device);
}

grte_status grte_set_inflow(grte_ctx *ctx, const double *b_left, const double *b_right)
{
    if (!ctx || !b_left || !b_right) return GRTE_E_INVAL;
    grte_status s = copy_in(ctx, ctx->bL, b_left, ctx->P, 0);
    if (s != GRTE_OK) return s;
    return copy_in(ctx, ctx->bR, b_right, ctx->P, 0);
}

grte_status grte_set_state(grte_ctx *ctx, const double *E, const double *O, const double *T, int on_device)
{
    if (!ctx || !E || !O || !T) return GRTE_E_INVAL;
    if (!on_device)
        for (int j = 0; j < ctx->N; ++j)
            if (!(T[j] >= 0) || !std::isfinite(T[j])) return GRTE_E_INVAL;
    const size_t N = ctx->N, P = ctx->P;
    ctx->stepped = 0;                      // the pair log refers to a step from this state on
    ctx->warm = 0;
    grte_status s = copy_in(ctx, ctx->E, E, N * P, on_device);
    if (s == GRTE_OK) s = copy_in(ctx, ctx->O, O, (N + 1) * P, on_device);
    if (s == GRTE_OK) s = copy_in(ctx, ctx->T, T, N, on_device);
    if (s == GRTE_OK && ctx->f32) s = convert_state(ctx, 1);
    return s;
}

grte_status grte_get_state(grte_ctx *ctx, double *E, double *O, double *T, int on_device)
{
    if (!ctx) return GRTE_E_INVAL;
    const size_t N = ctx->N, P = ctx->P;
    grte_status s = GRTE_OK;
    if (ctx->f32) s = convert_state(ctx, 0);   // binary64 values of the stored state
    if (s == GRTE_OK && E) s = copy_out(ctx, E, ctx->E, N * P, on_device);
    if (s == GRTE_OK && O) s = copy_out(ctx, O, ctx->O, (N + 1) * P, on_device);
    if (s == GRTE_OK && T) s = copy_out(ctx, T, ctx->T, N, on_device);
    return s;
}

grte_status grte_get_intensity(grte_ctx *ctx, double eps, double *I, int on_device)
{
    if (!ctx || !I || !(eps > 0.0) || !std::isfinite(eps)) return GRTE_E_INVAL;
    const size_t N = ctx->N, P = ctx->P;
    if (ctx->f32) {
        grte_status s = convert_state(ctx, 0);   // binary64 values of the stored state
        if (s != GRTE_OK) return s;
    }
    double *dst = I;
    if (!on_device) {
        if (!ctx->ibuf) {
            void *q = nullptr;
            if (hipMalloc(&q, 2 * N * P * sizeof(double)) != hipSuccess) return GRTE_E_NOMEM;
            ctx->allocs.push_back((double *)q);
            ctx->ibuf = (double *)q;
        }
        dst = ctx->ibuf;
    }
    hipLaunchKernelGGL(intensity_kernel, dim3((unsigned)((N * P + 255) / 256)), dim3(256), 0, ctx->stream, (int)N,
                       (int)P, eps, ctx->E, ctx->O, dst);
    HIPCHK(hipGetLastError());
    if (!on_device) return copy_out(ctx, I, dst, 2 * N * P, 0);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return GRTE_OK;
}

grte_status grte_get_pred_history(grte_ctx *ctx, double *out, int cap, int *n)
{
    if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return GRTE_E_INVAL;
    int its = 0;
    HIPCHK(hipMemcpyAsync(&its, ctx->stat, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int k = std::min(std::min(its, cap), HIST_CAP);
    *n = k;
    if (k > 0) return copy_out(ctx, out, ctx->hist, (size_t)k, 0);
    return GRTE_OK;
}

grte_status grte_get_stage(grte_ctx *ctx, int stage, double *out, int on_device)
{
    if (!ctx || !out) return GRTE_E_INVAL;
    const size_t N = ctx->N, P = ctx->P;
    switch (stage) {
    case GRTE_STAGE_ESTAR: return copy_out(ctx, out, ctx->estar, N * P, on_device);
    case GRTE_STAGE_OSTAR: return copy_out(ctx, out, ctx->ostar, (N + 1) * P, on_device);
    case GRTE_STAGE_USTAR: return copy_out(ctx, out, ctx->ustar, N, on_device);
    case GRTE_STAGE_D: return copy_out(ctx, out, ctx->Dv, N, on_device);
    case GRTE_STAGE_RHO: return copy_out(ctx, out, ctx->rho1, N, on_device);
    }
    return GRTE_E_INVAL;
}

}  // extern "C"

namespace {

// One AP step of n contexts (n <= GMAX, same tile shape M) with one launch of
// each kernel, ordered on the stream of the first context.
grte_status step_group(grte_ctx *const *ctxs, int n, const double *dts, const double *epss,
                       grte_step_info *info)
{
    grte_ctx *c0 = ctxs[0];
    hipStream_t stream = c0->stream;
    const int M = c0->M;
    Group<CoefArgs> gc{};
    Group<PredArgs> gp{};
    Group<NewtonArgs> gn{};
    Group<CorrArgs> gr{};
    Group<ProjArgs> gj{};
    Group<AltArgs> ga{};
    gc.n = gp.n = gn.n = gr.n = gj.n = ga.n = n;
    const bool alt = c0->corr_kind == GRTE_CORRECTION_ALT;
    unsigned ncb_max = 1, maxP = 1;
    int grid = 0;
    for (int g = 0; g < n; ++g) {
        grte_ctx *ctx = ctxs[g];
        const double dt = dts[g], eps = epss[g];
        const int N = ctx->N, P = ctx->P;
        const double dx = ctx->L / N;
        ncb_max = std::max(ncb_max, (unsigned)((N + ctx->cpb - 1) / ctx->cpb));
        maxP = std::max(maxP, (unsigned)P);
        // coefficients of the prediction (K from T^n); also clears the step counters
        CoefArgs &ca = gc.a[g];
        ca.N = N; ca.P = P; ca.m = ctx->m; ca.mode = 0; ca.cpb = ctx->cpb;
        ca.a = ctx->a; ca.c = ctx->c; ca.cv = ctx->cv; ca.eps = eps; ca.dt = dt; ca.dx = dx;
        ca.T = ctx->T; ca.Tn = ctx->T; ca.sigma0 = ctx->sigma0; ca.mu = ctx->mu; ca.omega = ctx->omega;
        ca.bL = ctx->bL; ca.bR = ctx->bR; ca.E = ctx->E; ca.O = ctx->O;
        ca.mu1 = ctx->mu1; ca.mu2 = ctx->mu2;
        ca.Ll = ctx->Ll; ca.Lu = ctx->Lu; ca.Lam = ctx->Lam; ca.LmG = ctx->LmG; ca.Gt = ctx->Gt; ca.M = ctx->M;
        ca.Bd = ctx->Bd; ca.Aw = ctx->Aw; ca.Bc = ctx->Bc; ca.beta = ctx->beta;
        ca.Dl = ctx->Dl; ca.Dd = ctx->Dd; ca.Du = ctx->Du; ca.rho_n = ctx->rho_n; ca.r = ctx->r;
        ca.stat = ctx->stat;
        ca.E32 = ctx->E32; ca.O32 = ctx->O32; ca.f32 = ctx->f32;
        // prediction: work-groups [grid, grid + P) belong to this context
        PredArgs &pa = gp.a[g];
        pa.N = N; pa.P = P; pa.maxit = ctx->pred_maxit; pa.tol = ctx->pred_tol; pa.one_minus_W = ctx->one_minus_W;
        pa.accel = ctx->pred_accel;
        pa.hist = ctx->hist;
        pa.Ll = ctx->Ll; pa.Lu = ctx->Lu; pa.Lam = ctx->Lam; pa.LmG = ctx->LmG; pa.Gt = ctx->Gt;
        pa.Bd = ctx->Bd; pa.Dd = ctx->Dd; pa.mu2avg = ctx->mu2;
        pa.r = ctx->r; pa.mu = ctx->mu; pa.omega = ctx->omega; pa.rho0 = ctx->warm ? ctx->rho : ctx->rho_n;
        pa.part = ctx->part; pa.res = ctx->res; pa.estar = ctx->estar; pa.rho_out = ctx->rho_b; pa.stat = ctx->stat;
        pa.flags = ctx->flags;
        pa.gen0 = ctx->bar_gen;
        ctx->bar_gen += 2ull * (unsigned long long)ctx->pred_maxit + 4ull;   // never reused
        gp.first[g] = grid;
        grid += P;
        // correction substep 1
        NewtonArgs &na = gn.a[g];
        na.N = N; na.P = P; na.m = ctx->m; na.maxit = ctx->newton_maxit; na.keep = ctx->keep; na.cpb = ctx->cpb;
        na.Ecm = ctx->estar;
        na.a = ctx->a; na.c = ctx->c; na.cv = ctx->cv; na.eps = eps; na.dt = dt; na.dx = dx;
        na.O = ctx->O; na.Aw = ctx->Aw; na.Bc = ctx->Bc; na.beta = ctx->beta;
        na.rho_n = ctx->rho_n; na.Tn = ctx->T; na.sigma0 = ctx->sigma0; na.mu = ctx->mu; na.omega = ctx->omega;
        na.bL = ctx->bL; na.bR = ctx->bR; na.Tnew = ctx->T2; na.ustar = ctx->ustar; na.Dv = ctx->Dv;
        na.ostar = ctx->ostar; na.stat = ctx->stat; na.rstar = ctx->rstar;
        na.obnd = ctx->obnd;
        na.moments_only = alt ? 1 : 0;
        // the alternative correction (3.14): its operators, E_J into the scratch
        // `part` (cell-major), then the explicit temperature and the projection
        AltArgs &aa = ga.a[g];
        aa.N = N; aa.P = P; aa.m = ctx->m; aa.cpb = ctx->cpb; aa.M = ctx->M;
        aa.a = ctx->a; aa.c = ctx->c; aa.cv = ctx->cv; aa.eps = eps; aa.dt = dt; aa.dx = dx;
        aa.Tn = ctx->T; aa.sigma0 = ctx->sigma0; aa.mu = ctx->mu; aa.omega = ctx->omega;
        aa.bL = ctx->bL; aa.bR = ctx->bR; aa.En = ctx->E; aa.On = ctx->O; aa.Es = ctx->estar;
        aa.Os = ctx->ostar; aa.Us = ctx->ustar;
        aa.Ll = ctx->Ll; aa.Lu = ctx->Lu; aa.Lam = ctx->Lam; aa.Bd = ctx->Bd; aa.r = ctx->r;
        aa.EJ = ctx->part; aa.Enew = ctx->E2; aa.Onew = ctx->O2; aa.Tnew = ctx->T2; aa.rho_out = ctx->rho1;
        aa.rho_n = ctx->rho_n; aa.epart = ctx->epart; aa.energy = ctx->energy;
        aa.stat = ctx->stat;
        na.gw = ctx->guess_w; na.gnorm = ctx->guess_norm; na.gtol = ctx->guess_tol;
        na.O32 = ctx->O32; na.f32 = ctx->f32;
        ctx->last_dt = dt;
        ctx->last_eps = eps;
        ctx->stepped = 1;
        // correction substep 2: E^{n+1} straight into the next state
        CorrArgs &cc = gr.a[g];
        cc.N = N; cc.P = P; cc.Ll = ctx->Ll; cc.Lu = ctx->Lu; cc.Lam = ctx->Lam; cc.Bd = ctx->Bd;
        cc.r = ctx->r; cc.mu = ctx->mu; cc.Enew = alt ? ctx->part : ctx->E2;
        cc.E32new = ctx->E32b; cc.Tnew = ctx->T2; cc.ac = ctx->a * ctx->c; cc.f32 = alt ? 0 : ctx->f32;
        // projection: O^{n+1} at the nodes, rho^{n+1}
        ProjArgs &pj = gj.a[g];
        pj.N = N; pj.P = P; pj.keep = ctx->keep; pj.cpb = ctx->cpb; pj.eps = eps;
        pj.Enew = ctx->E2; pj.O = ctx->O; pj.Aw = ctx->Aw; pj.Bc = ctx->Bc;
        pj.mu = ctx->mu; pj.omega = ctx->omega; pj.bL = ctx->bL; pj.bR = ctx->bR;
        pj.Oout = ctx->O2; pj.rho_out = ctx->rho1;
        pj.O32 = ctx->O32; pj.O32out = ctx->O32b; pj.f32 = ctx->f32;
        pj.dx = dx; pj.c = ctx->c; pj.cv = ctx->cv; pj.dt = dt;
        pj.Tn = ctx->T; pj.Tnew = ctx->T2; pj.rho_n = ctx->rho_n; pj.obnd = ctx->obnd;
        pj.epart = ctx->epart; pj.energy = ctx->energy; pj.stat = ctx->stat;
    }
    gp.first[n] = grid;
    if (grid > c0->coop_capacity) return GRTE_E_UNSUPPORTED;

    int ev_step = -1, ev_pred = -1;
    // profiling samples every c0->profiling-th step (event records cost the
    // stream a few microseconds each)
    const bool sample = c0->profiling > 0 && (c0->prof_count++ % c0->profiling) == 0;
    grte_status st = sample ? prof_begin(c0, GRTE_TIMING_STEP, &ev_step) : GRTE_OK;
    if (st != GRTE_OK) return st;
    hipLaunchKernelGGL(coef_kernel, dim3(ncb_max, n), dim3(256), 0, stream, gc);
    HIPCHK(hipGetLastError());
    if (sample && (st = prof_begin(c0, GRTE_TIMING_PREDICT, &ev_pred)) != GRTE_OK) return st;
    switch (M) {
    case 2: st = launch_pred<2>(stream, gp, grid, c0->coop_launch != 0); break;
    case 4: st = launch_pred<4>(stream, gp, grid, c0->coop_launch != 0); break;
    case 8: st = launch_pred<8>(stream, gp, grid, c0->coop_launch != 0); break;
    default: st = launch_pred<16>(stream, gp, grid, c0->coop_launch != 0); break;
    }
    if (st != GRTE_OK) return st;
    if ((st = prof_end(c0, ev_pred)) != GRTE_OK) return st;
    bool any_guess = false;
    for (int g = 0; g < n; ++g) any_guess = any_guess || gn.a[g].gw != nullptr;
    if (any_guess) hipLaunchKernelGGL(newton_kernel<true>, dim3(ncb_max, n), dim3(256), 0, stream, gn);
    else hipLaunchKernelGGL(newton_kernel<false>, dim3(ncb_max, n), dim3(256), 0, stream, gn);
    HIPCHK(hipGetLastError());
    if (alt) {
        hipLaunchKernelGGL(alt_coef_kernel, dim3(ncb_max, n), dim3(256), 0, stream, ga);
    } else {
        for (int g = 0; g < n; ++g) {     // coefficients of the correction: K from T^{n+1}
            gc.a[g].mode = 1;
            gc.a[g].T = ctxs[g]->T2;
        }
        hipLaunchKernelGGL(coef_kernel, dim3(ncb_max, n), dim3(256), 0, stream, gc);
    }
    HIPCHK(hipGetLastError());
    switch (M) {
    case 2: st = launch_corr<2>(stream, gr, (int)maxP); break;
    case 4: st = launch_corr<4>(stream, gr, (int)maxP); break;
    case 8: st = launch_corr<8>(stream, gr, (int)maxP); break;
    default: st = launch_corr<16>(stream, gr, (int)maxP); break;
    }
    if (st != GRTE_OK) return st;
    if (alt) {
        hipLaunchKernelGGL(alt_project_kernel, dim3(ncb_max, n), dim3(256), 0, stream, ga);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(alt_energy_final_kernel, dim3(n), dim3(256), 0, stream, ga);
    } else {
        hipLaunchKernelGGL(project_kernel, dim3(ncb_max, n), dim3(256), 0, stream, gj);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(energy_final_kernel, dim3(n), dim3(256), 0, stream, gj);
    }
    HIPCHK(hipGetLastError());
    if ((st = prof_end(c0, ev_step)) != GRTE_OK) return st;   // whole step
    for (int g = 0; g < n; ++g) {
        grte_ctx *ctx = ctxs[g];
        std::swap(ctx->E, ctx->E2);
        std::swap(ctx->O, ctx->O2);
        std::swap(ctx->T, ctx->T2);
        std::swap(ctx->E32, ctx->E32b);
        std::swap(ctx->O32, ctx->O32b);
        std::swap(ctx->rho, ctx->rho_b);   // rho*: the next step's starting iterate
        ctx->warm = 1;
    }
    if (!info) return GRTE_OK;
    grte_status worst = GRTE_OK;
    for (int g = 0; g < n; ++g) {
        int h[NSTAT];
        double en[4];
        HIPCHK(hipMemcpyAsync(h, ctxs[g]->stat, sizeof(h), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipMemcpyAsync(en, ctxs[g]->energy, sizeof(en), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        grte_step_info &f = info[g];
        f.pred_iters = h[0];
        f.pred_converged = h[1] ? 1 : 0;
        f.pred_floor_stop = h[1] == 2 ? 1 : 0;
        f.newton_max_iters = h[2];
        f.newton_failed = h[3];
        f.kstar_clamped = h[4];
        f.negative_root = h[5];
        f.sync_error = h[6];
        f.guess_accepted = h[7];
        f.guess_rejected = h[8];
        f.newton_total_iters = h[9];
        f.guess_started = h[10];
        f.energy_before = en[0];
        f.energy_after = en[1];
        f.boundary_flux_dt = en[2];
        f.energy_defect = en[3];
        if (h[6]) worst = GRTE_E_HIP;
        else if ((!h[1] || h[3]) && worst == GRTE_OK) worst = GRTE_E_NOCONV;
    }
    return worst;
}

}  // namespace

extern "C" {

grte_status grte_step(grte_ctx *ctx, double dt, double eps, grte_step_info *info)
{
    if (!ctx || !(dt > 0) || !(eps > 0) || !std::isfinite(dt) || !std::isfinite(eps)) return GRTE_E_INVAL;
    grte_ctx *one[1] = {ctx};
    return step_group(one, 1, &dt, &eps, info);
}

grte_status grte_step_group(grte_ctx *const *ctxs, int n, const double *dt, const double *eps,
                            grte_step_info *info)
{
    if (!ctxs || !dt || !eps || n < 1) return GRTE_E_INVAL;
    if (n > GMAX) return GRTE_E_UNSUPPORTED;
    for (int g = 0; g < n; ++g) {
        if (!ctxs[g] || !(dt[g] > 0) || !(eps[g] > 0) || !std::isfinite(dt[g]) || !std::isfinite(eps[g]))
            return GRTE_E_INVAL;
        if (ctxs[g]->M != ctxs[0]->M || ctxs[g]->dev != ctxs[0]->dev) return GRTE_E_INVAL;
        if (ctxs[g]->corr_kind != ctxs[0]->corr_kind) return GRTE_E_INVAL;
        for (int h = 0; h < g; ++h)
            if (ctxs[h] == ctxs[g]) return GRTE_E_INVAL;
    }
    return step_group(ctxs, n, dt, eps, info);
}

grte_status grte_reference_step(grte_ctx *ctx, double dt, double eps, double tol, int maxit,
                                grte_reference_info *info)
{
    if (ctx) ctx->warm = 0;   // the Picard loop reuses the rho* buffer
    if (!ctx || !(dt > 0) || !(eps > 0) || !std::isfinite(dt) || !std::isfinite(eps) || !(tol > 0) || maxit < 1)
        return GRTE_E_INVAL;
    if (ctx->f32) return GRTE_E_UNSUPPORTED;
    const int N = ctx->N, P = ctx->P, M = ctx->M;
    const double dx = ctx->L / N;
    hipStream_t stream = ctx->stream;
    double *Tk = ctx->T2, *Tk1 = ctx->rstar;   // Picard iterates (scratch of the normal step)
    HIPCHK(hipMemcpyAsync(Tk, ctx->T, N * sizeof(double), hipMemcpyDeviceToDevice, stream));
    unsigned long long *dmax = ctx->flags + (size_t)(MAX_P - 1) * BAR_STRIDE + 8;   // spare words of the last flag line
    Group<CoefArgs> gc{};
    gc.n = 1;
    CoefArgs &ca = gc.a[0];
    ca.N = N; ca.P = P; ca.m = ctx->m; ca.mode = 0; ca.cpb = ctx->cpb;
    ca.a = ctx->a; ca.c = ctx->c; ca.cv = ctx->cv; ca.eps = eps; ca.dt = dt; ca.dx = dx;
    ca.Tn = ctx->T; ca.sigma0 = ctx->sigma0; ca.mu = ctx->mu; ca.omega = ctx->omega;
    ca.bL = ctx->bL; ca.bR = ctx->bR; ca.E = ctx->E; ca.O = ctx->O;
    ca.mu1 = ctx->mu1; ca.mu2 = ctx->mu2;
    ca.Ll = ctx->Ll; ca.Lu = ctx->Lu; ca.Lam = ctx->Lam; ca.LmG = ctx->LmG; ca.Gt = ctx->Gt; ca.M = M;
    ca.Bd = ctx->Bd; ca.Aw = ctx->Aw; ca.Bc = ctx->Bc; ca.beta = ctx->beta;
    ca.Dl = ctx->Dl; ca.Dd = ctx->Dd; ca.Du = ctx->Du; ca.rho_n = ctx->rho_n; ca.r = ctx->r;
    ca.stat = ctx->stat;
    Group<PredArgs> gp{};
    gp.n = 1;
    gp.first[0] = 0;
    gp.first[1] = P;
    PredArgs &pa = gp.a[0];
    pa.N = N; pa.P = P; pa.maxit = ctx->pred_maxit; pa.tol = ctx->pred_tol; pa.one_minus_W = ctx->one_minus_W;
        pa.accel = ctx->pred_accel;
        pa.hist = ctx->hist;
    pa.Ll = ctx->Ll; pa.Lu = ctx->Lu; pa.Lam = ctx->Lam; pa.LmG = ctx->LmG; pa.Gt = ctx->Gt;
    pa.Bd = ctx->Bd; pa.Dd = ctx->Dd; pa.mu2avg = ctx->mu2;
    pa.r = ctx->r; pa.mu = ctx->mu; pa.omega = ctx->omega; pa.rho0 = ctx->rho_n;
    pa.part = ctx->part; pa.res = ctx->res; pa.estar = ctx->E2; pa.rho_out = ctx->rho; pa.stat = ctx->stat;
    pa.flags = ctx->flags;
    const unsigned ncb = (unsigned)((N + ctx->cpb - 1) / ctx->cpb);
    const double ac = ctx->a * ctx->c;
    int k = 0, converged = 0, worst_pred = 0, pred_fail = 0, sync_err = 0;
    grte_status st = GRTE_OK;
    for (k = 1; k <= maxit; ++k) {
        ca.T = Tk;                                    // K from the current opacity temperature
        hipLaunchKernelGGL(coef_kernel, dim3(ncb, 1), dim3(256), 0, stream, gc);
        HIPCHK(hipGetLastError());
        pa.gen0 = ctx->bar_gen;
        ctx->bar_gen += 2ull * (unsigned long long)ctx->pred_maxit + 4ull;
        switch (M) {
        case 2: st = launch_pred<2>(stream, gp, P, ctx->coop_launch != 0); break;
        case 4: st = launch_pred<4>(stream, gp, P, ctx->coop_launch != 0); break;
        case 8: st = launch_pred<8>(stream, gp, P, ctx->coop_launch != 0); break;
        default: st = launch_pred<16>(stream, gp, P, ctx->coop_launch != 0); break;
        }
        if (st != GRTE_OK) return st;
        hipLaunchKernelGGL(clear_u64, dim3(1), dim3(64), 0, stream, dmax, 2);
        hipLaunchKernelGGL(picard_update_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream, N, ac,
                           ctx->T, ctx->beta, ctx->rho, Tk, Tk1, ctx->ustar, dmax);
        HIPCHK(hipGetLastError());
        unsigned long long h[2];
        int hs[8];
        HIPCHK(hipMemcpyAsync(h, dmax, sizeof(h), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipMemcpyAsync(hs, ctx->stat, sizeof(hs), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        worst_pred = std::max(worst_pred, hs[0]);
        if (!hs[1]) pred_fail = 1;
        if (hs[6]) { sync_err = 1; break; }
        double d, tmax;
        std::memcpy(&d, &h[0], sizeof(d));
        std::memcpy(&tmax, &h[1], sizeof(tmax));
        std::swap(Tk, Tk1);                           // Tk holds T^(k+1)
        if (d <= tol * tmax) { converged = 1; break; }
    }
    if (k > maxit) k = maxit;
    ctx->T2 = Tk;
    ctx->rstar = Tk1;
    if (!sync_err) {
        // E^{n+1} = E* (the last prediction wrote it into E2) and O^{n+1} = O*
        // of the last prediction (K from the last T^(k))
        hipLaunchKernelGGL(node_all_kernel, dim3((unsigned)(((size_t)(N + 1) * P + 255) / 256)), dim3(256), 0,
                           stream, N, P, eps, ctx->E2, ctx->O, ctx->Aw, ctx->Bc, ctx->mu, ctx->bL, ctx->bR, ctx->O2);
        HIPCHK(hipGetLastError());
        std::swap(ctx->E, ctx->E2);
        std::swap(ctx->O, ctx->O2);
        std::swap(ctx->T, ctx->T2);
        ctx->stepped = 0;
        ctx->warm = 0;
        HIPCHK(hipStreamSynchronize(stream));
    }
    if (info) {
        info->picard_iters = k;
        info->converged = converged;
        info->pred_max_iters = worst_pred;
        info->pred_failed = pred_fail;
        info->sync_error = sync_err;
    }
    if (sync_err) return GRTE_E_HIP;
    return (converged && !pred_fail) ? GRTE_OK : GRTE_E_NOCONV;
}

grte_status grte_set_correction(grte_ctx *ctx, int kind)
{
    if (!ctx || (kind != GRTE_CORRECTION_CONSERVATIVE && kind != GRTE_CORRECTION_ALT)) return GRTE_E_INVAL;
    if (kind == GRTE_CORRECTION_ALT && ctx->f32) return GRTE_E_UNSUPPORTED;
    ctx->corr_kind = kind;
    return GRTE_OK;
}

grte_status grte_get_error_flags(grte_ctx *ctx, int *flags, int clear)
{
    if (!ctx || !flags) return GRTE_E_INVAL;
    HIPCHK(hipMemcpyAsync(flags, ctx->stat + STAT_STICKY, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (clear) {
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->stat + STAT_STICKY, 1, 0);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return GRTE_OK;
}

grte_status grte_set_launch(grte_ctx *ctx, int cooperative)
{
    if (!ctx || (cooperative != 0 && cooperative != 1)) return GRTE_E_INVAL;
    ctx->coop_launch = cooperative;
    return GRTE_OK;
}

grte_status grte_set_storage(grte_ctx *ctx, int fp32)
{
    if (!ctx || (fp32 != 0 && fp32 != 1)) return GRTE_E_INVAL;
    if (fp32 == ctx->f32) return GRTE_OK;
    if (fp32 && ctx->corr_kind == GRTE_CORRECTION_ALT) return GRTE_E_UNSUPPORTED;
    if (fp32 && !ctx->E32) {
        const size_t ne = (size_t)ctx->N * ctx->P, no = (size_t)(ctx->N + 1) * ctx->P;
        float **bufs[] = {&ctx->E32, &ctx->E32b, &ctx->O32, &ctx->O32b};
        const size_t sizes[] = {ne, ne, no, no};
        for (int q = 0; q < 4; ++q) {
            void *p = nullptr;
            if (hipMalloc(&p, sizes[q] * sizeof(float)) != hipSuccess) return GRTE_E_NOMEM;
            ctx->allocs.push_back((double *)p);
            *bufs[q] = (float *)p;
        }
    }
    grte_status s = convert_state(ctx, fp32);
    if (s != GRTE_OK) return s;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->f32 = fp32;
    ctx->warm = 0;
    return GRTE_OK;
}

grte_status grte_set_guess(grte_ctx *ctx, const grte_mlp *model, double accept_tol)
{
    if (!ctx || !(accept_tol >= 0) || !std::isfinite(accept_tol)) return GRTE_E_INVAL;
    ctx->guess_w = model ? model->wbf : nullptr;
    ctx->guess_norm = model ? model->norm : nullptr;
    ctx->guess_tol = accept_tol;
    return GRTE_OK;
}

grte_status grte_log_pairs(grte_ctx *ctx, float *dev_rows, long long cap_rows, long long *n_rows)
{
    if (!ctx || !dev_rows || !n_rows) return GRTE_E_INVAL;
    *n_rows = 0;
    if (!ctx->stepped) return GRTE_E_INVAL;
    if (cap_rows < ctx->N) return GRTE_E_INVAL;
    // after the step the previous temperature sits in the second buffer
    hipLaunchKernelGGL(log_pairs_kernel, dim3((unsigned)((ctx->N + 255) / 256)), dim3(256), 0, ctx->stream,
                       ctx->N, ctx->m, ctx->last_eps, ctx->last_dt, ctx->rstar, ctx->T2, ctx->T, ctx->sigma0,
                       dev_rows);
    HIPCHK(hipGetLastError());
    *n_rows = ctx->N;
    return GRTE_OK;
}

grte_status grte_set_profiling(grte_ctx *ctx, int on)
{
    if (!ctx || on < 0) return GRTE_E_INVAL;
    ctx->profiling = on;
    ctx->prof_count = 0;
    ctx->ev_used = 0;
    return GRTE_OK;
}

grte_status grte_read_timing(grte_ctx *ctx, double *total_ms, int *count)
{
    if (!ctx || !total_ms || !count) return GRTE_E_INVAL;
    for (int q = 0; q < GRTE_TIMING_NSTAGES; ++q) {
        total_ms[q] = 0.0;
        count[q] = 0;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (size_t k = 0; k < ctx->ev_used; ++k) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev_pool[2 * k], ctx->ev_pool[2 * k + 1]));
        const int q = ctx->ev_stage[k];
        total_ms[q] += ms;
        count[q] += 1;
    }
    ctx->ev_used = 0;
    return GRTE_OK;
}

}  // extern "C"
