// ap2d.hip -- the AP step of Algorithm 2 on a 2-D rectangle, staggered parity:
// E_p in the cells, the odd parity O_p on the faces (x-faces and y-faces), the
// O-equation (second equation of (4.3)) at every interior face, the E-equation
// in every cell, the inflow relation (4.6) at the centre of every edge cell.
//
// Both linear systems of the step -- the prediction (4.5)/(5.2) in (E*, O*) and
// the correction (4.11) in (E_J, O_J) -- have the same structure once the face
// unknowns are eliminated (each face value is an explicit function of its
// neighbouring cell values):
//
//   A X = d_c X_p - g_c sum_q omega_q X_q + k_c div_p O(X)  =  rhs,
//
//   O(X) at an interior face = alpha_f O^n_f - gamma_f (Omega_p . grad X)_f  [+ known part],
//   O(X) at an edge face     = (2 s / eps)(b - fe X_cell) - O(X) at the opposite face,
//
// where the discrete Omega_p . grad at an x-face is the compact x-difference
// plus the mean of the two cells' centred y-differences (one-sided at a wall),
// and the y-faces likewise.  g_c (the angular coupling of (4.5c)) is zero in the
// correction.  The system is solved matrix-free by BiCGStab in binary64 with a
// right preconditioner: the exact inverse of each cell's P x P block (diagonal
// plus the rank-one coupling, by the Sherman-Morrison formula) and, in the
// prediction, an isotropic correction -- an approximate inverse of the operator's
// angular average over isotropic fields (a 5-point diffusion operator) by fixed
// Chebyshev steps or one multigrid V-cycle.  The true residual is recomputed
// from the equations after every pass of iterations and the solve restarted from
// it.  The state between steps may be stored in binary32 (E as its deviation
// from a c T^4); the arithmetic is binary64 throughout.
//
// Data layout (device, binary64): cell-major, pair index fastest:
//   E[(iy*nx + ix)*P + p], Ox[(iy*(nx+1) + fx)*P + p], Oy[(fy*nx + ix)*P + p].
// A thread owns one (cell, pair); the P threads of a cell are adjacent lanes of
// one wavefront (P a power of two <= 64), so angular sums are lane shuffles and
// the stencil reads of a neighbouring cell are one contiguous P*8-byte run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/grte.h"
#include "mlp_common.hpp"
#include "solver_common.hpp"

namespace {

constexpr int B2 = 256;        // threads per block of the (cell, pair) kernels
constexpr int MAXB = 2048;     // blocks of the grid-stride kernels outside the Krylov loop
// the Krylov kernels over the N*P items run KRY_ITEMS items per thread (up to
// KRYB blocks); their per-block partial sums are reduced by one block of
// FIN_T threads, or in two levels (RED_B partials per block of the first
// level, then that block) when there are more than RED_B of them (both figures
// can be set per context; by default every count takes the one level)
constexpr int KRYB = 16384, KRY_ITEMS = 4, RED_B = KRYB;
constexpr int OPC_N = 8;       // doubles per cell of the operator's packed coefficients (opc2d_kernel)
constexpr int CHUNK = 8;       // most BiCGStab iterations enqueued between convergence checks
constexpr int KRY_RESTARTS = 12;     // restarts from the true residual per solve
// a pass of binary32-stored iterations ends once the recursion's residual is
// this fraction of the pass's true starting residual (the recursion and the
// true residual part at the level of binary32 rounding)
constexpr double KRY_PASS_RED = 1e-5;
// binary32 Krylov vectors only where every cell's block inverse amplifies
// rounding by at most 1 / KRY_F32_GAP (its Sherman-Morrison denominator 1 - g
// sum_p omega_p / d_p is at least KRY_F32_GAP; it falls like 1 / (a c beta) in
// stiff cells, where a binary32 direction carries less and less of the
// near-isotropic mode: below ~1e-8 the binary32 solve can diverge (a c beta
// ~ 1e13), just above it it takes more iterations than a binary64 one, each
// cheaper)
constexpr double KRY_F32_GAP = 1e-8;
// the recursion runs on to this fraction of the tolerance before the true
// residual is taken: a restarted binary32 recursion stopped at the tolerance
// itself leaves, on stiff systems whose residual sits at the rounding floor,
// errors in modes with small residuals (E* up to 1e-11 where one binary64
// Krylov space reaches 2e-13 at the same residual)
constexpr double KRY_REC = 0.1;
constexpr double CHEB2_A = 0.01, CHEB2_B = 2.0;   // eigenvalue interval of the Jacobi-scaled isotropic operator
constexpr double KRY_FLOOR = 64.0;   // floor stop: true residual within this factor of its rounding level

// scalars of the Krylov solve, in device memory
enum { S_RHO = 0, S_ALPHA, S_OMEGA, S_BETA, S_RR, S_BB, S_RV, S_TS, S_TT, S_MM, S_R0, S_NS };
enum { F_STATE = 0, F_ITS, F_NF };          // F_STATE: 0 running, 1 converged, 2 breakdown

struct Sys {
    int nx, ny, P, lgP, corr;
    double dx, dy, eps, fe, W1;
    double idx, idy, inx, k2;            // 1/dx, 1/dy, 1/nx, 2/eps
    const double *mu, *eta, *om, *b;     // pairs and inflow b[4*P]
    const double *Ox0, *Oy0;             // O^n
    const double *ax, *gx, *ay, *gy;     // face alpha, gamma (gamma includes fe)
    const double *lam, *dmg, *cg, *kco;  // cell: Lambda, Lambda - g W1, g, K co c dt
    const double *rb1, *rb0, *acU;       // rhs = rb1 E^n_p + rb0; acU (correction's known part)
    const double *sab, *ue;              // residual in difference form (see residual_at)
    const double *pgc;                   // cell: g / (1 - g sum_p omega_p / d_p) of the block inverse
    const double *opc;                   // cell: the operator's coefficients packed, OPC_N per cell (opc2d_kernel)
};

// (iy, ix) of cell j without an integer division: the binary64 product is off
// by at most one for j < 2^31
__device__ __forceinline__ void cell_yx(const Sys &S, int j, int &iy, int &ix)
{
    iy = (int)((double)j * S.inx);
    ix = j - iy * S.nx;
    if (ix < 0) {
        --iy;
        ix += S.nx;
    } else if (ix >= S.nx) {
        ++iy;
        ix -= S.nx;
    }
}

__device__ __forceinline__ double group_sum(double v, int P)
{
    for (int o = P >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double group_lane0(double v, int P)
{
    const int lane = __lane_id();
    return __shfl(v, lane & ~(P - 1), 64);
}

// 3 x 3 neighbourhood of a cell field (indices clamped at the walls)
struct Nb {
    double v[3][3];
};

__device__ __forceinline__ Nb load_nb(const double *x, int nx, int ny, int iy, int ix, int P, int p)
{
    Nb n;
    const int r[3] = {max(iy - 1, 0), iy, min(iy + 1, ny - 1)};
    const int c[3] = {max(ix - 1, 0), ix, min(ix + 1, nx - 1)};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) n.v[a][k] = x[(r[a] * nx + c[k]) * P + p];
    return n;
}

// Omega . grad of a neighbourhood at the cell's four faces (left, right, bottom, top)
struct Grad {
    double l, r, b, t;
};

__device__ __forceinline__ Grad face_grad(const Nb &n, double mu, double eta, const Sys &S, int iy, int ix)
{
    // centred differences, one-sided next to a wall (the clamped neighbourhood
    // turns the centred formula into the one-sided one with the weight 1/h)
    const double wy = (iy == 0 || iy == S.ny - 1) ? S.idy : 0.5 * S.idy;
    const double wx = (ix == 0 || ix == S.nx - 1) ? S.idx : 0.5 * S.idx;
    double dy[3], dx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dy[k] = (n.v[2][k] - n.v[0][k]) * wy;
        dx[k] = (n.v[k][2] - n.v[k][0]) * wx;
    }
    Grad g;
    g.l = mu * (n.v[1][1] - n.v[1][0]) * S.idx + eta * 0.5 * (dy[0] + dy[1]);
    g.r = mu * (n.v[1][2] - n.v[1][1]) * S.idx + eta * 0.5 * (dy[1] + dy[2]);
    g.b = eta * (n.v[1][1] - n.v[0][1]) * S.idy + mu * 0.5 * (dx[0] + dx[1]);
    g.t = eta * (n.v[2][1] - n.v[1][1]) * S.idy + mu * 0.5 * (dx[1] + dx[2]);
    return g;
}

// Face values of O at the cell's four faces.  KNOWN: the part independent of X
// (O^n, the inflow data and, in the correction, a c U^{n+1}); LIN: the part linear
// in X (a neighbourhood of X for this pair).
template <bool KNOWN, bool LIN>
__device__ __forceinline__ void faces(const Sys &S, int iy, int ix, int p, const Nb *X, Grad &O)
{
    const int nx = S.nx, ny = S.ny, P = S.P;
    const double mu = S.mu[p], eta = S.eta[p];
    const int fl = iy * (nx + 1) + ix, fb = iy * nx + ix;
    const int fr = fl + 1, ft = fb + nx;
    O.l = O.r = O.b = O.t = 0.0;
    if (LIN) {
        const Grad g = face_grad(*X, mu, eta, S, iy, ix);
        O.l = -S.gx[fl] * g.l;
        O.r = -S.gx[fr] * g.r;
        O.b = -S.gy[fb] * g.b;
        O.t = -S.gy[ft] * g.t;
    }
    double uc = 0.0;
    if (KNOWN) {
        O.l += S.ax[fl] * S.Ox0[fl * P + p];
        O.r += S.ax[fr] * S.Ox0[fr * P + p];
        O.b += S.ay[fb] * S.Oy0[fb * P + p];
        O.t += S.ay[ft] * S.Oy0[ft * P + p];
        if (S.corr) {
            const Nb U = load_nb(S.acU, nx, ny, iy, ix, 1, 0);
            const Grad g = face_grad(U, mu, eta, S, iy, ix);
            const double ife = 1.0 / S.fe;
            O.l -= S.gx[fl] * ife * g.l;
            O.r -= S.gx[fr] * ife * g.r;
            O.b -= S.gy[fb] * ife * g.b;
            O.t -= S.gy[ft] * ife * g.t;
            uc = U.v[1][1];
        }
    }
    // inflow relations: E_cell + s (eps/2)(O_edge + O_opposite) = b, s = +1 when
    // +Omega_p enters through that edge
    const double xc = LIN ? X->v[1][1] : 0.0;
    const double k2 = S.k2;
    // (the difference inflow - cell value is formed first: both terms carry 2/eps)
    auto edge = [&](int e, double s) {
        double d = 0.0;
        if (KNOWN && LIN) d = (S.b[e * P + p] - uc) - S.fe * xc;
        else if (KNOWN) d = S.b[e * P + p] - uc;
        else d = -S.fe * xc;
        return s * k2 * d;
    };
    const double sx = mu > 0.0 ? 1.0 : -1.0, sy = eta > 0.0 ? 1.0 : -1.0;
    if (ix == 0) O.l = edge(0, sx) - O.r;
    if (ix == nx - 1) O.r = edge(1, -sx) - O.l;
    if (iy == 0) O.b = edge(2, sy) - O.t;
    if (iy == ny - 1) O.t = edge(3, -sy) - O.b;
}

__device__ __forceinline__ double divergence(const Sys &S, const Grad &O, int p)
{
    return S.mu[p] * (O.r - O.l) * S.idx + S.eta[p] * (O.t - O.b) * S.idy;
}

// ---------------------------------------------------------------------------
// per-step coefficients
// ---------------------------------------------------------------------------
struct CoefArgs {
    int nx, ny, m, corr;
    double a, c, cv, eps, dt, fe, W1;
    const double *T, *sigma0;
    double *ax, *gx, *ay, *gy, *lam, *dmg, *cg, *kco, *rb0, *rb1, *acU, *beta, *sab, *ue;
};


__device__ __forceinline__ double harm(double a, double b)
{
    const double s = a + b;
    return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

__global__ void __launch_bounds__(B2) coef2d_kernel(CoefArgs A)
{
    const int n = A.nx * A.ny;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        const int iy = j / A.nx, ix = j - iy * A.nx;
        const double T = A.T[j], s0 = A.sigma0[j];
        const double K = kpow(T, A.m);
        const double e2 = A.eps * A.eps, cdt = A.c * A.dt, ac = A.a * A.c;
        const double U = T * T * T * T;
        const double lam = K * e2 + s0 * cdt;
        A.lam[j] = lam;
        if (!A.corr) {
            // (4.5c): U* = (U^n + beta rho*)/(1 + ac beta), substituted into (4.5b)
            const double beta = 4.0 * s0 * A.dt * (A.m == 0 ? T * T * T : 1.0) / (e2 * A.cv);
            const double g = s0 * cdt * ac * beta / (1.0 + ac * beta);
            A.beta[j] = beta;
            A.cg[j] = g;
            // Lambda - g W1 formed directly: K eps^2 + sigma0 c dt / (1 + ac beta) + g (1 - W1)
            A.dmg[j] = K * e2 + s0 * cdt / (1.0 + ac * beta) + g * (1.0 - A.W1);
            A.kco[j] = K * e2 * cdt;
            A.rb1[j] = K * e2;
            A.rb0[j] = s0 * cdt * ac * U / (1.0 + ac * beta);
            A.sab[j] = s0 * cdt / (1.0 + ac * beta);
            A.ue[j] = ac * U;
        } else {
            A.cg[j] = 0.0;
            A.dmg[j] = lam;
            A.kco[j] = K * A.eps * cdt;
            A.rb1[j] = K * A.eps;
            A.rb0[j] = -K * A.eps * ac * U;
            A.acU[j] = ac * U;
            A.sab[j] = s0 * cdt;
            A.ue[j] = ac * U;
        }
        // faces owned by this cell: its left x-face and bottom y-face (interior ones)
        auto face = [&](int jn, double &alpha, double &gamma) {
            const double Kf = 0.5 * (K + kpow(A.T[jn], A.m));
            const double sf = harm(s0, A.sigma0[jn]);
            const double den = Kf * e2 + sf * cdt;
            alpha = Kf * e2 / den;
            gamma = Kf * cdt * A.fe / den;
        };
        const size_t fl = (size_t)iy * (A.nx + 1) + ix, fb = (size_t)iy * A.nx + ix;
        double al = 0.0, gl = 0.0, ab = 0.0, gb = 0.0;
        if (ix > 0) face(j - 1, al, gl);
        if (iy > 0) face(j - A.nx, ab, gb);
        A.ax[fl] = al;
        A.gx[fl] = gl;
        A.ay[fb] = ab;
        A.gy[fb] = gb;
        if (ix == A.nx - 1) A.ax[fl + 1] = A.gx[fl + 1] = 0.0;
        if (iy == A.ny - 1) A.ay[fb + A.nx] = A.gy[fb + A.nx] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// right-hand side, residual, operator
// ---------------------------------------------------------------------------
struct VecArgs {
    Sys S;
    size_t n;                  // N * P
    const double *En;          // E^n (rhs)
    double *bv, *x;            // right-hand side, iterate (binary64)
    // the Krylov vectors and the block inverse's 1/d_p, stored in binary32 or
    // binary64 (the kernels' template type V; the arithmetic is binary64): a
    // pass of iterations ends when the recursion has reduced the residual by
    // KRY_PASS_RED, and the next starts from the binary64 true residual
    void *r, *p, *ph, *v, *s, *sh, *t;
    void *dx;                  // the pass's correction of x (added to x when the pass ends)
    const void *idg;
    double pass_red, rec;      // a pass ends at pass_red x its start, or at rec x tol
    double *part;              // [k * KRYB + block]
    double *part2;             // [k * KRYB + block] (first reduction level)
    int red_b;                 // partials per block of the first reduction level
    double *sc;                // scalars
    int *fl;                   // flags
    double tol;
    int maxit;
    // isotropic (diffusion) correction of the preconditioner (null: none): the
    // preconditioned vectors are B^{-1} p + dP[cell] and B^{-1} s + dS[cell], dP and
    // dS the correction applied to yP = sum_p omega_p p_p and yS = sum_p omega_p s_p.
    // yP and yS are formed per cell from the moments mr = sum_p omega_p r_p and
    // mv = sum_p omega_p v_p, which the kernels producing r and v also write
    // (p = r + beta (p - omega v), s = r - alpha v are linear), so that the
    // correction can be solved before the update that adds it
    const double *dP, *dS;
    double *yP, *yS, *mr, *mv;
};

__device__ __forceinline__ void block_sums(double *vals, int k, double *part)
{
    __shared__ double red[4][B2 / 64];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    for (int q = 0; q < k; ++q) {
        double v = vals[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[q][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < k) {
        double v = 0.0;
        for (int i = 0; i < B2 / 64; ++i) v += red[threadIdx.x][i];
        part[threadIdx.x * KRYB + blockIdx.x] = v;
    }
}

// the shadow vector of BiCGStab: a fixed pseudo-random value in [-1, 1) per
// item (the splitmix64 output function of the item index), computed where used
__device__ __forceinline__ double shadow(int t)
{
    unsigned long long z = (unsigned long long)(unsigned)t + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-52 - 1.0;
}

// rhs: rb1 E^n_p + rb0 - k div O(known)   (rb1 = K eps^2 prediction, K eps correction)
__global__ void __launch_bounds__(B2) rhs2d_kernel(VecArgs A)
{
    const Sys &S = A.S;
    const int P = S.P;
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)A.n; t += gridDim.x * B2) {
        const int j = t >> S.lgP, p = t & (P - 1);
        int iy, ix;
        cell_yx(S, j, iy, ix);
        Grad O;
        faces<true, false>(S, iy, ix, p, nullptr, O);
        A.bv[t] = S.rb1[j] * A.En[t] + S.rb0[j] - S.kco[j] * divergence(S, O, p);
    }
}

// b - A x evaluated from the full face values and differences of nearly equal
// quantities (E^n - x, a c U - x), so that its rounding stays at the level of the
// residual itself rather than of the large terms that cancel in it (the inflow
// relations carry 2/eps times the inflow and the cell value):
//   prediction  K eps^2 (E^n_p - x_p) + s (a c U^n - x_p) - g (1 - W1) x_p
//               - g (W1 x_p - sum_q omega_q x_q) - k div O(x),   s = sigma0 c dt / (1 + ac beta)
//   correction  K eps (E^n_p - a c U - eps x_p) - sigma0 c dt x_p - k div O(x)
__device__ __forceinline__ double residual_at(const Sys &S, const double *En, const double *x, int t, int j,
                                              int p, double &mag)
{
    const int P = S.P;
    int iy, ix;
    cell_yx(S, j, iy, ix);
    const Nb X = load_nb(x, S.nx, S.ny, iy, ix, P, p);
    Grad O;
    faces<true, true>(S, iy, ix, p, &X, O);
    const double xp = X.v[1][1];
    const double mu = S.mu[p], eta = S.eta[p];
    const double k = S.kco[j];
    const double div = k * divergence(S, O, p);
    // mag: an upper estimate of (|A| |x| + |b|) for this row -- the scale of the
    // rounding a binary64 iterate and its residual cannot avoid (normwise
    // backward error): the face terms bounded by the largest |x| of the
    // neighbourhood, the inflow and O^n terms by their magnitudes
    double xm = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) xm = fmax(xm, fabs(X.v[a][c]));
    const int fl = iy * (S.nx + 1) + ix, fb = iy * S.nx + ix;
    const double gsum = S.gx[fl] + S.gx[fl + 1] + S.gy[fb] + S.gy[fb + S.nx];
    const double grad_bound = 2.0 * (fabs(mu) * S.idx + fabs(eta) * S.idy) * xm;
    const double k2 = S.k2;
    const double edge_bound = ((ix == 0 || ix == S.nx - 1) + (iy == 0 || iy == S.ny - 1)) * k2 *
                              (4.0 * S.fe * xm + fabs(S.ue[j]));
    const double dmag = fabs(k) * (fabs(mu) * S.idx + fabs(eta) * S.idy) *
                        (fabs(O.l) + fabs(O.r) + fabs(O.b) + fabs(O.t) + gsum * grad_bound + edge_bound);
    if (S.corr) {
        const double a1 = S.rb1[j] * ((En[t] - S.ue[j]) - S.eps * xp), a2 = S.sab[j] * xp;
        mag = fabs(S.rb1[j]) * (fabs(En[t]) + fabs(S.ue[j]) + S.eps * fabs(xp)) + fabs(a2) + dmag;
        return a1 - a2 - div;
    }
    const double xr = group_lane0(xp, P);
    const double w = S.om[p];
    const double cpl = S.W1 * (xp - xr) - group_sum(w * (xp - xr), P);
    const double g = S.cg[j];
    mag = fabs(S.rb1[j]) * (fabs(En[t]) + fabs(xp)) + S.sab[j] * (fabs(S.ue[j]) + fabs(xp)) +
          fabs(g) * (S.W1 * fabs(xp) + group_sum(w * fabs(xp), P)) + dmag;
    return S.rb1[j] * (En[t] - xp) + S.sab[j] * (S.ue[j] - xp) - g * (1.0 - S.W1) * xp - g * cpl - div;
}

// r = b - A x (the pass's starting residual, stored as V), partial (r, r)
// of the binary64 residual, (b, b), the backward-error scale and (h, r)
// (h: the shadow vector)
template <class V>
__global__ void __launch_bounds__(B2) residual2d_kernel(VecArgs A)
{
    const Sys &S = A.S;
    const int P = S.P;
    V *r = (V *)A.r;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)A.n; t += gridDim.x * B2) {
        const int j = t >> A.S.lgP, p = t & (P - 1);
        double mag;
        const double rr = residual_at(S, A.En, A.x, t, j, p, mag);
        const V rf = (V)rr;
        r[t] = rf;
        if (A.mr) {
            const double m = group_sum(S.om[p] * (double)rf, P);
            if (p == 0) A.mr[j] = m;
        }
        acc[0] += rr * rr;
        acc[1] += A.bv[t] * A.bv[t];
        acc[2] += mag * mag;
        acc[3] += shadow(t) * (double)rf;
    }
    block_sums(acc, 4, A.part);
}

// The operator products of the iteration by columns: the grid is cut into tiles
// of (B2 / P) cells across by OP_ROWS cells down; thread (cell c, pair p) of a
// tile walks down its column keeping the 3 x 3 neighbourhood of its pair in
// registers, so that a row costs three new loads of x instead of nine and the
// shared face coefficient of two rows one, and it loads the next row's values
// and coefficients before it computes the current row (their latency overlaps
// the arithmetic).  Per (cell, pair): y = (Lambda - g W1) x_p + g (W1 x_p -
// sum_q omega_q x_q) + k div O(x) with O(x) the part of faces() linear in x (the
// coupling referred to the cell's first pair, exact for a nearly isotropic x).
// A block takes tiles blockIdx.x, + gridDim.x, ...; its partial sums go to
// part[k * KRYB + blockIdx.x].  The products are stored as V.
// MODE 1: v = A ph, partial (h, v) and, with the isotropic correction, the moment
// of v;  MODE 2: t = A sh, partial (t, s), (t, t)
constexpr int OP_ROWS = 16;

__device__ __forceinline__ void block_sums_at(double *vals, int k, double *part, int bid)
{
    __shared__ double red[4][B2 / 64];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    for (int q = 0; q < k; ++q) {
        double v = vals[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[q][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < k) {
        double v = 0.0;
        for (int i = 0; i < B2 / 64; ++i) v += red[threadIdx.x][i];
        part[threadIdx.x * KRYB + bid] = v;
    }
}

template <int MODE, class V>
__global__ void __launch_bounds__(B2, 5) apply2d_col_kernel(VecArgs A, int ncol, int ntile)
{
    if (A.fl[F_STATE] != 0) return;
    const Sys &S = A.S;
    const int P = S.P, lgP = S.lgP, nx = S.nx, ny = S.ny;
    const int c = threadIdx.x >> lgP, p = threadIdx.x & (P - 1);
    const int cw = B2 >> lgP, rs = nx * P;
    const V *xv = (const V *)(MODE == 1 ? A.ph : A.sh);
    const V *sa = (const V *)A.s;
    V *out = (V *)(MODE == 1 ? A.v : A.t);
    const double mu = S.mu[p], eta = S.eta[p], w = S.om[p];
    const double sx = mu > 0.0 ? 1.0 : -1.0, sy = eta > 0.0 ? 1.0 : -1.0;
    double acc[2] = {0.0, 0.0};
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int ty = tile / ncol, tx = tile - ty * ncol;
        const int ix = tx * cw + c;
        if (ix >= nx) continue;                 // whole cells: a cell's P lanes agree
        const int iy0 = ty * OP_ROWS, iy1 = min(iy0 + OP_ROWS, ny);
        const int o0 = max(ix - 1, 0) * P + p, o1 = ix * P + p, o2 = min(ix + 1, nx - 1) * P + p;
        auto ldrow = [&](int row, double(&v)[3]) {
            const V *q = xv + row * rs;
            v[0] = q[o0];
            v[1] = q[o1];
            v[2] = q[o2];
        };
        Nb X;
        ldrow(max(iy0 - 1, 0), X.v[0]);
        ldrow(iy0, X.v[1]);
        ldrow(min(iy0 + 1, ny - 1), X.v[2]);
        int j = iy0 * nx + ix;
        auto ldc = [&](int jj, double2(&c)[4]) {
            const double2 *q = (const double2 *)(S.opc + (size_t)OPC_N * jj);
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = q[k];
        };
        double2 cf[4];
        ldc(j, cf);
        double sv = MODE == 2 ? (double)sa[j * P + p] : 0.0;
        for (int iy = iy0; iy < iy1; ++iy) {
            // the next row's loads (row indices clamped in range; unused after
            // the tile's last row)
            const int yn = min(iy + 1, ny - 1), jn = yn * nx + ix;
            double xn[3];
            ldrow(min(iy + 2, ny - 1), xn);
            double2 cfn[4];
            ldc(jn, cfn);
            const double svn = MODE == 2 ? (double)sa[jn * P + p] : 0.0;
            // row iy: faces<false, true> with the coefficients in registers
            const double dm = cf[0].x, cgv = cf[0].y, kc = cf[1].x;
            const Grad g = face_grad(X, mu, eta, S, iy, ix);
            Grad O;
            O.l = -cf[2].x * g.l;
            O.r = -cf[2].y * g.r;
            O.b = -cf[3].x * g.b;
            O.t = -cf[3].y * g.t;
            const double xp = X.v[1][1];
            const double k2 = S.k2;
            auto edge = [&](double sg) {
                const double d = -S.fe * xp;
                return sg * k2 * d;
            };
            if (ix == 0) O.l = edge(sx) - O.r;
            if (ix == nx - 1) O.r = edge(-sx) - O.l;
            if (iy == 0) O.b = edge(sy) - O.t;
            if (iy == ny - 1) O.t = edge(-sy) - O.b;
            const double div = mu * (O.r - O.l) * S.idx + eta * (O.t - O.b) * S.idy;
            double y;
            if (S.corr) {
                y = dm * xp + kc * div;             // no angular coupling (g = 0)
            } else {
                const double xr = group_lane0(xp, P);
                const double cpl = S.W1 * (xp - xr) - group_sum(w * (xp - xr), P);
                y = dm * xp + cgv * cpl + kc * div;
            }
            const int t = j * P + p;
            const double yf = (double)(V)y;         // the stored product
            out[t] = (V)y;
            if (MODE == 1) {
                if (A.mv) {
                    const double m = group_sum(w * yf, P);
                    if (p == 0) A.mv[j] = m;
                }
                acc[0] += shadow(t) * yf;
            } else {
                acc[0] += yf * sv;
                acc[1] += yf * yf;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                X.v[0][k] = X.v[1][k];
                X.v[1][k] = X.v[2][k];
                X.v[2][k] = xn[k];
            }
            j = jn;
#pragma unroll
            for (int k = 0; k < 4; ++k) cf[k] = cfn[k];
            sv = svn;
        }
    }
    block_sums_at(acc, MODE == 1 ? 1 : 2, A.part, blockIdx.x);
}

// 1 / d_p: the inverse of the direction-diagonal part of a cell's block
__device__ __forceinline__ double block_idiag(const Sys &S, int j, int p)
{
    int iy, ix;
    cell_yx(S, j, iy, ix);
    const double mu = S.mu[p], eta = S.eta[p];
    const double mx = mu * mu * S.idx * S.idx, my = eta * eta * S.idy * S.idy;
    const int fl = iy * (S.nx + 1) + ix, fb = iy * S.nx + ix;
    const double gl = S.gx[fl], gr = S.gx[fl + 1], gb = S.gy[fb], gt = S.gy[fb + S.nx];
    // diagonal of k div O(X) with respect to X_cell (the compact terms; an edge
    // face doubles the opposite face and adds the inflow term 2|Omega_n| fe/(eps h))
    double tr = 0.0;
    const double k2 = S.k2 * S.fe;
    if (ix == 0) tr += 2.0 * gr * mx + k2 * fabs(mu) * S.idx;
    else if (ix == S.nx - 1) tr += 2.0 * gl * mx + k2 * fabs(mu) * S.idx;
    else tr += (gl + gr) * mx;
    if (iy == 0) tr += 2.0 * gt * my + k2 * fabs(eta) * S.idy;
    else if (iy == S.ny - 1) tr += 2.0 * gb * my + k2 * fabs(eta) * S.idy;
    else tr += (gb + gt) * my;
    return 1.0 / (S.lam[j] + S.kco[j] * tr);
}

// the system-dependent parts of each cell's block inverse, once per solve:
// 1 / d_p for every (cell, pair) and, with angular coupling (the prediction),
// the Sherman-Morrison scalar g / (1 - g sum_p omega_p / d_p) of the cell
// (1/d_p in binary64 and binary32; *narrow cleared where a cell's denominator
// is below KRY_F32_GAP)
__global__ void __launch_bounds__(B2) pgc2d_kernel(Sys S, double *idg, float *idg32, double *pgc, int *narrow,
                                                   size_t n)
{
    const int P = S.P;
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)n; t += gridDim.x * B2) {
        const int j = t >> S.lgP, p = t & (P - 1);
        const double id = block_idiag(S, j, p);
        idg[t] = id;
        idg32[t] = (float)id;
        if (S.corr) continue;
        const double s2 = group_sum(S.om[p] * id, P);
        const double g = S.cg[j];
        const double den = 1.0 - g * s2;
        if (p == 0) {
            pgc[j] = g / den;
            if (!(den >= KRY_F32_GAP)) *narrow = 0;
        }
    }
}

__global__ void set_int_kernel(int *a, int v)
{
    if (threadIdx.x == 0) *a = v;
}

// The coefficients the operator products read per cell and row, packed once per
// solve so that a row takes four 16-byte loads instead of six 8-byte ones:
// {Lambda - g W1, g, k, 0, gamma of the left, right, bottom and top faces}

__global__ void __launch_bounds__(B2) opc2d_kernel(Sys S, double *opc)
{
    const int n = S.nx * S.ny;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        int iy, ix;
        cell_yx(S, j, iy, ix);
        const int fl = j + iy;
        double2 *q = (double2 *)(opc + (size_t)OPC_N * j);
        q[0] = make_double2(S.dmg[j], S.cg[j]);
        q[1] = make_double2(S.kco[j], 0.0);
        q[2] = make_double2(S.gx[fl], S.gx[fl + 1]);
        q[3] = make_double2(S.gy[j], S.gy[j + S.nx]);
    }
}

// cell-block Jacobi: z = B^{-1} y, B = diag(d_p) - g 1 omega^T (Sherman-Morrison);
// the correction's blocks have g = 0 and are diagonal
// (id = 1/d_p of the item, pg = the cell's g / (1 - g sum_p omega_p / d_p),
// wp = omega_p)
__device__ __forceinline__ double precond_at(const Sys &S, double y, double id, double pg, double wp)
{
    const double u = y * id;
    if (S.corr) return u;
    const double s1 = group_sum(wp * u, S.P);
    return u + pg * s1 * id;
}

// The vector updates take KI items per thread and loop trip (items t, t + G,
// t + 2G, ... for a grid of G threads, the order of the grid-stride loop they
// replace): every load of a trip is issued before its arithmetic and stores,
// through restrict-qualified pointers, so that one wave keeps several
// independent loads in flight.  Items past the end read item t (always in
// range) and store nothing; a cell's P lanes are in or out together, so the
// angular sums stay within whole cells.
constexpr int KI = 4;

// p = r + beta (p - omega v), p = r in the first iteration of a pass (p and v
// are not read then: they hold the last pass's vectors); ph = B^{-1} p (+ dP)
template <class V>
__global__ void __launch_bounds__(B2) pupd2d_kernel(VecArgs A)
{
    if (A.fl[F_STATE] != 0) return;
    const bool first = A.fl[F_ITS] == 0;
    const double beta = A.sc[S_BETA], omega = A.sc[S_OMEGA];
    const int P = A.S.P, lgP = A.S.lgP, n = (int)A.n, G = gridDim.x * B2;
    const V *__restrict__ r = (const V *)A.r;
    const V *__restrict__ v = (const V *)A.v;
    const V *__restrict__ idg = (const V *)A.idg;
    V *__restrict__ pp = (V *)A.p;
    V *__restrict__ ph = (V *)A.ph;
    const double *__restrict__ dP = A.dP;
    const double *__restrict__ pgc = A.S.pgc;
    // the pair of every item of this thread (G is a multiple of P)
    const double wp = A.S.om[(blockIdx.x * B2 + threadIdx.x) & (P - 1)];
    for (int t0 = blockIdx.x * B2 + threadIdx.x; t0 < n; t0 += KI * G) {
        double rv[KI], pv[KI], vv[KI], id[KI], dd[KI], pg[KI];
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int t = t0 + k * G < n ? t0 + k * G : t0;
            rv[k] = r[t];
            pv[k] = first ? 0.0 : (double)pp[t];
            vv[k] = first ? 0.0 : (double)v[t];
            id[k] = idg[t];
            dd[k] = dP ? dP[t >> lgP] : 0.0;
            pg[k] = A.S.corr ? 0.0 : pgc[t >> lgP];
        }
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int t = t0 + k * G;
            if (t >= n) break;
            const V pn = first ? (V)rv[k] : (V)(rv[k] + beta * (pv[k] - omega * vv[k]));
            pp[t] = pn;
            ph[t] = (V)(precond_at(A.S, pn, id[k], pg[k], wp) + dd[k]);
        }
    }
}

// s = r - alpha v; sh = B^{-1} s (+ dS)
template <class V>
__global__ void __launch_bounds__(B2) supd2d_kernel(VecArgs A)
{
    if (A.fl[F_STATE] != 0) return;
    const double alpha = A.sc[S_ALPHA];
    const int P = A.S.P, lgP = A.S.lgP, n = (int)A.n, G = gridDim.x * B2;
    const V *__restrict__ r = (const V *)A.r;
    const V *__restrict__ v = (const V *)A.v;
    const V *__restrict__ idg = (const V *)A.idg;
    V *__restrict__ sa = (V *)A.s;
    V *__restrict__ sh = (V *)A.sh;
    const double *__restrict__ dS = A.dS;
    const double *__restrict__ pgc = A.S.pgc;
    // the pair of every item of this thread (G is a multiple of P)
    const double wp = A.S.om[(blockIdx.x * B2 + threadIdx.x) & (P - 1)];
    for (int t0 = blockIdx.x * B2 + threadIdx.x; t0 < n; t0 += KI * G) {
        double rv[KI], vv[KI], id[KI], dd[KI], pg[KI];
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int t = t0 + k * G < n ? t0 + k * G : t0;
            rv[k] = r[t];
            vv[k] = v[t];
            id[k] = idg[t];
            dd[k] = dS ? dS[t >> lgP] : 0.0;
            pg[k] = A.S.corr ? 0.0 : pgc[t >> lgP];
        }
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int t = t0 + k * G;
            if (t >= n) break;
            const V sv = (V)(rv[k] - alpha * vv[k]);
            sa[t] = sv;
            sh[t] = (V)(precond_at(A.S, sv, id[k], pg[k], wp) + dd[k]);
        }
    }
}

// the isotropic correction's inputs from the moments:
// which 0: yP = mr + beta (yP - omega mv) (yP holds the last direction's moment);
// which 1: yS = mr - alpha mv
__global__ void __launch_bounds__(B2) ymom2d_kernel(VecArgs A, int which, int n)
{
    if (A.fl[F_STATE] != 0) return;
    const double alpha = A.sc[S_ALPHA], beta = A.sc[S_BETA], omega = A.sc[S_OMEGA];
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        if (which == 0) A.yP[j] = A.mr[j] + beta * (A.yP[j] - omega * A.mv[j]);
        else A.yS[j] = A.mr[j] - alpha * A.mv[j];
    }
}

// dx += alpha ph + omega sh (the pass's correction of x, stored as V and added
// to the binary64 x when the pass ends; dx = alpha ph + omega sh in the first
// iteration of a pass, the last pass's dx not read); r = s - omega t (and its
// moment); partial (h, r), (r, r)
template <class V>
__global__ void __launch_bounds__(B2) xupd2d_kernel(VecArgs A)
{
    if (A.fl[F_STATE] != 0) return;
    const bool first = A.fl[F_ITS] == 0;
    const double alpha = A.sc[S_ALPHA], omega = A.sc[S_OMEGA];
    const int P = A.S.P, lgP = A.S.lgP, n = (int)A.n, G = gridDim.x * B2;
    const V *__restrict__ ph = (const V *)A.ph;
    const V *__restrict__ sh = (const V *)A.sh;
    const V *__restrict__ sa = (const V *)A.s;
    const V *__restrict__ ta = (const V *)A.t;
    V *__restrict__ r = (V *)A.r;
    V *__restrict__ dx = (V *)A.dx;
    double acc[2] = {0.0, 0.0};
    // the pair of every item of this thread (G is a multiple of P)
    const double wp = A.S.om[(blockIdx.x * B2 + threadIdx.x) & (P - 1)];
    for (int t0 = blockIdx.x * B2 + threadIdx.x; t0 < n; t0 += KI * G) {
        double xv[KI], pv[KI], hv[KI], sv[KI], tv[KI];
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int t = t0 + k * G < n ? t0 + k * G : t0;
            xv[k] = first ? 0.0 : (double)dx[t];
            pv[k] = ph[t];
            hv[k] = sh[t];
            sv[k] = sa[t];
            tv[k] = ta[t];
        }
#pragma unroll
        for (int k = 0; k < KI; ++k) {
            const int t = t0 + k * G;
            if (t >= n) break;
            const int j = t >> lgP, p = t & (P - 1);
            dx[t] = first ? (V)(alpha * pv[k] + omega * hv[k]) : (V)(xv[k] + (alpha * pv[k] + omega * hv[k]));
            const V rs = (V)(sv[k] - omega * tv[k]);
            r[t] = rs;
            const double rv = rs;
            if (A.mr) {
                const double m = group_sum(wp * rv, P);
                if (p == 0) A.mr[j] = m;
            }
            acc[0] += shadow(t) * rv;
            acc[1] += rv * rv;
        }
    }
    block_sums(acc, 2, A.part);
}

// ---------------------------------------------------------------------------
// isotropic correction of the preconditioner: D z = y with D the operator's
// angular average on isotropic fields (sum_p omega_p A_p applied to 1 z; the
// angular coupling cancels on them), a 5-point diffusion operator
//   D z_c = W1 (Lambda - g W1)_c z_c + k_c [ sum_faces M h^-2 gamma_f (z_c - z_nb) (x2 next to an edge)
//                                           + edge cells: 2 fe S / (eps h) z_c ],
// M = sum_p omega_p mu_p^2 (x-faces) or eta_p^2 (y-faces), S = sum_p omega_p |mu_p| or |eta_p|
// (the mixed moment sum_p omega_p mu_p eta_p vanishes for direction sets symmetric
// under x -> -x, as the equally spaced one is, and is not carried).  Solved
// approximately by a fixed number of Chebyshev steps on the Jacobi-scaled
// operator over the eigenvalue interval [CHEB2_A, CHEB2_B]: a fixed linear map,
// as the Krylov method requires of its preconditioner.
// ---------------------------------------------------------------------------
struct IsoArgs {
    Sys S;
    double Mxx, Myy, Sx, Sy;
    const double *y;
    const double *xin;
    double *xout, *d;
    double c1, c2, th;
    const int *fl;
};

// the four face values around a cell (left, right, bottom, top)
struct Faces {
    double l, r, b, t;
};

// a cell's faces in the isotropic operator's form: at a wall the face on the
// far side counts twice and the wall face drops out
__device__ __forceinline__ Faces iso_walls(const Sys &S, int iy, int ix, Faces g)
{
    if (ix == 0) { g.r *= 2.0; g.l = 0.0; }
    else if (ix == S.nx - 1) { g.l *= 2.0; g.r = 0.0; }
    if (iy == 0) { g.t *= 2.0; g.b = 0.0; }
    else if (iy == S.ny - 1) { g.b *= 2.0; g.t = 0.0; }
    return g;
}

// the diagonal of a cell's row (wall-form faces g; a wall adds the inflow term)
__device__ __forceinline__ double iso_diag(const IsoArgs &A, int iy, int ix, int j, const Faces &g)
{
    const Sys &S = A.S;
    const double k = S.kco[j];
    const double cx = A.Mxx * S.idx * S.idx, cy = A.Myy * S.idy * S.idy;
    double ed = 0.0;
    const double e2 = S.k2 * S.fe;
    if (ix == 0 || ix == S.nx - 1) ed += e2 * A.Sx * S.idx;
    if (iy == 0 || iy == S.ny - 1) ed += e2 * A.Sy * S.idy;
    return S.W1 * S.dmg[j] + k * (cx * (g.l + g.r) + cy * (g.b + g.t) + ed);
}

// A cell's Jacobi-scaled row: the Chebyshev steps need r = (y - D x) / diag,
// formed as y / diag - x_c + sum_nb w_nb x_nb with w_nb = k c g_nb / diag
// (c = M h^-2 of the face's direction; 0 beyond a wall), the weights held per
// cell for all of a launch's steps
struct IsoRow {
    double diag, rdg, wl, wr, wb, wt;
};

__device__ __forceinline__ IsoRow iso_row_coefs(const IsoArgs &A, int iy, int ix, int j, double gl, double gr,
                                                double gb, double gt)
{
    const Sys &S = A.S;
    const Faces g = iso_walls(S, iy, ix, Faces{gl, gr, gb, gt});
    IsoRow R;
    R.diag = iso_diag(A, iy, ix, j, g);
    R.rdg = 1.0 / R.diag;
    const double k = S.kco[j];
    const double cx = A.Mxx * S.idx * S.idx, cy = A.Myy * S.idy * S.idy;
    R.wl = k * cx * g.l * R.rdg;
    R.wr = k * cx * g.r * R.rdg;
    R.wb = k * cy * g.b * R.rdg;
    R.wt = k * cy * g.t * R.rdg;
    return R;
}

// (y - D x) / diag from y / diag, the cell's value and its neighbours' (0 beyond a wall)
// (no contraction into fused multiply-adds: the tiled and the per-step kernels
// then round every term alike, whatever the code around them)
__device__ __forceinline__ double iso_jres(double yr, double wl, double wr, double wb, double wt, double xc,
                                           double xl, double xr, double xb, double xt)
{
#pragma clang fp contract(off)
    return (yr - xc) + ((wl * xl + wr * xr) + (wb * xb + wt * xt));
}

__device__ __forceinline__ IsoRow iso_row_at(const IsoArgs &A, int j, int &iy, int &ix)
{
    const Sys &S = A.S;
    cell_yx(S, j, iy, ix);
    const int fl = iy * (S.nx + 1) + ix, fb = iy * S.nx + ix;
    return iso_row_coefs(A, iy, ix, j, S.gx[fl], S.gx[fl + 1], S.gy[fb], S.gy[fb + S.nx]);
}

// first step: x1 = d0 = (y / diag) / theta
__global__ void __launch_bounds__(B2) iso_first_kernel(IsoArgs A)
{
    if (A.fl[F_STATE] != 0) return;
    const int n = A.S.nx * A.S.ny;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        int iy, ix;
        const IsoRow R = iso_row_at(A, j, iy, ix);
        const double d0 = A.y[j] / (R.diag * A.th);
        A.d[j] = d0;
        A.xout[j] = d0;
    }
}

// later steps: r = (y - D x)/diag; d = c1 d + c2 r; x_out = x + d
__global__ void __launch_bounds__(B2) iso_step_kernel(IsoArgs A)
{
    if (A.fl[F_STATE] != 0) return;
    const Sys &S = A.S;
    const int n = S.nx * S.ny;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        int iy, ix;
        const IsoRow R = iso_row_at(A, j, iy, ix);
        const double *x = A.xin;
        const double xc = x[j];
        const double xl = ix > 0 ? x[j - 1] : 0.0, xr = ix < S.nx - 1 ? x[j + 1] : 0.0;
        const double xb = iy > 0 ? x[j - S.nx] : 0.0, xt = iy < S.ny - 1 ? x[j + S.nx] : 0.0;
        const double r = iso_jres(A.y[j] * R.rdg, R.wl, R.wr, R.wb, R.wt, xc, xl, xr, xb, xt);
        const double dn = A.c1 * A.d[j] + A.c2 * r;
        A.d[j] = dn;
        A.xout[j] = xc + dn;
    }
}

// Up to ISO_HALO stencil steps of the Chebyshev map in one launch, preceded
// by the local first step (first = 1) or continuing from a stored iterate and
// direction.  A block owns a tile of ISO_T x ISO_T cells and works on the tile
// plus a halo of as many cells as it takes stencil steps: the iterate sits in
// LDS, each cell's own values (its Jacobi-scaled row, y / diag, the Chebyshev
// direction) in registers.  Stencil step s updates the region cells
// at least s + 1 cells inside its border (their neighbours hold step-s
// values), so after the launch's steps the tile's cells are exact; cells
// outside the grid are never read (their neighbours' weights are zero and
// their values taken as 0, as in the per-step form).  The arithmetic is the
// per-step kernels' own, term for term, so the result is the same to the bit.
constexpr int ISO_T = 32, ISO_HALO = 9, ISO_RMAX = ISO_T + 2 * ISO_HALO, ISO_TB = 1024;
constexpr int ISO_CPT = (ISO_RMAX * ISO_RMAX + ISO_TB - 1) / ISO_TB;

struct IsoFused {
    IsoArgs A;                  // A.xin: the iterate to continue from (first = 0); A.xout: the result
    int first;                  // 1: start with the local first step from A.y
    int nsteps;                 // stencil steps of this launch, 0 .. ISO_HALO
    const double *din;          // the direction to continue from (first = 0)
    double *dout;               // the direction after the launch (null: not kept)
    double c1[ISO_HALO], c2[ISO_HALO];
};

__global__ void __launch_bounds__(ISO_TB, 8) iso_fused_kernel(IsoFused F)
{
    const IsoArgs &A = F.A;
    if (A.fl[F_STATE] != 0) return;
    const Sys &S = A.S;
    const int h = F.nsteps, R = ISO_T + 2 * h;
    const int ox = blockIdx.x * ISO_T - h, oy = blockIdx.y * ISO_T - h;   // grid position of region cell (0, 0)
    __shared__ double X[ISO_RMAX * ISO_RMAX];
    const int t = threadIdx.x;
    // per cell: its Jacobi-scaled row and y / diag in registers, and its region
    // position packed as rx | ry << 8 | (depth + 1) << 16, depth = distance to
    // the region's border (-1: outside the region or the grid), so that stencil
    // step s updates the cells of depth > s and the tile is the cells of depth >= h
    double yr[ISO_CPT], wl[ISO_CPT], wr[ISO_CPT], wb[ISO_CPT], wt[ISO_CPT], d[ISO_CPT], xn[ISO_CPT];
    int pk[ISO_CPT];
#pragma unroll
    for (int i = 0; i < ISO_CPT; ++i) {
        const int c = t + i * ISO_TB;
        yr[i] = wl[i] = wr[i] = wb[i] = wt[i] = d[i] = xn[i] = 0.0;
        pk[i] = 0;
        if (c >= R * R) continue;
        const int ry = c / R, rx = c - ry * R;
        const int iy = oy + ry, ix = ox + rx;
        if (iy < 0 || iy >= S.ny || ix < 0 || ix >= S.nx) continue;
        const int dep = min(min(rx, R - 1 - rx), min(ry, R - 1 - ry));
        pk[i] = rx | (ry << 8) | ((dep + 1) << 16);
        const int j = iy * S.nx + ix, fl = iy * (S.nx + 1) + ix;
        const IsoRow Rw = iso_row_coefs(A, iy, ix, j, S.gx[fl], S.gx[fl + 1], S.gy[j], S.gy[j + S.nx]);
        wl[i] = Rw.wl;
        wr[i] = Rw.wr;
        wb[i] = Rw.wb;
        wt[i] = Rw.wt;
        const double y = A.y[j];
        yr[i] = y * Rw.rdg;
        if (F.first) {
            d[i] = y / (Rw.diag * A.th);   // the first step: x1 = d0
            xn[i] = d[i];
        } else {
            d[i] = F.din[j];
            xn[i] = A.xin[j];
        }
    }
#pragma unroll
    for (int i = 0; i < ISO_CPT; ++i) {
        const int c = t + i * ISO_TB;
        if (c < R * R) X[c] = xn[i];
    }
    __syncthreads();
    for (int s = 0; s < h; ++s) {
        const double c1 = F.c1[s], c2 = F.c2[s];
#pragma unroll
        for (int i = 0; i < ISO_CPT; ++i) {
            if ((pk[i] >> 16) - 1 <= s) continue;
            const int c = t + i * ISO_TB;
            const int rx = pk[i] & 0xff, ry = (pk[i] >> 8) & 0xff;
            const int iy = oy + ry, ix = ox + rx;
            const double xc = X[c];
            const double xl = ix > 0 ? X[c - 1] : 0.0, xr = ix < S.nx - 1 ? X[c + 1] : 0.0;
            const double xb = iy > 0 ? X[c - R] : 0.0, xt = iy < S.ny - 1 ? X[c + R] : 0.0;
            const double r = iso_jres(yr[i], wl[i], wr[i], wb[i], wt[i], xc, xl, xr, xb, xt);
            const double dn = c1 * d[i] + c2 * r;
            d[i] = dn;
            xn[i] = xc + dn;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ISO_CPT; ++i)
            if ((pk[i] >> 16) - 1 > s) X[t + i * ISO_TB] = xn[i];
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < ISO_CPT; ++i) {
        if ((pk[i] >> 16) - 1 < h) continue;
        const int rx = pk[i] & 0xff, ry = (pk[i] >> 8) & 0xff;
        const int j = (oy + ry) * S.nx + ox + rx;
        A.xout[j] = X[t + i * ISO_TB];
        if (F.dout) F.dout[j] = d[i];
    }
}

// ---------------------------------------------------------------------------
// the isotropic operator by multigrid: Galerkin coarse operators of 2 x 2 cell
// aggregates (piecewise-constant prolongation, summing restriction), weighted
// Jacobi smoothing, one V-cycle per application -- again a fixed linear map.
// Each level stores its 5-point rows: diagonal d and the couplings wl, wr, wb, wt
// to the left, right, bottom and top neighbours (zero at a wall).
// ---------------------------------------------------------------------------
struct MgRows {
    int nx, ny;
    double *d, *wl, *wr, *wb, *wt;
};

constexpr double MG_COUPLE = 0.5;   // coarse coupling = this x the summed fine couplings across a side

__global__ void __launch_bounds__(B2) mg_fine_kernel(IsoArgs A, MgRows L)
{
    const Sys &S = A.S;
    const int n = S.nx * S.ny;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        int iy, ix;
        cell_yx(S, j, iy, ix);
        const int fl = iy * (S.nx + 1) + ix, fb = iy * S.nx + ix;
        const double k = S.kco[j];
        const double cx = A.Mxx * S.idx * S.idx, cy = A.Myy * S.idy * S.idy;
        double gl = S.gx[fl], gr = S.gx[fl + 1], gb = S.gy[fb], gt = S.gy[fb + S.nx];
        double ed = 0.0;
        const double e2 = S.k2 * S.fe;
        if (ix == 0) { gr *= 2.0; gl = 0.0; ed += e2 * A.Sx * S.idx; }
        else if (ix == S.nx - 1) { gl *= 2.0; gr = 0.0; ed += e2 * A.Sx * S.idx; }
        if (iy == 0) { gt *= 2.0; gb = 0.0; ed += e2 * A.Sy * S.idy; }
        else if (iy == S.ny - 1) { gb *= 2.0; gt = 0.0; ed += e2 * A.Sy * S.idy; }
        L.d[j] = S.W1 * S.dmg[j] + k * (cx * (gl + gr) + cy * (gb + gt) + ed);
        L.wl[j] = -k * cx * gl;
        L.wr[j] = -k * cx * gr;
        L.wb[j] = -k * cy * gb;
        L.wt[j] = -k * cy * gt;
    }
}

// coarse rows: the children's row sums (absorption and inflow terms) add up; a
// coupling to a neighbouring aggregate is half the sum of the children's
// couplings across that side (the rediscretised coarse operator: two fine faces
// of unchanged face/distance ratio make one coarse face); the diagonal closes the
// row with the same row sum
__global__ void __launch_bounds__(B2) mg_coarsen_kernel(MgRows F, MgRows C)
{
    const int n = C.nx * C.ny;
    for (int J = blockIdx.x * B2 + threadIdx.x; J < n; J += gridDim.x * B2) {
        const int cy = J / C.nx, cx = J - cy * C.nx;
        const int x0 = 2 * cx, x1 = min(2 * cx + 1, F.nx - 1), y0 = 2 * cy, y1 = min(2 * cy + 1, F.ny - 1);
        double rs = 0.0, wl = 0.0, wr = 0.0, wb = 0.0, wt = 0.0;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const int c = y * F.nx + x;
                rs += F.d[c] + F.wl[c] + F.wr[c] + F.wb[c] + F.wt[c];
                if (x - 1 < x0) wl += F.wl[c];
                if (x + 1 > x1) wr += F.wr[c];
                if (y - 1 < y0) wb += F.wb[c];
                if (y + 1 > y1) wt += F.wt[c];
            }
        wl *= MG_COUPLE;
        wr *= MG_COUPLE;
        wb *= MG_COUPLE;
        wt *= MG_COUPLE;
        C.d[J] = rs - (wl + wr + wb + wt);
        C.wl[J] = wl;
        C.wr[J] = wr;
        C.wb[J] = wb;
        C.wt[J] = wt;
    }
}

__device__ __forceinline__ double mg_Az(const MgRows &L, const double *z, int j, int x, int y)
{
    double a = L.d[j] * z[j];
    if (x > 0) a += L.wl[j] * z[j - 1];
    if (x < L.nx - 1) a += L.wr[j] * z[j + 1];
    if (y > 0) a += L.wb[j] * z[j - L.nx];
    if (y < L.ny - 1) a += L.wt[j] * z[j + L.nx];
    return a;
}

// one weighted Jacobi sweep: zout = zin + om (b - A zin) / d  (zin = null: zero)
__global__ void __launch_bounds__(B2) mg_jacobi_kernel(MgRows L, const double *b, const double *zin, double *zout,
                                                       double om, const int *fl)
{
    if (fl[F_STATE] != 0) return;
    const int n = L.nx * L.ny;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        const int y = j / L.nx, x = j - y * L.nx;
        const double z = zin ? zin[j] : 0.0;
        const double az = zin ? mg_Az(L, zin, j, x, y) : 0.0;
        zout[j] = z + om * (b[j] - az) / L.d[j];
    }
}

// coarse right-hand side: the sum of the children's residuals b - A z
__global__ void __launch_bounds__(B2) mg_restrict_kernel(MgRows F, const double *b, const double *z, MgRows C,
                                                         double *bc, const int *fl)
{
    if (fl[F_STATE] != 0) return;
    const int n = C.nx * C.ny;
    for (int J = blockIdx.x * B2 + threadIdx.x; J < n; J += gridDim.x * B2) {
        const int cy = J / C.nx, cx = J - cy * C.nx;
        const int x0 = 2 * cx, x1 = min(2 * cx + 1, F.nx - 1), y0 = 2 * cy, y1 = min(2 * cy + 1, F.ny - 1);
        double r = 0.0;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const int c = y * F.nx + x;
                r += b[c] - mg_Az(F, z, c, x, y);
            }
        bc[J] = r;
    }
}

// z += (coarse correction of the parent aggregate)
__global__ void __launch_bounds__(B2) mg_prolong_kernel(MgRows F, double *z, MgRows C, const double *zc,
                                                        const int *fl)
{
    if (fl[F_STATE] != 0) return;
    const int n = F.nx * F.ny;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        const int y = j / F.nx, x = j - y * F.nx;
        z[j] += zc[(y >> 1) * C.nx + (x >> 1)];
    }
}

__global__ void __launch_bounds__(B2) copy_kernel(double *dst, const double *src, int n, const int *fl)
{
    if (fl[F_STATE] != 0) return;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) dst[j] = src[j];
}

// sum of the partials of dot k over nb blocks, in a fixed order (one block of B2 threads)
__device__ __forceinline__ double block_reduce(double v)
{
    __shared__ double red[B2];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = B2 / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// first reduction level: block b sums partials b*red_b .. of each of k sums
__global__ void __launch_bounds__(B2) red2d_kernel(VecArgs A, int which, int k, int nb)
{
    if (which != 0 && A.fl[F_STATE] != 0) return;
    const int base = blockIdx.x * A.red_b, cnt = min(A.red_b, nb - base);
    for (int q = 0; q < k; ++q) {
        double v = 0.0;
        for (int i = threadIdx.x; i < cnt; i += B2) v += A.part[q * KRYB + base + i];
        v = block_reduce(v);
        if (threadIdx.x == 0) A.part2[q * KRYB + blockIdx.x] = v;
    }
}

// the final reduction: one block of FIN_T threads
constexpr int FIN_T = 1024;

// the K sums of nb partials each (through the first level when nb > red_b):
// thread i adds partials i, i + FIN_T, ... in that order, then each wavefront
// reduces by a butterfly and the wavefronts are added in order (a fixed order,
// independent of timing); every thread gets the totals
template <int K>
__device__ __forceinline__ void fin_sums(const VecArgs &A, int nb, double (&s)[K])
{
    __shared__ double red[K][FIN_T / 64];
    const bool two = nb > A.red_b;
    const double *part = two ? A.part2 : A.part;
    const int cnt = two ? (nb + A.red_b - 1) / A.red_b : nb;
    double v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < cnt; i += FIN_T)
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] += part[q * KRYB + i];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
        if (lane == 0) red[q][w] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double t = 0.0;
        for (int i = 0; i < FIN_T / 64; ++i) t += red[q][i];
        s[q] = t;
    }
}

// which: 0 = start (rho = (h, r), rr = (r, r), bb, test), 1 = alpha, 2 = omega, 3 = rho/beta/test
__global__ void __launch_bounds__(FIN_T) fin2d_kernel(VecArgs A, int which, int nb)
{
    if (which != 0 && A.fl[F_STATE] != 0) return;
    double *sc = A.sc;
    if (which == 0) {
        double f[4];
        fin_sums<4>(A, nb, f);
        const double rr = f[0], bb = f[1], mm = f[2], hr = f[3];
        if (threadIdx.x == 0) {
            sc[S_RHO] = hr;
            sc[S_RR] = rr;
            sc[S_R0] = rr;
            sc[S_BB] = bb;
            sc[S_MM] = mm;
            sc[S_ALPHA] = sc[S_OMEGA] = 1.0;
            sc[S_BETA] = 0.0;
            A.fl[F_STATE] = (rr <= A.tol * A.tol * bb) ? 1 : 0;
        }
    } else if (which == 1) {
        double f[1];
        fin_sums<1>(A, nb, f);
        const double rv = f[0];
        if (threadIdx.x == 0) {
            sc[S_RV] = rv;
            if (rv == 0.0 || !isfinite(rv)) A.fl[F_STATE] = 2;
            else sc[S_ALPHA] = sc[S_RHO] / rv;
        }
    } else if (which == 2) {
        double f[2];
        fin_sums<2>(A, nb, f);
        const double ts = f[0], tt = f[1];
        if (threadIdx.x == 0) {
            sc[S_TS] = ts;
            sc[S_TT] = tt;
            // t = A sh vanishes only with s: omega = 0 lets the last update still
            // take x += alpha ph, and the test after it stops on r = s
            if (!isfinite(tt) || !isfinite(ts)) A.fl[F_STATE] = 2;
            else sc[S_OMEGA] = tt == 0.0 ? 0.0 : ts / tt;
        }
    } else {
        double f[2];
        fin_sums<2>(A, nb, f);
        const double rho = f[0], rr = f[1];
        if (threadIdx.x == 0) {
            const int its = A.fl[F_ITS] + 1;
            A.fl[F_ITS] = its;
            sc[S_RR] = rr;
            const double rec = A.rec * A.tol;
            const bool done = rr <= rec * rec * sc[S_BB] || rr <= A.pass_red * A.pass_red * sc[S_R0];
            if (!done && its >= A.maxit) {
                A.fl[F_STATE] = 3;
            } else if (done) {
                A.fl[F_STATE] = 1;              // the end of the pass
            } else if (sc[S_OMEGA] == 0.0 || rho == 0.0 || !isfinite(rho)) {
                A.fl[F_STATE] = 2;
            } else {
                sc[S_BETA] = (rho / sc[S_RHO]) * (sc[S_ALPHA] / sc[S_OMEGA]);
                sc[S_RHO] = rho;
            }
        }
    }
}

__global__ void __launch_bounds__(B2) zero2_kernel(double *a, double *b, size_t n)
{
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)n; t += gridDim.x * B2) a[t] = b[t] = 0.0;
}

// x += dx at the end of a pass
template <class V>
__global__ void __launch_bounds__(B2) xadd_kernel(double *x, const void *dv, size_t n, const int *fl)
{
    // no iteration of the pass completed (a breakdown in its first): dx holds
    // the last pass's correction, already added
    if (fl[F_ITS] == 0) return;
    const V *d = (const V *)dv;
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)n; t += gridDim.x * B2) x[t] += (double)d[t];
}

__global__ void reset_flags_kernel(int *fl)
{
    if (threadIdx.x < F_NF) fl[threadIdx.x] = 0;
}

// x0 of the correction: E_J = (E* - a c U^{n+1}) / eps
__global__ void __launch_bounds__(B2) xcorr0_kernel(double *x, const double *Es, const double *acU, int P,
                                                    double ieps, size_t n)
{
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)n; t += gridDim.x * B2)
        x[t] = (Es[t] - acU[t / P]) * ieps;
}

// between the binary64 state and its binary32 storage (E stored as its deviation
// from a c T^4, O as is)
__global__ void __launch_bounds__(B2) conv2d_kernel(int nE, int nOx, int nOy, int lgP, double ac, const double *T,
                                                    double *E, double *Ox, double *Oy, float *E32, float *Ox32,
                                                    float *Oy32, int to32)
{
    const int n = max(nE, max(nOx, nOy));
    for (int t = blockIdx.x * B2 + threadIdx.x; t < n; t += gridDim.x * B2) {
        if (t < nE) {
            const double tj = T[t >> lgP];
            const double base = ac * (tj * tj) * (tj * tj);
            if (to32) E32[t] = (float)(E[t] - base);
            else E[t] = base + (double)E32[t];
        }
        if (t < nOx) {
            if (to32) Ox32[t] = (float)Ox[t];
            else Ox[t] = (double)Ox32[t];
        }
        if (t < nOy) {
            if (to32) Oy32[t] = (float)Oy[t];
            else Oy[t] = (double)Oy32[t];
        }
    }
}

// cell-centre intensities I(+-Omega_p) = E_p +- eps O_p, O at the cell centre the
// mean of its four faces; out[c*2P + p] = I(+Omega_p), out[c*2P + P + p] = I(-Omega_p)
__global__ void __launch_bounds__(B2) intensity2d_kernel(int nx, int ny, int lgP, double eps, const double *E,
                                                         const double *Ox, const double *Oy, double *out)
{
    const int P = 1 << lgP;
    const int n = nx * ny * P;
    for (int t = blockIdx.x * B2 + threadIdx.x; t < n; t += gridDim.x * B2) {
        const int j = t >> lgP, p = t & (P - 1);
        const int iy = j / nx, ix = j - iy * nx;
        const int fl = iy * (nx + 1) + ix, fb = iy * nx + ix;
        const double oc = 0.25 * (Ox[fl * P + p] + Ox[(fl + 1) * P + p] + Oy[fb * P + p] + Oy[(fb + nx) * P + p]);
        out[j * 2 * P + p] = E[t] + eps * oc;
        out[j * 2 * P + P + p] = E[t] - eps * oc;
    }
}

// ---------------------------------------------------------------------------
// correction substep 1: moments, D, U*, K*, scalar Newton per cell
// ---------------------------------------------------------------------------
struct NewtArgs {
    Sys S;                       // the prediction's system (its faces give O*)
    const double *Es, *En, *Tn, *sigma0, *beta;
    double a, c, cv, dt;
    int m, maxit;
    double *Tnew, *ustar, *Dv, *rhon, *rstar;
    double *bflux;               // edge cells: outflow through their edge faces, sum_p omega_p (...)
    int *stat;                   // [0] max its, [1] failed, [2] K* clamped, [3] negative root, [4] sum its,
                                 // [5] guesses accepted, [6] guesses not used, [7] Newton started from a guess
    const double *tg;            // learned starting values (guess2d_kernel; GUESS kernels only)
    double gtol;                 // residual below which the guess is taken as the root
};

// The learned starting values of the temperature solve, one thread per cell:
// the network's features from (rho*, T^n, sigma0, eps, dt), rho* = sum_p
// omega_p E*_p, and T_g = T^n exp(mean + sd y) into tg (NaN where the network
// has no input: sigma0 = 0 or T^n <= 0).  A kernel of its own, so that the
// network's 64 hidden values live in the registers of every lane rather than
// in one lane per cell of the temperature kernel.
struct GuessArgs {
    int n, P, m;
    double eps, dt;
    const double *Es, *Tn, *sigma0, *om;
    const uint16_t *gw;
    const float *gnorm;
    double *tg;
};

__global__ void __launch_bounds__(B2) guess2d_kernel(GuessArgs A)
{
    __shared__ uint16_t sW[MLP_NPARAM + 3];
    __shared__ float sN[MLP_NNORM];
    for (int e = threadIdx.x; e < MLP_NPARAM; e += B2) sW[e] = A.gw[e];
    if (threadIdx.x < MLP_NNORM) sN[threadIdx.x] = A.gnorm[threadIdx.x];
    __syncthreads();
    for (int j = blockIdx.x * B2 + threadIdx.x; j < A.n; j += gridDim.x * B2) {
        const double Tn = A.Tn[j], s0 = A.sigma0[j];
        double tg = NAN;
        if (s0 > 0.0 && Tn > 0.0) {
            double rho = 0.0;
            for (int p = 0; p < A.P; ++p) rho += A.om[p] * A.Es[(size_t)j * A.P + p];
            float f[MLP_IN];
            mlp_features(rho, Tn, s0, A.m, A.eps, A.dt, f);
            const float y = mlp_eval_streamed(sW, sN, f);
            tg = Tn * exp((double)sN[10] + (double)sN[11] * (double)y);
        }
        A.tg[j] = tg;
    }
}

// The prediction's moments, one thread per (cell, pair): rho* = sum_p omega_p
// E*_p, rho^n, the flux divergence D of the prediction's face values and, at
// the domain's edges, the outflow through the cell's edge faces (the face
// values are those whose divergence is D; interior faces cancel in the sum of D)
__global__ void __launch_bounds__(B2) moments2d_kernel(NewtArgs A)
{
    const Sys &S = A.S;
    const int P = S.P;
    const size_t n = (size_t)S.nx * S.ny * P;
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)n; t += gridDim.x * B2) {
        const int j = t >> S.lgP, p = t & (P - 1);
        int iy, ix;
        cell_yx(S, j, iy, ix);
        const Nb X = load_nb(A.Es, S.nx, S.ny, iy, ix, P, p);
        Grad O;
        faces<true, true>(S, iy, ix, p, &X, O);
        const double w = S.om[p];
        const double D = group_sum(w * divergence(S, O, p), P);
        const double rhs_s = group_sum(w * X.v[1][1], P);
        const double rn = group_sum(w * A.En[t], P);
        double fo = 0.0;
        if (ix == S.nx - 1) fo += S.mu[p] * O.r * S.dy;
        if (ix == 0) fo -= S.mu[p] * O.l * S.dy;
        if (iy == S.ny - 1) fo += S.eta[p] * O.t * S.dx;
        if (iy == 0) fo -= S.eta[p] * O.b * S.dx;
        const double fout = group_sum(w * fo, P);
        if (p != 0) continue;
        if (ix == 0 || iy == 0 || ix == S.nx - 1 || iy == S.ny - 1) A.bflux[j] = fout;
        A.Dv[j] = D;
        A.rhon[j] = rn;
        A.rstar[j] = rhs_s;
    }
}

// U* of (4.5c) and the temperature of (4.13), one thread per cell (from the
// moments above)
template <bool GUESS>
__global__ void __launch_bounds__(B2) newton2d_kernel(NewtArgs A)
{
    int acc = 0, unused = 0, started = 0;
    const Sys &S = A.S;
    const int n = S.nx * S.ny;
    int mx = 0, sum = 0, failed = 0, clamped = 0, neg = 0;
    for (int j = blockIdx.x * B2 + threadIdx.x; j < n; j += gridDim.x * B2) {
        const double D = A.Dv[j], rn = A.rhon[j], rhs_s = A.rstar[j];
        const double ac = A.a * A.c;
        const double Tn = A.Tn[j];
        const double Un = Tn * Tn * Tn * Tn;
        const double beta = A.beta[j];
        const double us = (Un + beta * rhs_s) / (1.0 + ac * beta);
        A.ustar[j] = us;
        double Ks = 1.0;
        if (A.m == 3) {
            if (us < 0.0) {
                Ks = 0.0;
                ++clamped;
            } else {
                Ks = pow(us, 0.75);
            }
        }
        // (4.13) times c sigma0 dt^2:
        //   a c sigma0 dt T^4 + Cv (eps^2 K* + c sigma0 dt)(T - T^n) - sigma0 dt (rho^n - c dt D) = 0
        const double s0 = A.sigma0[j];
        const double lin = A.cv * (S.eps * S.eps * Ks + A.c * s0 * A.dt);
        const double q4 = ac * s0 * A.dt;
        const double rhs = s0 * A.dt * (rn - A.c * A.dt * D);
        double T = Tn;
        int its = 0;
        if (!(s0 == 0.0 && Ks == 0.0)) {
            if (Tn + rhs / lin < 0.0) ++neg;
            bool ok = false, done = false;
            if (GUESS && s0 > 0.0 && Tn > 0.0) {
                // learned starting value (guess2d_kernel), judged by the normalised
                // residual of (4.13): taken as the root below gtol, used as Newton's
                // start if its residual is below that of T^n, otherwise Newton starts
                // from T^n
                const double Tg = A.tg[j];
                if (isfinite(Tg) && Tg > 0.0) {
                    const double T2 = Tg * Tg;
                    const double rg = fabs(q4 * T2 * T2 + lin * (Tg - Tn) - rhs) / lin;
                    const double Tn2 = Tn * Tn;
                    const double rr = fabs(q4 * Tn2 * Tn2 - rhs) / lin;
                    if (rg <= A.gtol * fmax(fabs(Tn + rhs / lin), 1e-300)) {
                        T = Tg;
                        ok = done = true;
                        ++acc;
                    } else if (rg < rr) {
                        ok = done = newton_quartic(Tg, Tn, q4, lin, rhs, A.maxit, T, its);
                        if (done) ++started;
                    }
                }
                if (!done) ++unused;
            }
            if (!done) ok = newton_quartic(Tn, Tn, q4, lin, rhs, A.maxit, T, its);
            if (!ok) ++failed;
        }
        A.Tnew[j] = T;
        mx = max(mx, its);
        sum += its;
    }
    // one atomic per wavefront and counter
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, __shfl_xor(mx, o, 64));
        sum += __shfl_xor(sum, o, 64);
        failed += __shfl_xor(failed, o, 64);
        clamped += __shfl_xor(clamped, o, 64);
        neg += __shfl_xor(neg, o, 64);
        acc += __shfl_xor(acc, o, 64);
        unused += __shfl_xor(unused, o, 64);
        started += __shfl_xor(started, o, 64);
    }
    if (__lane_id() == 0) {
        if (mx) atomicMax(&A.stat[0], mx);
        if (failed) atomicAdd(&A.stat[1], failed);
        if (clamped) atomicAdd(&A.stat[2], clamped);
        if (neg) atomicAdd(&A.stat[3], neg);
        if (sum) atomicAdd(&A.stat[4], sum);
        if (acc) atomicAdd(&A.stat[5], acc);
        if (unused) atomicAdd(&A.stat[6], unused);
        if (started) atomicAdd(&A.stat[7], started);
    }
}

// training rows of the learned guess for the last step: features of (rho*, T^n,
// sigma0, eps, dt) and the target log(T^{n+1}/T^n), six binary32 values per cell
__global__ void __launch_bounds__(B2) log2d_kernel(int n, int m, double eps, double dt, const double *rstar,
                                                   const double *Told, const double *Tnew, const double *sigma0,
                                                   float *out)
{
    const int j = blockIdx.x * B2 + threadIdx.x;
    if (j >= n) return;
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

// ---------------------------------------------------------------------------
// projection (4.14): E^{n+1} = a c U^{n+1} + eps E_J, O^{n+1} = O_J
// ---------------------------------------------------------------------------
struct ProjArgs {
    Sys S;                    // the correction's system
    const double *EJ;
    double *E1, *Ox1, *Oy1;
    double *rho1;             // rho^{n+1} per cell (energy balance)
};

__global__ void __launch_bounds__(B2) project2d_kernel(ProjArgs A)
{
    const Sys &S = A.S;
    const int P = S.P;
    const size_t n = (size_t)S.nx * S.ny * P;
    for (int t = blockIdx.x * B2 + threadIdx.x; t < (int)n; t += gridDim.x * B2) {
        const int j = t >> S.lgP, p = t & (P - 1);
        int iy, ix;
        cell_yx(S, j, iy, ix);
        const Nb X = load_nb(A.EJ, S.nx, S.ny, iy, ix, P, p);
        Grad O;
        faces<true, true>(S, iy, ix, p, &X, O);
        const double e1 = S.acU[j] + S.eps * X.v[1][1];
        A.E1[t] = e1;
        const double r1 = group_sum(S.om[p] * e1, P);
        if (p == 0) A.rho1[j] = r1;
        const int fl = iy * (S.nx + 1) + ix, fb = iy * S.nx + ix;
        A.Ox1[fl * P + p] = O.l;
        if (ix == S.nx - 1) A.Ox1[(fl + 1) * P + p] = O.r;
        A.Oy1[fb * P + p] = O.b;
        if (iy == S.ny - 1) A.Oy1[(fb + S.nx) * P + p] = O.t;
    }
}

// energy balance of the step ((3.12)-(3.13)): E_tot = sum dx dy (rho / c + Cv T)
// before and after, and the outflow through the domain's edges of the
// prediction's face values times dt.  Binary64 sums in a fixed order: each
// thread takes cells j = t, t + G, ... (G threads in the grid) in order, a tree
// over the block, per-block partials, and the last block to finish sums those
// by index.
struct EnergyArgs {
    int n, nb;
    double dxdy, c, cv, dt;
    int nx, ny;
    const double *rhon, *Tn, *rho1, *Tnew, *bflux;
    double *epart;            // 3 per block
    unsigned *ecnt;           // blocks done (reset to 0 by the last one)
    double *energy;           // E_before, E_after, outflow dt, defect
};

__global__ void __launch_bounds__(B2) energy2d_kernel(EnergyArgs A)
{
    __shared__ double s0[B2], s1[B2], s2[B2];
    __shared__ int s_last;
    const int t = threadIdx.x;
    double e0 = 0.0, e1 = 0.0, fo = 0.0;
    for (int j = blockIdx.x * B2 + t; j < A.n; j += A.nb * B2) {
        e0 += A.dxdy * (A.rhon[j] / A.c + A.cv * A.Tn[j]);
        e1 += A.dxdy * (A.rho1[j] / A.c + A.cv * A.Tnew[j]);
        const int iy = j / A.nx, ix = j - iy * A.nx;
        if (ix == 0 || iy == 0 || ix == A.nx - 1 || iy == A.ny - 1) fo += A.bflux[j];
    }
    s0[t] = e0;
    s1[t] = e1;
    s2[t] = fo;
    __syncthreads();
    for (int o = B2 / 2; o > 0; o >>= 1) {
        if (t < o) {
            s0[t] += s0[t + o];
            s1[t] += s1[t + o];
            s2[t] += s2[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        A.epart[3 * blockIdx.x] = s0[0];
        A.epart[3 * blockIdx.x + 1] = s1[0];
        A.epart[3 * blockIdx.x + 2] = s2[0];
        __threadfence();                         // partials visible device-wide before the count
        s_last = atomicAdd(A.ecnt, 1u) == (unsigned)(A.nb - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();                             // every block's partials are in memory
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int b = t; b < A.nb; b += B2) {
        a0 += __hip_atomic_load(&A.epart[3 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a1 += __hip_atomic_load(&A.epart[3 * b + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a2 += __hip_atomic_load(&A.epart[3 * b + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    s0[t] = a0;
    s1[t] = a1;
    s2[t] = a2;
    __syncthreads();
    for (int o = B2 / 2; o > 0; o >>= 1) {
        if (t < o) {
            s0[t] += s0[t + o];
            s1[t] += s1[t + o];
            s2[t] += s2[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double eb = s0[0], ea = s1[0], fdt = A.dt * s2[0];
        A.energy[0] = eb;
        A.energy[1] = ea;
        A.energy[2] = fdt;
        A.energy[3] = (ea - eb) + fdt;
        *A.ecnt = 0u;
    }
}

}  // namespace

// ===========================================================================
// host side
// ===========================================================================
struct grte2d_ctx {
    int nx, ny, P, m;
    double lx, ly, a, c, cv, W1;
    size_t N, nE, nOx, nOy;
    hipStream_t stream = nullptr;
    double tol = 1e-14;
    int maxit = 2000;
    // pairs, inflow
    double *mu = nullptr, *eta = nullptr, *om = nullptr, *b = nullptr;
    // state
    double *E = nullptr, *Ox = nullptr, *Oy = nullptr, *T = nullptr, *sigma0 = nullptr;
    double *E1 = nullptr, *Ox1 = nullptr, *Oy1 = nullptr, *T1 = nullptr;
    // coefficients
    double *ax = nullptr, *gx = nullptr, *ay = nullptr, *gy = nullptr;
    double *lam = nullptr, *dmg = nullptr, *cg = nullptr, *kco = nullptr, *rb0 = nullptr, *rb1 = nullptr;
    double *acU = nullptr, *beta = nullptr, *ustar = nullptr, *Dv = nullptr, *rhon = nullptr;
    double *sab = nullptr, *ue = nullptr;
    // Krylov
    double *bv = nullptr, *x = nullptr, *Es = nullptr;
    // the Krylov vectors: binary64 arrays, used as binary32 ones when the
    // solve's vectors are narrow
    double *r = nullptr, *p = nullptr, *ph = nullptr, *v = nullptr, *s = nullptr, *sh = nullptr, *t = nullptr;
    double *dxv = nullptr;
    int *narrow = nullptr;               // the solve's vectors are binary32 (set per solve)
    int narrow_ok = 1;                   // binary32 Krylov vectors allowed (grte2d_set_krylov_storage)
    int last_narrow[2] = {-1, -1};       // the storage of the last prediction / correction solve
    int narrow_used[2] = {0, 0};         // (reported in the step info)
    double *part = nullptr, *part2 = nullptr, *sc = nullptr;
    int *fl = nullptr, *stat = nullptr;
    int *h_fl = nullptr;      // pinned
    double *h_sc = nullptr;   // pinned
    std::vector<void *> allocs;
    double *ibuf = nullptr;              // intensity readout for host destinations
    // binary32 storage of the state between steps (0: binary64)
    int f32 = 0;
    float *E32 = nullptr, *Ox32 = nullptr, *Oy32 = nullptr;
    // learned initial guess of the temperature solve
    const uint16_t *guess_w = nullptr;
    const float *guess_norm = nullptr;
    double guess_tol = 1e-10;
    double *rstar = nullptr;
    int stepped = 0;
    double last_eps = 0, last_dt = 0;
    // isotropic correction of the preconditioner
    int iso_kind = 1;                    // 0 none, 1 Chebyshev (tiled), 2 multigrid V-cycle, 3 Chebyshev per step
    int iso_k = 19;                      // Chebyshev steps (two tiled launches)
    // iterations of each pass of the last prediction / correction solve (-1: none yet)
    int last_its[2][KRY_RESTARTS + 1];
    int mg_nu = 2;                       // multigrid: Jacobi sweeps before and after the coarse correction
    struct Lv {
        MgRows R;
        double *b, *z0, *z1;
    };
    std::vector<Lv> mg;
    double Mxx = 0, Myy = 0, Sx = 0, Sy = 0;
    double *yP = nullptr, *yS = nullptr, *dP = nullptr, *dS = nullptr, *itmp = nullptr, *idir = nullptr;
    double *pgc = nullptr;               // per-cell scalar of the block inverse
    int kry_items = KRY_ITEMS;           // launch shape of the Krylov kernels (grte2d_set_launch_shape)
    int red_b = RED_B;
    // energy balance: edge outflow per edge cell, rho^{n+1}, block partials,
    // the blocks-done counter and the four results
    double *bflux = nullptr, *rho1 = nullptr, *epart = nullptr, *energy = nullptr;
    double *tguess = nullptr;            // learned starting values of the temperature solve
    unsigned *ecnt = nullptr;
    double *idg = nullptr;               // per-(cell, pair) inverse diagonal of the block inverse
    float *idg32 = nullptr;              // the same in binary32
    double *opc = nullptr;               // the operator's packed per-cell coefficients (OPC_N per cell)
    double *mr = nullptr, *mv = nullptr;  // angular moments of r and v (isotropic correction)
    double *idir2 = nullptr;             // second Chebyshev direction buffer of the tiled launches
    // sampled timing of the operator kernel (first iteration of every chunk)
    int profiling = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double prof_ms = 0.0;
    int prof_n = 0;
};

namespace {

grte_status hip_ok(hipError_t e) { return e == hipSuccess ? GRTE_OK : GRTE_E_HIP; }

template <class T>
bool dalloc(grte2d_ctx *c, T *&p, size_t n)
{
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
    c->allocs.push_back(q);
    p = (T *)q;
    return true;
}

constexpr int ENERGY_BLOCKS = 1024;    // most blocks of the energy reduction

int energy_blocks(size_t n)
{
    const size_t b = (n + B2 - 1) / B2;
    return (int)std::max<size_t>(1, std::min<size_t>(b, ENERGY_BLOCKS));
}

int nblocks(size_t n)
{
    const size_t b = (n + B2 - 1) / B2;
    return (int)std::max<size_t>(1, std::min<size_t>(b, MAXB));
}

int kblocks(size_t n, int items)
{
    const size_t b = (n + (size_t)B2 * items - 1) / ((size_t)B2 * items);
    return (int)std::max<size_t>(1, std::min<size_t>(b, KRYB));
}

Sys make_sys(grte2d_ctx *c, int corr, double eps)
{
    Sys S;
    S.opc = nullptr;                     // (set where the operator products run)
    S.nx = c->nx;
    S.ny = c->ny;
    S.P = c->P;
    S.corr = corr;
    S.dx = c->lx / c->nx;
    S.dy = c->ly / c->ny;
    S.idx = 1.0 / S.dx;
    S.idy = 1.0 / S.dy;
    S.inx = 1.0 / c->nx;
    S.k2 = 2.0 / eps;
    S.lgP = 0;
    while ((1 << S.lgP) < c->P) ++S.lgP;
    S.eps = eps;
    S.fe = corr ? eps : 1.0;
    S.W1 = c->W1;
    S.mu = c->mu;
    S.eta = c->eta;
    S.om = c->om;
    S.b = c->b;
    S.Ox0 = c->Ox;
    S.Oy0 = c->Oy;
    S.ax = c->ax;
    S.gx = c->gx;
    S.ay = c->ay;
    S.gy = c->gy;
    S.lam = c->lam;
    S.dmg = c->dmg;
    S.cg = c->cg;
    S.kco = c->kco;
    S.rb1 = c->rb1;
    S.rb0 = c->rb0;
    S.acU = c->acU;
    S.sab = c->sab;
    S.ue = c->ue;
    S.pgc = c->pgc;
    return S;
}

// widen (to32 = 0) or round (to32 = 1) the state held in E, Ox, Oy with temperature T
grte_status convert2d(grte2d_ctx *c, int to32)
{
    int lgP = 0;
    while ((1 << lgP) < c->P) ++lgP;
    const size_t n = std::max(c->nE, std::max(c->nOx, c->nOy));
    hipLaunchKernelGGL(conv2d_kernel, dim3(nblocks(n)), dim3(B2), 0, c->stream, (int)c->nE, (int)c->nOx, (int)c->nOy,
                       lgP, c->a * c->c, c->T, c->E, c->Ox, c->Oy, c->E32, c->Ox32, c->Oy32, to32);
    return hipGetLastError() == hipSuccess ? GRTE_OK : GRTE_E_HIP;
}

IsoArgs iso_args(grte2d_ctx *c, const Sys &S)
{
    IsoArgs I;
    I.S = S;
    I.Mxx = c->Mxx;
    I.Myy = c->Myy;
    I.Sx = c->Sx;
    I.Sy = c->Sy;
    I.fl = c->fl;
    I.y = nullptr;
    I.xin = nullptr;
    I.xout = nullptr;
    I.d = c->idir;
    I.c1 = I.c2 = I.th = 0.0;
    return I;
}

// rows of every multigrid level for the current prediction system
void mg_setup(grte2d_ctx *c, const Sys &S, hipStream_t st)
{
    hipLaunchKernelGGL(mg_fine_kernel, dim3(nblocks(c->N)), dim3(B2), 0, st, iso_args(c, S), c->mg[0].R);
    for (size_t l = 1; l < c->mg.size(); ++l) {
        const MgRows &C = c->mg[l].R;
        hipLaunchKernelGGL(mg_coarsen_kernel, dim3(nblocks((size_t)C.nx * C.ny)), dim3(B2), 0, st, c->mg[l - 1].R,
                           C);
    }
}

constexpr double MG_OMEGA = 0.8;       // Jacobi damping
constexpr int MG_COARSE_SWEEPS = 40;   // on the coarsest level (at most 4 x 4 cells on a side)

// k Jacobi sweeps on level L for right-hand side b, from z = 0 (zero) or from the
// values in L.z0; the result is left in L.z0
void mg_sweeps(grte2d_ctx *c, grte2d_ctx::Lv &L, const double *b, int k, bool zero, hipStream_t st)
{
    const int nb = nblocks((size_t)L.R.nx * L.R.ny);
    double *cur = zero ? nullptr : L.z0;
    for (int i = 0; i < k; ++i) {
        double *dst = (cur == L.z0) ? L.z1 : L.z0;
        hipLaunchKernelGGL(mg_jacobi_kernel, dim3(nb), dim3(B2), 0, st, L.R, b, (const double *)cur, dst, MG_OMEGA,
                           (const int *)c->fl);
        cur = dst;
    }
    if (cur == L.z1)
        hipLaunchKernelGGL(copy_kernel, dim3(nb), dim3(B2), 0, st, L.z0, (const double *)L.z1,
                           L.R.nx * L.R.ny, (const int *)c->fl);
}

void mg_vcycle(grte2d_ctx *c, size_t l, const double *b, hipStream_t st)
{
    grte2d_ctx::Lv &L = c->mg[l];
    if (l + 1 == c->mg.size()) {
        mg_sweeps(c, L, b, MG_COARSE_SWEEPS, true, st);
        return;
    }
    mg_sweeps(c, L, b, c->mg_nu, true, st);
    grte2d_ctx::Lv &C = c->mg[l + 1];
    hipLaunchKernelGGL(mg_restrict_kernel, dim3(nblocks((size_t)C.R.nx * C.R.ny)), dim3(B2), 0, st, L.R, b,
                       (const double *)L.z0, C.R, C.b, (const int *)c->fl);
    mg_vcycle(c, l + 1, C.b, st);
    hipLaunchKernelGGL(mg_prolong_kernel, dim3(nblocks((size_t)L.R.nx * L.R.ny)), dim3(B2), 0, st, L.R, L.z0, C.R,
                       (const double *)C.z0, (const int *)c->fl);
    mg_sweeps(c, L, b, c->mg_nu, false, st);
}

// K Chebyshev steps for D z = y; the result lands in out (tmp is scratch)
void iso_cheb(grte2d_ctx *c, const Sys &S, const double *y, double *out, hipStream_t st)
{
    const int K = c->iso_k;
    const int nbc = nblocks(c->N);
    IsoArgs I;
    I.S = S;
    I.Mxx = c->Mxx;
    I.Myy = c->Myy;
    I.Sx = c->Sx;
    I.Sy = c->Sy;
    I.y = y;
    I.d = c->idir;
    I.fl = c->fl;
    const double th = 0.5 * (CHEB2_B + CHEB2_A), de = 0.5 * (CHEB2_B - CHEB2_A), sg = th / de;
    I.th = th;
    if (c->iso_kind == 1) {
        // tiled launches of up to ISO_HALO stencil steps each (the first also
        // takes the local first step); the iterate alternates between itmp and
        // out so that the last launch writes out, the direction between idir
        // and idir2
        const int nl = K - 1 <= ISO_HALO ? 1 : 1 + (K - 1 - ISO_HALO + ISO_HALO - 1) / ISO_HALO;
        const dim3 grid((S.nx + ISO_T - 1) / ISO_T, (S.ny + ISO_T - 1) / ISO_T);
        double rho = 1.0 / sg;
        int k = 1;                          // global index of the next stencil step
        for (int l = 0; l < nl; ++l) {
            IsoFused F;
            F.A = I;
            F.first = l == 0;
            F.nsteps = std::min(ISO_HALO, K - k);
            F.A.xin = l == 0 ? nullptr : (((nl - l) % 2 == 0) ? out : c->itmp);
            F.A.xout = ((nl - 1 - l) % 2 == 0) ? out : c->itmp;
            F.din = l == 0 ? nullptr : ((l % 2 == 1) ? c->idir : c->idir2);
            F.dout = l == nl - 1 ? nullptr : ((l % 2 == 0) ? c->idir : c->idir2);
            for (int s = 0; s < F.nsteps; ++s, ++k) {
                const double rn = 1.0 / (2.0 * sg - rho);
                F.c1[s] = rn * rho;
                F.c2[s] = 2.0 * rn / de;
                rho = rn;
            }
            hipLaunchKernelGGL(iso_fused_kernel, grid, dim3(ISO_TB), 0, st, F);
        }
        return;
    }
    auto buf = [&](int k) { return ((K - k) % 2 == 0) ? out : c->itmp; };   // iterate k lands in buf(k)
    I.xin = nullptr;
    I.xout = buf(1);
    I.c1 = I.c2 = 0.0;
    hipLaunchKernelGGL(iso_first_kernel, dim3(nbc), dim3(B2), 0, st, I);
    double rho = 1.0 / sg;
    for (int k = 1; k < K; ++k) {
        const double rn = 1.0 / (2.0 * sg - rho);
        I.c1 = rn * rho;
        I.c2 = 2.0 * rn / de;
        rho = rn;
        I.xin = buf(k);
        I.xout = buf(k + 1);
        hipLaunchKernelGGL(iso_step_kernel, dim3(nbc), dim3(B2), 0, st, I);
    }
}

void iso_solve(grte2d_ctx *c, const Sys &S, const double *y, double *out, hipStream_t st)
{
    if (c->iso_kind == 1 || c->iso_kind == 3) {
        iso_cheb(c, S, y, out, st);
        return;
    }
    // one V-cycle; level 0's result buffer is `out`
    grte2d_ctx::Lv &L0 = c->mg[0];
    double *keep = L0.z0;
    L0.z0 = out;
    mg_vcycle(c, 0, y, st);
    L0.z0 = keep;
}

// BiCGStab on the system currently described by the coefficient arrays; x holds
// the start and receives the solution.  Returns iterations, state and the
// final true relative residual.
template <class V>
grte_status krylov_run(grte2d_ctx *c, const Sys &S, int &its_out, int &state_out, double &res_out, int &floor_out)
{
    int floor = 0;
    VecArgs A;
    A.S = S;
    A.S.opc = c->opc;
    A.n = c->nE;
    A.En = c->E;
    A.bv = c->bv;
    A.x = c->x;
    A.r = c->r;
    A.p = c->p;
    A.ph = c->ph;
    A.v = c->v;
    A.s = c->s;
    A.sh = c->sh;
    A.t = c->t;
    A.dx = c->dxv;
    const bool narrow = sizeof(V) == 4;
    A.idg = narrow ? (const void *)c->idg32 : (const void *)c->idg;
    // binary32 passes end at KRY_PASS_RED of their starting residual, with the
    // recursion run on to KRY_REC of the tolerance; binary64 passes at the tolerance
    A.pass_red = narrow ? KRY_PASS_RED : 0.0;
    A.rec = narrow ? KRY_REC : 1.0;
    // the pass lengths of the last solve of this kind size the batches when it
    // had the same storage
    if (c->last_narrow[S.corr] != (int)narrow)
        for (int &n : c->last_its[S.corr]) n = -1;
    c->last_narrow[S.corr] = narrow;
    A.part = c->part;
    A.part2 = c->part2;
    A.sc = c->sc;
    A.fl = c->fl;
    A.tol = c->tol;
    A.maxit = c->maxit;
    // the isotropic correction targets the angular coupling of the prediction;
    // the correction's systems have none
    const bool iso = c->iso_kind != 0 && !S.corr;
    if (iso && c->iso_kind == 2) mg_setup(c, S, c->stream);
    A.dP = iso ? c->dP : nullptr;
    A.dS = iso ? c->dS : nullptr;
    A.yP = iso ? c->yP : nullptr;
    A.yS = iso ? c->yS : nullptr;
    A.mr = iso ? c->mr : nullptr;
    A.mv = iso ? c->mv : nullptr;
    const int nbc = nblocks(c->N);
    const int nb = kblocks(c->nE, c->kry_items);
    A.red_b = c->red_b;
    hipStream_t st = c->stream;
    // the scalar step `which` of the iteration after a kernel that left k partial sums per block
    // (the operator products of the iteration run on their own grid of column tiles)
    const int ncol = (c->nx + (B2 / c->P) - 1) / (B2 / c->P), ntile = ncol * ((c->ny + OP_ROWS - 1) / OP_ROWS);
    const int nbo = std::min(ntile, KRYB);
    auto fin = [&](int which, int k, int nbk) {
        if (nbk > c->red_b)
            hipLaunchKernelGGL(red2d_kernel, dim3((nbk + c->red_b - 1) / c->red_b), dim3(B2), 0, st, A, which, k,
                               nbk);
        hipLaunchKernelGGL(fin2d_kernel, dim3(1), dim3(FIN_T), 0, st, A, which, nbk);
    };
    int its_total = 0, state = 0;
    // iterations are enqueued in batches between convergence checks; the
    // batches are sized to end where the same pass of the last solve of the
    // same kind ended (iteration counts change slowly from step to step), and
    // iterations enqueued past the end of a pass return at once
    double res = INFINITY;
    int pass_its[KRY_RESTARTS + 1];
    for (int k = 0; k <= KRY_RESTARTS; ++k) pass_its[k] = -1;
    for (int restart = 0; restart <= KRY_RESTARTS; ++restart) {
        hipLaunchKernelGGL(reset_flags_kernel, dim3(1), dim3(64), 0, st, c->fl);
        hipLaunchKernelGGL(residual2d_kernel<V>, dim3(nb), dim3(B2), 0, st, A);
        fin(0, 4, nb);
        // the recurrence of the isotropic correction's input starts from zero
        // moments (the pass's first iteration takes p = r and dx = alpha ph +
        // omega sh, so p, v and dx need no clearing)
        if (iso) hipLaunchKernelGGL(zero2_kernel, dim3(nbc), dim3(B2), 0, st, c->yP, c->mv, c->N);
        if (hipMemcpyAsync(c->h_fl, c->fl, F_NF * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
            return GRTE_E_HIP;
        if (hipMemcpyAsync(c->h_sc, c->sc, S_NS * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
            return GRTE_E_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return GRTE_E_HIP;
        const double prev = res;
        res = c->h_sc[S_BB] > 0 ? sqrt(c->h_sc[S_RR] / c->h_sc[S_BB]) : 0.0;
        // accept the iterate when its true residual meets the tolerance, or when
        // a pass of iterations no longer reduces it and it lies within KRY_FLOOR
        // units of binary64 rounding of || |A| |x| + |b| || / ||b|| (the
        // normwise backward-error floor) or of the tolerance, whichever is larger
        if (c->h_fl[F_STATE] == 1 || c->h_sc[S_BB] == 0.0) {
            state = 1;
            break;
        }
        const double lvl = c->h_sc[S_BB] > 0 ? 0x1p-53 * sqrt(c->h_sc[S_MM] / c->h_sc[S_BB]) : 0.0;
        if (restart > 0 && res > 0.5 * prev && res <= KRY_FLOOR * fmax(c->tol, lvl)) {
            state = 1;
            floor = 1;
            break;
        }
        if (restart == KRY_RESTARTS || its_total >= c->maxit) break;
        A.maxit = c->maxit - its_total;    // the cap holds for the whole solve
        int inpass = 0;                    // iterations enqueued in this pass
        while (true) {
            const bool timed = c->profiling != 0 && narrow;   // the binary32 products only
            const int last = c->last_its[S.corr][restart], left = last - inpass;
            const int batch = last < 0 ? CHUNK : (left >= 1 ? std::min(CHUNK, left) : 2);
            inpass += batch;
            for (int k = 0; k < batch; ++k) {
                if (iso) {
                    hipLaunchKernelGGL(ymom2d_kernel, dim3(nbc), dim3(B2), 0, st, A, 0, (int)c->N);
                    iso_solve(c, S, c->yP, c->dP, st);
                }
                hipLaunchKernelGGL(pupd2d_kernel<V>, dim3(nb), dim3(B2), 0, st, A);
                if (timed && k == 0) (void)hipEventRecord(c->ev0, st);
                hipLaunchKernelGGL((apply2d_col_kernel<1, V>), dim3(nbo), dim3(B2), 0, st, A, ncol, ntile);
                if (timed && k == 0) (void)hipEventRecord(c->ev1, st);
                fin(1, 1, nbo);
                if (iso) {
                    hipLaunchKernelGGL(ymom2d_kernel, dim3(nbc), dim3(B2), 0, st, A, 1, (int)c->N);
                    iso_solve(c, S, c->yS, c->dS, st);
                }
                hipLaunchKernelGGL(supd2d_kernel<V>, dim3(nb), dim3(B2), 0, st, A);
                hipLaunchKernelGGL((apply2d_col_kernel<2, V>), dim3(nbo), dim3(B2), 0, st, A, ncol, ntile);
                fin(2, 2, nbo);
                hipLaunchKernelGGL(xupd2d_kernel<V>, dim3(nb), dim3(B2), 0, st, A);
                fin(3, 2, nb);
            }
            if (hipGetLastError() != hipSuccess) return GRTE_E_HIP;
            if (hipMemcpyAsync(c->h_fl, c->fl, F_NF * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
                return GRTE_E_HIP;
            if (hipStreamSynchronize(st) != hipSuccess) return GRTE_E_HIP;
            if (timed) {
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) {
                    c->prof_ms += ms;
                    ++c->prof_n;
                }
            }
            if (c->h_fl[F_STATE] != 0) break;
        }
        its_total += c->h_fl[F_ITS];
        pass_its[restart] = c->h_fl[F_ITS];
        hipLaunchKernelGGL(xadd_kernel<V>, dim3(nb), dim3(B2), 0, st, c->x, (const void *)c->dxv, c->nE, c->fl);
        // the recursion's residual has met the tolerance (or broken down): the
        // next pass recomputes the true residual and restarts from it if needed
        if (c->h_fl[F_STATE] == 3 && its_total >= c->maxit) {
            // one more true residual for the report
            hipLaunchKernelGGL(reset_flags_kernel, dim3(1), dim3(64), 0, st, c->fl);
            hipLaunchKernelGGL(residual2d_kernel<V>, dim3(nb), dim3(B2), 0, st, A);
            fin(0, 4, nb);
            if (hipMemcpyAsync(c->h_sc, c->sc, S_NS * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
                return GRTE_E_HIP;
            if (hipStreamSynchronize(st) != hipSuccess) return GRTE_E_HIP;
            res = c->h_sc[S_BB] > 0 ? sqrt(c->h_sc[S_RR] / c->h_sc[S_BB]) : 0.0;
            state = 0;
            break;
        }
    }
    for (int k = 0; k <= KRY_RESTARTS; ++k) c->last_its[S.corr][k] = pass_its[k];
    its_out = its_total;
    state_out = state;
    res_out = res;
    floor_out = floor;
    return GRTE_OK;
}

// BiCGStab on the system currently described by the coefficient arrays, with
// binary32 Krylov vectors where allowed and where the block inverse is well
// enough conditioned for them (every cell's Sherman-Morrison denominator at
// least KRY_F32_GAP; the correction's blocks are diagonal), else binary64 ones
grte_status krylov(grte2d_ctx *c, const Sys &S, int &its_out, int &state_out, double &res_out, int &floor_out)
{
    hipStream_t st = c->stream;
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, st, c->narrow, c->narrow_ok);
    hipLaunchKernelGGL(pgc2d_kernel, dim3(nblocks(c->nE)), dim3(B2), 0, st, S, c->idg, c->idg32, c->pgc, c->narrow,
                       c->nE);
    hipLaunchKernelGGL(opc2d_kernel, dim3(nblocks(c->N)), dim3(B2), 0, st, S, c->opc);
    int narrow = c->narrow_ok;
    if (narrow && !S.corr) {
        if (hipMemcpyAsync(c->h_fl, c->narrow, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
            return GRTE_E_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return GRTE_E_HIP;
        narrow = c->h_fl[0];
    }
    c->narrow_used[S.corr] = narrow;
    return narrow ? krylov_run<float>(c, S, its_out, state_out, res_out, floor_out)
                  : krylov_run<double>(c, S, its_out, state_out, res_out, floor_out);
}

}  // namespace

extern "C" {

grte_status grte2d_circle_directions(int nv, double *mu, double *eta, double *omega)
{
    if (!mu || !eta || !omega || nv < 4 || nv % 4 || nv > 128) return GRTE_E_INVAL;
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < nv / 2; ++k) {
        const double th = 2.0 * pi * (k + 0.5) / nv;
        mu[k] = cos(th);
        eta[k] = sin(th);
        omega[k] = 2.0 / nv;
    }
    return GRTE_OK;
}

grte_status grte2d_create(const grte2d_problem *pb, const double *mu, const double *eta, const double *omega,
                          grte2d_ctx **out)
{
    if (!pb || !mu || !eta || !omega || !out) return GRTE_E_INVAL;
    *out = nullptr;
    const int P = pb->npairs;
    if (pb->nx < 2 || pb->ny < 2 || P < 1 || P > 64 || (P & (P - 1))) return GRTE_E_UNSUPPORTED;
    if (!(pb->lx > 0) || !(pb->ly > 0) || !(pb->a > 0) || !(pb->c > 0) || !(pb->cv > 0)) return GRTE_E_INVAL;
    if (pb->opacity_law != 0 && pb->opacity_law != 3) return GRTE_E_INVAL;
    if ((size_t)pb->nx * pb->ny > (size_t)1 << 28) return GRTE_E_UNSUPPORTED;
    // 32-bit indexing of the face arrays of every pair
    if ((size_t)(pb->nx + 1) * (pb->ny + 1) * P >= ((size_t)1 << 31)) return GRTE_E_UNSUPPORTED;
    for (int p = 0; p < P; ++p)
        if (!(eta[p] > 0.0) || mu[p] == 0.0 || !(omega[p] > 0.0)) return GRTE_E_INVAL;
    grte2d_ctx *c = new (std::nothrow) grte2d_ctx();
    if (!c) return GRTE_E_NOMEM;
    for (auto &kind : c->last_its)
        for (int &n : kind) n = -1;
    c->nx = pb->nx;
    c->ny = pb->ny;
    c->P = P;
    c->m = pb->opacity_law;
    c->lx = pb->lx;
    c->ly = pb->ly;
    c->a = pb->a;
    c->c = pb->c;
    c->cv = pb->cv;
    c->W1 = 0.0;
    for (int p = 0; p < P; ++p) {
        c->W1 += omega[p];
        c->Mxx += omega[p] * mu[p] * mu[p];
        c->Myy += omega[p] * eta[p] * eta[p];
        c->Sx += omega[p] * fabs(mu[p]);
        c->Sy += omega[p] * fabs(eta[p]);
    }
    c->N = (size_t)c->nx * c->ny;
    c->nE = c->N * P;
    // multigrid levels of the isotropic correction: halve while both sides exceed 4
    {
        int lx = c->nx, ly = c->ny;
        while (true) {
            grte2d_ctx::Lv L;
            L.R.nx = lx;
            L.R.ny = ly;
            L.R.d = L.R.wl = L.R.wr = L.R.wb = L.R.wt = nullptr;
            L.b = L.z0 = L.z1 = nullptr;
            c->mg.push_back(L);
            if (lx <= 4 || ly <= 4 || c->mg.size() >= 16) break;
            lx = (lx + 1) / 2;
            ly = (ly + 1) / 2;
        }
    }
    c->nOx = (size_t)c->ny * (c->nx + 1) * P;
    c->nOy = (size_t)(c->ny + 1) * c->nx * P;
    const size_t nfx = (size_t)c->ny * (c->nx + 1), nfy = (size_t)(c->ny + 1) * c->nx;
    bool ok = dalloc(c, c->mu, P) && dalloc(c, c->eta, P) && dalloc(c, c->om, P) && dalloc(c, c->b, 4 * P) &&
              dalloc(c, c->E, c->nE) && dalloc(c, c->Ox, c->nOx) && dalloc(c, c->Oy, c->nOy) &&
              dalloc(c, c->T, c->N) && dalloc(c, c->sigma0, c->N) && dalloc(c, c->E1, c->nE) &&
              dalloc(c, c->Ox1, c->nOx) && dalloc(c, c->Oy1, c->nOy) && dalloc(c, c->T1, c->N) &&
              dalloc(c, c->ax, nfx) && dalloc(c, c->gx, nfx) && dalloc(c, c->ay, nfy) && dalloc(c, c->gy, nfy) &&
              dalloc(c, c->lam, c->N) && dalloc(c, c->dmg, c->N) && dalloc(c, c->cg, c->N) &&
              dalloc(c, c->kco, c->N) && dalloc(c, c->rb0, c->N) && dalloc(c, c->rb1, c->N) &&
              dalloc(c, c->acU, c->N) && dalloc(c, c->beta, c->N) && dalloc(c, c->ustar, c->N) &&
              dalloc(c, c->Dv, c->N) && dalloc(c, c->rhon, c->N) && dalloc(c, c->bv, c->nE) &&
              dalloc(c, c->sab, c->N) && dalloc(c, c->ue, c->N) &&
              dalloc(c, c->yP, c->N) && dalloc(c, c->yS, c->N) && dalloc(c, c->dP, c->N) &&
              dalloc(c, c->rstar, c->N) && dalloc(c, c->bflux, c->N) && dalloc(c, c->rho1, c->N) && dalloc(c, c->tguess, c->N) &&
              dalloc(c, c->epart, 3 * ENERGY_BLOCKS) && dalloc(c, c->energy, 4) && dalloc(c, c->ecnt, 1) &&
              [&] {
                  for (auto &L : c->mg) {
                      const size_t m = (size_t)L.R.nx * L.R.ny;
                      if (!(dalloc(c, L.R.d, m) && dalloc(c, L.R.wl, m) && dalloc(c, L.R.wr, m) &&
                            dalloc(c, L.R.wb, m) && dalloc(c, L.R.wt, m) && dalloc(c, L.b, m) &&
                            dalloc(c, L.z0, m) && dalloc(c, L.z1, m)))
                          return false;
                  }
                  return true;
              }() &&
              dalloc(c, c->dS, c->N) && dalloc(c, c->itmp, c->N) && dalloc(c, c->idir, c->N) && dalloc(c, c->idir2, c->N) && dalloc(c, c->pgc, c->N) && dalloc(c, c->idg, c->nE) && dalloc(c, c->idg32, c->nE) && dalloc(c, c->opc, OPC_N * c->N) && dalloc(c, c->dxv, c->nE) && dalloc(c, c->narrow, 1) && dalloc(c, c->mr, c->N) && dalloc(c, c->mv, c->N) &&
              dalloc(c, c->x, c->nE) && dalloc(c, c->r, c->nE) &&
              dalloc(c, c->p, c->nE) && dalloc(c, c->ph, c->nE) && dalloc(c, c->v, c->nE) &&
              dalloc(c, c->s, c->nE) && dalloc(c, c->sh, c->nE) && dalloc(c, c->t, c->nE) &&
              dalloc(c, c->Es, c->nE) && dalloc(c, c->part, 4 * KRYB) && dalloc(c, c->part2, 4 * KRYB) && dalloc(c, c->sc, S_NS) &&
              dalloc(c, c->fl, F_NF) && dalloc(c, c->stat, 8);
    if (ok) ok = hipHostMalloc((void **)&c->h_fl, F_NF * sizeof(int)) == hipSuccess;
    if (ok) ok = hipHostMalloc((void **)&c->h_sc, S_NS * sizeof(double)) == hipSuccess;
    if (!ok) {
        grte2d_destroy(c);
        return GRTE_E_NOMEM;
    }
    bool hok = hipMemcpy(c->mu, mu, P * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
               hipMemcpy(c->eta, eta, P * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
               hipMemcpy(c->om, omega, P * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
               hipMemset(c->b, 0, 4 * P * sizeof(double)) == hipSuccess &&
               hipMemset(c->E, 0, c->nE * sizeof(double)) == hipSuccess &&
               hipMemset(c->Ox, 0, c->nOx * sizeof(double)) == hipSuccess &&
               hipMemset(c->Oy, 0, c->nOy * sizeof(double)) == hipSuccess &&
               hipMemset(c->T, 0, c->N * sizeof(double)) == hipSuccess &&
               hipMemset(c->bflux, 0, c->N * sizeof(double)) == hipSuccess &&
               hipMemset(c->energy, 0, 4 * sizeof(double)) == hipSuccess &&
               hipMemset(c->ecnt, 0, sizeof(unsigned)) == hipSuccess;
    if (hok) {
        std::vector<double> one(c->N, 1.0);
        hok = hipMemcpy(c->sigma0, one.data(), c->N * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!hok) {
        grte2d_destroy(c);
        return GRTE_E_HIP;
    }
    *out = c;
    return GRTE_OK;
}

grte_status grte2d_destroy(grte2d_ctx *c)
{
    if (!c) return GRTE_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (void *q : c->allocs) (void)hipFree(q);
    if (c->h_fl) (void)hipHostFree(c->h_fl);
    if (c->h_sc) (void)hipHostFree(c->h_sc);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return GRTE_OK;
}

grte_status grte2d_set_stream(grte2d_ctx *c, void *stream)
{
    if (!c) return GRTE_E_INVAL;
    c->stream = (hipStream_t)stream;
    return GRTE_OK;
}

grte_status grte2d_set_storage(grte2d_ctx *c, int fp32)
{
    if (!c || (fp32 != 0 && fp32 != 1)) return GRTE_E_INVAL;
    if (fp32 == c->f32) return GRTE_OK;
    if (fp32 && !c->E32) {
        if (!dalloc(c, c->E32, c->nE) || !dalloc(c, c->Ox32, c->nOx) || !dalloc(c, c->Oy32, c->nOy))
            return GRTE_E_NOMEM;
    }
    // switching on rounds the current state; switching off keeps the stored values
    grte_status s = convert2d(c, fp32 ? 1 : 0);
    if (s != GRTE_OK) return s;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return GRTE_E_HIP;
    c->f32 = fp32;
    return GRTE_OK;
}

grte_status grte2d_set_guess(grte2d_ctx *c, const grte_mlp *model, double accept_tol)
{
    if (!c || !(accept_tol >= 0) || !std::isfinite(accept_tol)) return GRTE_E_INVAL;
    c->guess_w = model ? model->wbf : nullptr;
    c->guess_norm = model ? model->norm : nullptr;
    c->guess_tol = accept_tol;
    return GRTE_OK;
}

grte_status grte2d_log_pairs(grte2d_ctx *c, float *dev_rows, long long cap_rows, long long *n_rows)
{
    if (!c || !dev_rows || !n_rows) return GRTE_E_INVAL;
    *n_rows = 0;
    if (!c->stepped || cap_rows < (long long)c->N) return GRTE_E_INVAL;
    // after the step T holds T^{n+1} and the second buffer T^n
    hipLaunchKernelGGL(log2d_kernel, dim3((unsigned)((c->N + B2 - 1) / B2)), dim3(B2), 0, c->stream, (int)c->N,
                       c->m, c->last_eps, c->last_dt, c->rstar, c->T1, c->T, c->sigma0, dev_rows);
    if (hipGetLastError() != hipSuccess) return GRTE_E_HIP;
    *n_rows = (long long)c->N;
    return GRTE_OK;
}

grte_status grte2d_set_isotropic_correction(grte2d_ctx *c, int kind, int steps)
{
    if (!c || kind < 0 || kind > 3 || steps < 1 || steps > 64) return GRTE_E_INVAL;
    c->iso_kind = kind;
    if (kind == 1 || kind == 3) c->iso_k = steps;
    if (kind == 2) c->mg_nu = steps;
    return GRTE_OK;
}

grte_status grte2d_set_profiling(grte2d_ctx *c, int on)
{
    if (!c) return GRTE_E_INVAL;
    if (on && !c->ev0) {
        if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) return GRTE_E_HIP;
    }
    c->profiling = on != 0;
    c->prof_ms = 0.0;
    c->prof_n = 0;
    return GRTE_OK;
}

grte_status grte2d_read_timing(grte2d_ctx *c, double *ms, int *count)
{
    if (!c || !ms || !count) return GRTE_E_INVAL;
    *ms = c->prof_ms;
    *count = c->prof_n;
    return GRTE_OK;
}

grte_status grte2d_set_solver(grte2d_ctx *c, double tol, int maxit)
{
    if (!c || !(tol > 0.0) || maxit < 1) return GRTE_E_INVAL;
    c->tol = tol;
    c->maxit = maxit;
    return GRTE_OK;
}

grte_status grte2d_set_launch_shape(grte2d_ctx *c, int items_per_thread, int first_level)
{
    if (!c || items_per_thread < 1 || items_per_thread > 64 || first_level < 1 || first_level > KRYB)
        return GRTE_E_INVAL;
    c->kry_items = items_per_thread;
    c->red_b = first_level;
    return GRTE_OK;
}

grte_status grte2d_set_krylov_storage(grte2d_ctx *c, int narrow)
{
    if (!c || (narrow != 0 && narrow != 1)) return GRTE_E_INVAL;
    c->narrow_ok = narrow;
    return GRTE_OK;
}

grte_status grte2d_set_opacity(grte2d_ctx *c, const double *sigma0, int on_device)
{
    if (!c || !sigma0) return GRTE_E_INVAL;
    if (!on_device) {
        for (size_t j = 0; j < c->N; ++j)
            if (!(sigma0[j] >= 0.0) || !std::isfinite(sigma0[j])) return GRTE_E_INVAL;
    }
    if (hipMemcpyAsync(c->sigma0, sigma0, c->N * sizeof(double),
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return GRTE_E_HIP;
    return hip_ok(hipStreamSynchronize(c->stream));
}

grte_status grte2d_set_inflow(grte2d_ctx *c, const double *b)
{
    if (!c || !b) return GRTE_E_INVAL;
    if (hipMemcpyAsync(c->b, b, 4 * c->P * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return GRTE_E_HIP;
    return hip_ok(hipStreamSynchronize(c->stream));
}

grte_status grte2d_set_state(grte2d_ctx *c, const double *E, const double *Ox, const double *Oy, const double *T,
                             int on_device)
{
    if (!c || !E || !Ox || !Oy || !T) return GRTE_E_INVAL;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipStream_t st = c->stream;
    c->stepped = 0;
    if (hipMemcpyAsync(c->E, E, c->nE * sizeof(double), k, st) != hipSuccess ||
        hipMemcpyAsync(c->Ox, Ox, c->nOx * sizeof(double), k, st) != hipSuccess ||
        hipMemcpyAsync(c->Oy, Oy, c->nOy * sizeof(double), k, st) != hipSuccess ||
        hipMemcpyAsync(c->T, T, c->N * sizeof(double), k, st) != hipSuccess)
        return GRTE_E_HIP;
    if (c->f32) {
        grte_status s = convert2d(c, 1);
        if (s != GRTE_OK) return s;
    }
    return hip_ok(hipStreamSynchronize(st));
}

grte_status grte2d_get_state(grte2d_ctx *c, double *E, double *Ox, double *Oy, double *T, int on_device)
{
    if (!c) return GRTE_E_INVAL;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipStream_t st = c->stream;
    if (c->f32) {   // the stored state: widen the binary32 arrays
        grte_status s = convert2d(c, 0);
        if (s != GRTE_OK) return s;
    }
    if ((E && hipMemcpyAsync(E, c->E, c->nE * sizeof(double), k, st) != hipSuccess) ||
        (Ox && hipMemcpyAsync(Ox, c->Ox, c->nOx * sizeof(double), k, st) != hipSuccess) ||
        (Oy && hipMemcpyAsync(Oy, c->Oy, c->nOy * sizeof(double), k, st) != hipSuccess) ||
        (T && hipMemcpyAsync(T, c->T, c->N * sizeof(double), k, st) != hipSuccess))
        return GRTE_E_HIP;
    return hip_ok(hipStreamSynchronize(st));
}

grte_status grte2d_get_intensity(grte2d_ctx *c, double eps, double *I, int on_device)
{
    if (!c || !I || !(eps > 0.0) || !std::isfinite(eps)) return GRTE_E_INVAL;
    if (c->f32) {   // the stored state
        grte_status s = convert2d(c, 0);
        if (s != GRTE_OK) return s;
    }
    int lgP = 0;
    while ((1 << lgP) < c->P) ++lgP;
    // a host destination is filled from a device buffer of 2 N P doubles,
    // allocated on first use
    if (!on_device && !c->ibuf && !dalloc(c, c->ibuf, 2 * c->nE)) return GRTE_E_NOMEM;
    double *dst = on_device ? I : c->ibuf;
    hipLaunchKernelGGL(intensity2d_kernel, dim3(nblocks(2 * c->nE)), dim3(B2), 0, c->stream, c->nx, c->ny, lgP, eps,
                       (const double *)c->E, (const double *)c->Ox, (const double *)c->Oy, dst);
    if (hipGetLastError() != hipSuccess) return GRTE_E_HIP;
    if (!on_device &&
        hipMemcpyAsync(I, dst, 2 * c->nE * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return GRTE_E_HIP;
    return hip_ok(hipStreamSynchronize(c->stream));
}

grte_status grte2d_get_stage(grte2d_ctx *c, int which, double *out, int on_device)
{
    if (!c || !out) return GRTE_E_INVAL;
    const double *src = nullptr;
    size_t n = c->N;
    switch (which) {
        case GRTE2D_STAGE_ESTAR: src = c->Es; n = c->nE; break;
        case GRTE2D_STAGE_USTAR: src = c->ustar; break;
        case GRTE2D_STAGE_D: src = c->Dv; break;
        case GRTE2D_STAGE_RHON: src = c->rhon; break;
        default: return GRTE_E_INVAL;
    }
    if (hipMemcpyAsync(out, src, n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
        return GRTE_E_HIP;
    return hip_ok(hipStreamSynchronize(c->stream));
}

grte_status grte2d_step(grte2d_ctx *c, double dt, double eps, grte2d_step_info *info)
{
    if (!c || !(dt > 0.0) || !(eps > 0.0) || !std::isfinite(dt) || !std::isfinite(eps)) return GRTE_E_INVAL;
    hipStream_t st = c->stream;
    const int nbc = nblocks(c->N), nb = nblocks(c->nE);
    grte2d_step_info inf;
    memset(&inf, 0, sizeof(inf));
    if (hipMemsetAsync(c->stat, 0, 8 * sizeof(int), st) != hipSuccess) return GRTE_E_HIP;
    if (c->f32) {   // the step reads the stored (binary32) state, widened to binary64
        grte_status s = convert2d(c, 0);
        if (s != GRTE_OK) return s;
    }

    // ---- prediction (4.5)/(5.2)
    CoefArgs ca;
    ca.nx = c->nx;
    ca.ny = c->ny;
    ca.m = c->m;
    ca.corr = 0;
    ca.a = c->a;
    ca.c = c->c;
    ca.cv = c->cv;
    ca.eps = eps;
    ca.dt = dt;
    ca.fe = 1.0;
    ca.W1 = c->W1;
    ca.T = c->T;
    ca.sigma0 = c->sigma0;
    ca.ax = c->ax;
    ca.gx = c->gx;
    ca.ay = c->ay;
    ca.gy = c->gy;
    ca.lam = c->lam;
    ca.dmg = c->dmg;
    ca.cg = c->cg;
    ca.kco = c->kco;
    ca.rb0 = c->rb0;
    ca.acU = c->acU;
    ca.beta = c->beta;
    ca.sab = c->sab;
    ca.ue = c->ue;
    ca.rb1 = c->rb1;
    hipLaunchKernelGGL(coef2d_kernel, dim3(nbc), dim3(B2), 0, st, ca);
    Sys Sp = make_sys(c, 0, eps);
    {
        VecArgs A;
        A.S = Sp;
        A.n = c->nE;
        A.En = c->E;
        A.bv = c->bv;
        hipLaunchKernelGGL(rhs2d_kernel, dim3(nb), dim3(B2), 0, st, A);
    }
    if (hipMemcpyAsync(c->x, c->E, c->nE * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return GRTE_E_HIP;
    if (hipGetLastError() != hipSuccess) return GRTE_E_HIP;
    int its, state;
    double res;
    int floor;
    grte_status s = krylov(c, Sp, its, state, res, floor);
    if (s != GRTE_OK) return s;
    inf.pred_iters = its;
    inf.pred_converged = state == 1;
    inf.pred_narrow = c->narrow_used[0];
    inf.pred_residual = res;
    inf.pred_floor_stop = floor;
    if (hipMemcpyAsync(c->Es, c->x, c->nE * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return GRTE_E_HIP;

    // ---- correction, substep 1: Newton per cell
    NewtArgs na;
    na.S = Sp;
    na.Es = c->Es;
    na.En = c->E;
    na.Tn = c->T;
    na.sigma0 = c->sigma0;
    na.beta = c->beta;
    na.a = c->a;
    na.c = c->c;
    na.cv = c->cv;
    na.dt = dt;
    na.m = c->m;
    na.maxit = 60;
    na.Tnew = c->T1;
    na.ustar = c->ustar;
    na.Dv = c->Dv;
    na.rhon = c->rhon;
    na.stat = c->stat;
    na.rstar = c->rstar;
    na.bflux = c->bflux;
    na.tg = c->tguess;
    na.gtol = c->guess_tol;
    hipLaunchKernelGGL(moments2d_kernel, dim3(kblocks(c->nE, KRY_ITEMS)), dim3(B2), 0, st, na);
    // (one thread per cell; fewer, longer-lived blocks: one atomic per wavefront and counter)
    const int nbn = std::min(nbc, 2048);
    if (c->guess_w) {
        GuessArgs ga;
        ga.n = (int)c->N;
        ga.P = c->P;
        ga.m = c->m;
        ga.eps = eps;
        ga.dt = dt;
        ga.Es = c->Es;
        ga.Tn = c->T;
        ga.sigma0 = c->sigma0;
        ga.om = c->om;
        ga.gw = c->guess_w;
        ga.gnorm = c->guess_norm;
        ga.tg = c->tguess;
        hipLaunchKernelGGL(guess2d_kernel, dim3(nbc), dim3(B2), 0, st, ga);
        hipLaunchKernelGGL(newton2d_kernel<true>, dim3(nbn), dim3(B2), 0, st, na);
    } else {
        hipLaunchKernelGGL(newton2d_kernel<false>, dim3(nbn), dim3(B2), 0, st, na);
    }

    // ---- correction, substep 2 (4.11) with K^{n+1}, U^{n+1}
    ca.corr = 1;
    ca.fe = eps;
    ca.T = c->T1;
    hipLaunchKernelGGL(coef2d_kernel, dim3(nbc), dim3(B2), 0, st, ca);
    Sys Sc = make_sys(c, 1, eps);
    {
        VecArgs A;
        A.S = Sc;
        A.n = c->nE;
        A.En = c->E;
        A.bv = c->bv;
        hipLaunchKernelGGL(rhs2d_kernel, dim3(nb), dim3(B2), 0, st, A);
    }
    hipLaunchKernelGGL(xcorr0_kernel, dim3(nb), dim3(B2), 0, st, c->x, c->Es, c->acU, c->P, 1.0 / eps, c->nE);
    if (hipGetLastError() != hipSuccess) return GRTE_E_HIP;
    s = krylov(c, Sc, its, state, res, floor);
    if (s != GRTE_OK) return s;
    inf.corr_iters = its;
    inf.corr_converged = state == 1;
    inf.corr_narrow = c->narrow_used[1];
    inf.corr_residual = res;
    inf.corr_floor_stop = floor;

    // ---- projection (4.14)
    ProjArgs pa;
    pa.S = Sc;
    pa.EJ = c->x;
    pa.E1 = c->E1;
    pa.Ox1 = c->Ox1;
    pa.Oy1 = c->Oy1;
    pa.rho1 = c->rho1;
    hipLaunchKernelGGL(project2d_kernel, dim3(nb), dim3(B2), 0, st, pa);
    {
        EnergyArgs ea;
        ea.n = (int)c->N;
        ea.nb = energy_blocks(c->N);
        ea.dxdy = (c->lx / c->nx) * (c->ly / c->ny);
        ea.c = c->c;
        ea.cv = c->cv;
        ea.dt = dt;
        ea.nx = c->nx;
        ea.ny = c->ny;
        ea.rhon = c->rhon;
        ea.Tn = c->T;
        ea.rho1 = c->rho1;
        ea.Tnew = c->T1;
        ea.bflux = c->bflux;
        ea.epart = c->epart;
        ea.ecnt = c->ecnt;
        ea.energy = c->energy;
        hipLaunchKernelGGL(energy2d_kernel, dim3(ea.nb), dim3(B2), 0, st, ea);
    }
    if (hipGetLastError() != hipSuccess) return GRTE_E_HIP;
    std::swap(c->E, c->E1);
    std::swap(c->Ox, c->Ox1);
    std::swap(c->Oy, c->Oy1);
    std::swap(c->T, c->T1);
    if (c->f32) {   // store the new state in binary32
        grte_status s2 = convert2d(c, 1);
        if (s2 != GRTE_OK) return s2;
    }
    int stat[8];
    double en[4];
    if (hipMemcpyAsync(stat, c->stat, 8 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return GRTE_E_HIP;
    if (hipMemcpyAsync(en, c->energy, sizeof(en), hipMemcpyDeviceToHost, st) != hipSuccess) return GRTE_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return GRTE_E_HIP;
    inf.energy_before = en[0];
    inf.energy_after = en[1];
    inf.boundary_flux_dt = en[2];
    inf.energy_defect = en[3];
    inf.newton_max_iters = stat[0];
    inf.newton_failed = stat[1];
    inf.kstar_clamped = stat[2];
    inf.negative_root = stat[3];
    inf.newton_total_iters = stat[4];
    inf.guess_accepted = stat[5];
    inf.guess_rejected = stat[6];
    inf.guess_started = stat[7];
    c->stepped = 1;
    c->last_eps = eps;
    c->last_dt = dt;
    if (info) *info = inf;
    const bool bad = !inf.pred_converged || !inf.corr_converged || inf.newton_failed;
    return bad ? GRTE_E_NOCONV : GRTE_OK;
}

}  // extern "C"
