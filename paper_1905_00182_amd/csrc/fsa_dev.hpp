// Device-side building blocks of the gfx950 solver: grid/physics descriptors passed to the
// kernels by value, boundary ghosts, the ideal-gas closure, the fifth-order reconstructions,
// the four-point delta and the sponge profile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsa {

enum : int { BC_PERIODIC = 0, BC_EXTRAP = 1, BC_INFLOW = 2, BC_NONREFLECT = 3 };
enum : int { WENO5JS = 0, TENO5 = 1, LEARNED = 2 };
enum : int { T_CONVX = 1, T_CONVY = 2, T_CONVZ = 4, T_VISC = 8, T_IB = 16, T_SPONGE = 32 };

// Grid and physics constants, copied into every kernel's argument block.
struct Grid {
    int dim;
    int n[3];
    long long ncell;
    double lo[3];
    double h, inv_h;
    int bc[3][2];
    // placement in a larger grid (a block of a decomposed domain): local cell i is global cell
    // i + org of a grid of gn cells (gncell in all); lo is the global grid's corner.  Cell
    // positions, the sponge and the inflow-noise counters are those of the global grid.
    int org[3];
    int gn[3];
    long long gncell;

    // global linear index of local cell (i, j, k)
    __host__ __device__ __forceinline__ long long glin(int i, int j, int k) const
    {
        return ((long long)(k + org[2]) * gn[1] + (j + org[1])) * gn[0] + (i + org[0]);
    }
};

struct Phys {
    double gamma, gm1, inv_gm1;
    double mu;
    double prim_inf[5];
    double q_inf[5];          // conserved far-field state
    double inflow_amp;
    unsigned long long seed;
    double sw[3][2];          // sponge widths
    double inv_sw[3][2];      // their reciprocals (0 where there is no sponge)
    double e_inf;             // far-field internal energy per volume, p_inf / (gamma - 1)
    double sigma;             // sponge sigma_max
    double weno_eps, teno_ct, teno_eps;
    int terms;
    // periodic Gaussian pressure source (3D): A_p = -src_amp exp(-src_bl2 |x - src_x|^2)
    // cos(src_omega t), src_bl2 = B log 2; src_amp = 0: none
    double src_amp, src_bl2, src_omega, src_x[3];
};

// ---------------------------------------------------------------------------------------
// Counter-based SplitMix64 (Steele, Lea & Flood 2014): output number ctr of the generator
// seeded with seed is the finaliser applied to seed + (ctr + 1) * golden increment.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

// Resolve one direction's index against its boundary; records the first inflow side.
__device__ __forceinline__ int resolve_index(int i, int n, int bclo, int bchi, int dir, int& inflow,
                                             int& side, int& depth)
{
    if (i < 0) {
        if (bclo == BC_PERIODIC) return ((i % n) + n) % n;
        if (bclo == BC_INFLOW && !inflow) { inflow = 1; side = 2 * dir; depth = -i; }
        return 0;
    }
    if (i >= n) {
        if (bchi == BC_PERIODIC) return i % n;
        if (bchi == BC_INFLOW && !inflow) { inflow = 1; side = 2 * dir + 1; depth = i - n + 1; }
        return n - 1;
    }
    return i;
}

// Conserved inflow ghost state: far field with the seeded velocity perturbation.  Evaluated
// without contraction, one rounding per operation, so that an unperturbed ghost equals the
// far-field state exactly (a uniform free stream then has an exactly zero right-hand side).
template <int DIM>
__device__ __forceinline__ void inflow_state(const Phys& P, long long step, long long ncell, long long lin, int side,
                                             int depth, double* q)
{
#pragma clang fp contract(off)
    const double rho = P.prim_inf[0];
    double ke = 0.0;
    q[0] = rho;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double u = P.prim_inf[1 + a];
        if (P.inflow_amp != 0.0) {
            const uint64_t ctr = ((((uint64_t)step * 6ull + (uint64_t)side) * 8ull + (uint64_t)depth)
                                      * (uint64_t)ncell + (uint64_t)lin) * 3ull + (uint64_t)a;
            u += P.inflow_amp * (2.0 * u01(splitmix64(P.seed, ctr)) - 1.0);
        }
        q[1 + a] = rho * u;
        ke += u * u;
    }
    q[DIM + 1] = P.e_inf + 0.5 * rho * ke;
}

// State at a possibly out-of-range cell (i, j, k): boundary ghosts resolved x, then y, then z.
template <int DIM>
__device__ __forceinline__ void fetch_state(const double* __restrict__ Q, const Grid& G, const Phys& P, long long step,
                                            int i, int j, int k, double* q)
{
    int inflow = 0, side = 0, depth = 0;
    i = resolve_index(i, G.n[0], G.bc[0][0], G.bc[0][1], 0, inflow, side, depth);
    j = resolve_index(j, G.n[1], G.bc[1][0], G.bc[1][1], 1, inflow, side, depth);
    if (DIM == 3) k = resolve_index(k, G.n[2], G.bc[2][0], G.bc[2][1], 2, inflow, side, depth);
    else k = 0;
    const long long lin = ((long long)k * G.n[1] + j) * G.n[0] + i;
    if (!inflow) {
#pragma unroll
        for (int c = 0; c < DIM + 2; ++c) q[c] = Q[c * G.ncell + lin];
        return;
    }
    inflow_state<DIM>(P, step, G.gncell, G.glin(i, j, k), side, depth, q);
}

// Reciprocal from the hardware estimate refined by two Newton steps (within an ulp or two of
// the correctly rounded 1/x for normal x), a quarter of the cost of an IEEE division.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// ---------------------------------------------------------------------------------------
// Fifth-order reconstruction at a face from five upwind-ordered values (a..e) =
// (v_{i-2}, ..., v_{i+2}): three third-order candidates with Jiang-Shu smoothness indicators,
// weighted WENO5-JS (alpha_k = d_k / (eps + beta_k)^2) or TENO5 (sharp cut-off of
// gamma_k = (1 + tau5 / (beta_k + eps))^6 at C_T, kept stencils weighted by d_k).
// Both are evaluated with reciprocals instead of divisions.
//
// TENO5's face value is a fixed linear form in (a..e) once the kept set is known: the
// candidates' coefficients weighted by d_k / (sum of kept d_j).  The eight keep patterns'
// forms are tabulated per block in LDS (row p, bit k = sub-stencil k kept; p = 0 does not
// occur and holds the full set), so the face value is one row lookup and five fused
// multiply-adds instead of three candidates, a weight sum and a reciprocal.
// ---------------------------------------------------------------------------------------
template <class T>
using KeepRows = T[8][8];   // [pattern][coefficient of a..e, 3 unused]

// Fill the table (lanes 0..7 of the block, one row each; the block synchronises before use).
// Each coefficient is formed in FP64 and rounded once to T.
template <class T>
__device__ __forceinline__ void init_keep_rows(KeepRows<T>& t, int tid)
{
    if (tid < 8) {
        const int p = tid == 0 ? 7 : tid;
        constexpr double dk[3] = {0.1, 0.6, 0.3};
        constexpr double cand[3][5] = {{1.0 / 3.0, -7.0 / 6.0, 11.0 / 6.0, 0.0, 0.0},
                                       {0.0, -1.0 / 6.0, 5.0 / 6.0, 1.0 / 3.0, 0.0},
                                       {0.0, 0.0, 1.0 / 3.0, 5.0 / 6.0, -1.0 / 6.0}};
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) sum += ((p >> k) & 1) ? dk[k] : 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) v += ((p >> k) & 1) ? dk[k] * cand[k][j] : 0.0;
            t[tid][j] = (T)(v / sum);
        }
#pragma unroll
        for (int j = 5; j < 8; ++j) t[tid][j] = T(0);
    }
}

// Face value of keep pattern p from its table row.
template <class T>
__device__ __forceinline__ T keep_sum(const T* row, T a, T b, T c, T d, T e)
{
    return fma(row[4], e, fma(row[3], d, fma(row[2], c, fma(row[1], b, row[0] * a))));
}

struct Recon {
    double eps;                  // WENO epsilon or TENO epsilon
    double ct;                   // TENO cut-off
    const double (*rows)[8];     // TENO5: keep-pattern table (LDS)
};

// TENO5 keeps every sub-stencil whenever tau5 <= T (beta_min + eps) with
// T = (3 C_T)^(-1/6) (1 - 1e-2) - 1: then each x_k = 1 + tau5 / (beta_k + eps) lies in
// [1, 1 + T], so gamma_k = x_k^6 >= 1 while C_T (gamma_0 + gamma_1 + gamma_2) <= 3 C_T (1 + T)^6
// < 0.95, below every gamma_k; the 1% margin covers the rounding of both evaluations many
// times over.  (The FP32 form's normalised test, x_k = (1 + a_k) / (1 + a_max) >= 1 / (1 + T),
// is certified by the same bound.)  Negative for C_T >= 1/3: the certificate never holds.
__host__ __device__ inline double teno_all_kept_bound(double ct)
{
    return ct > 0.0 ? pow(3.0 * ct, -1.0 / 6.0) * (1.0 - 1e-2) - 1.0 : -1.0;
}

// Jiang-Shu smoothness indicators of the three sub-stencils (FP64).
__device__ __forceinline__ void js_beta(double a, double b, double c, double d, double e, double& b0, double& b1,
                                        double& b2)
{
    const double s0 = fma(-2.0, b, a) + c, t0 = fma(-4.0, b, a) + 3.0 * c;
    const double s1 = fma(-2.0, c, b) + d, t1 = b - d;
    const double s2 = fma(-2.0, d, c) + e, t2 = fma(-4.0, d, 3.0 * c) + e;
    b0 = fma(13.0 / 12.0 * s0, s0, 0.25 * t0 * t0);
    b1 = fma(13.0 / 12.0 * s1, s1, 0.25 * t1 * t1);
    b2 = fma(13.0 / 12.0 * s2, s2, 0.25 * t2 * t2);
}

// TENO5 keep pattern (bit k = sub-stencil k kept) from the indicators: chi_k < C_T cuts,
// tested as gamma_k < C_T sum gamma.
__device__ __forceinline__ int teno_keep_beta(double b0, double b1, double b2, const Recon& R)
{
    const double tau = fabs(b0 - b2);
    const double e0 = b0 + R.eps, e1 = b1 + R.eps, e2 = b2 + R.eps;
    const double e01 = e0 * e1;
    const double inv = rcp_nr(e01 * e2);
    const double r0 = (e1 * e2) * inv, r1 = (e0 * e2) * inv, r2 = e01 * inv;  // 1 / e_k
    const double x0 = fma(tau, r0, 1.0), x1 = fma(tau, r1, 1.0), x2 = fma(tau, r2, 1.0);
    const double c0 = x0 * x0 * x0, c1 = x1 * x1 * x1, c2 = x2 * x2 * x2;
    const double g0 = c0 * c0, g1 = c1 * c1, g2 = c2 * c2;
    const double lim = R.ct * (g0 + g1 + g2);
    return (g0 < lim ? 0 : 1) | (g1 < lim ? 0 : 2) | (g2 < lim ? 0 : 4);
}

// TENO5 keep pattern of the five upwind-ordered values (what recon5<TENO5> decides).
__device__ __forceinline__ int teno_keep5(double a, double b, double c, double d, double e, const Recon& R)
{
    double b0, b1, b2;
    js_beta(a, b, c, d, e, b0, b1, b2);
    return teno_keep_beta(b0, b1, b2, R);
}

template <int SCHEME>
__device__ __forceinline__ double recon5(double a, double b, double c, double d, double e, const Recon& R);

// recon5 with a wave-wide shortcut for TENO5: when every active lane of the wave holds the
// all-kept certificate (teno_all_kept_bound(C_T) = tall), the face value takes the all-kept row of the
// table without the weights -- the decision the full test takes for these values, so the same
// value bit for bit.  Call with the whole wave converged at the call (a wave-uniform branch).
template <int SCHEME>
__device__ __forceinline__ double recon5w(double a, double b, double c, double d, double e, const Recon& R,
                                          double tall)
{
    if constexpr (SCHEME == TENO5) {
        double b0, b1, b2;
        js_beta(a, b, c, d, e, b0, b1, b2);
        const double bmin = fmin(b0, fmin(b1, b2));
        const bool cert = fabs(b0 - b2) <= tall * (bmin + R.eps);
        if (__ballot(!cert) == 0ull) return keep_sum(R.rows[7], a, b, c, d, e);
        return keep_sum(R.rows[teno_keep_beta(b0, b1, b2, R)], a, b, c, d, e);
    } else {
        return recon5<SCHEME>(a, b, c, d, e, R);
    }
}

template <int SCHEME>
__device__ __forceinline__ double recon5(double a, double b, double c, double d, double e, const Recon& R)
{
    double b0, b1, b2;
    js_beta(a, b, c, d, e, b0, b1, b2);
    if (SCHEME == WENO5JS) {
        const double q0 = fma(11.0 / 6.0, c, fma(-7.0 / 6.0, b, (1.0 / 3.0) * a));
        const double q1 = fma(1.0 / 3.0, d, fma(5.0 / 6.0, c, (-1.0 / 6.0) * b));
        const double q2 = fma(-1.0 / 6.0, e, fma(5.0 / 6.0, d, (1.0 / 3.0) * c));
        const double e0 = R.eps + b0, e1 = R.eps + b1, e2 = R.eps + b2;
        const double p0 = e0 * e0, p1 = e1 * e1, p2 = e2 * e2;
        // alpha_k proportional to d_k * prod_{j != k} (eps + beta_j)^2
        const double w0 = 0.1 * (p1 * p2), w1 = 0.6 * (p0 * p2), w2 = 0.3 * (p0 * p1);
        const double num = fma(w0, q0, fma(w1, q1, w2 * q2));
        return num * rcp_nr(w0 + w1 + w2);
    } else {
        return keep_sum(R.rows[teno_keep_beta(b0, b1, b2, R)], a, b, c, d, e);
    }
}

// FP32 reconstruction of the precision form.  Same candidates and indicators; WENO5-JS as in
// FP64; TENO5 in the normalised form gamma_k / gamma_max = ((1 + a_k) / (1 + a_max))^6,
// a_k = tau5 / (beta_k + eps32), which cannot overflow in FP32 (eps32 = 1e-30 replaces the
// FP64 1e-40, a subnormal in FP32); the cut-off test is the same ratio test.
struct Recon32 {
    float eps;
    float ct;
    const float (*rows)[8];   // TENO5 / learned: keep-pattern table (LDS)
};

template <int SCHEME>
__device__ __forceinline__ float recon5f(float a, float b, float c, float d, float e, const Recon32& R)
{
    const float s0 = fmaf(-2.0f, b, a) + c, t0 = fmaf(-4.0f, b, a) + 3.0f * c;
    const float s1 = fmaf(-2.0f, c, b) + d, t1 = b - d;
    const float s2 = fmaf(-2.0f, d, c) + e, t2 = fmaf(-4.0f, d, 3.0f * c) + e;
    const float b0 = fmaf(13.0f / 12.0f * s0, s0, 0.25f * t0 * t0);
    const float b1 = fmaf(13.0f / 12.0f * s1, s1, 0.25f * t1 * t1);
    const float b2 = fmaf(13.0f / 12.0f * s2, s2, 0.25f * t2 * t2);
    if (SCHEME == WENO5JS) {
        const float q0 = fmaf(11.0f / 6.0f, c, fmaf(-7.0f / 6.0f, b, (1.0f / 3.0f) * a));
        const float q1 = fmaf(1.0f / 3.0f, d, fmaf(5.0f / 6.0f, c, (-1.0f / 6.0f) * b));
        const float q2 = fmaf(-1.0f / 6.0f, e, fmaf(5.0f / 6.0f, d, (1.0f / 3.0f) * c));
        const float e0 = R.eps + b0, e1 = R.eps + b1, e2 = R.eps + b2;
        const float w0 = 0.1f * __builtin_amdgcn_rcpf(e0 * e0);
        const float w1 = 0.6f * __builtin_amdgcn_rcpf(e1 * e1);
        const float w2 = 0.3f * __builtin_amdgcn_rcpf(e2 * e2);
        const float num = fmaf(w0, q0, fmaf(w1, q1, w2 * q2));
        return num * __builtin_amdgcn_rcpf(w0 + w1 + w2);
    } else {
        const float tau = fabsf(b0 - b2);
        const float a0 = tau * __builtin_amdgcn_rcpf(b0 + R.eps);
        const float a1 = tau * __builtin_amdgcn_rcpf(b1 + R.eps);
        const float a2 = tau * __builtin_amdgcn_rcpf(b2 + R.eps);
        const float inv = __builtin_amdgcn_rcpf(1.0f + fmaxf(a0, fmaxf(a1, a2)));
        const float x0 = (1.0f + a0) * inv, x1 = (1.0f + a1) * inv, x2 = (1.0f + a2) * inv;
        const float c0 = x0 * x0 * x0, c1 = x1 * x1 * x1, c2 = x2 * x2 * x2;
        const float g0 = c0 * c0, g1 = c1 * c1, g2 = c2 * c2;
        const float lim = R.ct * (g0 + g1 + g2);
        const int keep = (g0 < lim ? 0 : 1) | (g1 < lim ? 0 : 2) | (g2 < lim ? 0 : 4);
        return keep_sum(R.rows[keep], a, b, c, d, e);
    }
}

// recon5f with the wave-wide all-kept shortcut of recon5w (TENO5).
template <int SCHEME>
__device__ __forceinline__ float recon5fw(float a, float b, float c, float d, float e, const Recon32& R, float tall)
{
    if constexpr (SCHEME == TENO5) {
        const float s0 = fmaf(-2.0f, b, a) + c, t0 = fmaf(-4.0f, b, a) + 3.0f * c;
        const float s1 = fmaf(-2.0f, c, b) + d, t1 = b - d;
        const float s2 = fmaf(-2.0f, d, c) + e, t2 = fmaf(-4.0f, d, 3.0f * c) + e;
        const float b0 = fmaf(13.0f / 12.0f * s0, s0, 0.25f * t0 * t0);
        const float b1 = fmaf(13.0f / 12.0f * s1, s1, 0.25f * t1 * t1);
        const float b2 = fmaf(13.0f / 12.0f * s2, s2, 0.25f * t2 * t2);
        const bool cert = fabsf(b0 - b2) <= tall * (fminf(b0, fminf(b1, b2)) + R.eps);
        if (__ballot(!cert) == 0ull) return keep_sum(R.rows[7], a, b, c, d, e);
    }
    return recon5f<SCHEME>(a, b, c, d, e, R);
}

// FP32 reconstruction with the sub-stencils given by keep bits (bit k = sub-stencil k, 1..7):
// the learned form.  The same table row as recon5f's TENO5 branch, so the same bits give the
// same value.
__device__ __forceinline__ float recon5_bits(float a, float b, float c, float d, float e, int bits,
                                             const float (*rows)[8])
{
    return keep_sum(rows[bits], a, b, c, d, e);
}

// ---------------------------------------------------------------------------------------
// Peskin four-point function (piecewise on |r| < 1, 1 <= |r| < 2).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double delta4(double r)
{
    const double x = fabs(r);
    if (x < 1.0) return 0.125 * (3.0 - 2.0 * x + sqrt(fma(-4.0 * x, x, fma(4.0, x, 1.0))));
    if (x < 2.0) return 0.125 * (5.0 - 2.0 * x - sqrt(fma(-4.0 * x, x, fma(12.0, x, -7.0))));
    return 0.0;
}

// Position in cell-index units along one direction: (X - lo) / h - 1/2.
__device__ __forceinline__ double cell_coord(double X, double lo, double h) { return (X - lo) / h - 0.5; }

// Four-point support along one direction: first cell j0 and the weights lambda(r0 - j) of
// cells j = j0..j0+3.
__device__ __forceinline__ void support4(double X, double lo, double h, int& j0, double* w)
{
    const double r0 = cell_coord(X, lo, h);
    j0 = (int)floor(r0) - 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) w[m] = delta4(r0 - (double)(j0 + m));
}

// ---------------------------------------------------------------------------------------
// Cubic sponge: depth ratio into the layers along one direction, clipped to [0, 1]; the
// rate is sigma_max * (max over directions of the ratio)^3.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double sponge_eta(double x, double lo, double hi, double wl, double wh, double iwl,
                                            double iwh)
{
    double eta = 0.0;
    if (wl > 0.0 && x < lo + wl) eta = fmax(eta, (lo + wl - x) * iwl);
    if (wh > 0.0 && x > hi - wh) eta = fmax(eta, (x - (hi - wh)) * iwh);
    return fmin(eta, 1.0);
}

// Grid and physics constants as the kernels read them: one block in device memory, so that
// rarely used fields are fetched with scalar loads where they are needed.
struct KConst {
    Grid G;
    Phys P;
    double inv12h;
    double Fx_inf[5], Fy_inf[5], Fz_inf[5];   // physical fluxes of the far-field state
    double sig[3];      // 1e-8 times the natural scales of rho, velocity and p (rho_inf, c_inf,
                        // rho_inf c_inf^2): significance threshold and feature floor of the
                        // learned selector
    double teno_tall;   // TENO5 all-kept certificate bound (teno_all_kept_bound)

    __device__ __forceinline__ double eta_dir(int d, int i) const
    {
        const double x = G.lo[d] + ((double)(i + G.org[d]) + 0.5) * G.h;
        return sponge_eta(x, G.lo[d], G.lo[d] + (double)G.gn[d] * G.h, P.sw[d][0], P.sw[d][1], P.inv_sw[d][0],
                          P.inv_sw[d][1]);
    }
};

// ---------------------------------------------------------------------------------------
// Characteristic-wise reconstruction: the eigenvectors of the flux Jacobian along D at the
// Roe average of a face's two cells (Roe 1981).  With r = sqrt(rho) weights, the velocity u
// and the total enthalpy H = (E + p)/rho are averaged, c^2 = (gamma - 1)(H - |u|^2/2),
// b1 = (gamma - 1)/c^2, b2 = b1 |u|^2/2.  Fields k = 0: u_n - c, 1: entropy, 2..DIM: shear
// along the tangential directions in increasing order, DIM + 1: u_n + c.  Left rows
//   u_n -+ c: [(b2 +- u_n/c)/2, -(b1 u +- e_n/c)/2, b1/2]
//   entropy:  [1 - b2, b1 u, -b1]        shear t: [-u_t, e_t, 0]
// and right columns
//   u_n -+ c: [1, u -+ c e_n, H -+ u_n c]
//   entropy:  [1, u, |u|^2/2]            shear t: [0, e_t, u_t].
// ---------------------------------------------------------------------------------------
template <int DIM, int D>
struct RoeVec {
    static constexpr int NQ = DIM + 2;
    double u[DIM];
    double H, c, ic, b1, b2, q2h;

    // tangential direction of shear field k (2 <= k <= DIM)
    static constexpr int tang(int k) { return (k - 2) < D ? k - 2 : k - 1; }

    // qa, qb conserved states [NQ], pa, pb their pressures
    __device__ __forceinline__ RoeVec(const double* qa, double pa, const double* qb, double pb, double gm1)
    {
        const double ra = sqrt(qa[0]), rb = sqrt(qb[0]);
        const double iw = 1.0 / (ra + rb);
        const double ira = 1.0 / ra, irb = 1.0 / rb;     // r / rho = 1 / r
        double q2 = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            u[a] = (qa[1 + a] * ira + qb[1 + a] * irb) * iw;
            q2 = fma(u[a], u[a], q2);
        }
        H = ((qa[NQ - 1] + pa) * ira + (qb[NQ - 1] + pb) * irb) * iw;
        q2h = 0.5 * q2;
        c = sqrt(gm1 * (H - q2h));
        ic = 1.0 / c;
        b1 = gm1 * ic * ic;
        b2 = b1 * q2h;
    }

    // g_k = l_k . f
    template <int K>
    __device__ __forceinline__ double left(const double* f) const
    {
        if constexpr (K == 0 || K == NQ - 1) {
            constexpr double sg = K == 0 ? 1.0 : -1.0;
            double g = 0.5 * fma(sg * u[D], ic, b2) * f[0];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const double la = a == D ? fma(b1, u[a], sg * ic) : b1 * u[a];
                g = fma(-0.5 * la, f[1 + a], g);
            }
            return fma(0.5 * b1, f[NQ - 1], g);
        } else if constexpr (K == 1) {
            double g = (1.0 - b2) * f[0];
#pragma unroll
            for (int a = 0; a < DIM; ++a) g = fma(b1 * u[a], f[1 + a], g);
            return fma(-b1, f[NQ - 1], g);
        } else {
            constexpr int t = tang(K);
            return fma(-u[t], f[0], f[1 + t]);
        }
    }

    // F += r_k g
    template <int K>
    __device__ __forceinline__ void right_add(double g, double* F) const
    {
        if constexpr (K == 0 || K == NQ - 1) {
            constexpr double sg = K == 0 ? -1.0 : 1.0;
            F[0] += g;
#pragma unroll
            for (int a = 0; a < DIM; ++a) F[1 + a] = fma(a == D ? fma(sg, c, u[a]) : u[a], g, F[1 + a]);
            F[NQ - 1] = fma(fma(sg * u[D], c, H), g, F[NQ - 1]);
        } else if constexpr (K == 1) {
            F[0] += g;
#pragma unroll
            for (int a = 0; a < DIM; ++a) F[1 + a] = fma(u[a], g, F[1 + a]);
            F[NQ - 1] = fma(q2h, g, F[NQ - 1]);
        } else {
            constexpr int t = tang(K);
            F[1 + t] += g;
            F[NQ - 1] = fma(u[t], g, F[NQ - 1]);
        }
    }
};

// One characteristic field KF of a face: the split fluxes of the six cells i-2..i+3,
// g+- = l_KF . (F +- alpha q)/2 = (l.F +- alpha l.q)/2, reconstructed (g+ from i-2..i+2,
// g- from i+3..i-1) and added to the face flux Fo along r_KF.
template <int SCHEME, int DIM, int D, int KF>
__device__ __forceinline__ void char_field(const RoeVec<DIM, D>& V, const double (&q)[6][DIM + 2],
                                           const double (&F)[6][DIM + 2], double alpha, const Recon& R, double* Fo)
{
    double gp[6], gm[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const double lq = V.template left<KF>(q[s]), lF = V.template left<KF>(F[s]);
        gp[s] = 0.5 * fma(alpha, lq, lF);
        gm[s] = 0.5 * fma(-alpha, lq, lF);
    }
    const double g = recon5<SCHEME>(gp[0], gp[1], gp[2], gp[3], gp[4], R) +
                     recon5<SCHEME>(gm[5], gm[4], gm[3], gm[2], gm[1], R);
    V.template right_add<KF>(g, Fo);
}

// Characteristic-wise face flux Fo[DIM + 2] from the six cells' conserved states q, their
// physical fluxes F along D and pressures p (the Roe average of cells 2 and 3, the two
// beside the face).
template <int SCHEME, int DIM, int D>
__device__ __forceinline__ void char_face(const double (&q)[6][DIM + 2], const double (&F)[6][DIM + 2],
                                          const double* p, double gm1, double alpha, const Recon& R, double* Fo)
{
    const RoeVec<DIM, D> V(q[2], p[2], q[3], p[3], gm1);
#pragma unroll
    for (int m = 0; m < DIM + 2; ++m) Fo[m] = 0.0;
    char_field<SCHEME, DIM, D, 0>(V, q, F, alpha, R, Fo);
    char_field<SCHEME, DIM, D, 1>(V, q, F, alpha, R, Fo);
    char_field<SCHEME, DIM, D, 2>(V, q, F, alpha, R, Fo);
    char_field<SCHEME, DIM, D, 3>(V, q, F, alpha, R, Fo);
    if constexpr (DIM == 3) char_field<SCHEME, DIM, D, 4>(V, q, F, alpha, R, Fo);
}

// NaN-propagating maximum of non-negative doubles through their bit patterns: for x >= 0
// the unsigned order of the bits is the numeric order, and every NaN pattern sorts above
// +Inf.
__device__ __forceinline__ unsigned long long max_bits(unsigned long long a, unsigned long long b)
{
    return a > b ? a : b;
}

}  // namespace fsa
