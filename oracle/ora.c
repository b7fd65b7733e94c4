/*
 * ora.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see ora.h).
 *
 * What it computes, in the paper's order (Wang, Tian & Lai, Sec. 2):
 *   1. the conservative compressible NS system dQ/dt + div(F,G,H) - div(F_v,G_v,H_v) = S
 *      (Sec. 2, Eqs. (2)-(6)) with the ideal-gas closure p = (gamma-1)(E - rho|u|^2/2);
 *   2. convective terms by conservative point-value finite differences with global
 *      Lax-Friedrichs flux splitting and fifth-order reconstruction: WENO5-JS (Jiang & Shu
 *      1996) or TENO5 (Fu, Hu & Adams 2016), the two schemes Sec. 2 names;
 *   3. viscous terms by the fourth-order central difference applied twice
 *      (velocity gradients at cells, then the divergence of the stress), no heat flux
 *      (Sec. 2, Eq. (5)-(6): b = u . tau);
 *   4. the penalty immersed boundary: interpolation of velocity to the markers (Eq. (8)),
 *      the feedback force F_f = alpha int(U_ib - U) dt + beta (U_ib - U) (Eq. (7)), and
 *      spreading of -F_f to the grid (Eq. (9)) with the tensor-product four-point
 *      delta function (Eqs. (10)-(11));
 *   5. a cubic sponge toward the far-field state;
 *   6. the third-order TVD (SSP) Runge-Kutta update (Shu & Osher 1988, cited in Sec. 2),
 *      the penalty integral advancing in lockstep with Q.
 *
 * The code is written to be read against the paper, not to be fast: every face flux is
 * computed from the six cells around it, every stress from the velocities around it.
 * Built with -O2 -fno-fast-math -ffp-contract=off; OpenMP only over loops with disjoint
 * writes; every sum runs in a fixed order.
 */
#include "ora.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Grids smaller than this run their loops on one thread: there a thread team's start-up and
 * barriers cost more than the loop (the results are the same either way: every loop has
 * disjoint writes and a fixed order per element). */
#define ORA_PAR_MIN_CELLS 16384

struct ora_ctx {
    ora_desc d;
    int nq;            /* dim + 2 conserved components */
    long nx, ny, nz;
    long ncell;
    double q_inf[5];   /* far-field conserved state */
    /* markers */
    int nm;
    double* X;         /* [dim][nm] */
    double* dV;        /* [nm] */
    double* U;         /* [dim][nm] */
    int motion;
    double omega;
    double* xi;        /* penalty integral [dim][nm] */
    double* F;         /* penalty force of the last right-hand side [dim][nm] */
    double* dxi;       /* U_ib - U of the last right-hand side [dim][nm] */
    /* probes */
    int np;
    double* Xp;
    double t;
    int64_t step;
    double* record;    /* if set: ora_rk3_step copies each stage's input state here (test hook) */
};

/* ------------------------------------------------------------------------------------ */
/* Small helpers                                                                          */
/* ------------------------------------------------------------------------------------ */

static long cell_index(const ora_ctx* c, long i, long j, long k) { return (k * c->ny + j) * c->nx + i; }

static long n_of(const ora_ctx* c, int d) { return d == 0 ? c->nx : (d == 1 ? c->ny : c->nz); }

uint64_t ora_splitmix64(uint64_t seed, uint64_t ctr)
{
    /* Steele, Lea & Flood (2014) SplitMix64: the state advances by the golden-ratio
     * increment, output number ctr is the finaliser applied to seed + (ctr+1) * increment. */
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform value in [0,1) from the top 53 bits. */
static double unit_uniform(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Far-field primitive state (rho, u_1..u_dim, p) -> conserved state. */
static void prim_to_cons(const ora_ctx* c, double rho, const double* u, double p, double* q)
{
    int dim = c->d.dim;
    double ke = 0.0;
    q[0] = rho;
    for (int a = 0; a < dim; ++a) {
        q[1 + a] = rho * u[a];
        ke += u[a] * u[a];
    }
    q[dim + 1] = p / (c->d.gamma - 1.0) + 0.5 * rho * ke;
}

/* Ideal-gas primitives of a conserved state: velocity u_a = m_a / rho, pressure
 * p = (gamma - 1)(E - 1/2 sum_a m_a u_a). */
static void primitives(const ora_ctx* c, const double* q, double* u, double* p)
{
    int dim = c->d.dim;
    double rho = q[0];
    double ke = 0.0;
    for (int a = 0; a < dim; ++a) {
        u[a] = q[1 + a] / rho;
        ke += q[1 + a] * u[a];
    }
    *p = (c->d.gamma - 1.0) * (q[dim + 1] - 0.5 * ke);
}

/* ------------------------------------------------------------------------------------ */
/* Boundary handling: the state at any (possibly out-of-range) cell index                */
/* ------------------------------------------------------------------------------------ */

/* Out-of-range indices are resolved direction by direction (x, then y, then z):
 * PERIODIC wraps, EXTRAP takes the nearest interior cell, INFLOW also clamps but marks the
 * cell as an inflow ghost.  An inflow ghost holds the far-field state with each velocity
 * component perturbed by inflow_amp * (2 r - 1), r uniform from SplitMix64 at counter
 * ((((step * 6 + side) * 8 + depth) * ncell + cell) * 3 + component), where side = 2 d + s
 * and depth >= 1 are those of the first inflow direction and cell is the clamped index. */
static void fetch(const ora_ctx* c, const double* Q, long i, long j, long k, double* q)
{
    long idx[3] = {i, j, k};
    int inflow = 0, side = 0;
    long depth = 0;
    for (int d = 0; d < c->d.dim; ++d) {
        long n = n_of(c, d);
        if (idx[d] < 0) {
            int bc = c->d.bc[d][0];
            long g = -idx[d];
            if (bc == ORA_BC_PERIODIC) {
                idx[d] = ((idx[d] % n) + n) % n;
            } else {
                idx[d] = 0;
                if (bc == ORA_BC_INFLOW && !inflow) { inflow = 1; side = 2 * d; depth = g; }
            }
        } else if (idx[d] >= n) {
            int bc = c->d.bc[d][1];
            long g = idx[d] - n + 1;
            if (bc == ORA_BC_PERIODIC) {
                idx[d] = idx[d] % n;
            } else {
                idx[d] = n - 1;
                if (bc == ORA_BC_INFLOW && !inflow) { inflow = 1; side = 2 * d + 1; depth = g; }
            }
        }
    }
    long lin = cell_index(c, idx[0], idx[1], idx[2]);
    if (!inflow) {
        for (int m = 0; m < c->nq; ++m) q[m] = Q[(long)m * c->ncell + lin];
        return;
    }
    double u[3];
    for (int a = 0; a < c->d.dim; ++a) {
        u[a] = c->d.prim_inf[1 + a];
        if (c->d.inflow_amp != 0.0) {
            uint64_t ctr = ((((uint64_t)c->step * 6u + (uint64_t)side) * 8u + (uint64_t)depth)
                                * (uint64_t)c->ncell + (uint64_t)lin) * 3u + (uint64_t)a;
            double r = unit_uniform(ora_splitmix64(c->d.seed, ctr));
            u[a] += c->d.inflow_amp * (2.0 * r - 1.0);
        }
    }
    prim_to_cons(c, c->d.prim_inf[0], u, c->d.prim_inf[4], q);
}

/* ------------------------------------------------------------------------------------ */
/* Global Lax-Friedrichs wave speeds                                                      */
/* ------------------------------------------------------------------------------------ */

/* max that keeps a NaN once one has been seen */
static double nan_max(double m, double v)
{
    if (isnan(m)) return m;
    if (isnan(v)) return v;
    return v > m ? v : m;
}

int ora_alpha(const ora_ctx* c, const double* Q, double* alpha)
{
    int dim = c->d.dim;
    double amax[3] = {0.0, 0.0, 0.0};
    for (long n = 0; n < c->ncell; ++n) {
        double q[5], u[3], p;
        for (int m = 0; m < c->nq; ++m) q[m] = Q[(long)m * c->ncell + n];
        primitives(c, q, u, &p);
        double snd = sqrt(c->d.gamma * p / q[0]);
        for (int a = 0; a < dim; ++a) amax[a] = nan_max(amax[a], fabs(u[a]) + snd);
    }
    for (int a = 0; a < 3; ++a) alpha[a] = a < dim ? amax[a] : 0.0;
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Fifth-order reconstruction                                                             */
/* ------------------------------------------------------------------------------------ */

/* Three third-order candidate values at the face from the five upwind-ordered values
 * (a,b,cc,d,e) = (v_{i-2}, v_{i-1}, v_i, v_{i+1}, v_{i+2}), and their Jiang-Shu smoothness
 * indicators. */
static void candidates(double a, double b, double cc, double d, double e, double q[3], double beta[3])
{
    q[0] = (2.0 * a - 7.0 * b + 11.0 * cc) / 6.0;
    q[1] = (-b + 5.0 * cc + 2.0 * d) / 6.0;
    q[2] = (2.0 * cc + 5.0 * d - e) / 6.0;
    double s0 = a - 2.0 * b + cc, t0 = a - 4.0 * b + 3.0 * cc;
    double s1 = b - 2.0 * cc + d, t1 = b - d;
    double s2 = cc - 2.0 * d + e, t2 = 3.0 * cc - 4.0 * d + e;
    beta[0] = 13.0 / 12.0 * s0 * s0 + 0.25 * t0 * t0;
    beta[1] = 13.0 / 12.0 * s1 * s1 + 0.25 * t1 * t1;
    beta[2] = 13.0 / 12.0 * s2 * s2 + 0.25 * t2 * t2;
}

static const double lin_w[3] = {0.1, 0.6, 0.3}; /* optimal linear weights d_k */

/* TENO5 sharp cut-off: gamma_k = (C + tau5 / (beta_k + eps))^q with C = 1, q = 6,
 * tau5 = |beta_0 - beta_2|; chi_k = gamma_k / sum gamma; sub-stencil k is kept unless
 * chi_k < C_T. */
static int teno_keep(const double beta[3], double ct, double eps)
{
    double tau = fabs(beta[0] - beta[2]);
    double g[3], sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        double x = 1.0 + tau / (beta[k] + eps);
        double x3 = x * x * x;
        g[k] = x3 * x3;
        sum += g[k];
    }
    int flags = 0;
    for (int k = 0; k < 3; ++k) {
        double chi = g[k] / sum;
        if (!(chi < ct)) flags |= 1 << k;
    }
    return flags;
}

int ora_teno_flags(double a, double b, double cc, double d, double e, double teno_ct, double teno_eps)
{
    double q[3], beta[3];
    candidates(a, b, cc, d, e, q, beta);
    return teno_keep(beta, teno_ct, teno_eps);
}

/* ora_teno_flags of n stencils v[n][5] into out[n] (a convenience for tests). */
int ora_teno_flags_n(const double* v, long n, double teno_ct, double teno_eps, int* out)
{
    for (long i = 0; i < n; ++i) {
        const double* w = v + 5 * i;
        out[i] = ora_teno_flags(w[0], w[1], w[2], w[3], w[4], teno_ct, teno_eps);
    }
    return 0;
}

double ora_recon5(double a, double b, double cc, double d, double e, int scheme,
                  double weno_eps, double teno_ct, double teno_eps)
{
    double q[3], beta[3], w[3];
    candidates(a, b, cc, d, e, q, beta);
    if (scheme == ORA_WENO5JS) {
        double al[3], sum = 0.0;
        for (int k = 0; k < 3; ++k) {
            double s = weno_eps + beta[k];
            al[k] = lin_w[k] / (s * s);
            sum += al[k];
        }
        for (int k = 0; k < 3; ++k) w[k] = al[k] / sum;
    } else {
        int flags = teno_keep(beta, teno_ct, teno_eps);
        double dd[3], sum = 0.0;
        for (int k = 0; k < 3; ++k) {
            dd[k] = ((flags >> k) & 1) ? lin_w[k] : 0.0;
            sum += dd[k];
        }
        for (int k = 0; k < 3; ++k) w[k] = dd[k] / sum;
    }
    return w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
}

/* ------------------------------------------------------------------------------------ */
/* Convective flux with global Lax-Friedrichs splitting                                   */
/* ------------------------------------------------------------------------------------ */

/* Physical flux along direction dir (Sec. 2, Eqs. (3)-(4)):
 * [m_dir, m_a u_dir + p delta_{a,dir}, (E + p) u_dir]. */
static void phys_flux(const ora_ctx* c, const double* q, int dir, double* f)
{
    int dim = c->d.dim;
    double u[3], p;
    primitives(c, q, u, &p);
    f[0] = q[1 + dir];
    for (int a = 0; a < dim; ++a) f[1 + a] = q[1 + a] * u[dir] + (a == dir ? p : 0.0);
    f[dim + 1] = (q[dim + 1] + p) * u[dir];
}

/* Eigenvectors of the flux Jacobian dF_dir/dQ at the Roe average of the conserved states qa
 * and qb (Roe 1981): with r = sqrt(rho), the velocity and the total enthalpy H = (E + p)/rho
 * averaged with weights r_a, r_b, |u|^2 = sum u_a^2 and c^2 = (gamma - 1)(H - |u|^2/2).  Along
 * the unit normal n = e_dir, u_n = u_dir, the right eigenvectors (columns, conserved
 * components rho, m_1..m_dim, E) are
 *   u_n - c:  [1, u - c n, H - u_n c]
 *   entropy:  [1, u, |u|^2/2]
 *   shear t:  [0, e_t, u_t]          for each tangential direction t != dir
 *   u_n + c:  [1, u + c n, H + u_n c]
 * and, with b1 = (gamma - 1)/c^2 and b2 = b1 |u|^2/2, the left ones (rows, R's inverse)
 *   u_n - c:  [(b2 + u_n/c)/2, -(b1 u + n/c)/2, b1/2]
 *   entropy:  [1 - b2, b1 u, -b1]
 *   shear t:  [-u_t, e_t, 0]
 *   u_n + c:  [(b2 - u_n/c)/2, -(b1 u - n/c)/2, b1/2]. */
static void roe_vectors(const ora_ctx* c, const double* qa, const double* qb, int dir, double L[5][5], double R[5][5])
{
    int dim = c->d.dim, nq = c->nq;
    double gm = c->d.gamma;
    double ua[3], ub[3], pa, pb;
    primitives(c, qa, ua, &pa);
    primitives(c, qb, ub, &pb);
    double ra = sqrt(qa[0]), rb = sqrt(qb[0]);
    double Ha = (qa[dim + 1] + pa) / qa[0], Hb = (qb[dim + 1] + pb) / qb[0];
    double u[3] = {0.0, 0.0, 0.0};
    double q2 = 0.0;
    for (int a = 0; a < dim; ++a) {
        u[a] = (ra * ua[a] + rb * ub[a]) / (ra + rb);
        q2 += u[a] * u[a];
    }
    double H = (ra * Ha + rb * Hb) / (ra + rb);
    double cs = sqrt((gm - 1.0) * (H - 0.5 * q2));
    double un = u[dir];
    double b1 = (gm - 1.0) / (cs * cs), b2 = 0.5 * b1 * q2;
    for (int m = 0; m < nq; ++m)
        for (int k = 0; k < nq; ++k) L[k][m] = R[m][k] = 0.0;
    /* field 0: u_n - c; field 1: entropy; fields 2..dim: shear; field dim + 1: u_n + c */
    R[0][0] = 1.0;
    R[0][1] = 1.0;
    R[0][nq - 1] = 1.0;
    for (int a = 0; a < dim; ++a) {
        double na = a == dir ? 1.0 : 0.0;
        R[1 + a][0] = u[a] - cs * na;
        R[1 + a][1] = u[a];
        R[1 + a][nq - 1] = u[a] + cs * na;
    }
    R[nq - 1][0] = H - un * cs;
    R[nq - 1][1] = 0.5 * q2;
    R[nq - 1][nq - 1] = H + un * cs;
    L[0][0] = 0.5 * (b2 + un / cs);
    L[1][0] = 1.0 - b2;
    L[nq - 1][0] = 0.5 * (b2 - un / cs);
    for (int a = 0; a < dim; ++a) {
        double na = a == dir ? 1.0 : 0.0;
        L[0][1 + a] = -0.5 * (b1 * u[a] + na / cs);
        L[1][1 + a] = b1 * u[a];
        L[nq - 1][1 + a] = -0.5 * (b1 * u[a] - na / cs);
    }
    L[0][nq - 1] = 0.5 * b1;
    L[1][nq - 1] = -b1;
    L[nq - 1][nq - 1] = 0.5 * b1;
    int k = 2;
    for (int t = 0; t < dim; ++t) {
        if (t == dir) continue;
        R[1 + t][k] = 1.0;
        R[nq - 1][k] = u[t];
        L[k][0] = -u[t];
        L[k][1 + t] = 1.0;
        ++k;
    }
}

int ora_char_vectors(const ora_ctx* c, const double* qa, const double* qb, int dir, double* L, double* R)
{
    if (!c || !qa || !qb || !L || !R || dir < 0 || dir >= c->d.dim) return -1;
    double Lm[5][5], Rm[5][5];
    roe_vectors(c, qa, qb, dir, Lm, Rm);
    for (int a = 0; a < c->nq; ++a)
        for (int b = 0; b < c->nq; ++b) {
            L[a * c->nq + b] = Lm[a][b];
            R[a * c->nq + b] = Rm[a][b];
        }
    return 0;
}

/* Numerical flux at the face between cell idx and idx + e_dir:
 * F_hat = rec+(f+_{i-2..i+2}) + rec-(f-_{i+3..i-1}), f+- = (F +- alpha Q)/2, component by
 * component; or, characteristic-wise (charwise = 1; the variables the schemes act on are a
 * reading, Jiang & Shu 1996 reconstruct characteristic fields), with L and R the eigenvectors
 * at the Roe average of cells i and i + 1: g+-_s = L f+-_s for the six cells, each field
 * reconstructed, F_hat = R (rec+(g+) + rec-(g-)).  A global Lax-Friedrichs splitting is
 * linear in Q and F, so projecting the split fluxes splits the projected ones alike. */
static void face_flux(const ora_ctx* c, const double* Q, int dir, const long* idx, double alpha, double* Fh)
{
    int nq = c->nq;
    double fp[6][5], fm[6][5];
    for (int s = 0; s < 6; ++s) {
        long id[3] = {idx[0], idx[1], idx[2]};
        id[dir] += s - 2;
        double q[5], f[5];
        fetch(c, Q, id[0], id[1], id[2], q);
        phys_flux(c, q, dir, f);
        for (int m = 0; m < nq; ++m) {
            fp[s][m] = 0.5 * (f[m] + alpha * q[m]);
            fm[s][m] = 0.5 * (f[m] - alpha * q[m]);
        }
    }
    const ora_desc* dd = &c->d;
    if (dd->charwise) {
        double qa[5], qb[5];
        fetch(c, Q, idx[0], idx[1], idx[2], qa);
        long ib[3] = {idx[0], idx[1], idx[2]};
        ib[dir] += 1;
        fetch(c, Q, ib[0], ib[1], ib[2], qb);
        double L[5][5], R[5][5];
        roe_vectors(c, qa, qb, dir, L, R);
        double gp[6][5], gm[6][5];
        for (int s = 0; s < 6; ++s)
            for (int k = 0; k < nq; ++k) {
                double a = 0.0, b = 0.0;
                for (int m = 0; m < nq; ++m) {
                    a += L[k][m] * fp[s][m];
                    b += L[k][m] * fm[s][m];
                }
                gp[s][k] = a;
                gm[s][k] = b;
            }
        double gh[5];
        for (int k = 0; k < nq; ++k) {
            double plus = ora_recon5(gp[0][k], gp[1][k], gp[2][k], gp[3][k], gp[4][k], dd->scheme,
                                     dd->weno_eps, dd->teno_ct, dd->teno_eps);
            double minus = ora_recon5(gm[5][k], gm[4][k], gm[3][k], gm[2][k], gm[1][k], dd->scheme,
                                      dd->weno_eps, dd->teno_ct, dd->teno_eps);
            gh[k] = plus + minus;
        }
        for (int m = 0; m < nq; ++m) {
            double a = 0.0;
            for (int k = 0; k < nq; ++k) a += R[m][k] * gh[k];
            Fh[m] = a;
        }
        return;
    }
    for (int m = 0; m < nq; ++m) {
        double plus = ora_recon5(fp[0][m], fp[1][m], fp[2][m], fp[3][m], fp[4][m], dd->scheme,
                                 dd->weno_eps, dd->teno_ct, dd->teno_eps);
        double minus = ora_recon5(fm[5][m], fm[4][m], fm[3][m], fm[2][m], fm[1][m], dd->scheme,
                                  dd->weno_eps, dd->teno_ct, dd->teno_eps);
        Fh[m] = plus + minus;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Viscous terms                                                                          */
/* ------------------------------------------------------------------------------------ */

/* Fourth-order central first derivative on the cell values g_{i-2..i+2} (g[0..4]). */
static double d1c4(const double* g, double h)
{
    return (8.0 * (g[3] - g[1]) - (g[4] - g[0])) / (12.0 * h);
}

static void velocity_at(const ora_ctx* c, const double* Q, const long* idx, double* u)
{
    double q[5], p;
    fetch(c, Q, idx[0], idx[1], idx[2], q);
    primitives(c, q, u, &p);
}

/* Stress tau_ab = mu (G_ab + G_ba - 2/3 delta_ab div u) with G_ab = D_b u_a, and the
 * viscous work b_a = sum_b u_b tau_ab (Sec. 2, Eqs. (5)-(6); no heat flux). */
static void stress_at(const ora_ctx* c, const double* Q, const long* idx, double tau[3][3], double* bw)
{
    int dim = c->d.dim;
    double G[3][3], u0[3];
    velocity_at(c, Q, idx, u0);
    for (int b = 0; b < dim; ++b) {
        double ub[5][3];
        for (int s = 0; s < 5; ++s) {
            long id[3] = {idx[0], idx[1], idx[2]};
            id[b] += s - 2;
            velocity_at(c, Q, id, ub[s]);
        }
        for (int a = 0; a < dim; ++a) {
            double g[5];
            for (int s = 0; s < 5; ++s) g[s] = ub[s][a];
            G[a][b] = d1c4(g, c->d.h);
        }
    }
    double div = 0.0;
    for (int a = 0; a < dim; ++a) div += G[a][a];
    for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
            double t = G[a][b] + G[b][a];
            if (a == b) t -= 2.0 / 3.0 * div;
            tau[a][b] = c->d.mu * t;
        }
    for (int a = 0; a < dim; ++a) {
        double s = 0.0;
        for (int b = 0; b < dim; ++b) s += u0[b] * tau[a][b];
        bw[a] = s;
    }
}

/* Viscous term at one cell from the stresses of the cells around it:
 * momentum a: sum_b D_b tau_ab; energy: sum_b D_b b_b.  tau_nb[b][s] holds the stress at
 * idx + (s-2) e_b. */
static void visc_from_stresses(const ora_ctx* c, double tau_nb[3][5][3][3], double bw_nb[3][5][3], double* out)
{
    int dim = c->d.dim;
    out[0] = 0.0;
    for (int a = 0; a < dim; ++a) {
        double s = 0.0;
        for (int b = 0; b < dim; ++b) {
            double g[5];
            for (int m = 0; m < 5; ++m) g[m] = tau_nb[b][m][a][b];
            s += d1c4(g, c->d.h);
        }
        out[1 + a] = s;
    }
    double e = 0.0;
    for (int b = 0; b < dim; ++b) {
        double g[5];
        for (int m = 0; m < 5; ++m) g[m] = bw_nb[b][m][b];
        e += d1c4(g, c->d.h);
    }
    out[dim + 1] = e;
}

/* ------------------------------------------------------------------------------------ */
/* Immersed boundary                                                                      */
/* ------------------------------------------------------------------------------------ */

/* Peskin's four-point function lambda(r) (Sec. 2, Eq. (11)). */
double ora_delta4(double r)
{
    double x = fabs(r);
    if (x < 1.0) return 0.125 * (3.0 - 2.0 * x + sqrt(1.0 + 4.0 * x - 4.0 * x * x));
    if (x < 2.0) return 0.125 * (5.0 - 2.0 * x - sqrt(-7.0 + 12.0 * x - 4.0 * x * x));
    return 0.0;
}

/* Support of the tensor-product delta at position X (Sec. 2, Eq. (10)) in direction d:
 * the four cells j0 .. j0+3 around X and their one-dimensional weights lambda((X - x_j)/h). */
static void support_1d(const ora_ctx* c, int d, double X, long* j0, double* w)
{
    double r0 = (X - c->d.lo[d]) / c->d.h - 0.5; /* X in cell-index units */
    long j = (long)floor(r0) - 1;
    *j0 = j;
    for (int m = 0; m < 4; ++m) w[m] = ora_delta4(r0 - (double)(j + m));
}

/* Check that every point's four-point support lies inside the grid. */
static int supports_inside(const ora_ctx* c, int n, const double* X)
{
    for (int k = 0; k < n; ++k)
        for (int d = 0; d < c->d.dim; ++d) {
            long j0;
            double w[4];
            double x = X[(long)d * n + k];
            if (!isfinite(x)) return 0;
            support_1d(c, d, x, &j0, w);
            if (j0 < 0 || j0 + 3 >= n_of(c, d)) return 0;
        }
    return 1;
}

/* Loop helper over the 4^dim support of point k of a point set: weight W = w_x w_y (w_z),
 * visited in z-major, x-fastest order. */
typedef struct {
    long j0[3];
    double w[3][4];
} support_t;

static void support_of(const ora_ctx* c, const double* X, int n, int k, support_t* s)
{
    for (int d = 0; d < 3; ++d) {
        if (d < c->d.dim) {
            support_1d(c, d, X[(long)d * n + k], &s->j0[d], s->w[d]);
        } else {
            s->j0[d] = 0;
            s->w[d][0] = 1.0;
            s->w[d][1] = s->w[d][2] = s->w[d][3] = 0.0;
        }
    }
}

/* Interpolation U_ib(X_k) = sum over the support of u(x) lambda lambda (lambda), the
 * discrete form of Eq. (8) with h^dim delta_h = prod lambda. */
static void interp_point(const ora_ctx* c, const support_t* s, const double* field, int ncomp, double* out)
{
    int mzn = c->d.dim == 3 ? 4 : 1;
    for (int a = 0; a < ncomp; ++a) out[a] = 0.0;
    for (int mz = 0; mz < mzn; ++mz)
        for (int my = 0; my < 4; ++my)
            for (int mx = 0; mx < 4; ++mx) {
                double W = s->w[0][mx] * s->w[1][my];
                if (c->d.dim == 3) W = W * s->w[2][mz];
                long lin = cell_index(c, s->j0[0] + mx, s->j0[1] + my, s->j0[2] + mz);
                for (int a = 0; a < ncomp; ++a) out[a] += field[(long)a * c->ncell + lin] * W;
            }
}

int ora_ib_interp(const ora_ctx* c, const double* field, int ncomp, double* out)
{
    if (ncomp < 1) return -1;
    for (int k = 0; k < c->nm; ++k) {
        support_t s;
        double v[8];
        support_of(c, c->X, c->nm, k, &s);
        interp_point(c, &s, field, ncomp, v);
        for (int a = 0; a < ncomp && a < 8; ++a) out[(long)a * c->nm + k] = v[a];
    }
    return 0;
}

/* Spreading f(x) = - sum_k F_k prod lambda dV_k / h^dim (Eq. (9)); contributions are added
 * to each cell in marker order. */
static void spread_add(const ora_ctx* c, const double* F, int ncomp, double* field, double scale)
{
    double hd = c->d.dim == 3 ? c->d.h * c->d.h * c->d.h : c->d.h * c->d.h;
    int mzn = c->d.dim == 3 ? 4 : 1;
    for (int k = 0; k < c->nm; ++k) {
        support_t s;
        support_of(c, c->X, c->nm, k, &s);
        for (int mz = 0; mz < mzn; ++mz)
            for (int my = 0; my < 4; ++my)
                for (int mx = 0; mx < 4; ++mx) {
                    double W = s.w[0][mx] * s.w[1][my];
                    if (c->d.dim == 3) W = W * s.w[2][mz];
                    long lin = cell_index(c, s.j0[0] + mx, s.j0[1] + my, s.j0[2] + mz);
                    for (int a = 0; a < ncomp; ++a) {
                        double fk = -(F[(long)a * c->nm + k] * W * c->dV[k]) / hd;
                        field[(long)a * c->ncell + lin] += scale * fk;
                    }
                }
    }
}

int ora_ib_spread(const ora_ctx* c, const double* F, int ncomp, double* field, double scale)
{
    if (ncomp < 1) return -1;
    spread_add(c, F, ncomp, field, scale);
    return 0;
}

/* Marker velocity at time t: STATIC and EXTERNAL markers carry the stored U; ROTATING
 * markers U = omega e_z x X. */
static void marker_velocity(const ora_ctx* c, int k, double t, double* U)
{
    (void)t;
    int dim = c->d.dim;
    if (c->motion == ORA_ROTATING) {
        double x = c->X[k], y = c->X[(long)c->nm + k];
        U[0] = -c->omega * y;
        U[1] = c->omega * x;
        if (dim == 3) U[2] = 0.0;
    } else {
        for (int a = 0; a < dim; ++a) U[a] = c->U[(long)a * c->nm + k];
    }
}

/* Penalty step (Eq. (7)): interpolate u = m / rho, form F_f and dxi/dt = U_ib - U.
 * Returns the force density on the grid, f = S(F_f), as a dense [dim][ncell] array. */
static double* ib_force(ora_ctx* c, const double* Q, double t)
{
    int dim = c->d.dim;
    long nc = c->ncell;
    double* vel = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)nc);
    #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS)
    for (long n = 0; n < nc; ++n)
        for (int a = 0; a < dim; ++a) vel[(long)a * nc + n] = Q[(long)(1 + a) * nc + n] / Q[n];
    for (int k = 0; k < c->nm; ++k) {
        support_t s;
        double uib[3], U[3];
        support_of(c, c->X, c->nm, k, &s);
        interp_point(c, &s, vel, dim, uib);
        marker_velocity(c, k, t, U);
        for (int a = 0; a < dim; ++a) {
            long o = (long)a * c->nm + k;
            c->dxi[o] = uib[a] - U[a];
            c->F[o] = c->d.ib_alpha * c->xi[o] + c->d.ib_beta * (uib[a] - U[a]);
        }
    }
    free(vel);
    double* f = (double*)calloc((size_t)dim * (size_t)nc, sizeof(double));
    spread_add(c, c->F, dim, f, 1.0);
    return f;
}

/* ------------------------------------------------------------------------------------ */
/* Sponge                                                                                 */
/* ------------------------------------------------------------------------------------ */

/* sigma(x) = sigma_max * eta^3, eta = max over directions of the depth into the layer
 * divided by the layer width (0 outside every layer). */
static double sponge_sigma_at(const ora_ctx* c, const long* idx)
{
    double eta = 0.0;
    for (int d = 0; d < c->d.dim; ++d) {
        double x = c->d.lo[d] + ((double)idx[d] + 0.5) * c->d.h;
        double lo = c->d.lo[d], hi = c->d.lo[d] + (double)n_of(c, d) * c->d.h;
        double wl = c->d.sponge_width[d][0], wh = c->d.sponge_width[d][1];
        if (wl > 0.0 && x < lo + wl) {
            double r = (lo + wl - x) / wl;
            if (r > eta) eta = r;
        }
        if (wh > 0.0 && x > hi - wh) {
            double r = (x - (hi - wh)) / wh;
            if (r > eta) eta = r;
        }
    }
    if (eta > 1.0) eta = 1.0;
    return c->d.sponge_sigma * eta * eta * eta;
}

/* ------------------------------------------------------------------------------------ */
/* Right-hand side                                                                        */
/* ------------------------------------------------------------------------------------ */

static void idx_of(const ora_ctx* c, long n, long* idx)
{
    idx[0] = n % c->nx;
    idx[1] = (n / c->nx) % c->ny;
    idx[2] = n / (c->nx * c->ny);
}

/* Add the IB source S = [0, f, f . u] (f the spread force density, u the fluid velocity)
 * and the sponge -sigma (Q - Q_inf) at one cell. */
/* Periodic Gaussian pressure source (Sec. 3, sphere scattering) at cell n and time t:
 * A_p = -A exp(-B log(2) r^2) cos(omega t), r the distance from the source point. */
static double pressure_source(const ora_ctx* c, long n, double t)
{
    long idx[3];
    idx_of(c, n, idx);
    double r2 = 0.0;
    for (int a = 0; a < c->d.dim; ++a) {
        double xa = c->d.lo[a] + ((double)idx[a] + 0.5) * c->d.h;
        r2 += (xa - c->d.src_x[a]) * (xa - c->d.src_x[a]);
    }
    return -c->d.src_amp * exp(-c->d.src_b * log(2.0) * r2) * cos(c->d.src_omega * t);
}

static void sources_at(const ora_ctx* c, const double* Q, const double* fib, long n, double* out)
{
    int dim = c->d.dim, nq = c->nq;
    long nc = c->ncell;
    if ((c->d.terms & ORA_IB) && fib) {
        double rho = Q[n], fu = 0.0;
        for (int a = 0; a < dim; ++a) {
            double fa = fib[(long)a * nc + n];
            out[1 + a] += fa;
            fu += fa * (Q[(long)(1 + a) * nc + n] / rho);
        }
        out[dim + 1] += fu;
    }
    if ((c->d.terms & ORA_SPONGE) && c->d.sponge_sigma != 0.0) {
        long idx[3];
        idx_of(c, n, idx);
        double sg = sponge_sigma_at(c, idx);
        for (int m = 0; m < nq; ++m) out[m] += -sg * (Q[(long)m * nc + n] - c->q_inf[m]);
    }
    if (c->d.src_amp != 0.0) out[dim + 1] += pressure_source(c, n, c->t) / (c->d.gamma - 1.0);
}

/* Non-reflecting boundary of Thompson (1987, 1990), the far-field treatment Sec. 2 applies:
 * at the boundary cell of a NONREFLECT side, the convective term along the boundary normal d
 * is replaced by its characteristic (locally one-dimensional) form, with the amplitudes of
 * the waves that enter the domain set to zero.  With primitives (rho, u_a, p), u_n = u_d,
 * c = sqrt(gamma p / rho) and one-sided second-order derivatives along d (the boundary cell
 * and the next two inward),
 *   L1 = (u_n - c)(p' - rho c u_n'),   L2 = u_n (c^2 rho' - p'),   L_a = u_n u_a' (a != d),
 *   L5 = (u_n + c)(p' + rho c u_n');
 * a wave whose speed points into the domain (negative at the high side, positive at the low
 * side) has its L set to zero.  Then
 *   d1 = (L2 + (L5 + L1)/2) / c^2,  d2 = (L5 + L1)/2,  dn = (L5 - L1)/(2 rho c),  d_a = L_a,
 * and the normal flux derivative dF/dx_d of the conserved variables is
 *   [d1,  u_d d1 + rho dn,  u_a d1 + rho d_a,  |u|^2/2 d1 + d2/(gamma-1) + rho u_d dn + sum_a rho u_a d_a];
 * out receives its negative (the convective term). */
static void nrbc_conv(const ora_ctx* c, const double* Q, int d, int side, const long* idx, double* out)
{
    int dim = c->d.dim;
    double rho[3], u[3][3], p[3];
    for (int s = 0; s < 3; ++s) {
        long id[3] = {idx[0], idx[1], idx[2]};
        id[d] += side == 0 ? s : -s;
        double q[5];
        for (int m = 0; m < c->nq; ++m) q[m] = Q[(long)m * c->ncell + cell_index(c, id[0], id[1], id[2])];
        rho[s] = q[0];
        primitives(c, q, u[s], &p[s]);
    }
    /* one-sided derivative along +x_d: (-3 f0 + 4 f1 - f2) / 2h at the low side, where f1, f2
     * lie inward (+x_d); at the high side they lie toward -x_d, which flips the sign.  Written
     * as (4 (f1 - f0) - (f2 - f0)) / 2h so that constant data give exactly zero. */
    double sg = side == 0 ? 1.0 : -1.0;
    double h2 = 2.0 * c->d.h;
#define ONE_SIDED(f0, f1, f2) (sg * (4.0 * ((f1) - (f0)) - ((f2) - (f0))) / h2)
    double drho = ONE_SIDED(rho[0], rho[1], rho[2]);
    double dp = ONE_SIDED(p[0], p[1], p[2]);
    double du[3];
    for (int a = 0; a < dim; ++a) du[a] = ONE_SIDED(u[0][a], u[1][a], u[2][a]);
#undef ONE_SIDED
    double r = rho[0], un = u[0][d];
    double cs = sqrt(c->d.gamma * p[0] / r);
    double lam1 = un - cs, lam2 = un, lam5 = un + cs;
    double L1 = lam1 * (dp - r * cs * du[d]);
    double L2 = lam2 * (cs * cs * drho - dp);
    double L5 = lam5 * (dp + r * cs * du[d]);
    double La[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a)
        if (a != d) La[a] = lam2 * du[a];
    /* incoming waves carry nothing in */
    int in_high = side == 1;
    if (in_high ? lam1 < 0.0 : lam1 > 0.0) L1 = 0.0;
    if (in_high ? lam2 < 0.0 : lam2 > 0.0) {
        L2 = 0.0;
        for (int a = 0; a < 3; ++a) La[a] = 0.0;
    }
    if (in_high ? lam5 < 0.0 : lam5 > 0.0) L5 = 0.0;
    double d1 = (L2 + 0.5 * (L5 + L1)) / (cs * cs);
    double d2 = 0.5 * (L5 + L1);
    double dn = (L5 - L1) / (2.0 * r * cs);
    double ke = 0.0;
    for (int a = 0; a < dim; ++a) ke += u[0][a] * u[0][a];
    out[0] = -d1;
    double e = 0.5 * ke * d1 + d2 / (c->d.gamma - 1.0) + r * un * dn;
    for (int a = 0; a < dim; ++a) {
        if (a == d) {
            out[1 + a] = -(un * d1 + r * dn);
        } else {
            out[1 + a] = -(u[0][a] * d1 + r * La[a]);
            e += r * u[0][a] * La[a];
        }
    }
    out[dim + 1] = -e;
}

static int conv_on(const ora_ctx* c, int d) { return (c->d.terms >> d) & 1; }
static int visc_on(const ora_ctx* c) { return (c->d.terms & ORA_VISC) && c->d.mu != 0.0; }

int ora_rhs(ora_ctx* c, const double* Q, double* L)
{
    int dim = c->d.dim, nq = c->nq;
    long nc = c->ncell;
    double alpha[3];
    ora_alpha(c, Q, alpha);
    memset(L, 0, sizeof(double) * (size_t)nq * (size_t)nc);

    /* convective terms: -(F_hat_{i+1/2} - F_hat_{i-1/2}) / h, one line of faces at a time */
    for (int d = 0; d < dim; ++d) {
        if (!conv_on(c, d)) continue;
        long nd = n_of(c, d);
        long nlines = nc / nd;
        #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS) schedule(dynamic, 16)
        for (long ln = 0; ln < nlines; ++ln) {
            long base[3];
            /* enumerate lines: the index along d is 0, the others run over the grid */
            long rest = ln;
            for (int e = 0; e < 3; ++e) {
                if (e == d) { base[e] = 0; continue; }
                long ne = (e < dim) ? n_of(c, e) : 1;
                base[e] = rest % ne;
                rest /= ne;
            }
            double* Fh = (double*)malloc(sizeof(double) * (size_t)(nd + 1) * (size_t)nq);
            for (long f = -1; f < nd; ++f) {
                long idx[3] = {base[0], base[1], base[2]};
                idx[d] = f;
                face_flux(c, Q, d, idx, alpha[d], &Fh[(f + 1) * nq]);
            }
            for (long i = 0; i < nd; ++i) {
                long idx[3] = {base[0], base[1], base[2]};
                idx[d] = i;
                long n = cell_index(c, idx[0], idx[1], idx[2]);
                int side = (i == 0 && c->d.bc[d][0] == ORA_BC_NONREFLECT) ? 0
                           : ((i == nd - 1 && c->d.bc[d][1] == ORA_BC_NONREFLECT) ? 1 : -1);
                if (side >= 0 && nd >= 3) {
                    double cv[5];
                    nrbc_conv(c, Q, d, side, idx, cv);
                    for (int m = 0; m < nq; ++m) L[(long)m * nc + n] += cv[m];
                    continue;
                }
                for (int m = 0; m < nq; ++m)
                    L[(long)m * nc + n] += -(Fh[(i + 1) * nq + m] - Fh[i * nq + m]) / c->d.h;
            }
            free(Fh);
        }
    }

    /* viscous terms: stresses on the grid plus a two-cell ring, then their divergence */
    if (visc_on(c)) {
        long ex = c->nx + 4, ey = c->ny + 4, ez = dim == 3 ? c->nz + 4 : 1;
        long ne = ex * ey * ez;
        int ntau = 9, nbw = 3;
        double* tau = (double*)malloc(sizeof(double) * (size_t)ne * (size_t)ntau);
        double* bw = (double*)malloc(sizeof(double) * (size_t)ne * (size_t)nbw);
        long zoff = dim == 3 ? 2 : 0;
        #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS) schedule(dynamic, 64)
        for (long e = 0; e < ne; ++e) {
            long idx[3] = {e % ex - 2, (e / ex) % ey - 2, e / (ex * ey) - zoff};
            double t3[3][3] = {{0}}, b3[3] = {0};
            stress_at(c, Q, idx, t3, b3);
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) tau[e * ntau + a * 3 + b] = t3[a][b];
                bw[e * nbw + a] = b3[a];
            }
        }
        #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS) schedule(dynamic, 64)
        for (long n = 0; n < nc; ++n) {
            long idx[3];
            idx_of(c, n, idx);
            double tnb[3][5][3][3], bnb[3][5][3], v[5];
            for (int b = 0; b < dim; ++b)
                for (int s = 0; s < 5; ++s) {
                    long id[3] = {idx[0] + 2, idx[1] + 2, idx[2] + zoff};
                    id[b] += s - 2;
                    long e = (id[2] * ey + id[1]) * ex + id[0];
                    for (int a = 0; a < 3; ++a) {
                        for (int bb = 0; bb < 3; ++bb) tnb[b][s][a][bb] = tau[e * ntau + a * 3 + bb];
                        bnb[b][s][a] = bw[e * nbw + a];
                    }
                }
            visc_from_stresses(c, tnb, bnb, v);
            for (int m = 0; m < nq; ++m) L[(long)m * nc + n] += v[m];
        }
        free(tau);
        free(bw);
    }

    /* immersed-boundary source and sponge */
    double* fib = NULL;
    if ((c->d.terms & ORA_IB) && c->nm > 0) fib = ib_force(c, Q, c->t);
    #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS)
    for (long n = 0; n < nc; ++n) {
        double s[5] = {0, 0, 0, 0, 0};
        sources_at(c, Q, fib, n, s);
        for (int m = 0; m < nq; ++m) L[(long)m * nc + n] += s[m];
    }
    free(fib);
    return 0;
}

int ora_rhs_cells(ora_ctx* c, const double* Q, int64_t nlist, const int64_t* cells, double* out)
{
    int dim = c->d.dim, nq = c->nq;
    long nc = c->ncell;
    for (int64_t l = 0; l < nlist; ++l)
        if (cells[l] < 0 || cells[l] >= nc) return -1;
    double alpha[3];
    ora_alpha(c, Q, alpha);
    /* IB force only at the requested cells: contributions in marker order */
    double* fl = (double*)calloc((size_t)dim * (size_t)(nlist > 0 ? nlist : 1), sizeof(double));
    if ((c->d.terms & ORA_IB) && c->nm > 0) {
        double* f = ib_force(c, Q, c->t);
        for (int64_t l = 0; l < nlist; ++l)
            for (int a = 0; a < dim; ++a) fl[(long)a * nlist + l] = f[(long)a * nc + cells[l]];
        free(f);
    }
    #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS) schedule(dynamic, 4)
    for (int64_t l = 0; l < nlist; ++l) {
        long n = cells[l];
        long idx[3];
        idx_of(c, n, idx);
        double acc[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < dim; ++d) {
            if (!conv_on(c, d)) continue;
            long nd = n_of(c, d);
            int side = (idx[d] == 0 && c->d.bc[d][0] == ORA_BC_NONREFLECT) ? 0
                       : ((idx[d] == nd - 1 && c->d.bc[d][1] == ORA_BC_NONREFLECT) ? 1 : -1);
            if (side >= 0 && nd >= 3) {
                double cv[5];
                nrbc_conv(c, Q, d, side, idx, cv);
                for (int m = 0; m < nq; ++m) acc[m] += cv[m];
                continue;
            }
            double Fr[5], Fl[5];
            long id[3] = {idx[0], idx[1], idx[2]};
            face_flux(c, Q, d, id, alpha[d], Fr);
            id[d] -= 1;
            face_flux(c, Q, d, id, alpha[d], Fl);
            for (int m = 0; m < nq; ++m) acc[m] += -(Fr[m] - Fl[m]) / c->d.h;
        }
        if (visc_on(c)) {
            double tnb[3][5][3][3], bnb[3][5][3], v[5];
            memset(tnb, 0, sizeof tnb);
            memset(bnb, 0, sizeof bnb);
            for (int b = 0; b < dim; ++b)
                for (int s = 0; s < 5; ++s) {
                    long id[3] = {idx[0], idx[1], idx[2]};
                    id[b] += s - 2;
                    stress_at(c, Q, id, tnb[b][s], bnb[b][s]);
                }
            visc_from_stresses(c, tnb, bnb, v);
            for (int m = 0; m < nq; ++m) acc[m] += v[m];
        }
        /* sources: reuse the per-cell routine with the requested cells' force values */
        double s[5] = {0, 0, 0, 0, 0};
        if ((c->d.terms & ORA_IB) && c->nm > 0) {
            double rho = Q[n], fu = 0.0;
            for (int a = 0; a < dim; ++a) {
                double fa = fl[(long)a * nlist + l];
                s[1 + a] += fa;
                fu += fa * (Q[(long)(1 + a) * nc + n] / rho);
            }
            s[dim + 1] += fu;
        }
        if ((c->d.terms & ORA_SPONGE) && c->d.sponge_sigma != 0.0) {
            double sg = sponge_sigma_at(c, idx);
            for (int m = 0; m < nq; ++m) s[m] += -sg * (Q[(long)m * nc + n] - c->q_inf[m]);
        }
        if (c->d.src_amp != 0.0) s[dim + 1] += pressure_source(c, n, c->t) / (c->d.gamma - 1.0);
        for (int m = 0; m < nq; ++m) out[(long)m * nlist + l] = acc[m] + s[m];
    }
    free(fl);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Learned-weight inputs and labels (not in the paper: this library's definitions)        */
/* ------------------------------------------------------------------------------------ */

/* The five cells of one face side in upwind order: side 0 ("+") uses cells i-2..i+2 of the
 * face between i and i+1 along dir; side 1 ("-") uses i+3..i-1.  Centre = position 2. */
static void side_cells(int dir, const long* idx, int side, long cells[5][3])
{
    for (int s = 0; s < 5; ++s) {
        long off = side == 0 ? (long)s - 2 : 3 - (long)s;
        cells[s][0] = idx[0];
        cells[s][1] = idx[1];
        cells[s][2] = idx[2];
        cells[s][dir] += off;
    }
}

/* Natural scales of rho, velocity and p: rho_inf, c_inf and rho_inf c_inf^2 of the far field. */
static void natural_scales(const ora_ctx* c, double* srho, double* svel, double* sp)
{
    const double cinf = sqrt(c->d.gamma * c->d.prim_inf[4] / c->d.prim_inf[0]);
    *srho = c->d.prim_inf[0];
    *svel = cinf;
    *sp = c->d.prim_inf[0] * cinf * cinf;
}

/* Features: for rho, the normal velocity (negated on side 1, so that both sides see the
 * stencil in their upwind orientation) and p at the five cells, each variable's deviations
 * from the centre divided by (their largest magnitude + 1e-8 times the variable's natural
 * scale): 15 values in [-1, 1].  The floor maps variations at rounding level to ~0. */
int ora_face_features(const ora_ctx* c, const double* Q, int dir, long i, long j, long k, int side, double* out)
{
    if (dir < 0 || dir >= c->d.dim || side < 0 || side > 1) return -1;
    long idx[3] = {i, j, k}, cells[5][3];
    side_cells(dir, idx, side, cells);
    double v[3][5], sc[3];
    natural_scales(c, &sc[0], &sc[1], &sc[2]);
    for (int s = 0; s < 5; ++s) {
        double q[5], u[3], p;
        fetch(c, Q, cells[s][0], cells[s][1], cells[s][2], q);
        primitives(c, q, u, &p);
        v[0][s] = q[0];
        v[1][s] = side == 0 ? u[dir] : -u[dir];
        v[2][s] = p;
    }
    for (int m = 0; m < 3; ++m) {
        double mx = 0.0;
        for (int s = 0; s < 5; ++s) {
            double dv = fabs(v[m][s] - v[m][2]);
            if (dv > mx) mx = dv;
        }
        for (int s = 0; s < 5; ++s) out[m * 5 + s] = (v[m][s] - v[m][2]) / (mx + 1e-8 * sc[m]);
    }
    return 0;
}

/* Significance: 1 when rho, some velocity component or p varies over the five cells of the
 * side by more than 1e-8 of its natural scale, else 0.  Every split-flux component of an
 * insignificant side is constant to O(1e-8) of its scale, so its sub-stencil choice moves
 * the face value by no more than that. */
int ora_face_significant(const ora_ctx* c, const double* Q, int dir, long i, long j, long k, int side)
{
    if (dir < 0 || dir >= c->d.dim || side < 0 || side > 1) return -1;
    long idx[3] = {i, j, k}, cells[5][3];
    side_cells(dir, idx, side, cells);
    double sc[3];
    natural_scales(c, &sc[0], &sc[1], &sc[2]);
    const int nv = c->d.dim + 2;   /* rho, velocity components, p */
    double lo[5], hi[5];
    for (int s = 0; s < 5; ++s) {
        double q[5], u[3], p, v[5];
        fetch(c, Q, cells[s][0], cells[s][1], cells[s][2], q);
        primitives(c, q, u, &p);
        v[0] = q[0];
        for (int a = 0; a < c->d.dim; ++a) v[1 + a] = u[a];
        v[nv - 1] = p;
        for (int m = 0; m < nv; ++m) {
            lo[m] = s == 0 || v[m] < lo[m] ? v[m] : lo[m];
            hi[m] = s == 0 || v[m] > hi[m] ? v[m] : hi[m];
        }
    }
    for (int m = 0; m < nv; ++m) {
        const double scale = m == 0 ? sc[0] : (m == nv - 1 ? sc[2] : sc[1]);
        if (hi[m] - lo[m] > 1e-8 * scale) return 1;
    }
    return 0;
}

/* Label: bit k set when TENO5 keeps sub-stencil k for every conserved component of this
 * face side's split flux (f+ on side 0, f- on side 1) at wave speed alpha.  A component
 * whose five values agree to 1e-12 of their magnitude counts as keeping every sub-stencil:
 * its TENO decision is then set by rounding noise and cannot change its face value. */
int ora_face_label(const ora_ctx* c, const double* Q, int dir, long i, long j, long k, int side, double alpha)
{
    if (dir < 0 || dir >= c->d.dim || side < 0 || side > 1) return -1;
    long idx[3] = {i, j, k}, cells[5][3];
    side_cells(dir, idx, side, cells);
    double f[5][5];
    for (int s = 0; s < 5; ++s) {
        double q[5], F[5];
        fetch(c, Q, cells[s][0], cells[s][1], cells[s][2], q);
        phys_flux(c, q, dir, F);
        for (int m = 0; m < c->nq; ++m) f[s][m] = 0.5 * (F[m] + (side == 0 ? alpha : -alpha) * q[m]);
    }
    int all = 7;
    for (int m = 0; m < c->nq; ++m) {
        double lo = f[0][m], hi = f[0][m], mag = 0.0;
        for (int s = 0; s < 5; ++s) {
            if (f[s][m] < lo) lo = f[s][m];
            if (f[s][m] > hi) hi = f[s][m];
            if (fabs(f[s][m]) > mag) mag = fabs(f[s][m]);
        }
        if (hi - lo <= 1e-12 * mag) continue;
        all &= ora_teno_flags(f[0][m], f[1][m], f[2][m], f[3][m], f[4][m], c->d.teno_ct, c->d.teno_eps);
    }
    return all;
}

/* ------------------------------------------------------------------------------------ */
/* SSP-RK3 (Shu & Osher 1988)                                                             */
/* ------------------------------------------------------------------------------------ */

/* Q1 = Qn + dt L(Qn);  Q2 = 3/4 Qn + 1/4 (Q1 + dt L(Q1));  Qn+1 = 1/3 Qn + 2/3 (Q2 + dt L(Q2)),
 * with the penalty integral xi advanced by the same three stages using dxi/dt = U_ib - U. */
int ora_rk3_step(ora_ctx* c, double* Q, double dt)
{
    long len = (long)c->nq * c->ncell;
    long lm = (long)c->d.dim * c->nm;
    double* Qn = (double*)malloc(sizeof(double) * (size_t)len);
    double* Qs = (double*)malloc(sizeof(double) * (size_t)len);
    double* L = (double*)malloc(sizeof(double) * (size_t)len);
    double* xin = (double*)malloc(sizeof(double) * (size_t)(lm > 0 ? lm : 1));
    memcpy(Qn, Q, sizeof(double) * (size_t)len);
    if (lm > 0) memcpy(xin, c->xi, sizeof(double) * (size_t)lm);
    double t0 = c->t;
    int ib = (c->d.terms & ORA_IB) && c->nm > 0;

    /* stage 1 at time t */
    c->t = t0;
    if (c->record) memcpy(c->record, Qn, sizeof(double) * (size_t)len);
    ora_rhs(c, Qn, L);
    #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS)
    for (long i = 0; i < len; ++i) Qs[i] = Qn[i] + dt * L[i];
    if (ib)
        for (long i = 0; i < lm; ++i) c->xi[i] = xin[i] + dt * c->dxi[i];

    /* stage 2 at time t + dt */
    c->t = t0 + dt;
    if (c->record) memcpy(c->record + len, Qs, sizeof(double) * (size_t)len);
    ora_rhs(c, Qs, L);
    #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS)
    for (long i = 0; i < len; ++i) Qs[i] = 0.75 * Qn[i] + 0.25 * (Qs[i] + dt * L[i]);
    if (ib)
        for (long i = 0; i < lm; ++i) c->xi[i] = 0.75 * xin[i] + 0.25 * (c->xi[i] + dt * c->dxi[i]);

    /* stage 3 at time t + dt/2 */
    c->t = t0 + 0.5 * dt;
    if (c->record) memcpy(c->record + 2 * len, Qs, sizeof(double) * (size_t)len);
    ora_rhs(c, Qs, L);
    #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS)
    for (long i = 0; i < len; ++i) Q[i] = (1.0 / 3.0) * Qn[i] + (2.0 / 3.0) * (Qs[i] + dt * L[i]);
    if (ib)
        for (long i = 0; i < lm; ++i)
            c->xi[i] = (1.0 / 3.0) * xin[i] + (2.0 / 3.0) * (c->xi[i] + dt * c->dxi[i]);

    c->t = t0 + dt;
    c->step += 1;
    free(Qn);
    free(Qs);
    free(L);
    free(xin);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Test hooks on the TENO5 decisions (they compute nothing the solver uses)               */
/* ------------------------------------------------------------------------------------ */

/* Threads of the OpenMP loops (n < 1: leave as is); returns the count in effect. */
int ora_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

int ora_record_stages(ora_ctx* c, double* buf)
{
    c->record = buf;
    return 0;
}

/* Split fluxes of the six cells around face `f` (between cells f-1 and f along dir) of the
 * line through (i, j, k): fp[s][m], fm[s][m] for cells f-3+s, s = 0..5. */
static void face_splits(const ora_ctx* c, const double* Q, int dir, long f, long i, long j, long k, double alpha,
                        double fp[6][5], double fm[6][5])
{
    long idx[3] = {i, j, k};
    idx[dir] = f - 3;
    for (int s = 0; s < 6; ++s) {
        long id[3] = {idx[0], idx[1], idx[2]};
        id[dir] += s;
        double q[5], fl[5];
        fetch(c, Q, id[0], id[1], id[2], q);
        phys_flux(c, q, dir, fl);
        for (int m = 0; m < c->nq; ++m) {
            fp[s][m] = 0.5 * (fl[m] + alpha * q[m]);
            fm[s][m] = 0.5 * (fl[m] - alpha * q[m]);
        }
    }
}

/* Number of faces along dir: x faces [nz][ny][nx+1], y faces [nz][ny+1][nx], z faces
 * [nz+1][ny][nx]. */
static long faces_along(const ora_ctx* c, int dir)
{
    return (c->nx + (dir == 0)) * (c->ny + (dir == 1)) * (c->nz + (dir == 2));
}

static void face_coords(const ora_ctx* c, int dir, long lin, long* f, long* i, long* j, long* k)
{
    long mx = c->nx + (dir == 0), my = c->ny + (dir == 1);
    long a = lin % mx, b = (lin / mx) % my, d = lin / (mx * my);
    *i = a;
    *j = b;
    *k = d;
    *f = dir == 0 ? a : (dir == 1 ? b : d);
}

/* The TENO5 keep patterns the oracle's reconstruction takes at every face of Q (its own wave
 * speeds), in the face layout above, directions one after the other: bits 3m+k for side "+"
 * (values f+_{f-3..f+1}), 16+3m+k for side "-" (f-_{f+2..f-2}), component m, sub-stencil k. */
int ora_teno_bits(const ora_ctx* c, const double* Q, uint32_t* out)
{
    double alpha[3];
    ora_alpha(c, Q, alpha);
    long off = 0;
    for (int dir = 0; dir < c->d.dim; ++dir) {
        long nf = faces_along(c, dir);
        #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS)
        for (long lin = 0; lin < nf; ++lin) {
            long f, i, j, k;
            double fp[6][5], fm[6][5];
            face_coords(c, dir, lin, &f, &i, &j, &k);
            face_splits(c, Q, dir, f, i, j, k, alpha[dir], fp, fm);
            uint32_t w = 0;
            for (int m = 0; m < c->nq; ++m) {
                int kp = ora_teno_flags(fp[0][m], fp[1][m], fp[2][m], fp[3][m], fp[4][m], c->d.teno_ct, c->d.teno_eps);
                int km = ora_teno_flags(fm[5][m], fm[4][m], fm[3][m], fm[2][m], fm[1][m], c->d.teno_ct, c->d.teno_eps);
                w |= (uint32_t)kp << (3 * m);
                w |= (uint32_t)km << (16 + 3 * m);
            }
            out[off + lin] = w;
        }
        off += nf;
    }
    return 0;
}

/* For n entries (face g[i] in the layout of ora_teno_bits, component m[i], side sd[i]: 0 "+",
 * 1 "-") of Q at the wave speeds alpha[3]: the five upwind-ordered split-flux values
 * v[i][5] and chi_k = gamma_k / sum gamma of TENO5 on them, chi[i][3]. */
int ora_teno_values_n(const ora_ctx* c, const double* Q, const double* alpha, long n, const long* g, const int* m,
                      const int* sd, double* v, double* chi)
{
    for (long e = 0; e < n; ++e) {
        long lin = g[e];
        int dir = 0;
        while (dir < c->d.dim && lin >= faces_along(c, dir)) lin -= faces_along(c, dir++);
        if (dir >= c->d.dim || m[e] < 0 || m[e] >= c->nq) return -1;
    }
    #pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS)
    for (long e = 0; e < n; ++e) {
        long lin = g[e];
        int dir = 0;
        while (lin >= faces_along(c, dir)) lin -= faces_along(c, dir++);
        long f, i, j, k;
        double fp[6][5], fm[6][5];
        face_coords(c, dir, lin, &f, &i, &j, &k);
        face_splits(c, Q, dir, f, i, j, k, alpha[dir], fp, fm);
        double* w = v + 5 * e;
        for (int s = 0; s < 5; ++s) w[s] = sd[e] == 0 ? fp[s][m[e]] : fm[5 - s][m[e]];
        double q[3], beta[3];
        candidates(w[0], w[1], w[2], w[3], w[4], q, beta);
        double tau = fabs(beta[0] - beta[2]), gk[3], sum = 0.0;
        for (int kk = 0; kk < 3; ++kk) {
            double x = 1.0 + tau / (beta[kk] + c->d.teno_eps);
            double x3 = x * x * x;
            gk[kk] = x3 * x3;
            sum += gk[kk];
        }
        for (int kk = 0; kk < 3; ++kk) chi[3 * e + kk] = gk[kk] / sum;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Probes, state, life cycle                                                              */
/* ------------------------------------------------------------------------------------ */

int ora_probe_dp(const ora_ctx* c, const double* Q, double* dp)
{
    long nc = c->ncell;
    double* p = (double*)malloc(sizeof(double) * (size_t)nc);
    for (long n = 0; n < nc; ++n) {
        double q[5], u[3];
        for (int m = 0; m < c->nq; ++m) q[m] = Q[(long)m * nc + n];
        primitives(c, q, u, &p[n]);
    }
    for (int k = 0; k < c->np; ++k) {
        support_t s;
        double v;
        support_of(c, c->Xp, c->np, k, &s);
        interp_point(c, &s, p, 1, &v);
        dp[k] = v - c->d.prim_inf[4];
    }
    free(p);
    return 0;
}

/* Field totals (diagnostics of Sec. 3): out[m] = sum over cells, in cell order, of q_m h^dim. */
int ora_totals(const ora_ctx* c, const double* Q, double* out)
{
    long nc = c->ncell;
    double hd = 1.0;
    for (int d = 0; d < c->d.dim; ++d) hd *= c->d.h;
    for (int m = 0; m < c->nq; ++m) {
        double s = 0.0;
        for (long n = 0; n < nc; ++n) s += Q[(long)m * nc + n];
        out[m] = s * hd;
    }
    return 0;
}

/* Dilatation div u at every cell: the fourth-order central difference of u_d = m_d / rho
 * along d, summed over directions (ghosts by the boundary conditions). */
int ora_dilatation(const ora_ctx* c, const double* Q, double* out)
{
    int dim = c->d.dim;
    long nc = c->ncell;
#pragma omp parallel for if (c->ncell >= ORA_PAR_MIN_CELLS) schedule(static)
    for (long n = 0; n < nc; ++n) {
        long idx[3];
        idx_of(c, n, idx);
        double div = 0.0;
        for (int d = 0; d < dim; ++d) {
            double g[5];
            for (int s = 0; s < 5; ++s) {
                long id[3] = {idx[0], idx[1], idx[2]};
                double u[3];
                id[d] += s - 2;
                velocity_at(c, Q, id, u);
                g[s] = u[d];
            }
            div += d1c4(g, c->d.h);
        }
        out[n] = div;
    }
    return 0;
}

int ora_marker_force(const ora_ctx* c, double* F)
{
    memcpy(F, c->F, sizeof(double) * (size_t)c->d.dim * (size_t)c->nm);
    return 0;
}

int ora_get_state(const ora_ctx* c, double* xi, double* t, int64_t* step)
{
    if (xi && c->nm > 0) memcpy(xi, c->xi, sizeof(double) * (size_t)c->d.dim * (size_t)c->nm);
    if (t) *t = c->t;
    if (step) *step = c->step;
    return 0;
}

int ora_set_state(ora_ctx* c, const double* xi, double t, int64_t step)
{
    if (xi && c->nm > 0) memcpy(c->xi, xi, sizeof(double) * (size_t)c->d.dim * (size_t)c->nm);
    c->t = t;
    c->step = step;
    return 0;
}

static void free_markers(ora_ctx* c)
{
    free(c->X); free(c->dV); free(c->U); free(c->xi); free(c->F); free(c->dxi);
    c->X = c->dV = c->U = c->xi = c->F = c->dxi = NULL;
    c->nm = 0;
}

int ora_set_markers(ora_ctx* c, int n, const double* X, const double* dV, const double* U,
                    int motion, double omega)
{
    int dim = c->d.dim;
    if (n < 0 || (n > 0 && (!X || !dV))) return -1;
    if (motion < ORA_STATIC || motion > ORA_EXTERNAL) return -1;
    if (n > 0 && !supports_inside(c, n, X)) return -1;
    free_markers(c);
    c->nm = n;
    c->motion = motion;
    c->omega = omega;
    size_t lm = (size_t)dim * (size_t)(n > 0 ? n : 1);
    c->X = (double*)calloc(lm, sizeof(double));
    c->dV = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    c->U = (double*)calloc(lm, sizeof(double));
    c->xi = (double*)calloc(lm, sizeof(double));
    c->F = (double*)calloc(lm, sizeof(double));
    c->dxi = (double*)calloc(lm, sizeof(double));
    if (n > 0) {
        memcpy(c->X, X, sizeof(double) * (size_t)dim * (size_t)n);
        memcpy(c->dV, dV, sizeof(double) * (size_t)n);
        if (U) memcpy(c->U, U, sizeof(double) * (size_t)dim * (size_t)n);
    }
    return 0;
}

int ora_set_marker_kinematics(ora_ctx* c, const double* X, const double* U)
{
    int dim = c->d.dim, n = c->nm;
    if (n == 0 || c->motion != ORA_EXTERNAL || !X) return -1;
    if (!supports_inside(c, n, X)) return -1;
    memcpy(c->X, X, sizeof(double) * (size_t)dim * (size_t)n);
    if (U) memcpy(c->U, U, sizeof(double) * (size_t)dim * (size_t)n);
    else memset(c->U, 0, sizeof(double) * (size_t)dim * (size_t)n);
    return 0;
}

int ora_set_probes(ora_ctx* c, int n, const double* Xp)
{
    if (n < 0 || (n > 0 && !Xp)) return -1;
    if (n > 0 && !supports_inside(c, n, Xp)) return -1;
    free(c->Xp);
    c->np = n;
    c->Xp = (double*)calloc((size_t)c->d.dim * (size_t)(n > 0 ? n : 1), sizeof(double));
    if (n > 0) memcpy(c->Xp, Xp, sizeof(double) * (size_t)c->d.dim * (size_t)n);
    return 0;
}

ora_ctx* ora_create(const ora_desc* desc)
{
    if (!desc || (desc->dim != 2 && desc->dim != 3)) return NULL;
    for (int d = 0; d < desc->dim; ++d)
        if (desc->n[d] < 1) return NULL;
    if (desc->dim == 2 && desc->n[2] != 1) return NULL;
    if (!(desc->h > 0.0)) return NULL;
    if (desc->charwise != 0 && desc->charwise != 1) return NULL;
    ora_ctx* c = (ora_ctx*)calloc(1, sizeof(ora_ctx));
    c->d = *desc;
    c->nq = desc->dim + 2;
    c->nx = desc->n[0];
    c->ny = desc->n[1];
    c->nz = desc->dim == 3 ? desc->n[2] : 1;
    c->ncell = c->nx * c->ny * c->nz;
    double u[3] = {desc->prim_inf[1], desc->prim_inf[2], desc->prim_inf[3]};
    prim_to_cons(c, desc->prim_inf[0], u, desc->prim_inf[4], c->q_inf);
    ora_set_markers(c, 0, NULL, NULL, NULL, ORA_STATIC, 0.0);
    return c;
}

void ora_destroy(ora_ctx* c)
{
    if (!c) return;
    free_markers(c);
    free(c->Xp);
    free(c);
}
