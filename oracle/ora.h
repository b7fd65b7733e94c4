/*
 * ora.h -- plain FP64 CPU oracle for the immersed-boundary compressible Navier-Stokes
 * right-hand side and its SSP-RK3 update (Wang, Tian & Lai, "An immersed boundary method
 * for fluid-structure-acoustics interactions involving large deformations and complex
 * geometries", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and ora.c are the reference the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load this code.  It shares no source, header, table or constant with the GPU
 * library; every constant below is stated here on its own.
 *
 * Conventions
 *   - Uniform cell-centred grid: x_i = lo + (i + 1/2) h, i = 0..n-1, same h in every direction.
 *   - Conserved state Q = [rho, m_1 .. m_dim, E] (Sec. 2, the conservative NS system), stored
 *     structure-of-arrays, component-major: Q[c * ncell + (k * ny + j) * nx + i].
 *     nq = dim + 2 components.  In 2D n[2] must be 1.
 *   - Marker arrays are [dim][nm], also component-major.
 *   - All functions return 0 on success and a negative code on a bad argument.
 */
#ifndef ORA_H
#define ORA_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_BC_PERIODIC = 0, ORA_BC_EXTRAP = 1, ORA_BC_INFLOW = 2, ORA_BC_NONREFLECT = 3 };
enum { ORA_WENO5JS = 0, ORA_TENO5 = 1 };
enum { ORA_STATIC = 0, ORA_ROTATING = 1, ORA_EXTERNAL = 2 };
/* Terms of the right-hand side that are evaluated (bit mask). */
enum {
    ORA_CONV_X = 1, ORA_CONV_Y = 2, ORA_CONV_Z = 4, ORA_VISC = 8,
    ORA_IB = 16, ORA_SPONGE = 32, ORA_ALL = 63
};

typedef struct ora_desc {
    int32_t  dim;              /* 2 or 3 */
    int32_t  n[3];             /* cells per direction (n[2] = 1 in 2D) */
    double   lo[3];            /* lower domain corner */
    double   h;                /* uniform grid spacing */
    int32_t  bc[3][2];         /* boundary type per direction and side (0 = low, 1 = high) */
    double   gamma;            /* ratio of specific heats */
    double   mu;               /* dynamic viscosity (1/Re folded in) */
    int32_t  scheme;           /* ORA_WENO5JS or ORA_TENO5 */
    int32_t  terms;            /* ORA_* bit mask */
    double   weno_eps;         /* WENO5-JS epsilon */
    double   teno_ct;          /* TENO5 cut-off C_T */
    double   teno_eps;         /* TENO5 epsilon */
    double   prim_inf[5];      /* far-field primitive state rho, u, v, w, p */
    double   inflow_amp;       /* amplitude of the seeded inflow velocity perturbation */
    uint64_t seed;             /* seed of that perturbation */
    double   sponge_width[3][2];
    double   sponge_sigma;     /* sigma_max of the cubic sponge */
    double   ib_alpha;         /* penalty constant on the integral term */
    double   ib_beta;          /* penalty constant on the proportional term */
    /* periodic Gaussian pressure source of the sphere-scattering case (Sec. 3):
       A_p = -src_amp exp(-src_b log(2) |x - src_x|^2) cos(src_omega t), added to the energy
       equation as A_p / (gamma - 1) (the pressure rate it makes at fixed rho and u);
       src_amp = 0: none */
    double   src_amp;
    double   src_b;
    double   src_omega;
    double   src_x[3];
    /* variables the reconstruction acts on: 0 = the conserved components, one by one;
       1 = the characteristic fields of the flux Jacobian along the face normal at the Roe
       average of the two cells beside the face (see ora.c) */
    int32_t  charwise;
} ora_desc;

typedef struct ora_ctx ora_ctx;

ora_ctx* ora_create(const ora_desc* desc);
void     ora_destroy(ora_ctx* c);

/* Markers: positions X[dim][n], quadrature weights dV[n], velocities U[dim][n] (NULL = 0).
 * ROTATING markers move with U = omega e_z x X (rotation about the origin).
 * Resets the penalty integral xi to zero. */
int ora_set_markers(ora_ctx* c, int n, const double* X, const double* dV, const double* U,
                    int motion, double omega);
/* EXTERNAL markers: new positions X and velocities U (NULL: zero) for the steps that follow;
 * the penalty integral and the forces are kept (prescribed or structure-driven motion). */
int ora_set_marker_kinematics(ora_ctx* c, const double* X, const double* U);
int ora_set_probes(ora_ctx* c, int n, const double* Xp);

/* Global Lax-Friedrichs speeds alpha[d] = max over cells of |u_d| + c. */
int ora_alpha(const ora_ctx* c, const double* Q, double* alpha);
/* L(Q) at the context's current time, step and penalty integral. */
int ora_rhs(ora_ctx* c, const double* Q, double* L);
/* L(Q) at a list of cells only (linear cell indices); out[nq][ncell_list]. */
int ora_rhs_cells(ora_ctx* c, const double* Q, int64_t nlist, const int64_t* cells, double* out);
/* One SSP-RK3 step in place; advances xi, t and step. */
int ora_rk3_step(ora_ctx* c, double* Q, double dt);
/* Interpolate ncomp cell fields (component-major) to the markers: out[ncomp][nm]. */
int ora_ib_interp(const ora_ctx* c, const double* field, int ncomp, double* out);
/* field[a] += scale * S_a(F), S the spreading operator with the paper's minus sign. */
int ora_ib_spread(const ora_ctx* c, const double* F, int ncomp, double* field, double scale);
/* Acoustic pressure p - p_inf interpolated to the probes. */
int ora_probe_dp(const ora_ctx* c, const double* Q, double* dp);
/* Penalty force of the most recent right-hand-side evaluation, [dim][nm]. */
int ora_marker_force(const ora_ctx* c, double* F);
/* Field totals sum q_m h^dim [nq]; dilatation div u at every cell [ncell]. */
int ora_totals(const ora_ctx* c, const double* Q, double* out);
int ora_dilatation(const ora_ctx* c, const double* Q, double* out);
int ora_get_state(const ora_ctx* c, double* xi, double* t, int64_t* step);
int ora_set_state(ora_ctx* c, const double* xi, double t, int64_t step);

/* Learned-weight inputs and label of one face side (side 0 = f+ stencil i-2..i+2 of the face
 * between cell idx and idx + e_dir, side 1 = f- stencil i+3..i-1); see ora.c. */
int ora_face_features(const ora_ctx* c, const double* Q, int dir, long i, long j, long k, int side, double* out);
int ora_face_label(const ora_ctx* c, const double* Q, int dir, long i, long j, long k, int side, double alpha);
int ora_face_significant(const ora_ctx* c, const double* Q, int dir, long i, long j, long k, int side);

/* Test hooks on the TENO5 decisions (nothing the solver uses):
 * ora_record_stages: while buf is set, ora_rk3_step copies the input state of each of its
 *   three stages into buf[stage][nq][ncell] (NULL stops);
 * ora_teno_bits: the keep patterns of every face of Q at Q's own wave speeds, x faces
 *   [nz][ny][nx+1], y faces [nz][ny+1][nx], (z faces [nz+1][ny][nx]) one after the other,
 *   bits 3m+k (side "+") and 16+3m+k (side "-") for component m and sub-stencil k;
 * ora_teno_values_n: for n (face in that layout, component, side 0 "+" / 1 "-") entries at
 *   the wave speeds alpha[3], the five upwind-ordered split-flux values v[n][5] and
 *   chi_k[n][3]. */
int ora_record_stages(ora_ctx* c, double* buf);
/* The characteristic-wise reconstruction's eigenvectors (a test hook): left rows L[nq][nq]
 * and right columns R[nq][nq] (row-major, R[m * nq + k] = component m of field k) of the flux
 * Jacobian along dir at the Roe average of the conserved states qa and qb; fields in the
 * order u_n - c, entropy, the shear waves of the tangential directions in increasing order,
 * u_n + c. */
int ora_char_vectors(const ora_ctx* c, const double* qa, const double* qb, int dir, double* L, double* R);
/* Threads of the oracle's OpenMP loops (n < 1: unchanged); returns the count in effect. */
int ora_threads(int n);
int ora_teno_bits(const ora_ctx* c, const double* Q, uint32_t* out);
int ora_teno_values_n(const ora_ctx* c, const double* Q, const double* alpha, long n, const long* g, const int* m,
                      const int* sd, double* v, double* chi);

/* Scalar building blocks exposed for the pins. */
double ora_delta4(double r);
/* Reconstruction at a face from five upwind-ordered values. */
double ora_recon5(double a, double b, double cc, double d, double e, int scheme,
                  double weno_eps, double teno_ct, double teno_eps);
/* TENO5 keep flags of one stencil (bit k set = sub-stencil k kept). */
int ora_teno_flags(double a, double b, double cc, double d, double e,
                   double teno_ct, double teno_eps);
/* The same for n stencils v[n][5] into out[n]. */
int ora_teno_flags_n(const double* v, long n, double teno_ct, double teno_eps, int* out);
/* Counter-based SplitMix64: output number ctr of the generator seeded with seed. */
uint64_t ora_splitmix64(uint64_t seed, uint64_t ctr);

#ifdef __cplusplus
}
#endif
#endif
