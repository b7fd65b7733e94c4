/* Flexible plate for the flapping-plate coupling (Sec. 2, the beam equation of the flexible
 * structure solved by absolute nodal coordinates; Sec. 4.1, the clamped leading edge's heave
 * and pitch).  Host code (no device memory): the structure side of the explicit staggered
 * coupling, fed by fsa_marker_force and feeding fsa_set_marker_kinematics (fsa.h).
 *
 * Model.  A planar plate of length L in n_elements equal elements; per node the position X
 * and the slope dX/ds (four coordinates, cubic Hermite interpolation along the arc length s).
 * Equation (the sign reading under which both rigidities restore; the printed bracket is
 * garbled):  rho_s X_tt = d/ds[K_S (|X_s| - 1) X_s] - K_B X_ssss + F_f,
 * in weak form  M e_tt + K e + f_s(e) = Q  with the consistent mass and bending matrices, the
 * stretching force f_s by five-point Gauss-Legendre quadrature per element and the load
 * Q = sum_k S(s_k)^T F_k dV_k from the IB markers' forces (force per unit length on the plate).
 * The leading edge (s = 0) is clamped: its position X0(t) = edge + (A0/2) cos(2 pi f t)
 * [cos beta, sin beta] and its slope (cos alpha, -sin alpha), alpha = (alpha_m/2)
 * sin(2 pi f t + phi), are prescribed.
 *
 * Step.  Newmark's average-acceleration rule (beta = 1/4, gamma = 1/2) for the free
 * coordinates with M and K implicit and the stretching force explicit at the Newmark
 * predictor, stable while the step times omega_s (the largest stretching frequency) is below 2:
 * a call of size dt takes n = ceil(dt omega_s / 1.9) equal sub-steps under the same load (at
 * most 16; larger steps are rejected).  The load is the fluid force of the step just taken.
 *
 * Status codes are those of fsa.h.  Not thread-safe per plate. */
#ifndef FSA_PLATE_H
#define FSA_PLATE_H

#include <stdint.h>

#include "fsa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsa_plate fsa_plate;

typedef struct fsa_plate_desc {
    double  length;        /* L */
    int32_t n_elements;    /* >= 1; nodes n_elements + 1 */
    double  rho_s;         /* linear density, > 0 */
    double  k_s;           /* stretching rigidity K_S, >= 0 */
    double  k_b;           /* bending rigidity K_B, >= 0 */
    int32_t n_markers;     /* IB markers on the plate, >= 1 */
    const double* s_mark;  /* [n_markers] arc positions in [0, L] (copied) */
    const double* dv_mark; /* [n_markers] quadrature weights, arc length (copied) */
    double  edge[2];       /* leading-edge rest point */
    double  a0;            /* heave: X0 moves by (a0/2) cos(2 pi f t) along (cos beta, sin beta) */
    double  beta;
    double  alpha_m;       /* pitch: alpha = (alpha_m/2) sin(2 pi f t + phi) */
    double  freq;          /* f */
    double  phi;
    double  t0;            /* start time: straight along the clamp's slope, moving with it */
} fsa_plate_desc;

/* FSA_EINVAL for a bad descriptor, FSA_ENOMEM. */
int32_t fsa_plate_create(const fsa_plate_desc* desc, fsa_plate** out);
int32_t fsa_plate_destroy(fsa_plate* plate);
/* Marker positions X[2][n] and velocities U[2][n] (host arrays): S(s_k) e and S(s_k) e_t. */
int32_t fsa_plate_markers(const fsa_plate* plate, double* X, double* U);
/* One step of size dt under the marker forces F[2][n] (host; the force on the plate per unit
 * length, as fsa_marker_force returns it), in ceil(dt omega_s / 1.9) equal sub-steps.
 * FSA_EINVAL when dt <= 0 or dt needs more than 16 sub-steps (the message names the explicit
 * stretching limit 1.9 / omega_s). */
int32_t fsa_plate_step(fsa_plate* plate, const double* F, double dt);
/* Checkpoint: coordinates e[4(n_elements + 1)] (node j: x, y, x_s, y_s), their velocities and
 * accelerations (the Newmark state) and the time; outputs may be NULL.  set_state with a NULL
 * takes the accelerations from the unloaded equation (a restart then differs from the run by
 * the last load's share of them). */
int32_t fsa_plate_get_state(const fsa_plate* plate, double* e, double* v, double* a, double* t);
int32_t fsa_plate_set_state(fsa_plate* plate, const double* e, const double* v, const double* a,
                            double t);
/* nsteps steps of the explicit staggered coupling of the solver ctx (2D, EXTERNAL markers:
 * the plate's) and the plate, each: the plate's marker positions and velocities to the
 * solver (fsa_set_marker_kinematics), one SSP-RK3 step of d_Q (fsa_rk3_steps_resume when
 * resume is nonzero or after the first step, else fsa_rk3_steps), the step's marker forces
 * (fsa_marker_force, synchronising) and the plate's step under them (fsa_plate_step): what a
 * caller would do per step, without the round trips through the caller.  FSA_ESTATE (before
 * any step) unless the solver's markers are EXTERNAL and as many as the plate's.  Returns the
 * first failing call's status (its message in fsa_last_error or fsa_plate_last_error). */
int32_t fsa_plate_coupled_steps(fsa_ctx* ctx, fsa_plate* plate, double* d_Q, double dt,
                                int32_t nsteps, int32_t resume);
/* Message of the last failed call on the plate (plate-owned). */
const char* fsa_plate_last_error(const fsa_plate* plate);

#ifdef __cplusplus
}
#endif

#endif
