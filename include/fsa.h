/*
 * fsa.h -- C ABI of the MI355X (gfx950) immersed-boundary compressible Navier-Stokes library.
 *
 * The library computes the fluid hot path of the immersed-boundary method of Wang, Tian &
 * Lai (fluid-structure-acoustics interactions, Sec. 2):
 *   - the right-hand side L(Q) of the conservative compressible NS system (Sec. 2,
 *     Eqs. (2)-(6)): convective fluxes by global Lax-Friedrichs splitting and fifth-order
 *     WENO5-JS or TENO5 reconstruction per direction, viscous fluxes by fourth-order
 *     central differences, the penalty immersed-boundary source and a sponge;
 *   - the penalty immersed boundary: interpolation of velocity to Lagrangian markers
 *     (Eq. (8)), the feedback force F_f = alpha int (U_ib - U) dt + beta (U_ib - U)
 *     (Eq. (7)), spreading of -F_f to the grid (Eq. (9)) with the four-point delta function
 *     (Eqs. (10)-(11));
 *   - the third-order TVD (SSP) Runge-Kutta update the paper uses for time integration.
 *
 * Conventions
 *   - Grid: uniform, cell-centred, x_i = lo + (i + 1/2) h, the same h in every direction.
 *   - Field arrays are DEVICE pointers to FP64 structure-of-arrays, component-major:
 *     Q[c * ncell + (k * ny + j) * nx + i], components [rho, m_1..m_dim, E] (nq = dim + 2),
 *     interior cells only (ghost values are generated from the boundary conditions).
 *   - Marker and probe arrays passed in are HOST pointers, [dim][n] component-major; they are
 *     copied before the call returns, so the caller may free them at once.
 *   - Every call that takes device pointers is enqueued on the context's HIP stream and
 *     returns without waiting; the buffers must stay alive until the stream has passed the
 *     call.  Calls documented as synchronising wait for the stream.
 *   - A context belongs to one host thread at a time.
 *   - Ownership: the caller owns all device memory.  fsa_workspace_bytes states how much one
 *     context needs for its descriptor (RK stage buffers, reduction partials, marker, window
 *     and probe arrays up to the descriptor's capacities, 3D stress and face buffers, the
 *     selector network); the caller allocates it (e.g. a torch tensor) and hands it to
 *     fsa_init, and keeps it alive, unused by anything else, until fsa_destroy returns.  The
 *     library never allocates, frees or resizes device memory.  It allocates only small pinned
 *     host buffers (the wave-speed read-back and the double-buffered marker placement
 *     staging, 2 x the placement size at the marker capacity) and HIP events, all freed by
 *     fsa_destroy.
 *
 * Errors: every function returns FSA_OK (0) or a negative status.  Argument and shape errors
 * are reported synchronously as FSA_EINVAL with a message from fsa_last_error.  Device
 * errors surface as FSA_EDEVICE.  With nan_check set, a NaN or Inf seen by the global
 * wave-speed reduction makes the next fsa_rk3_step / fsa_sync return FSA_ENONFINITE (the
 * state is not rolled back).  No C++ exception crosses this interface.
 */
#ifndef FSA_H
#define FSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSA_ABI_VERSION 4

enum {
    FSA_OK = 0,
    FSA_EINVAL = -1,
    FSA_ENOMEM = -2,
    FSA_EDEVICE = -3,
    FSA_ENONFINITE = -4,
    FSA_ESTATE = -5,
    FSA_EUNSUPPORTED = -6
};

/* Boundary conditions per direction and side.  NONREFLECT is the non-reflecting boundary of
 * Thompson (1987, 1990) that Sec. 2 applies on the outer boundaries: ghosts as EXTRAP for the
 * stencils, and at the boundary cell the convective term along the boundary normal in its
 * characteristic form with the amplitudes of incoming waves set to zero (see fsa_desc). */
enum { FSA_BC_PERIODIC = 0, FSA_BC_EXTRAP = 1, FSA_BC_INFLOW = 2, FSA_BC_NONREFLECT = 3 };
/* Convective reconstruction. */
enum { FSA_WENO5JS = 0, FSA_TENO5 = 1 };
/* Arithmetic of the face reconstruction and viscous fluxes (the state is always FP64):
 * FP64; FP32 on deviations from the far field (precision form); FP32 with the sub-stencils
 * chosen by the learned selector (fsa_mlp_set), plain TENO5 on low-confidence faces. */
enum { FSA_FP64 = 0, FSA_MIXED32 = 1, FSA_LEARNED32 = 2 };
/* Variables the reconstruction acts on.  COMPONENT: the conserved components, one by one
 * (global Lax-Friedrichs splitting, component-wise).  CHARACTERISTIC (FP64 only; other
 * precisions: FSA_EUNSUPPORTED): at each face the split fluxes of the six cells are projected
 * on the left eigenvectors of the flux Jacobian along the face normal at the Roe average of
 * the face's two cells, each characteristic field is reconstructed by the scheme, and the
 * face flux is recombined with the right eigenvectors (Jiang & Shu 1996); the paper does not
 * state which variables its schemes act on.  Fields are ordered u_n - c, entropy, shear
 * (tangential directions in increasing order), u_n + c; with r = sqrt(rho) weights the Roe
 * average takes u and H = (E + p)/rho, c^2 = (gamma - 1)(H - |u|^2/2).  In 2D this form runs
 * as separate stress, face and stage passes. */
enum { FSA_COMPONENT = 0, FSA_CHARACTERISTIC = 1 };
/* Cell layers a stage's output at one cell depends on along each direction (the viscous
 * terms: two for the stress, two for its divergence), the halo depth of a block. */
enum { FSA_HALO = 4 };
/* Marker motion. */
enum { FSA_STATIC = 0, FSA_ROTATING = 1, FSA_EXTERNAL = 2 };
/* Right-hand-side terms (bit mask). */
enum {
    FSA_TERM_CONV_X = 1, FSA_TERM_CONV_Y = 2, FSA_TERM_CONV_Z = 4, FSA_TERM_VISC = 8,
    FSA_TERM_IB = 16, FSA_TERM_SPONGE = 32, FSA_TERM_ALL = 63
};

/* Problem description (Sec. 2 problem statement plus the readings the paper leaves open).
 *
 * Boundary ghosts: PERIODIC wraps, EXTRAP copies the nearest interior cell, INFLOW holds the
 * far-field state prim_inf with each velocity component perturbed by
 * inflow_amp * (2 r - 1), r uniform in [0,1) from the counter-based SplitMix64 stream of
 * seed at counter ((((step * 6 + side) * 8 + depth) * ncell + cell) * 3 + component),
 * side = 2 * direction + (0 low | 1 high), depth >= 1 the ghost layer, cell the linear index
 * of the nearest interior cell.  Directions are resolved in the order x, y, z.
 *
 * Sponge: S = -sigma(x) (Q - Q_inf), sigma = sponge_sigma * eta^3, eta = max over
 * directions of (depth into the layer) / (layer width), clipped to 1.
 *
 * Non-reflecting side (FSA_BC_NONREFLECT, a direction with at least 3 cells): at its boundary
 * cell, with primitives rho, u, p, c = sqrt(gamma p / rho), u_n the normal velocity and
 * one-sided derivatives along the normal from the boundary cell and the next two inward,
 * (4 (f1 - f0) - (f2 - f0)) / 2h pointing outward-in, the wave amplitudes
 * L1 = (u_n - c)(p' - rho c u_n'), L2 = u_n (c^2 rho' - p'), L_t = u_n u_t' (tangential),
 * L5 = (u_n + c)(p' + rho c u_n') are zeroed where their speed points into the domain, and
 * the normal flux derivative is [d1, u d1 + rho (dn e_n + d_t e_t), |u|^2/2 d1 + d2/(gamma-1)
 * + rho (u_n dn + u_t d_t)] with d1 = (L2 + (L5+L1)/2)/c^2, d2 = (L5+L1)/2,
 * dn = (L5-L1)/(2 rho c), d_t = L_t.  Computed in FP64 in every form. */
typedef struct fsa_desc {
    int32_t  dim;                 /* 2 or 3 */
    int32_t  n[3];                /* cells per direction; n[2] = 1 in 2D */
    double   lo[3];               /* lower corner of the domain */
    double   h;                   /* uniform grid spacing */
    int32_t  bc[3][2];            /* FSA_BC_* per direction and side */
    double   gamma;               /* ratio of specific heats (ideal gas) */
    double   mu;                  /* dynamic viscosity, 1/Re folded in; 0 disables viscosity */
    int32_t  scheme;              /* FSA_WENO5JS or FSA_TENO5 */
    int32_t  precision;           /* FSA_FP64, FSA_MIXED32 or FSA_LEARNED32 */
    int32_t  terms;               /* FSA_TERM_* mask */
    int32_t  nan_check;           /* 1: report non-finite wave speeds as FSA_ENONFINITE */
    double   weno_eps;            /* WENO5-JS epsilon (1e-6) */
    double   teno_ct;             /* TENO5 cut-off C_T (1e-6) */
    double   teno_eps;            /* TENO5 epsilon (1e-40) */
    double   prim_inf[5];         /* far-field rho, u, v, w, p */
    double   inflow_amp;          /* inflow velocity perturbation amplitude */
    uint64_t seed;                /* its seed */
    double   sponge_width[3][2];  /* sponge layer widths per direction and side */
    double   sponge_sigma;        /* sigma_max */
    double   ib_alpha;            /* penalty constant on the integral term, Eq. (7) */
    double   ib_beta;             /* penalty constant on the proportional term, Eq. (7) */
    int32_t  selector_stride;     /* learned form: 1 (or 0) = keep patterns from every stage's
                                     state; 3 = from each step's first stage, reused by its
                                     other two stages.  Other values: FSA_EINVAL */
    /* Periodic Gaussian pressure source of the sphere-scattering case (Sec. 3), 3D only:
     * A_p = -src_amp exp(-src_b log(2) |x - src_x|^2) cos(src_omega t) at the cell centres,
     * added to the energy equation as A_p / (gamma - 1) (the pressure rate it makes at fixed
     * density and velocity), t the time of each SSP-RK3 stage (t, t + dt, t + dt/2).
     * src_amp = 0: no source; nonzero in 2D: FSA_EUNSUPPORTED. */
    double   src_amp;
    double   src_b;
    double   src_omega;
    double   src_x[3];
    /* Capacities of the workspace (fsa_workspace_bytes): markers and probes the context can
     * hold (fsa_set_markers / fsa_set_probes with more: FSA_EINVAL), and cells of the box that
     * holds every marker's four-point support (0: the whole grid, always enough; a placement
     * whose box is larger: FSA_EINVAL). */
    int32_t  max_markers;
    int32_t  max_probes;
    int64_t  max_window_cells;
    int32_t  variables;           /* FSA_COMPONENT or FSA_CHARACTERISTIC */
    /* Placement in a larger grid (a block of a decomposed domain; global_n[d] = 0: none):
     * local cell i along d is global cell i + origin[d] of a grid of global_n[d] cells whose
     * lower corner is lo.  Cell positions (sponge, markers, probes, source) and the inflow
     * noise counters are then those of the global grid, so a block computes its cells as the
     * whole grid would.  origin may reach FSA_HALO cells below 0 and the block as far beyond
     * global_n (halo layers wrapped across a periodic direction); otherwise FSA_EINVAL. */
    int32_t  origin[3];
    int32_t  global_n[3];
} fsa_desc;

typedef struct fsa_ctx fsa_ctx;

/* Run statistics.  Synchronising. */
typedef struct fsa_stats {
    double   alpha[3];            /* last global Lax-Friedrichs speeds max(|u_d| + c) */
    double   t;                   /* current time */
    int64_t  step;                /* completed RK3 steps */
    int32_t  nonfinite;           /* 1 if a NaN/Inf reached the wave-speed reduction */
    int32_t  n_markers;
    int32_t  n_probes;
    int32_t  window_cells;        /* cells of the box that holds every marker's support */
    int32_t  rows_per_wave;       /* segment height the 2D stage kernel runs with (0 = not tuned yet) */
    int64_t  learned_sides;       /* face sides the learned selector has decided (cumulative) */
    int64_t  fallback_sides;      /* of which fell back to plain TENO5 */
    int64_t  significant_sides;   /* of which were significant (evaluated by the network) */
} fsa_stats;

int32_t     fsa_abi_version(void);
const char* fsa_status_str(int32_t status);
/* Message of the last error on ctx (owned by ctx, valid until the next call on ctx). */
const char* fsa_last_error(const fsa_ctx* ctx);

/* Device bytes a context for desc needs (*bytes; 0 on error).  Validates desc (FSA_EINVAL).
 * Depends on the descriptor only: the grid, dimension, precision, boundary kinds and the
 * three capacities. */
int32_t fsa_workspace_bytes(const fsa_desc* desc, size_t* bytes);
/* Create a context on the current HIP device, enqueuing on hip_stream (a hipStream_t; NULL
 * is the null stream), its device buffers carved from the caller's d_workspace (a device
 * pointer to at least fsa_workspace_bytes(desc) bytes, any alignment; its contents need not
 * be initialised).  FSA_EINVAL: invalid desc, NULL or too small a workspace.  Synchronising
 * (the constants are copied in). */
int32_t fsa_init(const fsa_desc* desc, void* d_workspace, size_t ws_bytes, void* hip_stream, fsa_ctx** out);
/* Free everything the context owns.  Synchronising.  NULL is accepted. */
int32_t fsa_destroy(fsa_ctx* ctx);

/* Lagrangian markers (Sec. 2, Eqs. (7)-(9)): positions X[dim][n], quadrature weights
 * dV[n] (arc length in 2D, area in 3D), velocities U[dim][n] (NULL = 0; ignored for
 * ROTATING, where U = omega e_z x X about the origin).  Every marker's four-point support
 * must lie inside the grid (FSA_EINVAL otherwise).  Resets the penalty integral to zero.
 * n = 0 removes the markers.  Synchronising. */
int32_t fsa_set_markers(fsa_ctx* ctx, int32_t n, const double* X, const double* dV,
                        const double* U, int32_t motion, double omega);
/* New positions and velocities for EXTERNAL markers (same count), e.g. from a structure
 * solver; keeps the penalty integral.  Stream-ordered: the arrays are read before the call
 * returns and take effect for work enqueued after it; the host waits at most for the
 * previous update's host-to-device copy, and for the stream when the markers' window box
 * outgrows its buffers. */
int32_t fsa_set_marker_kinematics(fsa_ctx* ctx, const double* X, const double* U);
/* Probe points Xp[dim][n] for fsa_probe_dp; supports must lie inside the grid. */
int32_t fsa_set_probes(fsa_ctx* ctx, int32_t n, const double* Xp);

/* Global Lax-Friedrichs speeds alpha[d] = max over cells of |u_d| + c of d_Q, written to the
 * host array alpha[3] (NaN-propagating).  Synchronising. */
int32_t fsa_alpha(fsa_ctx* ctx, const double* d_Q, double* alpha);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc), and need no context: the global Lax-Friedrichs
 * speeds of fsa_alpha, max over the cells of d_Q (the grid and gas of desc, FP64 state as
 * above) of |u_d| + c, NaN-propagating, written to the DEVICE array d_alpha[3] (directions
 * beyond dim: 0) on hip_stream, without synchronising.  Allocates nothing: its per-block
 * partial maxima (at most 2048 blocks x 3) live in a static device array of the library, one
 * per GPU (48 KB, held until the process ends), which every call on that GPU shares and which
 * keeps the last call's partials; calls that overlap on one GPU (on different streams, or
 * from different threads without ordering) race and give wrong results.  Any grid desc
 * accepts fits (larger grids fold into the same number of partials); FSA_EINVAL for an invalid
 * desc or NULL pointers, FSA_EDEVICE if the launch fails. */
int32_t fsa_alpha_noalloc(const fsa_desc* desc, const double* d_Q, double* d_alpha, void* hip_stream);
/* d_L = L(d_Q) at the context's time, step and penalty integral (Sec. 2, Eq. (2) with the
 * IB source of Eqs. (7)-(9)).  d_L must not alias d_Q.  Also records the penalty force. */
int32_t fsa_rhs(fsa_ctx* ctx, const double* d_Q, double* d_L);
/* One SSP-RK3 step of size dt in place on d_Q:
 *   Q1 = Qn + dt L(Qn);  Q2 = 3/4 Qn + 1/4 (Q1 + dt L(Q1));  Qn+1 = 1/3 Qn + 2/3 (Q2 + dt L(Q2)),
 * the penalty integral advancing through the same stages; then t += dt, step += 1. */
int32_t fsa_rk3_step(fsa_ctx* ctx, double* d_Q, double dt);
/* nsteps consecutive fsa_rk3_step calls in one enqueue: the global Lax-Friedrichs speeds of
 * each stage input are taken from the kernel that wrote that state, so only the first stage
 * reduces d_Q on its own. */
int32_t fsa_rk3_steps(fsa_ctx* ctx, double* d_Q, double dt, int32_t nsteps);
/* fsa_rk3_steps continuing from the previous step call on this context: d_Q must be the
 * buffer that call advanced, holding what it wrote (the caller has not changed it since).
 * The first stage then takes the Lax-Friedrichs speeds of d_Q from the kernel that wrote it,
 * and the learned form's first keep-pattern pass its quiet-tile ranges, instead of computing
 * them afresh, so that k calls of one step each do what one call of k steps does (bit for
 * bit).  For callers that change something else between steps (the markers' kinematics, the
 * probes read-out).  FSA_ESTATE when the context holds no such state for d_Q: no step call
 * yet, another buffer, or an fsa_rhs call since.  A change to d_Q in between is not seen and
 * gives wrong results. */
int32_t fsa_rk3_steps_resume(fsa_ctx* ctx, double* d_Q, double dt, int32_t nsteps);
/* Interpolate ncomp fields d_field[ncomp][ncell] to the markers (Eq. (8)):
 * d_out[a][k] = sum over the support of field_a * prod lambda. */
int32_t fsa_ib_interp(fsa_ctx* ctx, const double* d_field, int32_t ncomp, double* d_out);
/* d_field[a] += scale * f_a with f = -sum_k F_k prod lambda dV_k / h^dim (Eq. (9)), F given
 * on the markers as d_F[ncomp][n].  Each cell sums its markers in index order. */
int32_t fsa_ib_spread(fsa_ctx* ctx, const double* d_F, int32_t ncomp, double* d_field,
                      double scale);
/* Acoustic pressure p - p_inf interpolated to the probes, d_dp[np]. */
int32_t fsa_probe_dp(fsa_ctx* ctx, const double* d_Q, double* d_dp);
/* Penalty force on the structure from the most recent right-hand side, host h_F[dim][n]
 * (the force on the fluid is its negative, Sec. 2).  Synchronising. */
int32_t fsa_marker_force(fsa_ctx* ctx, double* h_F);
/* The markers' count, motion (FSA_STATIC, FSA_ROTATING, FSA_EXTERNAL) and the solver's
 * dimension, e.g. for a structure solver to check that its arrays fit before it exchanges X,
 * U and F ([dim][n] each; host; any output may be NULL). */
int32_t fsa_marker_info(const fsa_ctx* ctx, int32_t* n, int32_t* motion, int32_t* dim);
/* Checkpoint: penalty integral h_xi[dim][n], time and step.  Synchronising. */
int32_t fsa_get_state(fsa_ctx* ctx, double* h_xi, double* t, int64_t* step);
int32_t fsa_set_state(fsa_ctx* ctx, const double* h_xi, double t, int64_t step);
/* Diagnostics (Sec. 3: field totals; the dilatation of the precision-form discussion).
 * h_totals (host, nullable) receives sum over cells of q_m h^dim for every component
 * (deterministic summation order; synchronising when given); d_dilatation (device, nullable,
 * [ncell] in the state's cell order) receives div u by fourth-order central differences of
 * u_d = m_d / rho, ghosts by the boundary conditions.  FSA_EINVAL if both are NULL. */
int32_t fsa_diagnostics(fsa_ctx* ctx, const double* d_Q, double* h_totals, double* d_dilatation);

/* Learned TENO5 sub-stencil selector (not in the paper; the library's addition).  A face side
 * is significant when rho, a velocity component or p varies over its five cells by more than
 * 1e-8 of its natural scale (rho_inf, c_inf, rho_inf c_inf^2); an insignificant side keeps
 * every sub-stencil.  For significant sides a network 15 -> 32 -> 32 -> 3 (ReLU, logits) maps
 * the features -- rho, the normal velocity (negated on the "-" side) and p at the five
 * upwind-ordered cells, each as deviations from the centre over (their largest magnitude +
 * 1e-8 of the natural scale) -- to keep probabilities of the three TENO5 sub-stencils, shared
 * by all conserved components.  Flat parameters (FP32, 1667): W1[15][32], b1[32], W2[32][32],
 * b2[32], W3[32][3], b3[3].  Inference and training run on BF16 MFMA with FP32 accumulation.
 * A side whose confidence min_k |2 sigmoid(z_k) - 1| is below conf_threshold, or with no
 * sub-stencil predicted, uses plain TENO5 per component.  Labels: bit k set when FP64 TENO5
 * keeps sub-stencil k for every component (a component whose five values agree to 1e-12
 * counts as keeping all). */
int32_t fsa_mlp_set(fsa_ctx* ctx, const float* h_params, int32_t nparams, double conf_threshold);
/* As fsa_mlp_set from BF16 parameters (HOST uint16 bit patterns, the same flat layout): each is
 * widened exactly to the FP32 master copy, so inference uses these BF16 values unchanged. */
int32_t fsa_set_mlp(fsa_ctx* ctx, const uint16_t* h_bf16_params, int32_t nparams, double conf_threshold);
int32_t fsa_mlp_get(fsa_ctx* ctx, float* h_params, int32_t nparams);            /* synchronising */
/* Logits d_logits[n][3] of features d_feats[n][16] (column 15 ignored). */
int32_t fsa_mlp_forward(fsa_ctx* ctx, const float* d_feats, int64_t n, float* d_logits);
/* Mean binary cross-entropy d_loss[1] and its gradient d_grad[1667] over n samples. */
int32_t fsa_mlp_grad(fsa_ctx* ctx, const float* d_feats, const uint8_t* d_labels, int64_t n, float* d_grad,
                     float* d_loss);
/* One Adam step (beta 0.9/0.999, eps 1e-8) on the gradient of this batch; d_loss may be NULL. */
int32_t fsa_mlp_train_step(fsa_ctx* ctx, const float* d_feats, const uint8_t* d_labels, int64_t n, float lr,
                           float* d_loss);
/* Harvest training samples from a 2D or 3D state at its own wave speeds: every significant
 * face side with a TENO5 cut-off and a seeded fraction keep_rate of the significant all-kept
 * ones (side s of face f is kept when the SplitMix64 number 2 f' + s of seed, as a uniform in
 * [0, 1), is below keep_rate; f' counts x faces first, then y faces, then z faces), written
 * in face order (x faces [nz][ny][nx+1], y faces [nz][ny+1][nx], z faces [nz+1][ny][nx]) as
 * d_feats[max_out][16], d_labels[max_out].  In 3D the features are those of 2D (rho, the
 * normal velocity and p of the five cells) and the label ANDs the five components.
 * *h_count receives the number selected (only the first max_out are written).
 * Synchronising. */
int32_t fsa_harvest(fsa_ctx* ctx, const double* d_Q, double keep_rate, uint64_t seed, int64_t max_out,
                    float* d_feats, uint8_t* d_labels, int64_t* h_count);
/* Keep patterns the learned form uses for d_Q: x faces [(nx+1) ny], y faces [nx (ny+1)];
 * bits 3c..3c+2 (side "+") and 16+3c.. (side "-") for component c. */
int32_t fsa_face_flags(fsa_ctx* ctx, const double* d_Q, uint32_t* d_flags_x, uint32_t* d_flags_y);

/* Test read-out of the TENO5 sub-stencil decisions (component-wise FP64 TENO5 only;
 * FSA_EUNSUPPORTED otherwise): while d_bits (DEVICE, uint32) is set, every right-hand side and SSP-RK3 stage
 * enqueued on ctx also writes the keep pattern its reconstruction chose at every face, for
 * the state that stage evaluates, into d_bits[stage][faces] (a lone fsa_rhs: stage 0; RK3
 * stages 0, 1, 2; a multi-step call leaves its last step's): x faces [nz][ny][nx+1], then y
 * faces [nz][ny+1][nx], then (3D) z faces [nz+1][ny][nx], one word per face with bits 3c+k
 * (side "+", component c, sub-stencil k kept) and 16+3c+k (side "-") -- the layout of
 * fsa_face_flags.  The kernels then run an instantiation that adds these stores to the same
 * arithmetic.  NULL turns the read-out off.  Used by tests to check that where the library
 * and an independent implementation decide differently, the decision is a tie. */
int32_t fsa_debug_teno_bits(fsa_ctx* ctx, uint32_t* d_bits);

/* Measurement: with timing on, a pair of HIP events on the context's stream brackets every
 * launch of the fused stencil/update kernel.  fsa_timing_read (synchronising) returns the
 * summed kernel milliseconds and the number of launches since the previous read. */
int32_t fsa_timing_enable(fsa_ctx* ctx, int32_t on);
int32_t fsa_timing_read(fsa_ctx* ctx, double* ms, int64_t* launches);
/* Wait for the stream; returns FSA_ENONFINITE if nan_check saw a NaN/Inf. */
int32_t fsa_sync(fsa_ctx* ctx);
int32_t fsa_stats_get(fsa_ctx* ctx, fsa_stats* out);

/* ---------------------------------------------------------------------------------------
 * Several blocks of one domain on one GPU: the one-GPU stand-in for the domain decomposition
 * across processes that the paper's solver runs with MPI (Sec. 2).
 *
 * The domain desc describes is cut into nblocks slabs along its last direction (y in 2D, z
 * in 3D), the first (n % nblocks) of them one cell layer thicker.  Each block is a context
 * over its own layers plus FSA_HALO layers of each neighbouring block (across the domain's
 * ends too when that direction is periodic), placed in the global grid with origin /
 * global_n; the block's own boundary rule at a halo side is EXTRAP and only ever shapes the
 * halo layers' output.  Every SSP-RK3 stage is enqueued on all blocks, then explicit device
 * copies refresh each block's halo layers from its neighbours' stage output, and the global
 * Lax-Friedrichs speeds of that output are the maximum over the blocks' own (the all-reduce
 * of a multi-process run).  Each block holds the markers whose supports reach its own
 * layers, in their global order (re-dealt when EXTERNAL markers move, their penalty integrals
 * going with them).  The result equals one context's over the whole domain bit for bit.
 * Probes and diagnostics are taken on the gathered state.  Every call is stream-ordered on hip_stream unless it says
 * synchronising: the blocks' stages run side by side on streams of their own (created with
 * the default priority), which wait for hip_stream before each stage and which hip_stream
 * waits for after it.
 *
 * Device memory: one workspace of fsa_mb_workspace_bytes (the blocks' contexts and states
 * and the copy tables) owned by the caller; the library allocates host memory only.
 * --------------------------------------------------------------------------------------- */
typedef struct fsa_mb fsa_mb;
/* Workspace bytes for desc in nblocks blocks.  FSA_EINVAL: invalid desc (its origin and
 * global_n must be zero), nblocks < 1, or a block thinner than FSA_HALO layers. */
int32_t fsa_mb_workspace_bytes(const fsa_desc* desc, int32_t nblocks, size_t* bytes);
int32_t fsa_mb_init(const fsa_desc* desc, int32_t nblocks, void* d_workspace, size_t ws_bytes, void* hip_stream,
                    fsa_mb** out);
int32_t fsa_mb_destroy(fsa_mb* mb);
const char* fsa_mb_last_error(const fsa_mb* mb);
/* Block b's first global layer, layer count, and halo layers below and above. */
int32_t fsa_mb_block_info(const fsa_mb* mb, int32_t b, int32_t* first, int32_t* count, int32_t* halo_lo,
                          int32_t* halo_hi);
/* Markers of the whole domain (HOST arrays as fsa_set_markers), shared out to the blocks
 * whose layers their supports reach; resets the penalty integral.  Synchronising.
 * FSA_EINVAL: a support leaves the grid (nothing changed).  After another error (a block's
 * own rejection, e.g. more markers than its desc.max_markers) the markers are undefined:
 * fsa_mb_rk3_steps, fsa_mb_marker_force and fsa_mb_set_marker_kinematics return FSA_ESTATE
 * until a call of this function succeeds. */
int32_t fsa_mb_set_markers(fsa_mb* mb, int32_t n, const double* X, const double* dV, const double* U,
                           int32_t motion, double omega);
/* EXTERNAL markers: new positions X and velocities U (HOST [dim][n], U NULL: zero) for the
 * steps that follow, as fsa_set_marker_kinematics.  A block whose markers stay the same takes
 * the kinematics; one whose set changes is given its new markers with their penalty integrals
 * (read back from the blocks that held them: synchronising then).  FSA_ESTATE: the markers
 * are not EXTERNAL, or undefined after a failed call; FSA_EINVAL: a support leaves the grid
 * (nothing changed).  After another error the markers are undefined (as above) until
 * fsa_mb_set_markers. */
int32_t fsa_mb_set_marker_kinematics(fsa_mb* mb, const double* X, const double* U);
/* The whole domain's state (DEVICE, [nq][cells] as fsa_rk3_step) into the blocks, halo
 * layers included; a fresh start: time, step and the penalty integral zero. */
int32_t fsa_mb_scatter(fsa_mb* mb, const double* d_Q);
/* The blocks' own layers into the whole domain's state d_Q (DEVICE). */
int32_t fsa_mb_gather(const fsa_mb* mb, double* d_Q);
/* nsteps SSP-RK3 steps of size dt on the blocks, halo copies and the wave-speed maximum
 * after every stage. */
int32_t fsa_mb_rk3_steps(fsa_mb* mb, double dt, int32_t nsteps);
/* Penalty force of the last stage per marker, h_F[dim][n] (HOST), each marker from a block
 * holding it.  Synchronising. */
int32_t fsa_mb_marker_force(fsa_mb* mb, double* h_F);

#ifdef __cplusplus
}
#endif
#endif /* FSA_H */
