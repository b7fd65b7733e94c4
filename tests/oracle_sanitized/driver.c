/*
 * Sanitizer driver for the oracle (test infrastructure): every entry point of ora.h on small
 * grids -- 2D and 3D, every boundary kind, static, rotating and external markers, probes,
 * both schemes and both reconstruction variables, the test hooks -- built together with
 * ora.c under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitized.py.  Exits non-zero when a call fails or returns a non-finite
 * value; the sanitizers abort on any invalid access, leak or undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ora.h"

static int failures = 0;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);   \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static int all_finite(const double* a, long n)
{
    for (long k = 0; k < n; ++k)
        if (!isfinite(a[k])) return 0;
    return 1;
}

static ora_desc base_desc(int dim, int nx, int ny, int nz, int bc, int scheme)
{
    ora_desc d;
    memset(&d, 0, sizeof d);
    d.dim = dim;
    d.n[0] = nx;
    d.n[1] = ny;
    d.n[2] = dim == 3 ? nz : 1;
    d.h = 1.0 / 16.0;
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = -0.5 * (a < dim ? d.n[a] : 1) * d.h;
        d.bc[a][0] = d.bc[a][1] = bc;
    }
    d.gamma = 1.4;
    d.mu = 0.004;
    d.scheme = scheme;
    d.terms = ORA_ALL;
    d.weno_eps = 1e-6;
    d.teno_ct = 1e-6;
    d.teno_eps = 1e-40;
    d.prim_inf[0] = 1.0;
    d.prim_inf[1] = 0.2;
    d.prim_inf[4] = 1.0 / 1.4;
    d.inflow_amp = 1e-4;
    d.seed = 1905;
    for (int a = 0; a < dim; ++a) d.sponge_width[a][0] = d.sponge_width[a][1] = 0.25;
    d.sponge_sigma = 2.0;
    d.ib_alpha = 40.0;
    d.ib_beta = 4.0;
    return d;
}

/* A smooth state with a density step: rho, u, (w,) p from cell centres. */
static void fill_state(const ora_desc* d, double* Q)
{
    const int dim = d->dim, nx = d->n[0], ny = d->n[1], nz = dim == 3 ? d->n[2] : 1;
    const long nc = (long)nx * ny * nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long n = ((long)k * ny + j) * nx + i;
                const double x = (i + 0.5) / nx, y = (j + 0.5) / ny, z = (k + 0.5) / nz;
                const double rho = 1.0 + 0.05 * sin(6.3 * x) * cos(6.3 * y) + (x > 0.6 ? 0.1 : 0.0);
                double u[3] = {0.2 + 0.03 * sin(6.3 * y), 0.02 * cos(6.3 * x), 0.01 * sin(6.3 * z)};
                const double p = (1.0 + 0.04 * cos(6.3 * (x + y + z))) / 1.4;
                double ke = 0.0;
                Q[n] = rho;
                for (int a = 0; a < dim; ++a) {
                    Q[(1 + a) * nc + n] = rho * u[a];
                    ke += u[a] * u[a];
                }
                Q[(dim + 1) * nc + n] = p / 0.4 + 0.5 * rho * ke;
            }
}

static void circle_markers(int dim, int nm, double r, double* X, double* dV)
{
    for (int k = 0; k < nm; ++k) {
        const double th = 6.283185307179586 * (k + 0.5) / nm;
        X[k] = r * cos(th);
        X[nm + k] = r * sin(th);
        if (dim == 3) X[2 * nm + k] = 0.05 * sin(3.0 * th);
        dV[k] = 6.283185307179586 * r / nm;
    }
}

static void exercise(int dim, int bc, int scheme, int charwise, int motion)
{
    ora_desc d = base_desc(dim, 30, 26, 22, bc, scheme);
    d.charwise = charwise;
    if (bc == ORA_BC_INFLOW) d.bc[0][1] = ORA_BC_EXTRAP;   /* inflow on x- only */
    ora_ctx* c = ora_create(&d);
    CHECK(c != NULL);
    if (!c) return;
    const int nq = dim + 2;
    const long nc = (long)d.n[0] * d.n[1] * d.n[2];
    double* Q = calloc((size_t)nq * nc, sizeof(double));
    double* L = calloc((size_t)nq * nc, sizeof(double));
    fill_state(&d, Q);

    enum { NM = 24, NP = 5 };
    double X[3 * NM], dV[NM], U[3 * NM], F[3 * NM], xi[3 * NM], out[3 * NM];
    circle_markers(dim, NM, 0.3, X, dV);
    for (int k = 0; k < 3 * NM; ++k) U[k] = 0.01 * (k % 5);
    CHECK(ora_set_markers(c, NM, X, dV, motion == ORA_EXTERNAL ? U : NULL, motion, 0.3) == 0);
    double Xp[3 * NP];
    for (int k = 0; k < NP; ++k) {
        Xp[k] = -0.4 + 0.2 * k;
        Xp[NP + k] = 0.35;
        Xp[2 * NP + k] = 0.0;
    }
    CHECK(ora_set_probes(c, NP, Xp) == 0);

    double alpha[3];
    CHECK(ora_alpha(c, Q, alpha) == 0 && all_finite(alpha, 3));
    CHECK(ora_rhs(c, Q, L) == 0 && all_finite(L, (long)nq * nc));
    int64_t cells[4] = {0, 7, nc / 2, nc - 1};
    double Lc[5 * 4];
    CHECK(ora_rhs_cells(c, Q, 4, cells, Lc) == 0 && all_finite(Lc, (long)nq * 4));
    double* rec = calloc((size_t)3 * nq * nc, sizeof(double));
    CHECK(ora_record_stages(c, rec) == 0);
    for (int s = 0; s < 3; ++s) {
        if (motion == ORA_EXTERNAL) {
            for (int k = 0; k < NM; ++k) X[k] += 0.001;
            CHECK(ora_set_marker_kinematics(c, X, U) == 0);
        }
        CHECK(ora_rk3_step(c, Q, 0.004) == 0);
    }
    CHECK(ora_record_stages(c, NULL) == 0);
    CHECK(all_finite(Q, (long)nq * nc) && all_finite(rec, 3L * nq * nc));
    free(rec);

    double* field = calloc((size_t)dim * nc, sizeof(double));
    for (long n = 0; n < (long)dim * nc; ++n) field[n] = 0.1 * (n % 7);
    CHECK(ora_ib_interp(c, field, dim, out) == 0 && all_finite(out, (long)dim * NM));
    CHECK(ora_ib_spread(c, out, dim, field, 1.0) == 0 && all_finite(field, (long)dim * nc));
    free(field);
    double dp[NP], tot[5];
    CHECK(ora_probe_dp(c, Q, dp) == 0 && all_finite(dp, NP));
    CHECK(ora_marker_force(c, F) == 0 && all_finite(F, (long)dim * NM));
    CHECK(ora_totals(c, Q, tot) == 0 && all_finite(tot, nq));
    double* dil = calloc((size_t)nc, sizeof(double));
    CHECK(ora_dilatation(c, Q, dil) == 0 && all_finite(dil, nc));
    free(dil);
    double t;
    int64_t step;
    CHECK(ora_get_state(c, xi, &t, &step) == 0 && step == 3);
    CHECK(ora_set_state(c, xi, t, step) == 0);

    /* learned-part hooks and the TENO5 read-outs */
    double feat[16];
    CHECK(ora_face_features(c, Q, 0, 3, 4, 0, 0, feat) == 0);
    CHECK(ora_face_label(c, Q, dim - 1, 2, 3, dim == 3 ? 2 : 0, 1, alpha[dim - 1]) >= 0);
    CHECK(ora_face_significant(c, Q, 1, 5, 5, 0, 1) >= 0);
    long nfaces = 0;
    for (int a = 0; a < dim; ++a) nfaces += (long)(d.n[0] + (a == 0)) * (d.n[1] + (a == 1)) * (dim == 3 ? d.n[2] + (a == 2) : 1);
    uint32_t* bits = calloc((size_t)nfaces, sizeof(uint32_t));
    CHECK(ora_teno_bits(c, Q, bits) == 0);
    free(bits);
    long g[3] = {0, nfaces / 2, nfaces - 1};
    int m[3] = {0, 1, dim + 1}, sd[3] = {0, 1, 0};
    double v[15], chi[9];
    CHECK(ora_alpha(c, Q, alpha) == 0);
    CHECK(ora_teno_values_n(c, Q, alpha, 3, g, m, sd, v, chi) == 0 && all_finite(v, 15));
    double qa[5] = {1.0, 0.2, 0.1, 0.0, 2.0}, qb[5] = {1.1, 0.1, -0.1, 0.05, 2.2}, Lm[25], Rm[25];
    if (dim == 2) {
        qa[3] = qa[4];
        qb[3] = qb[4];
    }
    CHECK(ora_char_vectors(c, qa, qb, dim - 1, Lm, Rm) == 0 && all_finite(Lm, (long)nq * nq));
    free(Q);
    free(L);
    ora_destroy(c);
}

int main(void)
{
    CHECK(ora_threads(1) == 1);
    const int bcs[4] = {ORA_BC_PERIODIC, ORA_BC_EXTRAP, ORA_BC_INFLOW, ORA_BC_NONREFLECT};
    for (int dim = 2; dim <= 3; ++dim)
        for (int b = 0; b < 4; ++b)
            for (int scheme = 0; scheme < 2; ++scheme)
                exercise(dim, bcs[b], scheme, (b + scheme) & 1, b % 3);
    /* scalar building blocks and rejected descriptors */
    CHECK(isfinite(ora_delta4(0.3)) && isfinite(ora_recon5(1, 2, 3, 2, 1, ORA_TENO5, 1e-6, 1e-6, 1e-40)));
    double vv[10] = {1, 2, 3, 4, 5, 1, 1, 1, 1, 1};
    int flags[2];
    CHECK(ora_teno_flags_n(vv, 2, 1e-6, 1e-40, flags) == 0 && flags[1] == ora_teno_flags(1, 1, 1, 1, 1, 1e-6, 1e-40));
    CHECK(ora_splitmix64(1, 2) != ora_splitmix64(1, 3));
    ora_desc bad = base_desc(2, 8, 8, 1, ORA_BC_PERIODIC, ORA_WENO5JS);
    bad.charwise = 2;
    CHECK(ora_create(&bad) == NULL);
    bad.charwise = 0;
    bad.n[2] = 3;
    CHECK(ora_create(&bad) == NULL);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle under the sanitizers: every entry point ran clean\n");
    return 0;
}
