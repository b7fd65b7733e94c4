// Flexible plate by absolute nodal coordinates (Sec. 2's beam equation; the clamped leading
// edge's flapping of Sec. 4.1): the host side of the explicit staggered coupling, declared in
// fsa_plate.h.
//
// The matrices are the textbook consistent Hermite element matrices (mass rho l / 420 [...],
// bending K_B / l^3 [...]) per component, assembled as symmetric band matrices (two nodes of
// four coordinates: half-bandwidth 7).  The free block of M + dt^2/4 K is factored once per
// step size (band Cholesky); a step is then a band solve, three band products, the stretching
// quadrature and the marker load: O(elements + markers).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fsa_plate.h"

// Sub-steps of a plate step: dt_sub omega_s < SUBSTEP_LIMIT (the explicit stretching force
// is stable below 2), at most MAX_SUBSTEPS of them.
constexpr double SUBSTEP_LIMIT = 1.9;
constexpr int MAX_SUBSTEPS = 16;

namespace {

constexpr int BW = 7;
constexpr double PI = 3.14159265358979323846;

// Symmetric band matrix, lower part: A(i, j) for 0 <= i - j <= BW.
struct Band {
    int n = 0;
    std::vector<double> a;
    void init(int n_)
    {
        n = n_;
        a.assign((size_t)n * (BW + 1), 0.0);
    }
    double get(int i, int j) const
    {
        if (i < j) std::swap(i, j);
        return i - j > BW ? 0.0 : a[(size_t)i * (BW + 1) + (i - j)];
    }
    double& low(int i, int j) { return a[(size_t)i * (BW + 1) + (i - j)]; }   // i >= j
};

// Lower Cholesky factor of a band matrix in place; false if it is not positive definite.
bool band_cholesky(Band& A)
{
    for (int i = 0; i < A.n; ++i) {
        const int k0 = std::max(0, i - BW);
        for (int j = k0; j <= i; ++j) {
            double s = A.low(i, j);
            for (int k = k0; k < j; ++k)
                if (j - k <= BW) s -= A.low(i, k) * A.low(j, k);
            if (i == j) {
                if (!(s > 0.0)) return false;
                A.low(i, i) = std::sqrt(s);
            } else {
                A.low(i, j) = s / A.low(j, j);
            }
        }
    }
    return true;
}

// x = (L L^T)^-1 b for a factor from band_cholesky (b and x may alias).
void band_solve(const Band& Lf, const double* b, double* x)
{
    const int n = Lf.n;
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = std::max(0, i - BW); k < i; ++k) s -= Lf.get(i, k) * x[k];
        x[i] = s / Lf.get(i, i);
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k <= std::min(n - 1, i + BW); ++k) s -= Lf.get(k, i) * x[k];
        x[i] = s / Lf.get(i, i);
    }
}

// Five-point Gauss-Legendre rule on [0, 1] (nodes and weights in closed form).
void gauss5(double* x, double* w)
{
    const double a = std::sqrt(5.0 - 2.0 * std::sqrt(10.0 / 7.0)) / 3.0;
    const double b = std::sqrt(5.0 + 2.0 * std::sqrt(10.0 / 7.0)) / 3.0;
    const double wa = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0, wb = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
    const double xs[5] = {-b, -a, 0.0, a, b}, ws[5] = {wb, wa, 128.0 / 225.0, wa, wb};
    for (int g = 0; g < 5; ++g) {
        x[g] = 0.5 * (xs[g] + 1.0);
        w[g] = 0.5 * ws[g];
    }
}

// Hermite functions at xi of an element of length l (left position, left slope, right
// position, right slope), and their arc-length derivatives.
void hermite(double xi, double l, double* N, double* dN)
{
    const double x2 = xi * xi, x3 = x2 * xi;
    N[0] = 1.0 - 3.0 * x2 + 2.0 * x3;
    N[1] = l * (xi - 2.0 * x2 + x3);
    N[2] = 3.0 * x2 - 2.0 * x3;
    N[3] = l * (x3 - x2);
    dN[0] = (6.0 * x2 - 6.0 * xi) / l;
    dN[1] = 1.0 - 4.0 * xi + 3.0 * x2;
    dN[2] = (6.0 * xi - 6.0 * x2) / l;
    dN[3] = 3.0 * x2 - 2.0 * xi;
}

// Largest eigenvalue of k x = lambda m x for 4 x 4 symmetric k, positive definite m (power
// iteration on m^-1 k, Rayleigh quotient).
double max_eig4(const double k[4][4], const double m[4][4])
{
    double x[4] = {1.0, 0.3, -0.7, 0.2}, lam = 0.0;
    for (int it = 0; it < 400; ++it) {
        double y[4], A[4][5];
        for (int r = 0; r < 4; ++r) {
            y[r] = 0.0;
            for (int c = 0; c < 4; ++c) y[r] += k[r][c] * x[c];
            for (int c = 0; c < 4; ++c) A[r][c] = m[r][c];
            A[r][4] = y[r];
        }
        for (int p = 0; p < 4; ++p)   // Gaussian elimination (m is positive definite)
            for (int r = p + 1; r < 4; ++r) {
                const double f = A[r][p] / A[p][p];
                for (int c = p; c < 5; ++c) A[r][c] -= f * A[p][c];
            }
        double z[4];
        for (int r = 3; r >= 0; --r) {
            double s = A[r][4];
            for (int c = r + 1; c < 4; ++c) s -= A[r][c] * z[c];
            z[r] = s / A[r][r];
        }
        double nz = 0.0;
        for (double zi : z) nz = std::max(nz, std::fabs(zi));
        if (!(nz > 0.0)) return 0.0;
        for (int r = 0; r < 4; ++r) x[r] = z[r] / nz;
        double xk = 0.0, xm = 0.0;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                xk += x[r] * k[r][c] * x[c];
                xm += x[r] * m[r][c] * x[c];
            }
        lam = xk / xm;
    }
    return lam;
}

}  // namespace

struct fsa_plate {
    int nel = 0, ndof = 0, nm = 0;
    double L = 0, l = 0, rho = 0, ks = 0, kb = 0;
    std::vector<double> s, dv;
    double edge[2] = {0, 0}, a0 = 0, beta = 0, am = 0, f = 0, phi = 0;
    Band M, K;                 // all coordinates
    Band Mf;                   // factor of the free block of M
    Band A;                    // factor of the free block of M + dt^2/4 K
    double A_dt = -1.0;
    double omega_s = 0.0;      // bound on the largest stretching frequency (unstretched plate)
    std::vector<double> e, v, a, Q, fs, et, rhs;
    double t = 0.0;
    double gx[5], gw[5];
    std::string err;
};

namespace {

int fail(fsa_plate* p, int code, const char* msg)
{
    p->err = msg;
    return code;
}

// Clamp state at t: position, slope, their velocities and accelerations (4 coordinates each).
void clamp(const fsa_plate* p, double t, double* ep, double* vp, double* ap)
{
    const double w = 2.0 * PI * p->f, cb = std::cos(p->beta), sb = std::sin(p->beta);
    const double h = 0.5 * p->a0, c = std::cos(w * t), sn = std::sin(w * t);
    ep[0] = p->edge[0] + h * c * cb;
    ep[1] = p->edge[1] + h * c * sb;
    vp[0] = -h * w * sn * cb;
    vp[1] = -h * w * sn * sb;
    ap[0] = -h * w * w * c * cb;
    ap[1] = -h * w * w * c * sb;
    const double ph = w * t + p->phi;
    const double al = 0.5 * p->am * std::sin(ph), alt = 0.5 * p->am * w * std::cos(ph),
                 altt = -0.5 * p->am * w * w * std::sin(ph);
    const double ca = std::cos(al), sa = std::sin(al);
    // slope (cos alpha, -sin alpha); its alpha-derivative (-sin alpha, -cos alpha)
    ep[2] = ca;
    ep[3] = -sa;
    vp[2] = -sa * alt;
    vp[3] = -ca * alt;
    ap[2] = -ca * alt * alt - sa * altt;
    ap[3] = sa * alt * alt - ca * altt;
}

void stretch_force(const fsa_plate* p, const double* e, double* out)
{
    std::fill(out, out + p->ndof, 0.0);
    if (p->ks == 0.0) return;
    for (int j = 0; j < p->nel; ++j) {
        const double* ej = e + 4 * j;
        double* oj = out + 4 * j;
        for (int g = 0; g < 5; ++g) {
            double N[4], dN[4];
            hermite(p->gx[g], p->l, N, dN);
            double xs[2] = {0.0, 0.0};
            for (int q = 0; q < 4; ++q)
                for (int c = 0; c < 2; ++c) xs[c] += dN[q] * ej[2 * q + c];
            const double coef = p->ks * p->l * p->gw[g] * (std::hypot(xs[0], xs[1]) - 1.0);
            for (int q = 0; q < 4; ++q)
                for (int c = 0; c < 2; ++c) oj[2 * q + c] += coef * (dN[q] * xs[c]);
        }
    }
}

void locate(const fsa_plate* p, double s, int& j, double& xi)
{
    j = std::min((int)(s / p->l), p->nel - 1);
    xi = s / p->l - j;
}

// Accelerations of the free coordinates from the unloaded equation (start, set_state).
void rest_accelerations(fsa_plate* p)
{
    double ep[4], vp[4], ap[4];
    clamp(p, p->t, ep, vp, ap);
    for (int k = 0; k < 4; ++k) p->a[k] = ap[k];
    stretch_force(p, p->e.data(), p->fs.data());
    const int nf = p->ndof - 4;
    for (int i = 4; i < p->ndof; ++i) {
        double s = -p->fs[i];
        for (int j = std::max(0, i - BW); j <= std::min(p->ndof - 1, i + BW); ++j) {
            s -= p->K.get(i, j) * p->e[j];
            if (j < 4) s -= p->M.get(i, j) * ap[j];
        }
        p->rhs[i - 4] = s;
    }
    band_solve(p->Mf, p->rhs.data(), p->rhs.data());
    for (int i = 0; i < nf; ++i) p->a[4 + i] = p->rhs[i];
}

}  // namespace

extern "C" {

int32_t fsa_plate_create(const fsa_plate_desc* d, fsa_plate** out)
{
    if (!d || !out) return FSA_EINVAL;
    *out = nullptr;
    if (!(d->length > 0.0) || d->n_elements < 1 || d->n_elements > 100000 || !(d->rho_s > 0.0) ||
        !(d->k_s >= 0.0) || !(d->k_b >= 0.0) || d->n_markers < 1 || !d->s_mark || !d->dv_mark ||
        !std::isfinite(d->a0 + d->beta + d->alpha_m + d->freq + d->phi + d->t0 + d->edge[0] + d->edge[1]))
        return FSA_EINVAL;
    for (int k = 0; k < d->n_markers; ++k)
        if (!(d->s_mark[k] >= 0.0 && d->s_mark[k] <= d->length) || !std::isfinite(d->dv_mark[k])) return FSA_EINVAL;
    fsa_plate* p = new (std::nothrow) fsa_plate;
    if (!p) return FSA_ENOMEM;
    try {
        p->nel = d->n_elements;
        p->ndof = 4 * (p->nel + 1);
        p->nm = d->n_markers;
        p->L = d->length;
        p->l = d->length / d->n_elements;
        p->rho = d->rho_s;
        p->ks = d->k_s;
        p->kb = d->k_b;
        p->s.assign(d->s_mark, d->s_mark + p->nm);
        p->dv.assign(d->dv_mark, d->dv_mark + p->nm);
        p->edge[0] = d->edge[0];
        p->edge[1] = d->edge[1];
        p->a0 = d->a0;
        p->beta = d->beta;
        p->am = d->alpha_m;
        p->f = d->freq;
        p->phi = d->phi;
        gauss5(p->gx, p->gw);
        const double l = p->l;
        // consistent element matrices per component, coordinates (position, slope) x 2 nodes
        const double m4[4][4] = {{156.0, 22.0 * l, 54.0, -13.0 * l},
                                 {22.0 * l, 4.0 * l * l, 13.0 * l, -3.0 * l * l},
                                 {54.0, 13.0 * l, 156.0, -22.0 * l},
                                 {-13.0 * l, -3.0 * l * l, -22.0 * l, 4.0 * l * l}};
        const double k4[4][4] = {{12.0, 6.0 * l, -12.0, 6.0 * l},
                                 {6.0 * l, 4.0 * l * l, -6.0 * l, 2.0 * l * l},
                                 {-12.0, -6.0 * l, 12.0, -6.0 * l},
                                 {6.0 * l, 2.0 * l * l, -6.0 * l, 4.0 * l * l}};
        const double mf = p->rho * l / 420.0, kf = p->kb / (l * l * l);
        p->M.init(p->ndof);
        p->K.init(p->ndof);
        for (int j = 0; j < p->nel; ++j)
            for (int q = 0; q < 4; ++q)
                for (int r = 0; r < 4; ++r)
                    for (int c = 0; c < 2; ++c) {
                        const int gi = 4 * j + 2 * q + c, gj = 4 * j + 2 * r + c;
                        if (gi < gj) continue;
                        p->M.low(gi, gj) += mf * m4[q][r];
                        p->K.low(gi, gj) += kf * k4[q][r];
                    }
        const int nf = p->ndof - 4;
        p->Mf.init(nf);
        for (int i = 0; i < nf; ++i)
            for (int j = std::max(0, i - BW); j <= i; ++j) p->Mf.low(i, j) = p->M.get(i + 4, j + 4);
        if (!band_cholesky(p->Mf)) {
            delete p;
            return FSA_EINVAL;
        }
        // stretching frequency bound: the element's largest eigenvalue (no larger one exists
        // in the assembly) of K_S int dN dN^T ds against the element mass
        double ke[4][4], me[4][4];
        for (int q = 0; q < 4; ++q)
            for (int r = 0; r < 4; ++r) {
                me[q][r] = mf * m4[q][r];
                ke[q][r] = 0.0;
            }
        for (int g = 0; g < 5; ++g) {
            double N[4], dN[4];
            hermite(p->gx[g], l, N, dN);
            for (int q = 0; q < 4; ++q)
                for (int r = 0; r < 4; ++r) ke[q][r] += p->ks * l * p->gw[g] * dN[q] * dN[r];
        }
        p->omega_s = p->ks > 0.0 ? std::sqrt(max_eig4(ke, me)) : 0.0;
        p->e.assign(p->ndof, 0.0);
        p->v.assign(p->ndof, 0.0);
        p->a.assign(p->ndof, 0.0);
        p->Q.assign(p->ndof, 0.0);
        p->fs.assign(p->ndof, 0.0);
        p->et.assign(p->ndof, 0.0);
        p->rhs.assign(nf, 0.0);
        p->t = d->t0;
        double ep[4], vp[4], ap[4];
        clamp(p, p->t, ep, vp, ap);
        for (int i = 0; i <= p->nel; ++i) {
            const double si = i * l;
            for (int c = 0; c < 2; ++c) {
                p->e[4 * i + c] = ep[c] + si * ep[2 + c];
                p->e[4 * i + 2 + c] = ep[2 + c];
                p->v[4 * i + c] = vp[c] + si * vp[2 + c];
                p->v[4 * i + 2 + c] = vp[2 + c];
            }
        }
        rest_accelerations(p);
    } catch (...) {
        delete p;
        return FSA_ENOMEM;
    }
    *out = p;
    return FSA_OK;
}

int32_t fsa_plate_destroy(fsa_plate* p)
{
    delete p;
    return FSA_OK;
}

int32_t fsa_plate_markers(const fsa_plate* p, double* X, double* U)
{
    if (!p || !X) return FSA_EINVAL;
    for (int k = 0; k < p->nm; ++k) {
        int j;
        double xi, N[4], dN[4];
        locate(p, p->s[k], j, xi);
        hermite(xi, p->l, N, dN);
        for (int c = 0; c < 2; ++c) {
            double x = 0.0, u = 0.0;
            for (int q = 0; q < 4; ++q) {
                x += N[q] * p->e[4 * j + 2 * q + c];
                u += N[q] * p->v[4 * j + 2 * q + c];
            }
            X[c * p->nm + k] = x;
            if (U) U[c * p->nm + k] = u;
        }
    }
    return FSA_OK;
}

namespace {

// One Newmark step of size dt (within the explicit stretching limit).
int32_t plate_substep(fsa_plate* p, const double* F, double dt)
{
    const int nd = p->ndof, nf = nd - 4;
    if (dt != p->A_dt) {
        p->A.init(nf);
        const double c = 0.25 * dt * dt;
        for (int i = 0; i < nf; ++i)
            for (int j = std::max(0, i - BW); j <= i; ++j)
                p->A.low(i, j) = p->M.get(i + 4, j + 4) + c * p->K.get(i + 4, j + 4);
        if (!band_cholesky(p->A)) {
            p->A_dt = -1.0;
            return fail(p, FSA_EINVAL, "Newmark matrix not positive definite");
        }
        p->A_dt = dt;
    }
    const double b = 0.25 * dt * dt;
    for (int i = 0; i < nd; ++i) p->et[i] = p->e[i] + dt * p->v[i] + b * p->a[i];
    double ep[4], vp[4], ap[4];
    const double t1 = p->t + dt;
    clamp(p, t1, ep, vp, ap);
    // load of the marker forces minus the stretching force at the predictor
    stretch_force(p, p->et.data(), p->fs.data());
    for (int i = 0; i < nd; ++i) p->Q[i] = -p->fs[i];
    for (int k = 0; k < p->nm; ++k) {
        int j;
        double xi, N[4], dN[4];
        locate(p, p->s[k], j, xi);
        hermite(xi, p->l, N, dN);
        for (int q = 0; q < 4; ++q)
            for (int c = 0; c < 2; ++c) p->Q[4 * j + 2 * q + c] += N[q] * (F[c * p->nm + k] * p->dv[k]);
    }
    for (int i = 4; i < nd; ++i) {
        double s = p->Q[i];
        for (int j = std::max(0, i - BW); j <= std::min(nd - 1, i + BW); ++j) {
            if (j < 4) s -= p->M.get(i, j) * ap[j] + p->K.get(i, j) * ep[j];
            else s -= p->K.get(i, j) * p->et[j];
        }
        p->rhs[i - 4] = s;
    }
    band_solve(p->A, p->rhs.data(), p->rhs.data());
    bool finite = true;
    for (int i = 0; i < nf; ++i) {
        const double af = p->rhs[i];
        p->e[4 + i] = p->et[4 + i] + b * af;
        p->v[4 + i] = p->v[4 + i] + 0.5 * dt * (p->a[4 + i] + af);
        p->a[4 + i] = af;
        finite = finite && std::isfinite(p->e[4 + i]);
    }
    for (int k = 0; k < 4; ++k) {
        p->e[k] = ep[k];
        p->v[k] = vp[k];
        p->a[k] = ap[k];
    }
    p->t = t1;
    return finite ? FSA_OK : fail(p, FSA_ENONFINITE, "non-finite plate state");
}

}  // namespace

int32_t fsa_plate_step(fsa_plate* p, const double* F, double dt)
{
    if (!p) return FSA_EINVAL;
    if (!F) return fail(p, FSA_EINVAL, "F is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(p, FSA_EINVAL, "dt must be positive");
    // equal sub-steps under the same forces, each within the explicit stretching limit
    // (dt_sub omega_s < 1.9 < 2)
    const double ratio = dt * p->omega_s / SUBSTEP_LIMIT;
    if (!(ratio <= MAX_SUBSTEPS)) {
        p->err = "dt needs more than " + std::to_string(MAX_SUBSTEPS) +
                 " sub-steps of the explicit stretching limit 1.9 / omega_s = " + std::to_string(SUBSTEP_LIMIT / p->omega_s);
        return FSA_EINVAL;
    }
    const int nsub = std::max(1, (int)std::ceil(ratio));
    const double h = dt / nsub;
    for (int k = 0; k < nsub; ++k) {
        const int32_t rc = plate_substep(p, F, h);
        if (rc != FSA_OK) return rc;
    }
    return FSA_OK;
}

int32_t fsa_plate_get_state(const fsa_plate* p, double* e, double* v, double* a, double* t)
{
    if (!p) return FSA_EINVAL;
    if (e) std::memcpy(e, p->e.data(), sizeof(double) * p->ndof);
    if (v) std::memcpy(v, p->v.data(), sizeof(double) * p->ndof);
    if (a) std::memcpy(a, p->a.data(), sizeof(double) * p->ndof);
    if (t) *t = p->t;
    return FSA_OK;
}

int32_t fsa_plate_set_state(fsa_plate* p, const double* e, const double* v, const double* a, double t)
{
    if (!p) return FSA_EINVAL;
    if (!e || !v || !std::isfinite(t)) return fail(p, FSA_EINVAL, "bad plate state");
    p->e.assign(e, e + p->ndof);
    p->v.assign(v, v + p->ndof);
    p->t = t;
    if (a) p->a.assign(a, a + p->ndof);
    else rest_accelerations(p);
    return FSA_OK;
}

int32_t fsa_plate_coupled_steps(fsa_ctx* ctx, fsa_plate* p, double* d_Q, double dt, int32_t nsteps,
                                int32_t resume)
{
    if (!ctx || !p || !d_Q || nsteps < 0) return FSA_EINVAL;
    int32_t nm = 0, motion = -1, dim = 0;
    if (fsa_marker_info(ctx, &nm, &motion, &dim) != FSA_OK) return fail(p, FSA_EINVAL, "bad solver context");
    if (dim != 2) return fail(p, FSA_EUNSUPPORTED, "the plate is planar: the solver must be 2D");
    if (nm != p->nm || motion != FSA_EXTERNAL)
        return fail(p, FSA_ESTATE, "the solver's markers are not the plate's (count or EXTERNAL motion)");
    try {
        std::vector<double> X(2 * (size_t)p->nm), U(2 * (size_t)p->nm), F(2 * (size_t)p->nm);
        for (int n = 0; n < nsteps; ++n) {
            int rc = fsa_plate_markers(p, X.data(), U.data());
            if (rc == FSA_OK) rc = fsa_set_marker_kinematics(ctx, X.data(), U.data());
            if (rc == FSA_OK)
                rc = (resume || n > 0) ? fsa_rk3_steps_resume(ctx, d_Q, dt, 1) : fsa_rk3_steps(ctx, d_Q, dt, 1);
            if (rc == FSA_OK) rc = fsa_marker_force(ctx, F.data());
            if (rc != FSA_OK) return rc;
            if ((rc = fsa_plate_step(p, F.data(), dt)) != FSA_OK) return rc;
        }
    } catch (...) {
        return FSA_ENOMEM;
    }
    return FSA_OK;
}

const char* fsa_plate_last_error(const fsa_plate* p) { return p ? p->err.c_str() : "null plate"; }

}  // extern "C"
