// Fused 2D right-hand side / SSP-RK3 stage kernel for gfx950.
//
// One wave64 owns a column strip of 64 consecutive x cells (56 outputs plus a 4-cell halo
// on each side) and marches along y over a segment of rows.  Per front row it loads the
// state once, forms the y-split fluxes f+-_y and the velocities, and keeps them in register
// windows (five rows, slot = row mod 5 fixed at compile time by unrolling the march by 5),
// so every y-face is reconstructed exactly once.  x-neighbours come from the neighbouring
// lanes of the same wave.  The viscous stress (Sec. 2, Eqs. (5)-(6), fourth-order central
// differences applied twice) lags the front by two rows, the output row by four.  The
// output row combines, in this order, the x and y convective terms, the viscous term and
// the sources (penalty-IB force from the window array, sponge), and writes either L(Q) or
// the SSP-RK3 combination a Qn + b (Qs + dt L).
#include "fsa_impl.hpp"

namespace fsa {

namespace {

constexpr int HALO = 4;
constexpr int WAVE = 64;
constexpr int OUTW = WAVE - 2 * HALO;   // 56 output columns per wave

__device__ __forceinline__ double from_lower(double x, int k) { return __shfl_up(x, (unsigned)k, WAVE); }
__device__ __forceinline__ double from_upper(double x, int k) { return __shfl_down(x, (unsigned)k, WAVE); }

// Fourth-order central first derivative from the values at offsets -2..+2 (times 1/(12h)).
__device__ __forceinline__ double d1(double gm2, double gm1, double gp1, double gp2, double inv12h)
{
    return (8.0 * (gp1 - gm1) - (gp2 - gm2)) * inv12h;
}

__device__ __forceinline__ double d1_lanes(double g, double inv12h)
{
    return d1(from_lower(g, 2), from_lower(g, 1), from_upper(g, 1), from_upper(g, 2), inv12h);
}

template <int SCHEME>
struct Column2D {
    // problem
    Grid G;
    Phys P;
    Recon R;
    const double* __restrict__ Qs;
    const double* Qn;    // may alias out (last stage writes in place)
    double* out;
    const double* __restrict__ fwin;
    int wlo0, wlo1, wn0, wn1;
    double ax, ay, inv_h, inv12h, ca, cb, dt;
    int mode_rhs;
    int j0, j1, ic, i;
    bool out_lane;
    // register windows, slot = (row - first front row) mod 5
    double fp[5][4], fm[5][4];
    double uw[5], vw[5];
    double txx[5], txy[5], tyy[5], bx[5], by[5];
    double fy_prev[4], cy_queue[4], cy_new[4];

    template <int K>
    __device__ __forceinline__ void step(int Rw)
    {
        constexpr int S0 = K % 5;          // row Rw (and row Rw-5 before it is overwritten)
        constexpr int S1 = (K + 4) % 5;    // row Rw-1
        constexpr int S2 = (K + 3) % 5;    // row Rw-2
        constexpr int S3 = (K + 2) % 5;    // row Rw-3
        constexpr int S4 = (K + 1) % 5;    // row Rw-4

        // ---- front row: state, velocity, y-split fluxes
        double q[4];
        fetch_state<2>(Qs, G, P, ic, Rw, 0, q);
        const double inv_rho = 1.0 / q[0];
        const double u = q[1] * inv_rho, v = q[2] * inv_rho;
        const double p = P.gm1 * (q[3] - 0.5 * fma(q[1], u, q[2] * v));
        double fpr[4];
        {
            const double F[4] = {q[2], q[1] * v, fma(q[2], v, p), (q[3] + p) * v};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                fm[S0][c] = 0.5 * fma(-ay, q[c], F[c]);
                fpr[c] = 0.5 * fma(ay, q[c], F[c]);
            }
        }
        uw[S0] = u;
        vw[S0] = v;

        // ---- y face (Rw-3)+1/2: f+ rows Rw-5..Rw-1, f- rows Rw..Rw-4
        if ((P.terms & T_CONVY) && Rw >= j0 + 2 && Rw <= j1 + 3) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double fh = recon5<SCHEME>(fp[S0][c], fp[S4][c], fp[S3][c], fp[S2][c], fp[S1][c], R)
                                + recon5<SCHEME>(fm[S0][c], fm[S1][c], fm[S2][c], fm[S3][c], fm[S4][c], R);
                cy_new[c] = -(fh - fy_prev[c]) * inv_h;
                fy_prev[c] = fh;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) fp[S0][c] = fpr[c];

        // ---- stress at row Rw-2 (velocities of rows Rw-4..Rw in the window)
        if ((P.terms & T_VISC) && Rw >= j0) {
            const double uc = uw[S2], vc = vw[S2];
            const double dudx = d1_lanes(uc, inv12h), dvdx = d1_lanes(vc, inv12h);
            const double dudy = d1(uw[S4], uw[S3], uw[S1], uw[S0], inv12h);
            const double dvdy = d1(vw[S4], vw[S3], vw[S1], vw[S0], inv12h);
            const double div = dudx + dvdy;
            const double sxx = P.mu * fma(-2.0 / 3.0, div, dudx + dudx);
            const double syy = P.mu * fma(-2.0 / 3.0, div, dvdy + dvdy);
            const double sxy = P.mu * (dudy + dvdx);
            txx[S2] = sxx;
            txy[S2] = sxy;
            tyy[S2] = syy;
            bx[S2] = fma(uc, sxx, vc * sxy);
            by[S2] = fma(uc, sxy, vc * syy);
        }

        // ---- output row r = Rw-4
        if (Rw >= j0 + 4) {
            const int r = Rw - 4;
            double L[4] = {0.0, 0.0, 0.0, 0.0};
            // x convection: state of row r, velocities from the window
            double qr[4];
            fetch_state<2>(Qs, G, P, ic, r, 0, qr);
            if (P.terms & T_CONVX) {
                const double ur = uw[S4], vr = vw[S4];
                const double pr = P.gm1 * (qr[3] - 0.5 * fma(qr[1], ur, qr[2] * vr));
                const double F[4] = {qr[1], fma(qr[1], ur, pr), qr[2] * ur, (qr[3] + pr) * ur};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double fpx = 0.5 * fma(ax, qr[c], F[c]);
                    const double fmx = 0.5 * fma(-ax, qr[c], F[c]);
                    const double fh =
                        recon5<SCHEME>(from_lower(fpx, 2), from_lower(fpx, 1), fpx, from_upper(fpx, 1),
                                       from_upper(fpx, 2), R) +
                        recon5<SCHEME>(from_upper(fmx, 3), from_upper(fmx, 2), from_upper(fmx, 1), fmx,
                                       from_lower(fmx, 1), R);
                    L[c] = -(fh - from_lower(fh, 1)) * inv_h;
                }
            }
            if (P.terms & T_CONVY) {
#pragma unroll
                for (int c = 0; c < 4; ++c) L[c] += cy_queue[c];
            }
            if (P.terms & T_VISC) {
                // rows r-2..r+2 sit in slots S1, S0, S4, S3, S2
                const double vx = d1_lanes(txx[S4], inv12h) + d1(txy[S1], txy[S0], txy[S3], txy[S2], inv12h);
                const double vy = d1_lanes(txy[S4], inv12h) + d1(tyy[S1], tyy[S0], tyy[S3], tyy[S2], inv12h);
                const double ve = d1_lanes(bx[S4], inv12h) + d1(by[S1], by[S0], by[S3], by[S2], inv12h);
                L[1] += vx;
                L[2] += vy;
                L[3] += ve;
            }
            if (out_lane) {
                double s[4] = {0.0, 0.0, 0.0, 0.0};
                if ((P.terms & T_IB) && fwin) {
                    const int wi = i - wlo0, wj = r - wlo1;
                    if (wi >= 0 && wi < wn0 && wj >= 0 && wj < wn1) {
                        const long long wc = (long long)wj * wn0 + wi;
                        const long long wcells = (long long)wn0 * wn1;
                        const double f0 = fwin[wc], f1 = fwin[wcells + wc];
                        s[1] = f0;
                        s[2] = f1;
                        s[3] = fma(f0, uw[S4], f1 * vw[S4]);
                    }
                }
                if ((P.terms & T_SPONGE) && P.sigma != 0.0) {
                    const double sg = sponge_rate<2>(G, P, i, r, 0);
                    if (sg != 0.0) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) s[c] = fma(-sg, qr[c] - P.q_inf[c], s[c]);
                    }
                }
                const long long o = (long long)r * G.n[0] + i;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double l = L[c] + s[c];
                    double val;
                    if (mode_rhs) {
                        val = l;
                    } else {
                        const double stage = fma(dt, l, qr[c]);
                        val = (ca == 0.0) ? stage : fma(ca, Qn[c * G.ncell + o], cb * stage);
                    }
                    out[c * G.ncell + o] = val;
                }
            }
        }
        if ((P.terms & T_CONVY) && Rw >= j0 + 3 && Rw <= j1 + 3) {
#pragma unroll
            for (int c = 0; c < 4; ++c) cy_queue[c] = cy_new[c];
        }
    }
};

template <int SCHEME>
__global__ __launch_bounds__(64) void k_stage2d(Grid G, Phys P, StageArgs A)
{
    Column2D<SCHEME> C;
    C.G = G;
    C.P = P;
    C.R.eps = SCHEME == WENO5JS ? P.weno_eps : P.teno_eps;
    C.R.ct = P.teno_ct;
    C.Qs = A.Qs;
    C.Qn = A.Qn;
    C.out = A.out;
    C.fwin = A.fwin;
    C.wlo0 = A.wlo[0];
    C.wlo1 = A.wlo[1];
    C.wn0 = A.wn[0];
    C.wn1 = A.wn[1];
    C.ax = __longlong_as_double((long long)A.alpha_bits[0]);
    C.ay = __longlong_as_double((long long)A.alpha_bits[1]);
    C.inv_h = G.inv_h;
    C.inv12h = 1.0 / (12.0 * G.h);
    C.ca = A.ca;
    C.cb = A.cb;
    C.dt = A.dt;
    C.mode_rhs = A.mode_rhs;

    const int lane = threadIdx.x;
    const int nx = G.n[0], ny = G.n[1];
    C.i = blockIdx.x * OUTW - HALO + lane;
    C.ic = min(max(C.i, -HALO), nx + HALO - 1);
    C.out_lane = lane >= HALO && lane < WAVE - HALO && C.i < nx;
    C.j0 = blockIdx.y * A.ty;
    C.j1 = min(C.j0 + A.ty, ny) - 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        C.fy_prev[c] = 0.0;
        C.cy_queue[c] = 0.0;
        C.cy_new[c] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < 5; ++s) {
#pragma unroll
        for (int c = 0; c < 4; ++c) C.fp[s][c] = C.fm[s][c] = 0.0;
        C.uw[s] = C.vw[s] = 0.0;
        C.txx[s] = C.txy[s] = C.tyy[s] = C.bx[s] = C.by[s] = 0.0;
    }
    const int Rend = C.j1 + HALO;
    for (int Rw = C.j0 - HALO; Rw <= Rend; Rw += 5) {
        C.template step<0>(Rw);
        if (Rw + 1 > Rend) break;
        C.template step<1>(Rw + 1);
        if (Rw + 2 > Rend) break;
        C.template step<2>(Rw + 2);
        if (Rw + 3 > Rend) break;
        C.template step<3>(Rw + 3);
        if (Rw + 4 > Rend) break;
        C.template step<4>(Rw + 4);
    }
}

}  // namespace

int launch_stage2d(const Grid& G, const Phys& P, int scheme, const StageArgs& A, hipStream_t s)
{
    const int ncolx = (G.n[0] + OUTW - 1) / OUTW;
    const int nseg = (G.n[1] + A.ty - 1) / A.ty;
    dim3 grid(ncolx, nseg), block(WAVE);
    if (scheme == TENO5) hipLaunchKernelGGL(k_stage2d<TENO5>, grid, block, 0, s, G, P, A);
    else hipLaunchKernelGGL(k_stage2d<WENO5JS>, grid, block, 0, s, G, P, A);
    return (int)hipGetLastError();
}

int stage2d_ncolx(int nx) { return (nx + OUTW - 1) / OUTW; }

}  // namespace fsa
