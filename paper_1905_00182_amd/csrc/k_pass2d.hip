// 2D right-hand side / SSP-RK3 stage in three passes, the form the characteristic-wise
// reconstruction runs in (per face it projects six cells' split fluxes on four eigenvectors,
// which the fused column-march kernel has no registers for):
//
//  * k_pstress2d: for every cell of the grid extended by two ghost layers, the velocity
//    gradients by the fourth-order central difference (Sec. 2, Eqs. (5)-(6)), the Stokes
//    stress and b = u . tau, stored as [5][(nx+4)(ny+4)] (tau_xx, tau_yy, tau_xy, b_x, b_y);
//  * k_pfaces2d<D>: one thread per face along D: the face flux of the six cells i-2..i+3,
//    characteristic-wise (char_face: the split fluxes projected on the eigenvectors at the
//    Roe average of the face's two cells, each field reconstructed, recombined), [4][faces];
//  * k_pstage2d: per interior cell the face differences, the viscous divergence, the
//    penalty-IB force and its work from the window array, the sponge, the RK3 combination,
//    and one wave-speed partial per block.
//
// Threads of a block are 64 consecutive x cells by 4 rows: loads along x are coalesced and
// neighbours along y come through the caches.  Ghosts are resolved where they are read
// (fetch_state), inflow sides included.
#include "fsa_impl.hpp"

namespace fsa {

namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ void cell_state2(const KConst* K, const double* __restrict__ Q, long long step, int i, int j,
                                            double* q)
{
    const Grid& G = K->G;
    if (i >= 0 && i < G.n[0] && j >= 0 && j < G.n[1]) {
        const long long o = (long long)j * G.n[0] + i;
#pragma unroll
        for (int c = 0; c < 4; ++c) q[c] = Q[c * G.ncell + o];
    } else {
        fetch_state<2>(Q, G, K->P, step, i, j, 0, q);
    }
}

__device__ __forceinline__ void velocity2(const KConst* K, const double* Q, long long step, int i, int j, double* u)
{
    double q[4];
    cell_state2(K, Q, step, i, j, q);
    const double ir = rcp_nr(q[0]);
    u[0] = q[1] * ir;
    u[1] = q[2] * ir;
}

__device__ __forceinline__ double d1(double gm2, double gm1, double gp1, double gp2, double inv12h)
{
    return (8.0 * (gp1 - gm1) - (gp2 - gm2)) * inv12h;
}

__global__ __launch_bounds__(BX * BY) void k_pstress2d(const KConst* __restrict__ K, const double* __restrict__ Q,
                                                       long long step, double* __restrict__ S)
{
    const Grid& G = K->G;
    const int ex = G.n[0] + 4, ey = G.n[1] + 4;
    const int xi = blockIdx.x * BX + (threadIdx.x & (BX - 1)), yi = blockIdx.y * BY + threadIdx.x / BX;
    if (xi >= ex || yi >= ey) return;
    const int i = xi - 2, j = yi - 2;
    const double inv12h = K->inv12h, mu = K->P.mu;
    double um2[2], um1[2], up1[2], up2[2], vm2[2], vm1[2], vp1[2], vp2[2], uc[2];
    velocity2(K, Q, step, i - 2, j, um2);
    velocity2(K, Q, step, i - 1, j, um1);
    velocity2(K, Q, step, i + 1, j, up1);
    velocity2(K, Q, step, i + 2, j, up2);
    velocity2(K, Q, step, i, j - 2, vm2);
    velocity2(K, Q, step, i, j - 1, vm1);
    velocity2(K, Q, step, i, j + 1, vp1);
    velocity2(K, Q, step, i, j + 2, vp2);
    velocity2(K, Q, step, i, j, uc);
    double g[2][2];   // g[a][b] = d u_a / d x_b
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        g[a][0] = d1(um2[a], um1[a], up1[a], up2[a], inv12h);
        g[a][1] = d1(vm2[a], vm1[a], vp1[a], vp2[a], inv12h);
    }
    const double div = g[0][0] + g[1][1];
    const double sxx = mu * fma(-2.0 / 3.0, div, g[0][0] + g[0][0]);
    const double syy = mu * fma(-2.0 / 3.0, div, g[1][1] + g[1][1]);
    const double sxy = mu * (g[0][1] + g[1][0]);
    const long long ne = (long long)ex * ey, o = (long long)yi * ex + xi;
    S[0 * ne + o] = sxx;
    S[1 * ne + o] = syy;
    S[2 * ne + o] = sxy;
    S[3 * ne + o] = fma(uc[0], sxx, uc[1] * sxy);
    S[4 * ne + o] = fma(uc[0], sxy, uc[1] * syy);
}

// Faces along D: x faces [ny][nx+1], y faces [ny+1][nx]; face f lies between cells f-1 and f.
template <int D>
__host__ __device__ __forceinline__ long long pfaces_of(const Grid& G)
{
    return (long long)(G.n[0] + (D == 0)) * (G.n[1] + (D == 1));
}

template <int SCHEME, int D>
__global__ __launch_bounds__(BX * BY) void k_pfaces2d(const KConst* __restrict__ K, const double* __restrict__ Q,
                                                      long long step, const unsigned long long* __restrict__ abits,
                                                      double* __restrict__ Fh)
{
    const Grid& G = K->G;
    const int xi = blockIdx.x * BX + (threadIdx.x & (BX - 1)), yi = blockIdx.y * BY + threadIdx.x / BX;
    __shared__ __attribute__((aligned(16))) KeepRows<double> keep_rows;
    if (SCHEME != WENO5JS) {
        init_keep_rows<double>(keep_rows, threadIdx.x);
        __syncthreads();
    }
    if (xi >= G.n[0] + (D == 0) || yi >= G.n[1] + (D == 1)) return;
    const int i = D == 0 ? xi - 1 : xi, j = D == 1 ? yi - 1 : yi;   // cell below the face along D
    const double alpha = __longlong_as_double((long long)abits[D]);
    Recon R;
    R.eps = SCHEME == WENO5JS ? K->P.weno_eps : K->P.teno_eps;
    R.ct = K->P.teno_ct;
    R.rows = keep_rows;
    double q[6][4], F[6][4], p[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        cell_state2(K, Q, step, D == 0 ? i + s - 2 : i, D == 1 ? j + s - 2 : j, q[s]);
        const double ir = rcp_nr(q[s][0]);
        const double u = q[s][1] * ir, v = q[s][2] * ir;
        p[s] = K->P.gm1 * (q[s][3] - 0.5 * fma(q[s][1], u, q[s][2] * v));
        const double un = D == 0 ? u : v;
        F[s][0] = q[s][1 + D];
        F[s][1] = D == 0 ? fma(q[s][1], un, p[s]) : q[s][1] * un;
        F[s][2] = D == 1 ? fma(q[s][2], un, p[s]) : q[s][2] * un;
        F[s][3] = (q[s][3] + p[s]) * un;
    }
    double Fo[4];
    char_face<SCHEME, 2, D>(q, F, p, K->P.gm1, alpha, R, Fo);
    const long long nf = pfaces_of<D>(G), o = (long long)yi * (G.n[0] + (D == 0)) + xi;
#pragma unroll
    for (int c = 0; c < 4; ++c) Fh[c * nf + o] = Fo[c];
}

__global__ __launch_bounds__(BX * BY) void k_pstage2d(const KConst* __restrict__ K, StageArgs A,
                                                      const double* __restrict__ S, int visc,
                                                      const double* __restrict__ Fx, const double* __restrict__ Fy)
{
    const Grid& G = K->G;
    const int i = blockIdx.x * BX + (threadIdx.x & (BX - 1)), j = blockIdx.y * BY + threadIdx.x / BX;
    const bool inside = i < G.n[0] && j < G.n[1];
    const int terms = K->P.terms;
    unsigned long long am[2] = {0ull, 0ull};
    if (inside) {
        double L[4] = {0.0, 0.0, 0.0, 0.0};
        const double inv_h = G.inv_h;
        // -(F^_{i+1/2} - F^_{i-1/2}) / h per direction (a non-reflecting side's boundary cells
        // leave the normal term to launch_nrbc)
        const int nr = A.nrbc;
        const bool skx = ((nr & 1) && i == 0) || ((nr & 2) && i == G.n[0] - 1);
        const bool sky = ((nr & 4) && j == 0) || ((nr & 8) && j == G.n[1] - 1);
        if ((terms & T_CONVX) && !skx) {
            const long long nf = pfaces_of<0>(G), o = (long long)j * (G.n[0] + 1) + i;
#pragma unroll
            for (int c = 0; c < 4; ++c) L[c] += -(Fx[c * nf + o + 1] - Fx[c * nf + o]) * inv_h;
        }
        if ((terms & T_CONVY) && !sky) {
            const long long nf = pfaces_of<1>(G), o = (long long)j * G.n[0] + i;
#pragma unroll
            for (int c = 0; c < 4; ++c) L[c] += -(Fy[c * nf + o + G.n[0]] - Fy[c * nf + o]) * inv_h;
        }
        if (visc) {
            // momentum a: sum_b D_b(tau_ab); energy: sum_b D_b(b_b)
            const int ex = G.n[0] + 4, ey = G.n[1] + 4;
            const long long ne = (long long)ex * ey, oc = (long long)(j + 2) * ex + (i + 2);
            const long long st[2] = {1, ex};
            const double inv12h = K->inv12h;
            constexpr int tidx[2][2] = {{0, 2}, {2, 1}};
            double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int b = 0; b < 2; ++b) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int comp = a < 2 ? tidx[a][b] : 3 + b;
                    const double* P = S + comp * ne + oc;
                    acc[a] += d1(P[-2 * st[b]], P[-st[b]], P[st[b]], P[2 * st[b]], inv12h);
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) L[1 + a] += acc[a];
        }
        const long long o = (long long)j * G.n[0] + i;
        double qc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) qc[c] = A.Qs[c * G.ncell + o];
        double src[4] = {0.0, 0.0, 0.0, 0.0};
        if ((terms & T_IB) && A.fwin) {
            const int wi = i - A.wlo[0], wj = j - A.wlo[1];
            if (wi >= 0 && wi < A.wn[0] && wj >= 0 && wj < A.wn[1]) {
                const long long wc = (long long)wj * A.wn[0] + wi, wcells = (long long)A.wn[0] * A.wn[1];
                const double ir = rcp_nr(qc[0]);
                double fu = 0.0;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const double f = A.fwin[a * wcells + wc];
                    src[1 + a] = f;
                    fu = fma(f, qc[1 + a] * ir, fu);
                }
                src[3] = fu;
            }
        }
        if (terms & T_SPONGE) {
            const double eta = fmax(K->eta_dir(0, i), K->eta_dir(1, j));
            if (eta > 0.0) {
                const double sg = K->P.sigma * (eta * eta * eta);
#pragma unroll
                for (int c = 0; c < 4; ++c) src[c] = fma(-sg, qc[c] - K->P.q_inf[c], src[c]);
            }
        }
        double val[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double l = L[c] + src[c];
            if (A.mode_rhs) {
                val[c] = l;
            } else {
                const double stage = fma(A.dt, l, qc[c]);
                val[c] = (A.ca == 0.0) ? stage : fma(A.ca, A.Qn[c * G.ncell + o], A.cb * stage);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) A.out[c * G.ncell + o] = val[c];
        if (A.alpha_part && j >= A.arow0 && j < A.arow1) {
            const double ir = rcp_nr(val[0]);
            const double u = val[1] * ir, v = val[2] * ir;
            const double pn = K->P.gm1 * (val[3] - 0.5 * fma(val[1], u, val[2] * v));
            const double cn = sqrt(K->P.gamma * pn * ir);
            am[0] = (unsigned long long)__double_as_longlong(fabs(u) + cn);
            am[1] = (unsigned long long)__double_as_longlong(fabs(v) + cn);
        }
    }
    if (A.alpha_part) {
        // block maximum -> one partial per block (plain stores; reduced by launch_alpha_final)
        __shared__ unsigned long long red[BX * BY / 64][2];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            unsigned long long v = am[d];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v = max_bits(v, __shfl_xor(v, off, 64));
            if (lane == 0) red[wid][d] = v;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            unsigned long long v = 0ull;
            if (threadIdx.x < 2)
                for (int w = 0; w < BX * BY / 64; ++w) v = max_bits(v, red[w][threadIdx.x]);
            const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
            A.alpha_part[b * 3 + threadIdx.x] = v;
        }
    }
}

}  // namespace

long long pass2d_stress_elems(const Grid& G) { return 5ll * (G.n[0] + 4) * (G.n[1] + 4); }

long long pass2d_face_elems(const Grid& G) { return 4ll * (pfaces_of<0>(G) + pfaces_of<1>(G)); }

long long pass2d_blocks(const Grid& G) { return (long long)((G.n[0] + BX - 1) / BX) * ((G.n[1] + BY - 1) / BY); }

int launch_pass2d(const KConst* K, const Grid& G, int scheme, int terms, double mu, const StageArgs& A,
                  double* stress, double* faces, hipStream_t s)
{
    const dim3 block(BX * BY);
    const int visc = (terms & T_VISC) && mu != 0.0;
    if (visc) {
        const dim3 gs((G.n[0] + 4 + BX - 1) / BX, (G.n[1] + 4 + BY - 1) / BY);
        hipLaunchKernelGGL(k_pstress2d, gs, block, 0, s, K, A.Qs, A.step, stress);
    }
    double* Fx = faces;
    double* Fy = Fx + 4 * pfaces_of<0>(G);
    const dim3 gx((G.n[0] + 1 + BX - 1) / BX, (G.n[1] + BY - 1) / BY);
    const dim3 gy((G.n[0] + BX - 1) / BX, (G.n[1] + 1 + BY - 1) / BY);
    if (scheme == TENO5) {
        hipLaunchKernelGGL((k_pfaces2d<TENO5, 0>), gx, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx);
        hipLaunchKernelGGL((k_pfaces2d<TENO5, 1>), gy, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fy);
    } else {
        hipLaunchKernelGGL((k_pfaces2d<WENO5JS, 0>), gx, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx);
        hipLaunchKernelGGL((k_pfaces2d<WENO5JS, 1>), gy, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fy);
    }
    const dim3 gr((G.n[0] + BX - 1) / BX, (G.n[1] + BY - 1) / BY);
    hipLaunchKernelGGL(k_pstage2d, gr, block, 0, s, K, A, (const double*)stress, visc, (const double*)Fx,
                       (const double*)Fy);
    return (int)hipGetLastError();
}

}  // namespace fsa
