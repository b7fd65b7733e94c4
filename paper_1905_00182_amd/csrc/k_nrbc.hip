// Non-reflecting boundary of Thompson (1987, 1990), which Sec. 2 applies on the outer
// boundaries: at the boundary cell of a non-reflecting side the stage kernels leave out the
// convective term along the boundary normal, and this kernel adds its characteristic
// (locally one-dimensional) form, with the amplitudes of the waves that enter the domain set
// to zero, into the stage output (one thread per boundary cell; FP64 in every form).
#include "fsa_impl.hpp"

namespace fsa {

namespace {

template <int DIM>
__global__ __launch_bounds__(256) void k_nrbc(const KConst* __restrict__ K, StageArgs A, int d, int side)
{
    const Grid& G = K->G;
    const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;     // the tangential directions
    const long long n1 = G.n[a1], n2 = DIM == 3 ? G.n[a2] : 1;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n1 * n2) return;
    int idx[3] = {0, 0, 0};
    idx[a1] = (int)(t % n1);
    if (DIM == 3) idx[a2] = (int)(t / n1);
    const int b = side == 0 ? 0 : G.n[d] - 1, inward = side == 0 ? 1 : -1;
    // primitives of the boundary cell (s = 0) and the next two inward
    double rho[3], u[3][3], p[3];
    long long lin0 = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        int id[3] = {idx[0], idx[1], idx[2]};
        id[d] = b + inward * s;
        const long long lin = ((long long)id[2] * G.n[1] + id[1]) * G.n[0] + id[0];
        if (s == 0) lin0 = lin;
        const double r = A.Qs[lin];
        double ke = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double m = a < DIM ? A.Qs[(1 + a) * G.ncell + lin] : 0.0;
            u[s][a] = m / r;
            ke += m * u[s][a];
        }
        rho[s] = r;
        p[s] = K->P.gm1 * (A.Qs[(DIM + 1) * G.ncell + lin] - 0.5 * ke);
    }
    // derivative along +x_d from the boundary cell inward (exactly zero on constant data);
    // at the high side the inward cells lie toward -x_d, which flips the sign
    const double sg = side == 0 ? 1.0 : -1.0, inv2h = 0.5 * G.inv_h;
    auto dn = [&](double f0, double f1, double f2) { return sg * (4.0 * (f1 - f0) - (f2 - f0)) * inv2h; };
    const double drho = dn(rho[0], rho[1], rho[2]), dp = dn(p[0], p[1], p[2]);
    double du[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) du[a] = dn(u[0][a], u[1][a], u[2][a]);
    const double r = rho[0], un = u[0][d], cs = sqrt(K->P.gamma * p[0] / r);
    const double lam1 = un - cs, lam2 = un, lam5 = un + cs;
    // amplitudes of the waves; those entering the domain carry nothing
    const bool high = side == 1;
    const double L1 = (high ? lam1 < 0.0 : lam1 > 0.0) ? 0.0 : lam1 * (dp - r * cs * du[d]);
    const bool in2 = high ? lam2 < 0.0 : lam2 > 0.0;
    const double L2 = in2 ? 0.0 : lam2 * (cs * cs * drho - dp);
    const double L5 = (high ? lam5 < 0.0 : lam5 > 0.0) ? 0.0 : lam5 * (dp + r * cs * du[d]);
    const double d1 = (L2 + 0.5 * (L5 + L1)) / (cs * cs);
    const double d2 = 0.5 * (L5 + L1);
    const double dnn = (L5 - L1) / (2.0 * r * cs);
    double C[5];
    double ke = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) ke += u[0][a] * u[0][a];
    C[0] = -d1;
    double e = 0.5 * ke * d1 + d2 * K->P.inv_gm1 + r * un * dnn;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (a == d) {
            C[1 + a] = -(un * d1 + r * dnn);
        } else {
            const double La = in2 ? 0.0 : lam2 * du[a];
            C[1 + a] = -(u[0][a] * d1 + r * La);
            e += r * u[0][a] * La;
        }
    }
    C[DIM + 1] = -e;
    const double w = A.mode_rhs ? 1.0 : A.cb * A.dt;
#pragma unroll
    for (int c = 0; c < DIM + 2; ++c) A.out[c * G.ncell + lin0] += w * C[c];
}

}  // namespace

int launch_nrbc(const KConst* K, const Grid& G, int d, int side, const StageArgs& A, hipStream_t s)
{
    if (d < 0 || d >= G.dim || G.n[d] < 3) return (int)hipErrorInvalidValue;
    const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
    const long long cells = (long long)G.n[a1] * (G.dim == 3 ? G.n[a2] : 1);
    const unsigned blocks = (unsigned)((cells + 255) / 256);
    if (G.dim == 3) hipLaunchKernelGGL(k_nrbc<3>, dim3(blocks), dim3(256), 0, s, K, A, d, side);
    else hipLaunchKernelGGL(k_nrbc<2>, dim3(blocks), dim3(256), 0, s, K, A, d, side);
    return (int)hipGetLastError();
}

}  // namespace fsa
