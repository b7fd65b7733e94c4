// Immersed-boundary kernels (Sec. 2, Eqs. (7)-(11)), probes and the global Lax-Friedrichs
// wave-speed reduction.
//
// The penalty step per stage is two small launches: one thread per marker gathers the fluid
// velocity m / rho over the 4^dim support with the tensor-product four-point weights, forms
// F_f = alpha xi + beta (U_ib - U) and advances the penalty integral with the stage's SSP-RK3
// combination; then one thread per cell of the window box (the bounding box of all supports)
// sums the spread force -F_k W_k dV_k / h^dim over that cell's markers in increasing marker
// index (a deterministic gather).  The weights depend only on the marker positions and are
// computed once per position update, by one launch that also puts the staged positions,
// velocities and window lists in place.
#include <algorithm>

#include "fsa_impl.hpp"

namespace fsa {

namespace {

constexpr int RED_THREADS = 256;

__device__ __forceinline__ unsigned long long wave_max_bits(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = max_bits(v, o);
    }
    return v;
}

// alpha_d = max over cells of |u_d| + c, NaN-propagating (bits of non-negative doubles).
template <int DIM>
__global__ __launch_bounds__(RED_THREADS) void k_alpha(Grid G, Phys P, const double* __restrict__ Q,
                                                       unsigned long long* __restrict__ part, long long c0,
                                                       long long c1)
{
    unsigned long long* __restrict__ out = part;
    __shared__ unsigned long long wpart[RED_THREADS / 64][DIM];
    unsigned long long m[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) m[d] = 0ull;
    const long long nc = G.ncell;
    for (long long n = c0 + (long long)blockIdx.x * blockDim.x + threadIdx.x; n < c1;
         n += (long long)gridDim.x * blockDim.x) {
        // the stage kernels' expressions for the wave speeds of their output, operation for
        // operation, so that a stage input's speeds do not depend on which kernel took them
        const double inv = rcp_nr(Q[n]);
        double u[DIM], mom[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            mom[d] = Q[(1 + d) * nc + n];
            u[d] = mom[d] * inv;
        }
        const double ke = DIM == 3 ? fma(mom[0], u[0], fma(mom[1], u[1], mom[DIM - 1] * u[DIM - 1]))
                                   : fma(mom[0], u[0], mom[DIM - 1] * u[DIM - 1]);
        const double p = P.gm1 * (Q[(DIM + 1) * nc + n] - 0.5 * ke);
        const double c = sqrt(P.gamma * p * inv);
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            m[d] = max_bits(m[d], (unsigned long long)__double_as_longlong(fabs(u[d]) + c));
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const unsigned long long w = wave_max_bits(m[d]);
        if (lane == 0) wpart[wid][d] = w;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0ull;
        if (threadIdx.x < DIM)
            for (int w = 0; w < RED_THREADS / 64; ++w) v = max_bits(v, wpart[w][threadIdx.x]);
        out[(long long)blockIdx.x * 3 + threadIdx.x] = v;
    }
}

// One block of NT threads: bits[d] = max over the n partials (the order is irrelevant for a
// maximum).  With ~4000 partials each thread issues its few loads at once.
template <int NT>
__device__ __forceinline__ void alpha_final_block(const unsigned long long* __restrict__ part, long long n,
                                                  unsigned long long* __restrict__ bits)
{
    __shared__ unsigned long long red[NT / 64][3];
    unsigned long long m[3] = {0ull, 0ull, 0ull};
    for (long long k = threadIdx.x; k < n; k += NT) {
#pragma unroll
        for (int d = 0; d < 3; ++d) m[d] = max_bits(m[d], part[k * 3 + d]);
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const unsigned long long w = wave_max_bits(m[d]);
        if (lane == 0) red[wid][d] = w;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0ull;
        for (int w = 0; w < NT / 64; ++w) v = max_bits(v, red[w][threadIdx.x]);
        bits[threadIdx.x] = v;
    }
}

constexpr int FINAL_THREADS = 1024;
__global__ __launch_bounds__(FINAL_THREADS) void k_alpha_final(const unsigned long long* __restrict__ part,
                                                               long long n, unsigned long long* __restrict__ bits)
{
    alpha_final_block<FINAL_THREADS>(part, n, bits);
}

// Many partials (a 3D stage leaves one per block): blocks reduce contiguous chunks and merge
// their maxima into the slot with an atomic maximum on the bit patterns (non-negative
// doubles order as their bits; the slot is cleared by k_bits_clear first).
__global__ __launch_bounds__(64) void k_bits_clear(unsigned long long* __restrict__ bits)
{
    if (threadIdx.x < 3) bits[threadIdx.x] = 0ull;
}

constexpr int CHUNK_THREADS = 256;
__global__ __launch_bounds__(CHUNK_THREADS) void k_alpha_chunks(const unsigned long long* __restrict__ part,
                                                                long long n, long long chunk,
                                                                unsigned long long* __restrict__ bits)
{
    const long long a = (long long)blockIdx.x * chunk, b = min(n, a + chunk);
    __shared__ unsigned long long red[CHUNK_THREADS / 64][3];
    unsigned long long m[3] = {0ull, 0ull, 0ull};
    for (long long k = a + threadIdx.x; k < b; k += CHUNK_THREADS) {
#pragma unroll
        for (int d = 0; d < 3; ++d) m[d] = max_bits(m[d], part[k * 3 + d]);
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const unsigned long long w = wave_max_bits(m[d]);
        if (lane == 0) red[wid][d] = w;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0ull;
        for (int w = 0; w < CHUNK_THREADS / 64; ++w) v = max_bits(v, red[w][threadIdx.x]);
        atomicMax(&bits[threadIdx.x], v);
    }
}

// Marker support: first cell and four weights per direction.
template <int DIM>
__device__ __forceinline__ void marker_support(const Grid& G, const double* X, int n, int k, int* j0,
                                               double (*w)[4])
{
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        support4(X[(long long)d * n + k], G.lo[d], G.h, j0[d], w[d]);   // (global cell index)
        j0[d] -= G.org[d];
    }
}

// Tensor-product weight of cell (ci, cj, ck) for point k.
template <int DIM>
__device__ __forceinline__ double cell_weight(const Grid& G, const double* X, int n, int k, int ci, int cj, int ck)
{
    double W = delta4(cell_coord(X[k], G.lo[0], G.h) - (double)(ci + G.org[0])) *
               delta4(cell_coord(X[(long long)n + k], G.lo[1], G.h) - (double)(cj + G.org[1]));
    if (DIM == 3) W = W * delta4(cell_coord(X[2ll * n + k], G.lo[2], G.h) - (double)(ck + G.org[2]));
    return W;
}

// 16-byte words from a host-visible block into device memory, each read once.
__global__ __launch_bounds__(256) void k_stage_in(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// A marker placement from the staged lists (one contiguous host-to-device copy): per marker
// X and U into place, the first support cell and the one-dimensional weights per direction;
// the window's CSR lists into place; per CSR entry (window cell, marker) the spreading weight
// W(cell) dV_k / h^dim.  One thread per item of the longest list, so every thread's loads are
// at most two levels deep (entry -> marker position).
template <int DIM>
__global__ void k_ib_place(Grid G, WindowUpdate W)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nm = W.nm;
    if (t < (long long)DIM * nm) {
        W.X[t] = W.sX[t];
        W.U[t] = W.sU[t];
    }
    if (t < nm) {
        const int k = (int)t;
        int j0[3];
        double w[3][4];
        marker_support<DIM>(G, W.sX, nm, k, j0, w);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            W.mj0[k * 3 + d] = j0[d];
#pragma unroll
            for (int m = 0; m < 4; ++m) W.mw[(k * DIM + d) * 4 + m] = w[d][m];
        }
    }
    if (t <= W.wcells) W.cell_start[t] = W.s_start[t];
    if (t < W.nent) {
        const int k = W.s_marker[t];
        W.cell_marker[t] = k;
        const long long c = W.s_cell[t];
        const int ci = W.wlo[0] + (int)(c % W.wn[0]);
        const int cj = W.wlo[1] + (int)((c / W.wn[0]) % W.wn[1]);
        const int ck = W.wlo[2] + (int)(c / ((long long)W.wn[0] * W.wn[1]));
        const double hd = DIM == 3 ? G.h * G.h * G.h : G.h * G.h;
        W.cell_w[t] = (cell_weight<DIM>(G, W.sX, nm, k, ci, cj, ck) * W.dV[k]) / hd;
    }
}

// Penalty force of marker k: U_ib = sum over the support of (m / rho) W, d = U_ib - U and
// F_f = alpha xi + beta d (xi the stage value).  Returns d in dv and F_f in Fk.
template <int DIM>
__device__ __forceinline__ void marker_force(const Grid& G, const IBArgs& A, int k, double* dv, double* Fk)
{
    const long long nc = G.ncell;
    int j0[3];
    double w[3][4];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        j0[d] = A.mj0[k * 3 + d];
#pragma unroll
        for (int m = 0; m < 4; ++m) w[d][m] = A.mw[(k * DIM + d) * 4 + m];
    }
    double uib[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) uib[a] = 0.0;
    // (3D: one z layer of 16 cells at a time, so its loads fit the registers)
#pragma nounroll
    for (int mz = 0; mz < (DIM == 3 ? 4 : 1); ++mz)
#pragma unroll
        for (int my = 0; my < 4; ++my)
#pragma unroll
            for (int mx = 0; mx < 4; ++mx) {
                double W = w[0][mx] * w[1][my];
                if (DIM == 3) W = W * w[2][mz];
                const long long lin =
                    ((long long)(DIM == 3 ? j0[2] + mz : 0) * G.n[1] + (j0[1] + my)) * G.n[0] + (j0[0] + mx);
                const double irho = rcp_nr(A.Qs[lin]);   // one refined reciprocal, not DIM divisions
#pragma unroll
                for (int a = 0; a < DIM; ++a) uib[a] = fma(A.Qs[(1 + a) * nc + lin] * irho, W, uib[a]);
            }
    double U[DIM];
    if (A.motion == 1) {
        const double x = A.X[k], y = A.X[(long long)A.nm + k];
        U[0] = -A.omega * y;
        U[1] = A.omega * x;
        if (DIM == 3) U[DIM - 1] = 0.0;
    } else {
#pragma unroll
        for (int a = 0; a < DIM; ++a) U[a] = A.U[(long long)a * A.nm + k];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        dv[a] = uib[a] - U[a];
        Fk[a] = fma(A.alpha, A.xi[(long long)a * A.nm + k], A.beta * dv[a]);
    }
}

// F_f of marker k, and the stage's update of its penalty integral into xi_out (stage 1 also
// keeps the step-start value in xi_n).
template <int DIM>
__device__ __forceinline__ void marker_update(const IBArgs& A, int k, const double* dv, const double* Fk)
{
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const long long o = (long long)a * A.nm + k;
        const double xs = A.xi[o];
        double xn = xs;
        if (A.stage == 1) A.xi_n[o] = xs;
        else if (A.stage > 1) xn = A.xi_n[o];
        A.F[o] = Fk[a];
        if (A.stage == 1) A.xi_out[o] = fma(A.dt, dv[a], xn);
        else if (A.stage > 1) A.xi_out[o] = fma(A.ca, xn, A.cb * fma(A.dt, dv[a], xs));
    }
}

// Penalty step per marker (xi_out may be xi: each thread reads its values before writing).
template <int DIM>
__global__ __launch_bounds__(64) void k_ib_markers(Grid G, IBArgs A)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= A.nm) return;
    double dv[DIM], Fk[DIM];
    marker_force<DIM>(G, A, k, dv, Fk);
    marker_update<DIM>(A, k, dv, Fk);
}

// Spread force density on the window box: one wave per window cell; lane l sums the cell's
// CSR entries l, l+64, ... in increasing marker index, then the wave adds the lane sums in a
// fixed butterfly order, so the result is the same on every run.  With A.alpha_part set, the
// last block instead reduces the wave-speed partials (one launch fewer per stage).
template <int DIM>
__global__ __launch_bounds__(256) void k_ib_window(IBArgs A)
{
    if (A.alpha_part && blockIdx.x == gridDim.x - 1) {
        alpha_final_block<256>(A.alpha_part, A.alpha_n, A.alpha_bits);
        return;
    }
    const long long wcells = (long long)A.wn[0] * A.wn[1] * A.wn[2];
    const long long c = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= wcells) return;
    double f[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) f[a] = 0.0;
    const int e1 = A.cell_start[c + 1];
    for (int e = A.cell_start[c] + lane; e < e1; e += 64) {
        const int k = A.cell_marker[e];
        const double we = A.cell_w[e];
#pragma unroll
        for (int a = 0; a < DIM; ++a) f[a] = fma(-A.F[(long long)a * A.nm + k], we, f[a]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < DIM; ++a) f[a] += __shfl_xor(f[a], off, 64);
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) A.fwin[a * wcells + c] = f[a];
    }
}

// Penalty step and spreading in one launch (2D, few markers): as k_ib_window, but each lane
// forms the force of the marker of its CSR entry itself (marker_force, the operations of
// k_ib_markers, so the same values) instead of reading it from a previous launch.  The entry
// at the marker's first support cell also writes F and the integral's update, into
// xi_out != xi (the marker's other entries read xi during the launch).
__global__ __launch_bounds__(256) void k_ib_fused2d(Grid G, IBArgs A)
{
    if (A.alpha_part && blockIdx.x == gridDim.x - 1) {
        alpha_final_block<256>(A.alpha_part, A.alpha_n, A.alpha_bits);
        return;
    }
    const long long wcells = (long long)A.wn[0] * A.wn[1];
    const long long c = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= wcells) return;
    const int ci = A.wlo[0] + (int)(c % A.wn[0]), cj = A.wlo[1] + (int)(c / A.wn[0]);
    double f[2] = {0.0, 0.0};
    const int e1 = A.cell_start[c + 1];
    for (int e = A.cell_start[c] + lane; e < e1; e += 64) {
        const int k = A.cell_marker[e];
        const double we = A.cell_w[e];
        double dv[2], Fk[2];
        marker_force<2>(G, A, k, dv, Fk);
        if (ci == A.mj0[k * 3] && cj == A.mj0[k * 3 + 1]) marker_update<2>(A, k, dv, Fk);
#pragma unroll
        for (int a = 0; a < 2; ++a) f[a] = fma(-Fk[a], we, f[a]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < 2; ++a) f[a] += __shfl_xor(f[a], off, 64);
    if (lane == 0) {
#pragma unroll
        for (int a = 0; a < 2; ++a) A.fwin[a * wcells + c] = f[a];
    }
}

// Interpolation of ncomp fields to points (one thread per point).
template <int DIM>
__global__ void k_interp(Grid G, int npts, const double* __restrict__ X, const double* __restrict__ field,
                         int ncomp, double* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npts) return;
    int j0[3];
    double w[3][4];
    marker_support<DIM>(G, X, npts, k, j0, w);
    for (int a = 0; a < ncomp; ++a) {
        double acc = 0.0;
        for (int mz = 0; mz < (DIM == 3 ? 4 : 1); ++mz)
            for (int my = 0; my < 4; ++my)
                for (int mx = 0; mx < 4; ++mx) {
                    double W = w[0][mx] * w[1][my];
                    if (DIM == 3) W = W * w[2][mz];
                    const long long lin =
                        ((long long)(DIM == 3 ? j0[2] + mz : 0) * G.n[1] + (j0[1] + my)) * G.n[0] + (j0[0] + mx);
                    acc = fma(field[(long long)a * G.ncell + lin], W, acc);
                }
        out[(long long)a * npts + k] = acc;
    }
}

// field[a] += scale * (-sum_k F_k W_k dV_k / h^dim) on the window cells (gather per cell).
template <int DIM>
__global__ void k_spread(Grid G, IBArgs A, const double* __restrict__ F, int ncomp, double* __restrict__ field,
                         double scale)
{
    const long long wcells = (long long)A.wn[0] * A.wn[1] * A.wn[2];
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= wcells) return;
    const int ci = A.wlo[0] + (int)(c % A.wn[0]);
    const int cj = A.wlo[1] + (int)((c / A.wn[0]) % A.wn[1]);
    const int ck = A.wlo[2] + (int)(c / ((long long)A.wn[0] * A.wn[1]));
    const long long lin = ((long long)(DIM == 3 ? ck : 0) * G.n[1] + cj) * G.n[0] + ci;
    for (int a = 0; a < ncomp; ++a) {
        double f = 0.0;
        for (int e = A.cell_start[c]; e < A.cell_start[c + 1]; ++e)
            f = fma(-F[(long long)a * A.nm + A.cell_marker[e]], A.cell_w[e], f);
        field[(long long)a * G.ncell + lin] += scale * f;
    }
}

// p - p_inf at probe points.
template <int DIM>
__global__ void k_probe_dp(Grid G, Phys P, int np, const double* __restrict__ Xp, const double* __restrict__ Q,
                           double* __restrict__ dp)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    int j0[3];
    double w[3][4];
    marker_support<DIM>(G, Xp, np, k, j0, w);
    const long long nc = G.ncell;
    double acc = 0.0;
    for (int mz = 0; mz < (DIM == 3 ? 4 : 1); ++mz)
        for (int my = 0; my < 4; ++my)
            for (int mx = 0; mx < 4; ++mx) {
                double W = w[0][mx] * w[1][my];
                if (DIM == 3) W = W * w[2][mz];
                const long long lin =
                    ((long long)(DIM == 3 ? j0[2] + mz : 0) * G.n[1] + (j0[1] + my)) * G.n[0] + (j0[0] + mx);
                const double rho = Q[lin];
                double ke = 0.0;
                for (int a = 0; a < DIM; ++a) {
                    const double m = Q[(1 + a) * nc + lin];
                    ke = fma(m, m / rho, ke);
                }
                const double p = P.gm1 * (Q[(DIM + 1) * nc + lin] - 0.5 * ke);
                acc = fma(p, W, acc);
            }
    dp[k] = acc - P.prim_inf[4];
}

// Field totals, deterministic: every block sums a fixed contiguous range of cells in a fixed
// order (thread-strided, then a fixed tree), and one block sums the block partials the same way.
constexpr int TOT_THREADS = 256;
constexpr int TOT_BLOCKS = 1024;

__device__ __forceinline__ double block_sum_fixed(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = TOT_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(TOT_THREADS) void k_totals(const double* __restrict__ Q, long long ncell, int nq,
                                                        double* __restrict__ part)
{
    __shared__ double sh[TOT_THREADS];
    const long long per = (ncell + gridDim.x - 1) / gridDim.x;
    const long long b0 = (long long)blockIdx.x * per, b1 = min(b0 + per, ncell);
    for (int m = 0; m < nq; ++m) {
        double s = 0.0;
        for (long long n = b0 + threadIdx.x; n < b1; n += TOT_THREADS) s += Q[(long long)m * ncell + n];
        const double t = block_sum_fixed(s, sh);
        if (threadIdx.x == 0) part[(long long)blockIdx.x * nq + m] = t;
    }
}

__global__ __launch_bounds__(TOT_THREADS) void k_totals_final(const double* __restrict__ part, int nblocks, int nq,
                                                              double hd, double* __restrict__ out)
{
    __shared__ double sh[TOT_THREADS];
    for (int m = 0; m < nq; ++m) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += TOT_THREADS) s += part[(long long)b * nq + m];
        const double t = block_sum_fixed(s, sh);
        if (threadIdx.x == 0) out[m] = t * hd;
    }
}

// div u at every cell: fourth-order central differences of u_d = m_d / rho along d.
template <int DIM>
__global__ __launch_bounds__(256) void k_dilatation(Grid G, Phys P, const double* __restrict__ Q, long long step,
                                                    double* __restrict__ out)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= G.ncell) return;
    const int i = (int)(n % G.n[0]);
    const int j = (int)((n / G.n[0]) % G.n[1]);
    const int k = DIM == 3 ? (int)(n / ((long long)G.n[0] * G.n[1])) : 0;
    const double inv12h = 1.0 / (12.0 * G.h);
    double div = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        double g[5];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            if (s == 2) {
                g[s] = 0.0;
                continue;
            }
            int ii = i, jj = j, kk = k;
            if (d == 0) ii += s - 2;
            else if (d == 1) jj += s - 2;
            else kk += s - 2;
            double q[DIM + 2];
            fetch_state<DIM>(Q, G, P, step, ii, jj, kk, q);
            g[s] = q[1 + d] / q[0];
        }
        div += (8.0 * (g[3] - g[1]) - (g[4] - g[0])) * inv12h;
    }
    out[n] = div;
}

}  // namespace

long long alpha_blocks(const Grid& G)
{
    long long blocks = (G.ncell + RED_THREADS - 1) / RED_THREADS;
    if (blocks > ALPHA_MAX_BLOCKS) blocks = ALPHA_MAX_BLOCKS;
    return blocks < 1 ? 1 : blocks;
}

int launch_alpha(const Grid& G, const Phys& P, const double* Q, unsigned long long* part, unsigned long long* bits,
                 hipStream_t s)
{
    return launch_alpha_rows(G, P, Q, 0, G.n[G.dim - 1], part, bits, s);
}

int launch_alpha_rows(const Grid& G, const Phys& P, const double* Q, int row0, int row1, unsigned long long* part,
                      unsigned long long* bits, hipStream_t s)
{
    const long long blocks = alpha_blocks(G);
    const long long plane = G.dim == 3 ? (long long)G.n[0] * G.n[1] : (long long)G.n[0];
    const long long c0 = plane * row0, c1 = plane * row1;
    if (G.dim == 3)
        hipLaunchKernelGGL(k_alpha<3>, dim3((unsigned)blocks), dim3(RED_THREADS), 0, s, G, P, Q, part, c0, c1);
    else
        hipLaunchKernelGGL(k_alpha<2>, dim3((unsigned)blocks), dim3(RED_THREADS), 0, s, G, P, Q, part, c0, c1);
    return launch_alpha_final(part, blocks, bits, s);
}

int launch_alpha_final(const unsigned long long* part, long long n, unsigned long long* bits, hipStream_t s)
{
    if (n <= 16384) {
        hipLaunchKernelGGL(k_alpha_final, dim3(1), dim3(FINAL_THREADS), 0, s, part, n, bits);
    } else {
        // ~2048 partials per block (one CU alone reads them at a fraction of the chip's rate)
        const long long nb = std::min<long long>(1024, (n + 2047) / 2048), chunk = (n + nb - 1) / nb;
        hipLaunchKernelGGL(k_bits_clear, dim3(1), dim3(64), 0, s, bits);
        hipLaunchKernelGGL(k_alpha_chunks, dim3((unsigned)nb), dim3(CHUNK_THREADS), 0, s, part, n, chunk, bits);
    }
    return (int)hipGetLastError();
}

int launch_ib_stage(const Grid& G, const Phys& P, const IBArgs& A, hipStream_t s)
{
    (void)P;
    if (A.nm <= 0) return 0;
    const unsigned mb = (unsigned)((A.nm + 63) / 64);
    const long long wcells = (long long)A.wn[0] * A.wn[1] * A.wn[2];
    const unsigned wb = (unsigned)((wcells + 3) / 4) + (A.alpha_part ? 1u : 0u);   // four cells per block
    if (ib_stage_fused(G, A.nm)) {
        if (A.stage > 0 && A.xi_out == A.xi) return (int)hipErrorInvalidValue;
        hipLaunchKernelGGL(k_ib_fused2d, dim3(wb), dim3(256), 0, s, G, A);
    } else if (G.dim == 3) {
        hipLaunchKernelGGL(k_ib_markers<3>, dim3(mb), dim3(64), 0, s, G, A);
        hipLaunchKernelGGL(k_ib_window<3>, dim3(wb), dim3(256), 0, s, A);
    } else {
        hipLaunchKernelGGL(k_ib_markers<2>, dim3(mb), dim3(64), 0, s, G, A);
        hipLaunchKernelGGL(k_ib_window<2>, dim3(wb), dim3(256), 0, s, A);
    }
    return (int)hipGetLastError();
}

bool ib_stage_fused(const Grid& G, int nm) { return G.dim == 2 && nm <= 4096; }

int launch_stage_in(const void* src, void* dst, long long n16, hipStream_t s)
{
    if (n16 <= 0) return 0;
    long long b = (n16 + 255) / 256;
    if (b > 256) b = 256;
    hipLaunchKernelGGL(k_stage_in, dim3((unsigned)b), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
    return (int)hipGetLastError();
}

int launch_ib_place(const Grid& G, const WindowUpdate& W, hipStream_t s)
{
    long long n = (long long)G.dim * W.nm;
    n = n > W.wcells + 1 ? n : W.wcells + 1;
    n = n > W.nent ? n : W.nent;
    if (W.nm <= 0) return 0;
    const unsigned b = (unsigned)((n + 127) / 128);
    if (G.dim == 3) hipLaunchKernelGGL(k_ib_place<3>, dim3(b), dim3(128), 0, s, G, W);
    else hipLaunchKernelGGL(k_ib_place<2>, dim3(b), dim3(128), 0, s, G, W);
    return (int)hipGetLastError();
}

int launch_interp(const Grid& G, int npts, const double* X, const double* field, int ncomp, double* out,
                  hipStream_t s)
{
    if (npts <= 0) return 0;
    const int blocks = (npts + 127) / 128;
    if (G.dim == 3) hipLaunchKernelGGL(k_interp<3>, dim3(blocks), dim3(128), 0, s, G, npts, X, field, ncomp, out);
    else hipLaunchKernelGGL(k_interp<2>, dim3(blocks), dim3(128), 0, s, G, npts, X, field, ncomp, out);
    return (int)hipGetLastError();
}

int launch_spread(const Grid& G, const IBArgs& A, const double* F, int ncomp, double* field, double scale,
                  hipStream_t s)
{
    const long long wcells = (long long)A.wn[0] * A.wn[1] * A.wn[2];
    if (wcells <= 0) return 0;
    const unsigned blocks = (unsigned)((wcells + 127) / 128);
    if (G.dim == 3) hipLaunchKernelGGL(k_spread<3>, dim3(blocks), dim3(128), 0, s, G, A, F, ncomp, field, scale);
    else hipLaunchKernelGGL(k_spread<2>, dim3(blocks), dim3(128), 0, s, G, A, F, ncomp, field, scale);
    return (int)hipGetLastError();
}

int launch_probe_dp(const Grid& G, const Phys& P, int np, const double* Xp, const double* Q, double* dp,
                    hipStream_t s)
{
    if (np <= 0) return 0;
    const int blocks = (np + 127) / 128;
    if (G.dim == 3) hipLaunchKernelGGL(k_probe_dp<3>, dim3(blocks), dim3(128), 0, s, G, P, np, Xp, Q, dp);
    else hipLaunchKernelGGL(k_probe_dp<2>, dim3(blocks), dim3(128), 0, s, G, P, np, Xp, Q, dp);
    return (int)hipGetLastError();
}

int totals_part_size(int nq) { return TOT_BLOCKS * nq; }

int launch_totals(const Grid& G, int nq, const double* Q, double* part, double* out, hipStream_t s)
{
    const double hd = G.dim == 3 ? G.h * G.h * G.h : G.h * G.h;
    hipLaunchKernelGGL(k_totals, dim3(TOT_BLOCKS), dim3(TOT_THREADS), 0, s, Q, G.ncell, nq, part);
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(TOT_THREADS), 0, s, part, TOT_BLOCKS, nq, hd, out);
    return (int)hipGetLastError();
}

int launch_dilatation(const Grid& G, const Phys& P, const double* Q, long long step, double* out, hipStream_t s)
{
    const unsigned blocks = (unsigned)((G.ncell + 255) / 256);
    if (G.dim == 3) hipLaunchKernelGGL(k_dilatation<3>, dim3(blocks), dim3(256), 0, s, G, P, Q, step, out);
    else hipLaunchKernelGGL(k_dilatation<2>, dim3(blocks), dim3(256), 0, s, G, P, Q, step, out);
    return (int)hipGetLastError();
}

}  // namespace fsa
