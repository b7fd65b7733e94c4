// 3D right-hand side / SSP-RK3 stage for gfx950: stress, face and stage passes.
//
//  * k_stress3d: for every cell of the grid extended by two ghost layers, the velocity
//    gradients by the fourth-order central difference (Sec. 2, Eqs. (5)-(6)), the Stokes
//    stress tau and b = u . tau, stored as nine components [9][ext cells] (tau_xx, tau_yy,
//    tau_zz, tau_xy, tau_xz, tau_yz, b_x, b_y, b_z); a z march of 64 x 4 column tiles with
//    the velocities of each plane formed once into LDS.
//  * k_faces3d<D>: one thread per face along direction D: the six cells i-2..i+3 give the
//    split fluxes f+- = (F +- alpha Q)/2 of the five components (each block's cells' splits
//    formed once into LDS) and the face flux F^ = rec+(f+) + rec-(f-), stored per component
//    [5][faces] (each face once), with TENO5's wave-wide all-kept certificate (recon5w); in
//    the characteristic-wise instantiation (FP64) the split fluxes are projected on the
//    eigenvectors at the Roe average of the face's two cells, reconstructed field by field
//    and recombined (char_face).  k_xedge3d takes the x faces at x = n_x when n_x is a
//    multiple of 64.
//  * k_stage3d: per interior cell, the flux differences of the three face buffers, the
//    viscous divergence from the stress buffer, the penalty-IB source from the window
//    array, the sponge, the RK3 combination, and one wave-speed partial per block.
//
// Threads of a block are 64 (32 for y and z faces) consecutive x cells by 4 (8) rows, so
// every load along x is coalesced; neighbours along y and z come through the caches.  Arithmetic type T as in 2D:
// double (the method) or float (the precision form, on deviations from the far field).
#include <type_traits>

#include "fsa_impl.hpp"

namespace fsa {

namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ long long lin3(const Grid& G, int i, int j, int k)
{
    return ((long long)k * G.n[1] + j) * G.n[0] + i;
}

// Store into a buffer the next pass reads: FP64 values with a nontemporal store (the
// buffers far exceed the caches; measured faster for FP64, slower for the FP32 form).
template <class T>
__device__ __forceinline__ void store_buffer(T v, T* p)
{
    if constexpr (std::is_same<T, double>::value) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// State of cell (i, j, k), ghosts resolved by the boundary conditions.
__device__ __forceinline__ void cell_state(const KConst* K, const double* __restrict__ Q, long long step, int i, int j,
                                           int k, double* q)
{
    const Grid& G = K->G;
    if (i >= 0 && i < G.n[0] && j >= 0 && j < G.n[1] && k >= 0 && k < G.n[2]) {
        const long long o = lin3(G, i, j, k);
#pragma unroll
        for (int c = 0; c < 5; ++c) q[c] = Q[c * G.ncell + o];
    } else {
        fetch_state<3>(Q, G, K->P, step, i, j, k, q);
    }
}

template <class T>
__device__ __forceinline__ T d1(T gm2, T gm1, T gp1, T gp2, T inv12h)
{
    return (T(8) * (gp1 - gm1) - (gp2 - gm2)) * inv12h;
}

// ---------------------------------------------------------------------------------------
// Stress pass
// ---------------------------------------------------------------------------------------
// The stress pass marches a 64 x 4 column tile of the extended grid up z over a segment of
// SZ planes.  Each step stages the velocities of one front plane of the tile and its two-cell
// x and y halo (every cell's velocity once, instead of once per neighbour that needs it) in
// LDS, takes this thread's x and y derivatives of that plane there at once and keeps them,
// with its column's velocities of five planes for the z derivatives, in registers until the
// plane two above arrives; it then writes the stress of the plane two below.  The state of
// the next front plane is loaded before the current plane's arithmetic, so the loads are in
// flight while it runs.  Two LDS slots and one barrier per step: a slot is rewritten one step
// after its last read, and every thread has passed that step's barrier by then.
// The grid is one-dimensional, stress_tiles() blocks per z segment (its tiles rounded up to a
// multiple of 8), and within a segment XCD x takes the x-th eighth of the tiles in row order:
// a band of tile rows, so that a tile and its x and y neighbours, whose state planes overlap
// in the halo, are read by one XCD's L2 close together.
constexpr int SZ = 32, TXS = BX + 4, TYS = BY + 4;
constexpr int SCELLS = TXS * TYS;                        // staged cells per plane
constexpr int SPER = (SCELLS + BX * BY - 1) / (BX * BY);  // per thread

__host__ __device__ __forceinline__ int stress_tiles(const Grid& G)
{
    return (((G.n[0] + 4 + BX - 1) / BX) * ((G.n[1] + 4 + BY - 1) / BY) + 7) & ~7;
}

template <class T>
__global__ __launch_bounds__(BX * BY) void k_stress3d(const KConst* __restrict__ K, const double* __restrict__ Q,
                                                      long long step, T* __restrict__ S)
{
    constexpr bool F64 = std::is_same<T, double>::value;
    __shared__ T ring[2][3][TYS][TXS];
    const Grid& G = K->G;
    const int ex = G.n[0] + 4, ey = G.n[1] + 4, ez = G.n[2] + 4;
    const int gx = (ex + BX - 1) / BX, per = stress_tiles(G);
    const int seg = blockIdx.x / per, wg = blockIdx.x - seg * per;
    const int r = (wg % 8) * (per / 8) + wg / 8;          // (workgroups go round-robin to the XCDs)
    if (r >= gx * ((ey + BY - 1) / BY)) return;         // (padding: the whole block, before any barrier)
    const int bx = r % gx, by = r / gx;
    const int tx = threadIdx.x & (BX - 1), ty = threadIdx.x / BX;
    const int xi = bx * BX + tx, yi = by * BY + ty;
    const bool out = xi < ex && yi < ey;
    const int za = seg * SZ, zb = min(za + SZ, ez) - 1;   // extended output planes
    const int ka = za - 2, kb = zb - 2;                           // their cell indices
    const T inv12h = (T)K->inv12h, mu = (T)K->P.mu;
    const long long ne = (long long)ex * ey * ez;
    // this thread's staged cells (cell c = threadIdx.x + m * 256 of the tile with its halo)
    // and their state for the next front plane (interior cells; ghosts are resolved when used)
    int ci[SPER], cj[SPER];
    bool cin[SPER];
    double pq[SPER][5];
#pragma unroll
    for (int m = 0; m < SPER; ++m) {
        const int c = threadIdx.x + m * BX * BY;
        const int ly = c / TXS, lx = c - ly * TXS;
        ci[m] = bx * BX + lx - 4;
        cj[m] = by * BY + ly - 4;
        cin[m] = c < SCELLS && ci[m] >= 0 && ci[m] < G.n[0] && cj[m] >= 0 && cj[m] < G.n[1];
    }
    auto prefetch = [&](int kf) {
        const bool kin = kf >= 0 && kf < G.n[2];
#pragma unroll
        for (int m = 0; m < SPER; ++m) {
            if (cin[m] && kin) {
                const long long o = lin3(G, ci[m], cj[m], kf);
#pragma unroll
                for (int c = 0; c < 5; ++c) pq[m][c] = Q[c * G.ncell + o];
            }
        }
    };
    T w[5][3];    // this column's velocities at planes k-2 .. k+2
    T gd[3][6];   // its x and y derivatives d u_a / d x, d u_a / d y at planes k .. k+2
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
        for (int a = 0; a < 3; ++a) w[m][a] = T(0);
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int a = 0; a < 6; ++a) gd[m][a] = T(0);
    prefetch(ka - 2);
    for (int kf = ka - 2; kf <= kb + 2; ++kf) {
        // front plane kf of the tile with its halo, from the state loaded one step ago
        T (*pl)[TYS][TXS] = ring[kf & 1];
        const bool kin = kf >= 0 && kf < G.n[2];
#pragma unroll
        for (int m = 0; m < SPER; ++m) {
            const int c = threadIdx.x + m * BX * BY;
            if (c < SCELLS) {
                double q[5];
                if (cin[m] && kin) {
#pragma unroll
                    for (int a = 0; a < 5; ++a) q[a] = pq[m][a];
                } else {
                    fetch_state<3>(Q, G, K->P, step, ci[m], cj[m], kf, q);
                }
                const double ir = rcp_nr(q[0]);
                const int ly = c / TXS, lx = c - ly * TXS;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double v = q[1 + a] * ir;
                    pl[a][ly][lx] = F64 ? (T)v : (T)(v - K->P.prim_inf[1 + a]);
                }
            }
        }
        if (kf < kb + 2) prefetch(kf + 1);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int a = 0; a < 3; ++a) w[m][a] = w[m + 1][a];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int a = 0; a < 6; ++a) gd[m][a] = gd[m + 1][a];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            w[4][a] = pl[a][ty + 2][tx + 2];
            gd[2][2 * a] = d1(pl[a][ty + 2][tx], pl[a][ty + 2][tx + 1], pl[a][ty + 2][tx + 3], pl[a][ty + 2][tx + 4], inv12h);
            gd[2][2 * a + 1] =
                d1(pl[a][ty][tx + 2], pl[a][ty + 1][tx + 2], pl[a][ty + 3][tx + 2], pl[a][ty + 4][tx + 2], inv12h);
        }
        const int k = kf - 2;
        if (k < ka || !out) continue;
        // plane k: x and y derivatives taken when it was staged, z derivatives from the column
        T g[3][3];   // g[a][b] = d u_a / d x_b
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            g[a][0] = gd[0][2 * a];
            g[a][1] = gd[0][2 * a + 1];
            g[a][2] = d1(w[0][a], w[1][a], w[3][a], w[4][a], inv12h);
        }
        const T div = g[0][0] + g[1][1] + g[2][2];
        const T sxx = mu * fma(T(-2.0 / 3.0), div, g[0][0] + g[0][0]);
        const T syy = mu * fma(T(-2.0 / 3.0), div, g[1][1] + g[1][1]);
        const T szz = mu * fma(T(-2.0 / 3.0), div, g[2][2] + g[2][2]);
        const T sxy = mu * (g[0][1] + g[1][0]);
        const T sxz = mu * (g[0][2] + g[2][0]);
        const T syz = mu * (g[1][2] + g[2][1]);
        T uf[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) uf[a] = F64 ? w[2][a] : w[2][a] + (T)K->P.prim_inf[1 + a];
        const long long o = ((long long)(k + 2) * ey + yi) * ex + xi;
        store_buffer(sxx, &S[0 * ne + o]);
        store_buffer(syy, &S[1 * ne + o]);
        store_buffer(szz, &S[2 * ne + o]);
        store_buffer(sxy, &S[3 * ne + o]);
        store_buffer(sxz, &S[4 * ne + o]);
        store_buffer(syz, &S[5 * ne + o]);
        store_buffer(fma(uf[0], sxx, fma(uf[1], sxy, uf[2] * sxz)), &S[6 * ne + o]);
        store_buffer(fma(uf[0], sxy, fma(uf[1], syy, uf[2] * syz)), &S[7 * ne + o]);
        store_buffer(fma(uf[0], sxz, fma(uf[1], syz, uf[2] * szz)), &S[8 * ne + o]);
    }
}

// ---------------------------------------------------------------------------------------
// Stage pass
// ---------------------------------------------------------------------------------------
// (the wave-wide all-kept shortcut: callers are converged waves)
template <int SCHEME>
__device__ __forceinline__ double rec(double a, double b, double c, double d, double e, const Recon& R, const Recon32&,
                                      double tall)
{
    return recon5w<SCHEME>(a, b, c, d, e, R, tall);
}
template <int SCHEME>
__device__ __forceinline__ float rec(float a, float b, float c, float d, float e, const Recon&, const Recon32& R,
                                     double tall)
{
    return recon5fw<SCHEME>(a, b, c, d, e, R, (float)tall);
}

// Face index of face f (between cells f-1 and f along D) of the line through (i, j, k):
// x faces [nz][ny][nx+1], y faces [nz][ny+1][nx], z faces [nz+1][ny][nx].
template <int D>
__device__ __forceinline__ long long face_index(const Grid& G, int f, int i, int j, int k)
{
    if (D == 0) return ((long long)k * G.n[1] + j) * (G.n[0] + 1) + f;
    if (D == 1) return ((long long)k * (G.n[1] + 1) + f) * G.n[0] + i;
    return ((long long)f * G.n[1] + j) * G.n[0] + i;
}

template <int D>
__host__ __device__ __forceinline__ long long faces_of(const Grid& G)
{
    return (long long)(G.n[0] + (D == 0)) * (G.n[1] + (D == 1)) * (G.n[2] + (D == 2));
}

// A block's 256 faces along D: FX along x by FA along a second axis (y for D = 0 and 1, z for
// D = 2, the block then taking one y row) -- 64 x 4 for x faces, 32 x 8 for y and z faces,
// whose tiles then stage 1.75 cells per face instead of 2.5; the cells those faces read form a
// tile of TX x TA cells (3 more on either side along D), staged in LDS once per block instead
// of once per face that reads them (six), in the same expressions.
template <int D>
struct FaceTile {
    static constexpr int FX = D == 0 ? BX : 32;        // faces along x
    static constexpr int FA = BX * BY / FX;            // faces along the second axis
    static constexpr int TX = FX + (D == 0 ? 6 : 0);   // cells along x
    static constexpr int TA = D == 0 ? FA : FA + 6;    // cells along the second axis
};

// Pressure and velocity along D of a staged cell, in the expressions every face pass uses.
template <int D>
__device__ __forceinline__ void cell_prims(const KConst* K, const double* qc, double& p, double& ud)
{
    const double ir = rcp_nr(qc[0]);
    const double u = qc[1] * ir, v = qc[2] * ir, w = qc[3] * ir;
    p = K->P.gm1 * (qc[4] - 0.5 * fma(qc[1], u, fma(qc[2], v, qc[3] * w)));
    ud = D == 0 ? u : (D == 1 ? v : w);
}

// Split fluxes f+- = (F +- alpha Q) / 2 along D of one cell, each rounded once to T (FP64: of
// the state; the precision form: of its deviation from the far field, formed in FP64).
template <class T, int D>
__device__ __forceinline__ void cell_split(const KConst* K, const double* q, double p, double ud, double alpha, T* fp,
                                           T* fm)
{
    constexpr bool F64 = std::is_same<T, double>::value;
    const double* Finf = D == 0 ? K->Fx_inf : (D == 1 ? K->Fy_inf : K->Fz_inf);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        double F;
        if (c == 0) F = q[1 + D];
        else if (c == 4) F = (q[4] + p) * ud;
        else if (c - 1 == D) F = fma(q[c], ud, p);
        else F = q[c] * ud;
        if (F64) {
            fp[c] = (T)(0.5 * fma(alpha, q[c], F));
            fm[c] = (T)(0.5 * fma(-alpha, q[c], F));
        } else {
            const double dq = q[c] - K->P.q_inf[c], dF = F - Finf[c];
            fp[c] = (T)(0.5 * fma(alpha, dq, dF));
            fm[c] = (T)(0.5 * fma(-alpha, dq, dF));
        }
    }
}

template <int SCHEME, class T>
__device__ __forceinline__ void recon_setup(const KConst* K, const KeepRows<T>& keep_rows, Recon& R, Recon32& R32)
{
    R.eps = SCHEME == WENO5JS ? K->P.weno_eps : K->P.teno_eps;
    R.ct = K->P.teno_ct;
    R32.eps = SCHEME == WENO5JS ? (float)K->P.weno_eps : 1e-30f;
    R32.ct = (float)K->P.teno_ct;
    if constexpr (std::is_same<T, double>::value) {
        R.rows = keep_rows;
        R32.rows = nullptr;
    } else {
        R.rows = nullptr;
        R32.rows = keep_rows;
    }
}

// Face flux of component c from the split fluxes of the face's six cells i-2..i+3 (i below it
// along D): F^ = rec+(f+ of i-2..i+2) + rec-(f- of i+3..i-1); with DBG (FP64 TENO5) also the
// keep patterns of both sides into *word.
template <int SCHEME, class T, bool DBG>
__device__ __forceinline__ T face_comp(const T (&fp)[6], const T (&fm)[6], const Recon& R, const Recon32& R32,
                                       double tall, int c, unsigned* word)
{
    if constexpr (DBG) {
        *word |= (unsigned)teno_keep5(fp[0], fp[1], fp[2], fp[3], fp[4], R) << (3 * c);
        *word |= (unsigned)teno_keep5(fm[5], fm[4], fm[3], fm[2], fm[1], R) << (16 + 3 * c);
    } else {
        (void)c;
        (void)word;
    }
    return rec<SCHEME>(fp[0], fp[1], fp[2], fp[3], fp[4], R, R32, tall) +
           rec<SCHEME>(fm[5], fm[4], fm[3], fm[2], fm[1], R, R32, tall);
}

// Characteristic-wise face flux (FP64) from the face's six cells: state q, pressure p and
// velocity ud; written per component to Fh[c * nf + o].
template <int SCHEME, int D>
__device__ __forceinline__ void char_face_emit(const KConst* K, double alpha, const Recon& R, const double (&q)[6][5],
                                               const double (&p)[6], const double (&ud)[6], double* __restrict__ Fh,
                                               long long nf, long long o)
{
    double Fs[6][5];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        Fs[s][0] = q[s][1 + D];
#pragma unroll
        for (int a = 0; a < 3; ++a) Fs[s][1 + a] = a == D ? fma(q[s][1 + a], ud[s], p[s]) : q[s][1 + a] * ud[s];
        Fs[s][4] = (q[s][4] + p[s]) * ud[s];
    }
    double Fo[5];
    char_face<SCHEME, 3, D>(q, Fs, p, K->P.gm1, alpha, R, Fo);
#pragma unroll
    for (int c = 0; c < 5; ++c) store_buffer(Fo[c], &Fh[c * nf + o]);
}

// Face fluxes along D: threads cover the faces f = 0..n_D along D (x index for D = 0, y index
// for D = 1, z index for D = 2) and the cells of the two other directions; along x only the
// faces below 64 * ceil(n_x / 64), the last face of a grid whose n_x is a multiple of 64
// being left to k_xedge3d (a block column for one face would idle 63 of its 64 lanes).
// Component-wise, each staged cell's split fluxes along D are formed once into LDS (instead
// of once per face that reads them, six); characteristic-wise its state, pressure and
// velocity are staged.  DBG (FP64 TENO5 only) also writes each face's keep patterns to dbg,
// in the face layout.  CH (FP64 only): characteristic-wise reconstruction.
template <int SCHEME, class T, int D, bool DBG = false, bool CH = false>
__global__ __launch_bounds__(BX * BY) void k_faces3d(const KConst* __restrict__ K, const double* __restrict__ Q,
                                                     long long step, const unsigned long long* __restrict__ abits,
                                                     T* __restrict__ Fh, unsigned* __restrict__ dbg)
{
    constexpr int TX = FaceTile<D>::TX, TA = FaceTile<D>::TA, FX = FaceTile<D>::FX, FA = FaceTile<D>::FA;
    const Grid& G = K->G;
    __shared__ __attribute__((aligned(16))) KeepRows<T> keep_rows;
    if (SCHEME != WENO5JS) init_keep_rows<T>(keep_rows, threadIdx.x);
    const double alpha = __longlong_as_double((long long)abits[D]);
    // x faces: XCD bands as in the stage pass (within a plane, XCD x takes the tile rows of
    // band x), so the rows of neighbouring tiles are read by one XCD close together
    int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    if (D == 0 && gridDim.y % 8 == 0) {
        const int r = blockIdx.y * gridDim.x + blockIdx.x;
        const int xcd = r % 8, slot = r / 8;
        bx = slot % gridDim.x;
        by = xcd * (gridDim.y / 8) + slot / gridDim.x;
    }
    // characteristic-wise z faces: XCD x takes the y rows of band x, and within a row and x
    // tile the z tiles one after another, so that the six planes two consecutive z tiles both
    // stage are read by one XCD close together (the component-wise passes, which wait on
    // memory more than they compute, run faster in launch order, neighbouring rows of the same
    // planes together)
    if (CH && D == 2 && gridDim.y % 8 == 0) {
        const int r = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        const int xcd = r % 8, slot = r / 8;
        bz = slot % gridDim.z;
        const int t = slot / gridDim.z;
        bx = t % gridDim.x;
        by = xcd * (gridDim.y / 8) + t / gridDim.x;
    }
    const int x0 = bx * FX - (D == 0 ? 3 : 0);
    const int fx = threadIdx.x % FX, fa = threadIdx.x / FX;
    const int xi = bx * FX + fx;
    const int yi = D == 2 ? by : by * FA + fa;
    const int zi = D == 2 ? bz * FA + fa : bz;
    const bool face_in = xi < G.n[0] + (D == 0) && yi < G.n[1] + (D == 1) && zi < G.n[2] + (D == 2);
    const int f = D == 0 ? xi : (D == 1 ? yi : zi);
    const long long nf = faces_of<D>(G);
    const long long o = face_index<D>(G, f, D == 0 ? 0 : xi, D == 1 ? 0 : yi, D == 2 ? 0 : zi);
    Recon R;
    Recon32 R32;
    recon_setup<SCHEME, T>(K, keep_rows, R, R32);
    if constexpr (CH) {
        static_assert(std::is_same<T, double>::value && !DBG, "characteristic-wise faces are FP64");
        __shared__ double tq[5][TA][TX];
        __shared__ double tp[TA][TX], tu[TA][TX];
        for (int c = threadIdx.x; c < TA * TX; c += BX * BY) {
            const int ca = c / TX, cx = c - ca * TX;
            const int cj = D == 2 ? by : by * FA + ca - (D == 1 ? 3 : 0);
            const int ck = D == 2 ? bz * FA + ca - 3 : bz;
            double qc[5];
            cell_state(K, Q, step, x0 + cx, cj, ck, qc);   // (ghosts resolved by the boundary rules)
#pragma unroll
            for (int m = 0; m < 5; ++m) tq[m][ca][cx] = qc[m];
            cell_prims<D>(K, qc, tp[ca][cx], tu[ca][cx]);
        }
        __syncthreads();
        if (!face_in) return;
        double q[6][5], ud[6], p[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const int cx = D == 0 ? fx + s : fx, ca = D == 0 ? fa : fa + s;
#pragma unroll
            for (int m = 0; m < 5; ++m) q[s][m] = tq[m][ca][cx];
            p[s] = tp[ca][cx];
            ud[s] = tu[ca][cx];
        }
        char_face_emit<SCHEME, D>(K, alpha, R, q, p, ud, Fh, nf, o);
    } else {
        __shared__ T sp[5][TA][TX], sm[5][TA][TX];
        for (int c = threadIdx.x; c < TA * TX; c += BX * BY) {
            const int ca = c / TX, cx = c - ca * TX;
            const int cj = D == 2 ? by : by * FA + ca - (D == 1 ? 3 : 0);
            const int ck = D == 2 ? bz * FA + ca - 3 : bz;
            double qc[5], p, ud;
            T fpc[5], fmc[5];
            cell_state(K, Q, step, x0 + cx, cj, ck, qc);   // (ghosts resolved by the boundary rules)
            cell_prims<D>(K, qc, p, ud);
            cell_split<T, D>(K, qc, p, ud, alpha, fpc, fmc);
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                sp[m][ca][cx] = fpc[m];
                sm[m][ca][cx] = fmc[m];
            }
        }
        __syncthreads();
        if (!face_in) return;
        unsigned word = 0u;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            T fp[6], fm[6];
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const int cx = D == 0 ? fx + s : fx, ca = D == 0 ? fa : fa + s;
                fp[s] = sp[c][ca][cx];
                fm[s] = sm[c][ca][cx];
            }
            store_buffer(face_comp<SCHEME, T, DBG>(fp, fm, R, R32, K->teno_tall, c, &word), &Fh[c * nf + o]);
        }
        if constexpr (DBG) dbg[o] = word;
    }
}

// The x faces f = n_x of a grid whose n_x is a multiple of 64: one thread per (j, k), its six
// cells n_x-3 .. n_x+2 loaded directly (the last three are ghosts), the same primitives,
// split fluxes and face arithmetic as k_faces3d.
template <int SCHEME, class T, bool DBG = false, bool CH = false>
__global__ __launch_bounds__(BX * BY) void k_xedge3d(const KConst* __restrict__ K, const double* __restrict__ Q,
                                                     long long step, const unsigned long long* __restrict__ abits,
                                                     T* __restrict__ Fh, unsigned* __restrict__ dbg)
{
    const Grid& G = K->G;
    __shared__ __attribute__((aligned(16))) KeepRows<T> keep_rows;
    if (SCHEME != WENO5JS) init_keep_rows<T>(keep_rows, threadIdx.x);
    __syncthreads();
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)G.n[1] * G.n[2]) return;
    const int j = (int)(t % G.n[1]), k = (int)(t / G.n[1]);
    const int f = G.n[0];
    const double alpha = __longlong_as_double((long long)abits[0]);
    const long long nf = faces_of<0>(G), o = face_index<0>(G, f, 0, j, k);
    Recon R;
    Recon32 R32;
    recon_setup<SCHEME, T>(K, keep_rows, R, R32);
    double q[6][5], ud[6], p[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        cell_state(K, Q, step, f - 3 + s, j, k, q[s]);
        cell_prims<0>(K, q[s], p[s], ud[s]);
    }
    if constexpr (CH) {
        static_assert(std::is_same<T, double>::value && !DBG, "characteristic-wise faces are FP64");
        char_face_emit<SCHEME, 0>(K, alpha, R, q, p, ud, Fh, nf, o);
    } else {
        T sp[6][5], sm[6][5];
#pragma unroll
        for (int s = 0; s < 6; ++s) cell_split<T, 0>(K, q[s], p[s], ud[s], alpha, sp[s], sm[s]);
        unsigned word = 0u;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            T fp[6], fm[6];
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                fp[s] = sp[s][c];
                fm[s] = sm[s][c];
            }
            store_buffer(face_comp<SCHEME, T, DBG>(fp, fm, R, R32, K->teno_tall, c, &word), &Fh[c * nf + o]);
        }
        if constexpr (DBG) dbg[o] = word;
    }
}

template <class T>
__global__ __launch_bounds__(BX * BY) void k_stage3d(const KConst* __restrict__ K, StageArgs A, const T* __restrict__ S,
                                                     const T* __restrict__ Fx, const T* __restrict__ Fy,
                                                     const T* __restrict__ Fz)
{
    const Grid& G = K->G;
    // XCD bands: workgroups go round-robin to the 8 XCDs; within a plane, XCD x takes the
    // tile rows of band x (an eighth of the plane's rows, every x tile), so that the rows a
    // tile reads above and below it, and the planes above and below, are read by the same
    // XCD within a short time (its L2 holds a band over five planes).  Any bijection of the
    // blocks is correct; this one only serves locality.
    int bx = blockIdx.x, by = blockIdx.y;
    if (gridDim.y % 8 == 0) {
        const int r = blockIdx.y * gridDim.x + blockIdx.x;   // (blockIdx.z is the plane)
        const int xcd = r % 8, slot = r / 8, bw = gridDim.y / 8;
        bx = slot % gridDim.x;
        by = xcd * bw + slot / gridDim.x;
    }
    const int i = bx * BX + (threadIdx.x & (BX - 1));
    const int j = by * BY + (threadIdx.x / BX);
    const int k = blockIdx.z;
    const bool inside = i < G.n[0] && j < G.n[1];
    const int terms = K->P.terms;
    unsigned long long am[3] = {0ull, 0ull, 0ull};
    if (inside) {
        double L[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        const T inv_h = (T)G.inv_h;
        // -(F^_{i+1/2} - F^_{i-1/2}) / h per direction, each face read from its buffer
        // (a non-reflecting side's boundary cells leave the normal term to launch_nrbc)
        const int nr = A.nrbc;
        const bool skx = ((nr & 1) && i == 0) || ((nr & 2) && i == G.n[0] - 1);
        const bool sky = ((nr & 4) && j == 0) || ((nr & 8) && j == G.n[1] - 1);
        const bool skz = ((nr & 16) && k == 0) || ((nr & 32) && k == G.n[2] - 1);
        if ((terms & T_CONVX) && !skx) {
            const long long nf = faces_of<0>(G), o = face_index<0>(G, i, 0, j, k);
#pragma unroll
            for (int c = 0; c < 5; ++c) L[c] += (double)(-(Fx[c * nf + o + 1] - Fx[c * nf + o]) * inv_h);
        }
        if ((terms & T_CONVY) && !sky) {
            const long long nf = faces_of<1>(G), o = face_index<1>(G, j, i, 0, k), st = G.n[0];
#pragma unroll
            for (int c = 0; c < 5; ++c) L[c] += (double)(-(Fy[c * nf + o + st] - Fy[c * nf + o]) * inv_h);
        }
        if ((terms & T_CONVZ) && !skz) {
            const long long nf = faces_of<2>(G), o = face_index<2>(G, k, i, j, 0);
            const long long st = (long long)G.n[0] * G.n[1];
#pragma unroll
            for (int c = 0; c < 5; ++c) L[c] += (double)(-(Fz[c * nf + o + st] - Fz[c * nf + o]) * inv_h);
        }
        if (terms & T_VISC) {
            // momentum a: sum_b D_b(tau_ab); energy: sum_b D_b(b_b)
            const int ex = G.n[0] + 4, ey = G.n[1] + 4, ez = G.n[2] + 4;
            const long long ne = (long long)ex * ey * ez;
            const long long oc = ((long long)(k + 2) * ey + (j + 2)) * ex + (i + 2);
            const long long st[3] = {1, ex, (long long)ex * ey};
            const T inv12h = (T)K->inv12h;
            // stress component index of tau_ab
            constexpr int tidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
            T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int comp = a < 3 ? tidx[a][b] : 6 + b;
                    const T* P = S + comp * ne + oc;
                    acc[a] += d1(P[-2 * st[b]], P[-st[b]], P[st[b]], P[2 * st[b]], inv12h);
                }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) L[1 + a] += (double)acc[a];
        }
        const long long o = lin3(G, i, j, k);
        double qc[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) qc[c] = __builtin_nontemporal_load(&A.Qs[c * G.ncell + o]);
        double src[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if ((terms & T_IB) && A.fwin) {
            const int wi = i - A.wlo[0], wj = j - A.wlo[1], wk = k - A.wlo[2];
            if (wi >= 0 && wi < A.wn[0] && wj >= 0 && wj < A.wn[1] && wk >= 0 && wk < A.wn[2]) {
                const long long wc = ((long long)wk * A.wn[1] + wj) * A.wn[0] + wi;
                const long long wcells = (long long)A.wn[0] * A.wn[1] * A.wn[2];
                const double ir = rcp_nr(qc[0]);
                double fu = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double f = A.fwin[a * wcells + wc];
                    src[1 + a] = f;
                    fu = fma(f, qc[1 + a] * ir, fu);
                }
                src[4] = fu;
            }
        }
        if (terms & T_SPONGE) {
            const double eta = fmax(K->eta_dir(0, i), fmax(K->eta_dir(1, j), K->eta_dir(2, k)));
            if (eta > 0.0) {
                const double sg = K->P.sigma * (eta * eta * eta);
#pragma unroll
                for (int c = 0; c < 5; ++c) src[c] = fma(-sg, qc[c] - K->P.q_inf[c], src[c]);
            }
        }
        if (K->P.src_amp != 0.0) {
            // periodic Gaussian pressure source (Sec. 3), into the energy as A_p / (gamma - 1)
            const double x = G.lo[0] + ((double)(i + G.org[0]) + 0.5) * G.h,
                         y = G.lo[1] + ((double)(j + G.org[1]) + 0.5) * G.h,
                         z = G.lo[2] + ((double)(k + G.org[2]) + 0.5) * G.h;
            const double dx = x - K->P.src_x[0], dy = y - K->P.src_x[1], dz = z - K->P.src_x[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ap = -K->P.src_amp * exp(-K->P.src_bl2 * r2) * cos(K->P.src_omega * A.t);
            src[4] += ap * K->P.inv_gm1;
        }
        double val[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const double l = L[c] + src[c];
            if (A.mode_rhs) {
                val[c] = l;
            } else {
                const double stage = fma(A.dt, l, qc[c]);
                val[c] = (A.ca == 0.0) ? stage : fma(A.ca, __builtin_nontemporal_load(&A.Qn[c * G.ncell + o]), A.cb * stage);
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            // (the output state streams past the caches: far larger than they are)
            __builtin_nontemporal_store(val[c], &A.out[c * G.ncell + o]);
        }
        if (A.alpha_part && k >= A.arow0 && k < A.arow1) {
            const double ir = rcp_nr(val[0]);
            const double u = val[1] * ir, v = val[2] * ir, w = val[3] * ir;
            const double pn = K->P.gm1 * (val[4] - 0.5 * fma(val[1], u, fma(val[2], v, val[3] * w)));
            const double cn = sqrt(K->P.gamma * pn * ir);
            am[0] = (unsigned long long)__double_as_longlong(fabs(u) + cn);
            am[1] = (unsigned long long)__double_as_longlong(fabs(v) + cn);
            am[2] = (unsigned long long)__double_as_longlong(fabs(w) + cn);
        }
    }
    if (A.alpha_part) {
        // block maximum -> one partial per block (plain stores; reduced by launch_alpha_final)
        __shared__ unsigned long long red[BX * BY / 64][3];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            unsigned long long v = am[d];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v = max_bits(v, __shfl_xor(v, off, 64));
            if (lane == 0) red[wid][d] = v;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            unsigned long long v = 0ull;
#pragma unroll
            for (int w = 0; w < BX * BY / 64; ++w) v = max_bits(v, red[w][threadIdx.x]);
            const long long b = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            A.alpha_part[b * 3 + threadIdx.x] = v;
        }
    }
}

}  // namespace

long long stress3d_elems(const Grid& G)
{
    return 9ll * (G.n[0] + 4) * (G.n[1] + 4) * (G.n[2] + 4);
}

long long stage3d_blocks(const Grid& G)
{
    return (long long)((G.n[0] + BX - 1) / BX) * ((G.n[1] + BY - 1) / BY) * G.n[2];
}

long long faces3d_elems(const Grid& G)
{
    return 5ll * (faces_of<0>(G) + faces_of<1>(G) + faces_of<2>(G));
}

template <int SCHEME, class T>
static void launch_faces(const KConst* K, const Grid& G, const StageArgs& A, T* F, bool ch, hipStream_t s)
{
    const dim3 block(BX * BY);
    T* Fx = F;
    T* Fy = Fx + 5 * faces_of<0>(G);
    T* Fz = Fy + 5 * faces_of<1>(G);
    const dim3 gx((G.n[0] + BX - 1) / BX, (G.n[1] + BY - 1) / BY, G.n[2]);
    constexpr int FXa = FaceTile<1>::FX, FAa = FaceTile<1>::FA;   // (the same for z faces)
    const dim3 gy((G.n[0] + FXa - 1) / FXa, (G.n[1] + 1 + FAa - 1) / FAa, G.n[2]);
    const dim3 gz((G.n[0] + FXa - 1) / FXa, G.n[1], (G.n[2] + 1 + FAa - 1) / FAa);   // (x by z faces)
    // the x faces f = n_x when the x blocks end there
    const bool xedge = G.n[0] % BX == 0;
    const dim3 ge((unsigned)(((long long)G.n[1] * G.n[2] + BX * BY - 1) / (BX * BY)));
    if constexpr (std::is_same<T, double>::value) {
        if (ch) {
            hipLaunchKernelGGL((k_faces3d<SCHEME, T, 0, false, true>), gx, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx, nullptr);
            if (xedge)
                hipLaunchKernelGGL((k_xedge3d<SCHEME, T, false, true>), ge, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx, nullptr);
            hipLaunchKernelGGL((k_faces3d<SCHEME, T, 1, false, true>), gy, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fy, nullptr);
            hipLaunchKernelGGL((k_faces3d<SCHEME, T, 2, false, true>), gz, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fz, nullptr);
            return;
        }
    }
    if constexpr (SCHEME == TENO5 && std::is_same<T, double>::value) {
        if (A.dbg_x) {
            hipLaunchKernelGGL((k_faces3d<SCHEME, T, 0, true>), gx, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx, A.dbg_x);
            if (xedge)
                hipLaunchKernelGGL((k_xedge3d<SCHEME, T, true>), ge, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx, A.dbg_x);
            hipLaunchKernelGGL((k_faces3d<SCHEME, T, 1, true>), gy, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fy, A.dbg_y);
            hipLaunchKernelGGL((k_faces3d<SCHEME, T, 2, true>), gz, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fz, A.dbg_z);
            return;
        }
    }
    hipLaunchKernelGGL((k_faces3d<SCHEME, T, 0>), gx, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx, nullptr);
    if (xedge) hipLaunchKernelGGL((k_xedge3d<SCHEME, T>), ge, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fx, nullptr);
    hipLaunchKernelGGL((k_faces3d<SCHEME, T, 1>), gy, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fy, nullptr);
    hipLaunchKernelGGL((k_faces3d<SCHEME, T, 2>), gz, block, 0, s, K, A.Qs, A.step, A.alpha_bits, Fz, nullptr);
}

int launch_stage3d(const KConst* K, const Grid& G, int scheme, int precision, int variables, const StageArgs& A,
                   void* stress, void* faces, hipStream_t s)
{
    if (A.dbg_x && (scheme != TENO5 || precision != 0 || variables != 0 || !A.dbg_y || !A.dbg_z))
        return (int)hipErrorInvalidValue;
    if (variables != 0 && precision != 0) return (int)hipErrorInvalidValue;
    const bool ch = variables != 0;
    const dim3 block(BX * BY);
    const dim3 gs((unsigned)(stress_tiles(G) * ((G.n[2] + 4 + SZ - 1) / SZ)));
    const dim3 gr((G.n[0] + BX - 1) / BX, (G.n[1] + BY - 1) / BY, G.n[2]);
    if (precision == 1) {
        float* S = static_cast<float*>(stress);
        float* F = static_cast<float*>(faces);
        hipLaunchKernelGGL(k_stress3d<float>, gs, block, 0, s, K, A.Qs, A.step, S);
        if (scheme == TENO5) launch_faces<TENO5, float>(K, G, A, F, false, s);
        else launch_faces<WENO5JS, float>(K, G, A, F, false, s);
        const float* Fx = F;
        const float* Fy = Fx + 5 * faces_of<0>(G);
        const float* Fz = Fy + 5 * faces_of<1>(G);
        hipLaunchKernelGGL(k_stage3d<float>, gr, block, 0, s, K, A, (const float*)S, Fx, Fy, Fz);
    } else {
        double* S = static_cast<double*>(stress);
        double* F = static_cast<double*>(faces);
        hipLaunchKernelGGL(k_stress3d<double>, gs, block, 0, s, K, A.Qs, A.step, S);
        if (scheme == TENO5) launch_faces<TENO5, double>(K, G, A, F, ch, s);
        else launch_faces<WENO5JS, double>(K, G, A, F, ch, s);
        const double* Fx = F;
        const double* Fy = Fx + 5 * faces_of<0>(G);
        const double* Fz = Fy + 5 * faces_of<1>(G);
        hipLaunchKernelGGL(k_stage3d<double>, gr, block, 0, s, K, A, (const double*)S, Fx, Fy, Fz);
    }
    return (int)hipGetLastError();
}

}  // namespace fsa
