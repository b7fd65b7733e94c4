// Per-face kernels of the learned TENO5 selector on a 2D grid.
//
// A face lies between cells i and i+1 along direction d; its side 0 reconstructs f+ from
// cells i-2..i+2, its side 1 reconstructs f- from cells i+3..i-1 (upwind order, centre at
// position 2).  x faces are numbered j * (nx + 1) + (i + 1), y faces (j + 1) * nx + i, with
// i or j = -1 for the boundary face below the first cell.
//
// A side is significant when rho, a velocity component or p varies over its five cells by
// more than 1e-8 of its natural scale (rho_inf, c_inf, rho_inf c_inf^2).  An insignificant
// side keeps every sub-stencil: each of its split-flux components is constant to that
// level, so no sub-stencil choice moves its face value by more.
//
//  * k_flags2d: one 256-thread block per tile of 64 x 16 faces of each direction.  The
//    tile's cells (with a 3-cell halo) go to LDS once as FP32 deviations of rho, u, v, p
//    from the far field; each wave then takes four rows of x faces and four rows of y faces.
//    Features of significant sides -> BF16 MFMA network (16 samples per tile, biases in the
//    accumulators, tiles without a significant side skipped) -> a 12-bit keep pattern per
//    side (3 bits per conserved component).  Confident sides use the predicted bits for every
//    component; sides below the confidence threshold (or with no sub-stencil predicted) fall
//    back to plain TENO5 per component, evaluated in FP32 on far-field deviations exactly as
//    the precision form does.
//  * k_harvest2d: features and the FP64 TENO5 label (bit k = kept for every component; a
//    numerically constant component keeps everything) of every significant side; all sides
//    with a cut-off and a seeded fraction of the all-kept ones are written, in face order, by
//    a two-pass compaction (deterministic).
#include <algorithm>

#include "fsa_mlp.hpp"

namespace fsa {

namespace {

typedef short s2_t __attribute__((ext_vector_type(2)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef short s8_t __attribute__((ext_vector_type(8)));
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// Two floats to bf16 (nearest even, one v_cvt_pk_bf16_f32), then max(., 0) on the two
// halves as signed 16-bit integers: the ReLU of both (bf16 rounding is monotonic and keeps
// the sign, so the order of rounding and ReLU does not matter).
__device__ __forceinline__ int relu_pk_bf16(float a, float b)
{
    const f2_t x = {a, b};
    s2_t h = __builtin_bit_cast(s2_t, __builtin_convertvector(x, b2_t));
    const s2_t z = {0, 0};
    h = __builtin_elementwise_max(h, z);
    return __builtin_bit_cast(int, h);
}
__device__ __forceinline__ int pk_bf16(float a, float b)
{
    const f2_t x = {a, b};
    return __builtin_bit_cast(int, __builtin_convertvector(x, b2_t));
}

// The six cells i-2..i+3 of a face along dir: states and primitives (FP64).
struct FaceCells {
    double q[6][4];
    double rho[6], un[6], ut[6], p[6];
};

__device__ __forceinline__ bool face_origin(const KConst* K, int dir, long long f, int& i, int& j)
{
    const int nx = K->G.n[0], ny = K->G.n[1];
    if (dir == 0) {
        if (f >= (long long)(nx + 1) * ny) return false;
        j = (int)(f / (nx + 1));
        i = (int)(f % (nx + 1)) - 1;
    } else {
        if (f >= (long long)nx * (ny + 1)) return false;
        j = (int)(f / nx) - 1;
        i = (int)(f % nx);
    }
    return true;
}

__device__ __forceinline__ void load_face(const KConst* K, const double* Q, long long step, int dir, int i, int j,
                                          FaceCells& C)
{
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int ii = dir == 0 ? i + s - 2 : i, jj = dir == 1 ? j + s - 2 : j;
        fetch_state<2>(Q, K->G, K->P, step, ii, jj, 0, C.q[s]);
        const double ir = 1.0 / C.q[s][0];
        const double u = C.q[s][1] * ir, v = C.q[s][2] * ir;
        C.rho[s] = C.q[s][0];
        C.un[s] = dir == 0 ? u : v;
        C.ut[s] = dir == 0 ? v : u;
        C.p[s] = K->P.gm1 * (C.q[s][3] - 0.5 * (C.q[s][1] * u + C.q[s][2] * v));
    }
}

// Primitive m (0 rho, 1 normal velocity, 2 tangential velocity, 3 p) of cell s.
__device__ __forceinline__ double prim(const FaceCells& C, int m, int s)
{
    return m == 0 ? C.rho[s] : (m == 1 ? C.un[s] : (m == 2 ? C.ut[s] : C.p[s]));
}

// Stencil position k (0..4) of side SD in the six cells.
template <int SD>
__device__ __forceinline__ constexpr int cell_of(int k) { return SD == 0 ? k : 5 - k; }

// 15 features of one side: deviations from the centre over (their largest magnitude + the
// variable's floor); the normal velocity is negated on side 1.
template <int SD>
__device__ __forceinline__ void side_features(const KConst* K, const FaceCells& C, float* f)
{
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int pm = m == 2 ? 3 : m;   // rho, normal velocity, p
        const double sgn = (m == 1 && SD == 1) ? -1.0 : 1.0;
        const double c = sgn * prim(C, pm, cell_of<SD>(2));
        double dv[5], mx = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            dv[k] = sgn * prim(C, pm, cell_of<SD>(k)) - c;
            mx = fmax(mx, fabs(dv[k]));
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) f[m * 5 + k] = (float)(dv[k] / (mx + K->sig[m]));
    }
}

// Significance of one side in FP64.
template <int SD>
__device__ __forceinline__ bool side_significant(const KConst* K, const FaceCells& C)
{
    bool sig = false;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double lo = prim(C, m, cell_of<SD>(0)), hi = lo;
#pragma unroll
        for (int k = 1; k < 5; ++k) {
            lo = fmin(lo, prim(C, m, cell_of<SD>(k)));
            hi = fmax(hi, prim(C, m, cell_of<SD>(k)));
        }
        sig = sig || (hi - lo > K->sig[m == 0 ? 0 : (m == 3 ? 2 : 1)]);
    }
    return sig;
}

// Split flux of component c at cell s along dir: (F + a q)/2.
__device__ __forceinline__ double split_flux(const FaceCells& C, int dir, int s, int c, double a)
{
    const double* q = C.q[s];
    const double ud = C.un[s];
    double F;
    if (c == 0) F = dir == 0 ? q[1] : q[2];
    else if (c == 3) F = (q[3] + C.p[s]) * ud;
    else F = q[c] * ud + (c - 1 == dir ? C.p[s] : 0.0);
    return 0.5 * (F + a * q[c]);
}

// FP64 TENO5 keep flags of five upwind-ordered values for the training labels, with the
// operations in the order of the method's plain definition and no contraction: a label is
// an integer decided by floating point, so it is taken exactly as the FP64 reference takes
// it.  (Contraction matters: fma(-4, b, a) + 3c contracted to fma(3, c, fma(-4, b, a)) leaves
// a rounding-level beta on a constant sub-stencil instead of 0, which flips the choice
// between two constant sub-stencils.)
__device__ __forceinline__ int teno_flags64(double a, double b, double c, double d, double e, double eps, double ct)
{
#pragma clang fp contract(off)
    const double s0 = a - 2.0 * b + c, t0 = a - 4.0 * b + 3.0 * c;
    const double s1 = b - 2.0 * c + d, t1 = b - d;
    const double s2 = c - 2.0 * d + e, t2 = 3.0 * c - 4.0 * d + e;
    const double b0 = 13.0 / 12.0 * s0 * s0 + 0.25 * t0 * t0;
    const double b1 = 13.0 / 12.0 * s1 * s1 + 0.25 * t1 * t1;
    const double b2 = 13.0 / 12.0 * s2 * s2 + 0.25 * t2 * t2;
    const double tau = fabs(b0 - b2);
    const double x0 = 1.0 + tau / (b0 + eps), x1 = 1.0 + tau / (b1 + eps), x2 = 1.0 + tau / (b2 + eps);
    const double c0 = x0 * x0 * x0, c1 = x1 * x1 * x1, c2 = x2 * x2 * x2;
    const double g0 = c0 * c0, g1 = c1 * c1, g2 = c2 * c2;
    const double sum = g0 + g1 + g2;
    return (g0 / sum < ct ? 0 : 1) | (g1 / sum < ct ? 0 : 2) | (g2 / sum < ct ? 0 : 4);
}

// Split flux (F + a q)/2 of component c of one state along dir for the labels: primitives
// u = m / rho, p = (gamma - 1)(E - (m_x u + m_y v)/2), no contraction.
__device__ __forceinline__ double label_split_flux(const KConst* K, const double* q, int dir, int c, double a)
{
#pragma clang fp contract(off)
    const double u = q[1] / q[0], v = q[2] / q[0];
    double ke = 0.0;
    ke += q[1] * u;
    ke += q[2] * v;
    const double p = K->P.gm1 * (q[3] - 0.5 * ke);
    const double ud = dir == 0 ? u : v;
    double F;
    if (c == 0) F = dir == 0 ? q[1] : q[2];
    else if (c == 3) F = (q[3] + p) * ud;
    else F = q[c] * ud + (c - 1 == dir ? p : 0.0);
    return 0.5 * (F + a * q[c]);
}

// FP32 TENO5 keep flags in the normalised form of the precision path.
__device__ __forceinline__ int teno_flags32(float a, float b, float c, float d, float e, float eps, float ct)
{
    const float s0 = fmaf(-2.0f, b, a) + c, t0 = fmaf(-4.0f, b, a) + 3.0f * c;
    const float s1 = fmaf(-2.0f, c, b) + d, t1 = b - d;
    const float s2 = fmaf(-2.0f, d, c) + e, t2 = fmaf(-4.0f, d, 3.0f * c) + e;
    const float b0 = fmaf(13.0f / 12.0f * s0, s0, 0.25f * t0 * t0);
    const float b1 = fmaf(13.0f / 12.0f * s1, s1, 0.25f * t1 * t1);
    const float b2 = fmaf(13.0f / 12.0f * s2, s2, 0.25f * t2 * t2);
    const float tau = fabsf(b0 - b2);
    const float a0 = tau * __builtin_amdgcn_rcpf(b0 + eps);
    const float a1 = tau * __builtin_amdgcn_rcpf(b1 + eps);
    const float a2 = tau * __builtin_amdgcn_rcpf(b2 + eps);
    const float inv = __builtin_amdgcn_rcpf(1.0f + fmaxf(a0, fmaxf(a1, a2)));
    const float x0 = (1.0f + a0) * inv, x1 = (1.0f + a1) * inv, x2 = (1.0f + a2) * inv;
    const float c0 = x0 * x0 * x0, c1 = x1 * x1 * x1, c2 = x2 * x2 * x2;
    const float g0 = c0 * c0, g1 = c1 * c1, g2 = c2 * c2;
    const float lim = ct * (g0 + g1 + g2);
    return (g0 < lim ? 0 : 1) | (g1 < lim ? 0 : 2) | (g2 < lim ? 0 : 4);
}

// Label of one side: AND over components of the FP64 TENO5 flags; a component whose five
// values agree to 1e-12 of their magnitude keeps everything.
template <int SD>
__device__ __forceinline__ int side_label(const KConst* K, const FaceCells& C, int dir, double alpha)
{
    const double a = SD == 0 ? alpha : -alpha;
    int all = 7;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double v[5], lo = 0, hi = 0, mag = 0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            v[k] = label_split_flux(K, C.q[cell_of<SD>(k)], dir, c, a);
            lo = k ? fmin(lo, v[k]) : v[k];
            hi = k ? fmax(hi, v[k]) : v[k];
            mag = fmax(mag, fabs(v[k]));
        }
        if (hi - lo <= 1e-12 * mag) continue;
        all &= teno_flags64(v[0], v[1], v[2], v[3], v[4], K->P.teno_eps, K->P.teno_ct);
    }
    return all;
}

// Plain FP32 TENO5 flags of both sides of one face for every component (3 bits each, side 0
// in the low half): the split fluxes minus those of the far field, formed in FP64 and rounded
// to FP32 with the same operations the precision form's stage kernel uses for that direction
// (so the fallback takes the decisions that form takes).  Cells i-2..i+3 along dir.
__device__ __forceinline__ unsigned fallback_patterns(const KConst* K, const double* Q, long long step, int dir, int i,
                                                      int j, double alpha, bool want0, bool want1)
{
    const int nx = K->G.n[0], ny = K->G.n[1];
    const long long ncell = K->G.ncell;
    const bool inner = dir == 0 ? (i - 2 >= 0 && i + 3 < nx && j >= 0 && j < ny)
                                : (j - 2 >= 0 && j + 3 < ny && i >= 0 && i < nx);
    float fp[6][4], fm[6][4];
    const double* Finf = dir == 0 ? K->Fx_inf : K->Fy_inf;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int ii = dir == 0 ? i + s - 2 : i, jj = dir == 1 ? j + s - 2 : j;
        double q[4];
        if (inner) {
            const double* src = Q + (long long)jj * nx + ii;
#pragma unroll
            for (int c = 0; c < 4; ++c) q[c] = src[c * ncell];
        } else {
            fetch_state<2>(Q, K->G, K->P, step, ii, jj, 0, q);
        }
        const double ir = rcp_nr(q[0]);
        const double u = q[1] * ir, v = q[2] * ir;
        const double p = K->P.gm1 * (q[3] - 0.5 * fma(q[1], u, q[2] * v));
        double F[4];
        if (dir == 0) {
            F[0] = q[1];
            F[1] = fma(q[1], u, p);
            F[2] = q[2] * u;
            F[3] = (q[3] + p) * u;
        } else {
            F[0] = q[2];
            F[1] = q[1] * v;
            F[2] = fma(q[2], v, p);
            F[3] = (q[3] + p) * v;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double dq = q[c] - K->P.q_inf[c], dF = F[c] - Finf[c];
            fm[s][c] = (float)(0.5 * fma(-alpha, dq, dF));
            fp[s][c] = (float)(0.5 * fma(alpha, dq, dF));
        }
    }
    const float ct = (float)K->P.teno_ct;
    unsigned pat0 = 0, pat1 = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (want0) pat0 |= (unsigned)teno_flags32(fp[0][c], fp[1][c], fp[2][c], fp[3][c], fp[4][c], 1e-30f, ct) << (3 * c);
        if (want1) pat1 |= (unsigned)teno_flags32(fm[5][c], fm[4][c], fm[3][c], fm[2][c], fm[1][c], 1e-30f, ct) << (3 * c);
    }
    return pat0 | (pat1 << 16);
}

// ---------------------------------------------------------------------------------------
// Learned flags
// ---------------------------------------------------------------------------------------
constexpr int FT_X = 64, FT_Y = 16;                // faces per tile: 64 along x, 16 rows
constexpr int LT_X = FT_X + 6, LT_Y = FT_Y + 6;    // cells of the tile with its halo
constexpr unsigned FALLBACK = 0xFFFFu;             // pattern marker: evaluate plain TENO5

// Order LDS traffic between the lanes of one wave: its LDS operations execute in program
// order, so it suffices that neither the compiler nor the wave moves a later access above an
// earlier one (the LDS arrays used this way are private to the wave).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP32 features of one side from the six cells' deviations v[0..5] (rho, un, p rows of w):
// upwind order k -> cell SD == 0 ? k : 5 - k, normal velocity negated on side 1.
template <int SD>
__device__ __forceinline__ void features32(const float (&w)[3][6], const float (&floor3)[3], int (&pk)[8])
{
    float f[16];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const float sgn = (m == 1 && SD == 1) ? -1.0f : 1.0f;
        const float c = w[m][cell_of<SD>(2)];
        float dv[5], mx = 0.0f;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            dv[k] = sgn * (w[m][cell_of<SD>(k)] - c);
            mx = fmaxf(mx, fabsf(dv[k]));
        }
        const float inv = __builtin_amdgcn_rcpf(mx + floor3[m]);
#pragma unroll
        for (int k = 0; k < 5; ++k) f[m * 5 + k] = dv[k] * inv;
    }
    f[15] = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) pk[k] = pk_bf16(f[2 * k], f[2 * k + 1]);
}

__global__ __launch_bounds__(256) void k_flags2d(const KConst* __restrict__ K, FlagArgs A)
{
    __shared__ float sv[4][LT_Y][LT_X];            // rho', u', v', p' of the tile's cells
    __shared__ int4 sfeat[4][128][2];              // per wave: bf16 features of 128 samples
    __shared__ unsigned short spat[4][128];        // per wave: network decision of each sample
    __shared__ unsigned short fb_list[8 * 256 * 2]; // deferred fallback sides: pass | wave | lane | side
    __shared__ int fb_count;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int nx = K->G.n[0], ny = K->G.n[1];
    const int x0 = blockIdx.x * FT_X, y0 = blockIdx.y * FT_Y;
    const long long ncell = K->G.ncell;

    // ---- quiet tile: when every strip and segment of the stage kernel that wrote Q and that
    // holds a cell of this tile (with its halo; ghosts only on zero-gradient sides, which copy
    // such cells) spreads by no more than the thresholds, so does every stencil of the tile (a
    // rounded max - min over a subset cannot exceed the rounded one over the union), and every
    // side is insignificant: the words are written without loading the state.
    if (A.qrange) {
        __shared__ int quiet;
        if (w == 0) {
            const int xa = x0 - 3, xb = x0 + LT_X - 4, ya = y0 - 3, yb = y0 + LT_Y - 4;
            bool ok = (xa >= 0 || K->G.bc[0][0] == BC_EXTRAP) && (xb < nx || K->G.bc[0][1] == BC_EXTRAP) &&
                      (ya >= 0 || K->G.bc[1][0] == BC_EXTRAP) && (yb < ny || K->G.bc[1][1] == BC_EXTRAP);
            const int sa = max(xa, 0) / A.qr_w, sb = min(xb, nx - 1) / A.qr_w;
            const int ga = max(ya, 0) / A.qr_ty, gb = min(yb, ny - 1) / A.qr_ty;
            const int ns = sb - sa + 1, nwav = ns * (gb - ga + 1);
            ok = ok && nwav <= 64;
            float mn[4] = {INFINITY, INFINITY, INFINITY, INFINITY}, mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
            if (ok && lane < nwav) {
                const int s = sa + lane % ns, gseg = ga + lane / ns;
                const float* q = A.qrange + ((long long)gseg * A.qr_ncolx + s) * 8;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    mn[m] = q[2 * m];
                    mx[m] = q[2 * m + 1];
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    mn[m] = fminf(mn[m], __shfl_xor(mn[m], off, 64));
                    mx[m] = fmaxf(mx[m], __shfl_xor(mx[m], off, 64));
                }
            const float th[4] = {(float)K->sig[0], (float)K->sig[1], (float)K->sig[1], (float)K->sig[2]};
#pragma unroll
            for (int m = 0; m < 4; ++m) ok = ok && !(mx[m] - mn[m] > th[m]);
            if (lane == 0) quiet = ok ? 1 : 0;
        }
        __syncthreads();
        if (quiet) {
            int n_sides = 0;
            for (int pass = 0; pass < 8; ++pass) {
                const int dir = pass >> 2, rs = 4 * w + (pass & 3);
                if (dir == 0) {
                    const int fi = x0 + lane - 1, fj = y0 + rs;
                    if (fj < ny && fi + 1 <= nx) {
                        A.flags_x[(long long)fj * (nx + 1) + (fi + 1)] = 0x0FFF0FFFu;
                        n_sides += 2;
                    }
                } else {
                    const int fi = x0 + lane, fj = y0 + rs - 1;
                    if (fi < nx && fj + 1 <= ny) {
                        A.flags_y[(long long)(fj + 1) * nx + fi] = 0x0FFF0FFFu;
                        n_sides += 2;
                    }
                }
            }
            if (A.counters) {
                __shared__ int qcnt[4];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) n_sides += __shfl_xor(n_sides, off, 64);
                if (lane == 0) qcnt[w] = n_sides;
                __syncthreads();
                if (tid == 0) {
                    const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
                    A.counters[blk * 3] += (unsigned long long)(qcnt[0] + qcnt[1] + qcnt[2] + qcnt[3]);
                }
            }
            return;
        }
    }

    // ---- the tile's cells (halo 3) as FP32 deviations from the far field: every interior
    // load of the thread is issued before any is used (one memory latency, not seven)
    constexpr int NT = LT_X * LT_Y, PER = (NT + 255) / 256;
    double q[PER][4];
    bool ghost[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int c = tid + 256 * t;
        const int ly = c / LT_X, lx = c - ly * LT_X;
        const int i = min(max(x0 - 3 + lx, -3), nx + 2), j = min(max(y0 - 3 + ly, -3), ny + 2);
        ghost[t] = !(i >= 0 && i < nx && j >= 0 && j < ny);
        if (c < NT && !ghost[t]) {
            const double* src = A.Q + (long long)j * nx + i;
#pragma unroll
            for (int m = 0; m < 4; ++m) q[t][m] = src[m * ncell];
        }
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int c = tid + 256 * t;
        if (c >= NT) continue;
        const int ly = c / LT_X, lx = c - ly * LT_X;
        if (ghost[t]) {
            const int i = min(max(x0 - 3 + lx, -3), nx + 2), j = min(max(y0 - 3 + ly, -3), ny + 2);
            fetch_state<2>(A.Q, K->G, K->P, A.step, i, j, 0, q[t]);
        }
        const double ir = rcp_nr(q[t][0]);
        const double u = q[t][1] * ir, v = q[t][2] * ir;
        const double p = K->P.gm1 * (q[t][3] - 0.5 * fma(q[t][1], u, q[t][2] * v));
        sv[0][ly][lx] = (float)(q[t][0] - K->P.prim_inf[0]);
        sv[1][ly][lx] = (float)(u - K->P.prim_inf[1]);
        sv[2][ly][lx] = (float)(v - K->P.prim_inf[2]);
        sv[3][ly][lx] = (float)(p - K->P.prim_inf[4]);
    }

    // ---- network operands: weights as A (loaded once), biases as accumulator inputs
    const unsigned short* wb = A.M.wbf;
    const float* master = A.M.master;
    s4_t w1[2];
    s8_t w2[2], w3;
    f4_t c1[2], c2[2], c3;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int h = 16 * m + r;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int in = 4 * g + jj;
            w1[m][jj] = (short)(in < MLP_NIN ? wb[MLP_W1 + in * MLP_NH + h] : 0);
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int pi = jj < 4 ? 4 * g + jj : 16 + 4 * g + (jj - 4);
            w2[m][jj] = (short)wb[MLP_W2 + pi * MLP_NH + h];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            c1[m][v] = master[MLP_B1 + 16 * m + 4 * g + v];
            c2[m][v] = master[MLP_B2 + 16 * m + 4 * g + v];
        }
    }
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
        const int pi = jj < 4 ? 4 * g + jj : 16 + 4 * g + (jj - 4);
        w3[jj] = (short)(r < MLP_NOUT ? wb[MLP_W3 + pi * MLP_NOUT + r] : 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) c3[v] = (g == 0 && v < MLP_NOUT) ? master[MLP_B3 + v] : 0.0f;
    const float sig[4] = {(float)K->sig[0], (float)K->sig[1], (float)K->sig[1], (float)K->sig[2]};
    const float floor3[3] = {sig[0], sig[1], sig[3]};
    const float zthr = A.zthr;
    const double alpha[2] = {__longlong_as_double((long long)A.alpha_bits[0]),
                             __longlong_as_double((long long)A.alpha_bits[1])};
    int n_sides = 0, n_sig = 0, n_fb = 0;
    if (tid == 0) fb_count = 0;
    __syncthreads();

    for (int pass = 0; pass < 8; ++pass) {
        const int dir = pass >> 2, rs = 4 * w + (pass & 3);
        // this lane's face: x faces f = x0 + lane of row y0 + rs; y faces g = y0 + rs of column
        // x0 + lane; cells k = 0..5 of the face are i-2..i+3 along dir
        int fi, fj;
        bool valid;
        float vv[4][6];   // rho', un', ut', p'
        if (dir == 0) {
            fi = x0 + lane - 1;          // cell left of the face
            fj = y0 + rs;
            valid = fj < ny && fi + 1 <= nx;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                vv[0][k] = sv[0][rs + 3][lane + k];
                vv[1][k] = sv[1][rs + 3][lane + k];
                vv[2][k] = sv[2][rs + 3][lane + k];
                vv[3][k] = sv[3][rs + 3][lane + k];
            }
        } else {
            fi = x0 + lane;
            fj = y0 + rs - 1;            // cell below the face
            valid = fi < nx && fj + 1 <= ny;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                vv[0][k] = sv[0][rs + k][lane + 3];
                vv[1][k] = sv[2][rs + k][lane + 3];
                vv[2][k] = sv[1][rs + k][lane + 3];
                vv[3][k] = sv[3][rs + k][lane + 3];
            }
        }
        // significance of both sides: spreads over cells 0..4 and 1..5
        bool sg0 = false, sg1 = false;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            float lo = fminf(fminf(vv[m][1], vv[m][2]), fminf(vv[m][3], vv[m][4]));
            float hi = fmaxf(fmaxf(vv[m][1], vv[m][2]), fmaxf(vv[m][3], vv[m][4]));
            sg0 = sg0 || (fmaxf(hi, vv[m][0]) - fminf(lo, vv[m][0]) > sig[m]);
            sg1 = sg1 || (fmaxf(hi, vv[m][5]) - fminf(lo, vv[m][5]) > sig[m]);
        }
        sg0 = sg0 && valid;
        sg1 = sg1 && valid;
        const unsigned long long need = __ballot(sg0 || sg1);
        if (need) {
            const float w3v[3][6] = {
                {vv[0][0], vv[0][1], vv[0][2], vv[0][3], vv[0][4], vv[0][5]},
                {vv[1][0], vv[1][1], vv[1][2], vv[1][3], vv[1][4], vv[1][5]},
                {vv[3][0], vv[3][1], vv[3][2], vv[3][3], vv[3][4], vv[3][5]}};
            int p0[8], p1[8];
            features32<0>(w3v, floor3, p0);
            features32<1>(w3v, floor3, p1);
            sfeat[w][2 * lane][0] = make_int4(p0[0], p0[1], p0[2], p0[3]);
            sfeat[w][2 * lane][1] = make_int4(p0[4], p0[5], p0[6], p0[7]);
            sfeat[w][2 * lane + 1][0] = make_int4(p1[0], p1[1], p1[2], p1[3]);
            sfeat[w][2 * lane + 1][1] = make_int4(p1[4], p1[5], p1[6], p1[7]);
        }
        wave_sync();
        if (need) {
            // tile t holds samples 16t..16t+15 = both sides of lanes 8t..8t+7
            for (int t = 0; t < 8; ++t) {
                if (((need >> (8 * t)) & 0xFFull) == 0) continue;
                const short* fs = reinterpret_cast<const short*>(&sfeat[w][16 * t + r][0]);
                s4_t x;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) x[jj] = fs[4 * g + jj];
                f4_t a1[2], a2[2];
#pragma unroll
                for (int m = 0; m < 2; ++m) a1[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[m], x, c1[m], 0, 0, 0);
                int h1[4] = {relu_pk_bf16(a1[0][0], a1[0][1]), relu_pk_bf16(a1[0][2], a1[0][3]),
                             relu_pk_bf16(a1[1][0], a1[1][1]), relu_pk_bf16(a1[1][2], a1[1][3])};
                const s8_t hb1 = __builtin_bit_cast(s8_t, h1);
#pragma unroll
                for (int m = 0; m < 2; ++m)
                    a2[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8_t, w2[m]),
                                                                    __builtin_bit_cast(b8_t, hb1), c2[m], 0, 0, 0);
                int h2[4] = {relu_pk_bf16(a2[0][0], a2[0][1]), relu_pk_bf16(a2[0][2], a2[0][3]),
                             relu_pk_bf16(a2[1][0], a2[1][1]), relu_pk_bf16(a2[1][2], a2[1][3])};
                const s8_t hb2 = __builtin_bit_cast(s8_t, h2);
                const f4_t z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8_t, w3),
                                                                       __builtin_bit_cast(b8_t, hb2), c3, 0, 0, 0);
                if (g == 0) {
                    const int bits = (z[0] > 0.f ? 1 : 0) | (z[1] > 0.f ? 2 : 0) | (z[2] > 0.f ? 4 : 0);
                    const float zmin = fminf(fabsf(z[0]), fminf(fabsf(z[1]), fabsf(z[2])));
                    spat[w][16 * t + r] =
                        (unsigned short)((bits != 0 && zmin >= zthr) ? (unsigned)bits * 0x249u : FALLBACK);
                }
            }
        }
        wave_sync();
        if (!valid) continue;
        unsigned pat0 = 0x0FFFu, pat1 = 0x0FFFu;
        if (sg0) pat0 = spat[w][2 * lane];
        if (sg1) pat1 = spat[w][2 * lane + 1];
        // sides below the confidence threshold are evaluated after the passes by the whole
        // block (spreading that work over all its lanes); their halves are written then
        if (pat0 == FALLBACK || pat1 == FALLBACK) {
            const int base = (pass << 8) | (w << 6) | lane;
            if (pat0 == FALLBACK) {
                fb_list[atomicAdd(&fb_count, 1)] = (unsigned short)(base << 1);
                pat0 = 0;
                ++n_fb;
            }
            if (pat1 == FALLBACK) {
                fb_list[atomicAdd(&fb_count, 1)] = (unsigned short)((base << 1) | 1);
                pat1 = 0;
                ++n_fb;
            }
        }
        n_sides += 2;
        n_sig += (int)sg0 + (int)sg1;
        const unsigned word = pat0 | (pat1 << 16);
        if (dir == 0) A.flags_x[(long long)fj * (nx + 1) + (fi + 1)] = word;
        else A.flags_y[(long long)(fj + 1) * nx + fi] = word;
    }
    __syncthreads();
    const int nfb = fb_count;
    for (int k = tid; k < nfb; k += 256) {
        const int e = fb_list[k], sd = e & 1, lanek = (e >> 1) & 63, wk = (e >> 7) & 3, pass = e >> 9;
        const int dir = pass >> 2, rs = 4 * wk + (pass & 3);
        const int fi = dir == 0 ? x0 + lanek - 1 : x0 + lanek;
        const int fj = dir == 0 ? y0 + rs : y0 + rs - 1;
        const unsigned pats = fallback_patterns(K, A.Q, A.step, dir, fi, fj, alpha[dir], sd == 0, sd == 1);
        const long long f = dir == 0 ? (long long)fj * (nx + 1) + (fi + 1) : (long long)(fj + 1) * nx + fi;
        unsigned short* half = reinterpret_cast<unsigned short*>(dir == 0 ? A.flags_x : A.flags_y);
        half[2 * f + sd] = (unsigned short)(sd == 0 ? (pats & 0xFFFFu) : (pats >> 16));
    }
    if (A.counters) {
        // per-block totals added to this block's own slot (no atomics: every block owns its
        // three counters, and launches on one stream are ordered)
        __shared__ int wcnt[4][3];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            n_sides += __shfl_xor(n_sides, off, 64);
            n_sig += __shfl_xor(n_sig, off, 64);
            n_fb += __shfl_xor(n_fb, off, 64);
        }
        if (lane == 0) {
            wcnt[w][0] = n_sides;
            wcnt[w][1] = n_fb;
            wcnt[w][2] = n_sig;
        }
        __syncthreads();
        if (tid < 3) {
            const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
            A.counters[blk * 3 + tid] += (unsigned long long)(wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid]);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Harvest: features and labels of selected significant sides, written in face order.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ bool select_side(const HarvestArgs& H, long long gid, int label)
{
    if (label != 7) return true;
    return u01(splitmix64(H.seed, (unsigned long long)gid)) < H.keep_rate;
}

// pass 0 counts selected sides per block; pass 1 writes them at the block's offset.
__global__ __launch_bounds__(256) void k_harvest2d(const KConst* __restrict__ K, HarvestArgs H, int pass)
{
    const int dir = blockIdx.y;
    const long long nfx = (long long)(K->G.n[0] + 1) * K->G.n[1];
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i = 0, j = 0;
    const bool valid = face_origin(K, dir, f, i, j);
    FaceCells C;
    int lab0 = 7, lab1 = 7;
    bool sel0 = false, sel1 = false;
    const double alpha = __longlong_as_double((long long)H.alpha_bits[dir]);
    if (valid) {
        load_face(K, H.Q, H.step, dir, i, j, C);
        const long long gid = 2 * ((dir == 0 ? 0 : nfx) + f);
        if (side_significant<0>(K, C)) {
            lab0 = side_label<0>(K, C, dir, alpha);
            sel0 = select_side(H, gid, lab0);
        }
        if (side_significant<1>(K, C)) {
            lab1 = side_label<1>(K, C, dir, alpha);
            sel1 = select_side(H, gid + 1, lab1);
        }
    }
    const int mine = (int)sel0 + (int)sel1;
    // ordered prefix of the block (thread order = face order)
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < wid; ++q) before += wsum[q];
    const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    if (pass == 0) {
        if (threadIdx.x == blockDim.x - 1) H.block_count[blk] = before + incl;
        return;
    }
    long long pos = H.block_offset[blk] + before + incl - mine;
    if (sel0) {
        if (pos < H.max_out) {
            float ft[15];
            side_features<0>(K, C, ft);
#pragma unroll
            for (int k = 0; k < 15; ++k) H.feats[pos * 16 + k] = ft[k];
            H.feats[pos * 16 + 15] = 0.f;
            H.labels[pos] = (unsigned char)lab0;
        }
        ++pos;
    }
    if (sel1 && pos < H.max_out) {
        float ft[15];
        side_features<1>(K, C, ft);
#pragma unroll
        for (int k = 0; k < 15; ++k) H.feats[pos * 16 + k] = ft[k];
        H.feats[pos * 16 + 15] = 0.f;
        H.labels[pos] = (unsigned char)lab1;
    }
}

__global__ void k_scan_counts(const int* __restrict__ count, long long n, long long* __restrict__ offset,
                              long long* __restrict__ total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long s = 0;
    for (long long b = 0; b < n; ++b) {
        offset[b] = s;
        s += count[b];
    }
    *total = s;
}

// ---------------------------------------------------------------------------------------
// Harvest in 3D: the same features, significance gate and labels as in 2D, for the faces of
// all three directions (x faces [nz][ny][nx+1], then y faces [nz][ny+1][nx], then z faces
// [nz+1][ny][nx]); side s of face f' (counted over the directions in that order) is drawn
// with SplitMix64 number 2 f' + s.
// ---------------------------------------------------------------------------------------
struct FaceCells3 {
    double q[6][5];
    double rho[6], u[6][3], p[6];
};

__device__ __forceinline__ long long faces3_of(const Grid& G, int dir)
{
    return (long long)(G.n[0] + (dir == 0)) * (G.n[1] + (dir == 1)) * (G.n[2] + (dir == 2));
}

// Cell (i, j, k) below face f along dir.
__device__ __forceinline__ bool face_origin3(const Grid& G, int dir, long long f, int& i, int& j, int& k)
{
    const long long mx = G.n[0] + (dir == 0), my = G.n[1] + (dir == 1);
    if (f >= faces3_of(G, dir)) return false;
    i = (int)(f % mx) - (dir == 0);
    j = (int)((f / mx) % my) - (dir == 1);
    k = (int)(f / (mx * my)) - (dir == 2);
    return true;
}

__device__ __forceinline__ void load_face3(const KConst* K, const double* Q, long long step, int dir, int i, int j,
                                           int k, FaceCells3& C)
{
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int ii = i + (dir == 0 ? s - 2 : 0), jj = j + (dir == 1 ? s - 2 : 0), kk = k + (dir == 2 ? s - 2 : 0);
        fetch_state<3>(Q, K->G, K->P, step, ii, jj, kk, C.q[s]);
        const double ir = 1.0 / C.q[s][0];
        double ke = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C.u[s][a] = C.q[s][1 + a] * ir;
            ke += C.q[s][1 + a] * C.u[s][a];
        }
        C.rho[s] = C.q[s][0];
        C.p[s] = K->P.gm1 * (C.q[s][4] - 0.5 * ke);
    }
}

template <int SD>
__device__ __forceinline__ void side_features3(const KConst* K, const FaceCells3& C, int dir, float* f)
{
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double sgn = (m == 1 && SD == 1) ? -1.0 : 1.0;
        double v[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int s = cell_of<SD>(k);
            v[k] = sgn * (m == 0 ? C.rho[s] : (m == 1 ? C.u[s][dir] : C.p[s]));
        }
        double mx = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) mx = fmax(mx, fabs(v[k] - v[2]));
#pragma unroll
        for (int k = 0; k < 5; ++k) f[m * 5 + k] = (float)((v[k] - v[2]) / (mx + K->sig[m]));
    }
}

template <int SD>
__device__ __forceinline__ bool side_significant3(const KConst* K, const FaceCells3& C)
{
    bool sig = false;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        double lo = 0.0, hi = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int s = cell_of<SD>(k);
            const double v = m == 0 ? C.rho[s] : (m == 4 ? C.p[s] : C.u[s][m - 1]);
            lo = k ? fmin(lo, v) : v;
            hi = k ? fmax(hi, v) : v;
        }
        sig = sig || (hi - lo > K->sig[m == 0 ? 0 : (m == 4 ? 2 : 1)]);
    }
    return sig;
}

// Split flux (F + a q)/2 of component c of one 3D state along dir for the labels, no
// contraction (as label_split_flux).
__device__ __forceinline__ double label_split_flux3(const KConst* K, const double* q, int dir, int c, double a)
{
#pragma clang fp contract(off)
    const double u = q[1] / q[0], v = q[2] / q[0], w = q[3] / q[0];
    double ke = 0.0;
    ke += q[1] * u;
    ke += q[2] * v;
    ke += q[3] * w;
    const double p = K->P.gm1 * (q[4] - 0.5 * ke);
    const double ud = dir == 0 ? u : (dir == 1 ? v : w);
    double F;
    if (c == 0) F = q[1 + dir];
    else if (c == 4) F = (q[4] + p) * ud;
    else F = q[c] * ud + (c - 1 == dir ? p : 0.0);
    return 0.5 * (F + a * q[c]);
}

template <int SD>
__device__ __forceinline__ int side_label3(const KConst* K, const FaceCells3& C, int dir, double alpha)
{
    const double a = SD == 0 ? alpha : -alpha;
    int all = 7;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        double v[5], lo = 0, hi = 0, mag = 0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            v[k] = label_split_flux3(K, C.q[cell_of<SD>(k)], dir, c, a);
            lo = k ? fmin(lo, v[k]) : v[k];
            hi = k ? fmax(hi, v[k]) : v[k];
            mag = fmax(mag, fabs(v[k]));
        }
        if (hi - lo <= 1e-12 * mag) continue;
        all &= teno_flags64(v[0], v[1], v[2], v[3], v[4], K->P.teno_eps, K->P.teno_ct);
    }
    return all;
}

__global__ __launch_bounds__(256) void k_harvest3d(const KConst* __restrict__ K, HarvestArgs H, int pass)
{
    const int dir = blockIdx.y;
    const Grid& G = K->G;
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i = 0, j = 0, k = 0;
    const bool valid = face_origin3(G, dir, f, i, j, k);
    FaceCells3 C;
    int lab0 = 7, lab1 = 7;
    bool sel0 = false, sel1 = false;
    const double alpha = __longlong_as_double((long long)H.alpha_bits[dir]);
    if (valid) {
        load_face3(K, H.Q, H.step, dir, i, j, k, C);
        long long off = 0;
        for (int d = 0; d < dir; ++d) off += faces3_of(G, d);
        const long long gid = 2 * (off + f);
        if (side_significant3<0>(K, C)) {
            lab0 = side_label3<0>(K, C, dir, alpha);
            sel0 = select_side(H, gid, lab0);
        }
        if (side_significant3<1>(K, C)) {
            lab1 = side_label3<1>(K, C, dir, alpha);
            sel1 = select_side(H, gid + 1, lab1);
        }
    }
    const int mine = (int)sel0 + (int)sel1;
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < wid; ++q) before += wsum[q];
    const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    if (pass == 0) {
        if (threadIdx.x == blockDim.x - 1) H.block_count[blk] = before + incl;
        return;
    }
    long long pos = H.block_offset[blk] + before + incl - mine;
    float ft[15];
    if (sel0) {
        if (pos < H.max_out) {
            side_features3<0>(K, C, dir, ft);
#pragma unroll
            for (int m = 0; m < 15; ++m) H.feats[pos * 16 + m] = ft[m];
            H.feats[pos * 16 + 15] = 0.f;
            H.labels[pos] = (unsigned char)lab0;
        }
        ++pos;
    }
    if (sel1 && pos < H.max_out) {
        side_features3<1>(K, C, dir, ft);
#pragma unroll
        for (int m = 0; m < 15; ++m) H.feats[pos * 16 + m] = ft[m];
        H.feats[pos * 16 + 15] = 0.f;
        H.labels[pos] = (unsigned char)lab1;
    }
}

}  // namespace

long long flags2d_blocks(const Grid& G)
{
    return (long long)((G.n[0] + 1 + FT_X - 1) / FT_X) * ((G.n[1] + 1 + FT_Y - 1) / FT_Y);
}

int launch_flags2d(const KConst* K, const Grid& G, const FlagArgs& A, hipStream_t s)
{
    const unsigned gx = (unsigned)((G.n[0] + 1 + FT_X - 1) / FT_X), gy = (unsigned)((G.n[1] + 1 + FT_Y - 1) / FT_Y);
    hipLaunchKernelGGL(k_flags2d, dim3(gx, gy), dim3(256), 0, s, K, A);
    return (int)hipGetLastError();
}

long long harvest2d_blocks(const Grid& G)
{
    const long long nfx = (long long)(G.n[0] + 1) * G.n[1], nfy = (long long)G.n[0] * (G.n[1] + 1);
    const long long nf = nfx > nfy ? nfx : nfy;
    return 2 * ((nf + 255) / 256);
}

long long harvest3d_blocks(const Grid& G)
{
    long long nf = 0;
    for (int d = 0; d < 3; ++d)
        nf = std::max(nf, (long long)(G.n[0] + (d == 0)) * (G.n[1] + (d == 1)) * (G.n[2] + (d == 2)));
    return 3 * ((nf + 255) / 256);
}

int launch_harvest3d(const KConst* K, const Grid& G, const HarvestArgs& H, hipStream_t s)
{
    const unsigned bx = (unsigned)(harvest3d_blocks(G) / 3);
    hipLaunchKernelGGL(k_harvest3d, dim3(bx, 3), dim3(256), 0, s, K, H, 0);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(64), 0, s, H.block_count, 3ll * bx, H.block_offset, H.total);
    hipLaunchKernelGGL(k_harvest3d, dim3(bx, 3), dim3(256), 0, s, K, H, 1);
    return (int)hipGetLastError();
}

int launch_harvest2d(const KConst* K, const Grid& G, const HarvestArgs& H, hipStream_t s)
{
    const long long nfx = (long long)(G.n[0] + 1) * G.n[1], nfy = (long long)G.n[0] * (G.n[1] + 1);
    const long long nf = nfx > nfy ? nfx : nfy;
    const unsigned bx = (unsigned)((nf + 255) / 256);
    hipLaunchKernelGGL(k_harvest2d, dim3(bx, 2), dim3(256), 0, s, K, H, 0);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(64), 0, s, H.block_count, 2ll * bx, H.block_offset, H.total);
    hipLaunchKernelGGL(k_harvest2d, dim3(bx, 2), dim3(256), 0, s, K, H, 1);
    return (int)hipGetLastError();
}

}  // namespace fsa
