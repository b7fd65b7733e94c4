// Per-face kernels of the learned TENO5 selector on a 2D grid.
//
// A face lies between cells i and i+1 along direction d; its side 0 reconstructs f+ from
// cells i-2..i+2, its side 1 reconstructs f- from cells i+3..i-1 (upwind order, centre at
// position 2).  x faces are numbered j * (nx + 1) + (i + 1), y faces (j + 1) * nx + i, with
// i or j = -1 for the boundary face below the first cell.
//
//  * k_flags2d: features of both sides -> the BF16 MFMA network (LDS-staged, 16 samples per
//    tile) -> a 12-bit keep pattern per side (3 bits per conserved component).  Confident
//    sides use the predicted bits for every component; sides below the confidence threshold
//    (or with no sub-stencil predicted) fall back to plain TENO5 per component, evaluated in
//    FP32 on far-field deviations exactly as the precision form does.
//  * k_harvest2d: features and the FP64 TENO5 label (bit k = kept for every component; a
//    numerically constant component keeps everything) of every side; all sides with a cut-off
//    and a seeded fraction of the all-kept ones are written, in face order, by a two-pass
//    compaction (deterministic).
#include "fsa_mlp.hpp"

namespace fsa {

namespace {

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef short s8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// The six cells i-2..i+3 of face f along dir, their states, primitives and split fluxes.
struct FaceCells {
    double q[6][4];
    double rho[6], un[6], p[6];
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
    for (int s = 0; s < 6; ++s) {
        const int ii = dir == 0 ? i + s - 2 : i, jj = dir == 1 ? j + s - 2 : j;
        fetch_state<2>(Q, K->G, K->P, step, ii, jj, 0, C.q[s]);
        const double ir = 1.0 / C.q[s][0];
        const double u = C.q[s][1] * ir, v = C.q[s][2] * ir;
        C.rho[s] = C.q[s][0];
        C.un[s] = dir == 0 ? u : v;
        C.p[s] = K->P.gm1 * (C.q[s][3] - 0.5 * (C.q[s][1] * u + C.q[s][2] * v));
    }
}

// Stencil position k (0..4) of side sd in the six cells.
__device__ __forceinline__ int cell_of(int sd, int k) { return sd == 0 ? k : 5 - k; }

// 15 features of one side: deviations from the centre, scaled by their largest magnitude.
__device__ __forceinline__ void side_features(const FaceCells& C, int sd, float* f)
{
    const double* vars[3] = {C.rho, C.un, C.p};
    for (int m = 0; m < 3; ++m) {
        const double sgn = (m == 1 && sd == 1) ? -1.0 : 1.0;
        const double c = sgn * vars[m][cell_of(sd, 2)];
        double dv[5], mx = 0.0;
        for (int k = 0; k < 5; ++k) {
            dv[k] = sgn * vars[m][cell_of(sd, k)] - c;
            mx = fmax(mx, fabs(dv[k]));
        }
        for (int k = 0; k < 5; ++k) f[m * 5 + k] = (float)(dv[k] / (mx + 1e-30));
    }
}

// Split flux of component c at cell s along dir: (F +- alpha q)/2 (sign + for side 0).
__device__ __forceinline__ double split_flux(const KConst* K, const FaceCells& C, int dir, int s, int c, double a)
{
    const double* q = C.q[s];
    const double ud = C.un[s];
    double F;
    if (c == 0) F = q[1 + dir];
    else if (c == 3) F = (q[3] + C.p[s]) * ud;
    else F = q[c] * ud + (c - 1 == dir ? C.p[s] : 0.0);
    return 0.5 * (F + a * q[c]);
}

// FP64 TENO5 keep flags of five upwind-ordered values (same decision as the FP64 method).
__device__ __forceinline__ int teno_flags64(double a, double b, double c, double d, double e, double eps, double ct)
{
    const double s0 = fma(-2.0, b, a) + c, t0 = fma(-4.0, b, a) + 3.0 * c;
    const double s1 = fma(-2.0, c, b) + d, t1 = b - d;
    const double s2 = fma(-2.0, d, c) + e, t2 = fma(-4.0, d, 3.0 * c) + e;
    const double b0 = fma(13.0 / 12.0 * s0, s0, 0.25 * t0 * t0);
    const double b1 = fma(13.0 / 12.0 * s1, s1, 0.25 * t1 * t1);
    const double b2 = fma(13.0 / 12.0 * s2, s2, 0.25 * t2 * t2);
    const double tau = fabs(b0 - b2);
    const double x0 = 1.0 + tau / (b0 + eps), x1 = 1.0 + tau / (b1 + eps), x2 = 1.0 + tau / (b2 + eps);
    const double c0 = x0 * x0 * x0, c1 = x1 * x1 * x1, c2 = x2 * x2 * x2;
    const double g0 = c0 * c0, g1 = c1 * c1, g2 = c2 * c2;
    const double sum = g0 + g1 + g2;
    return (g0 / sum < ct ? 0 : 1) | (g1 / sum < ct ? 0 : 2) | (g2 / sum < ct ? 0 : 4);
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
__device__ __forceinline__ int side_label(const KConst* K, const FaceCells& C, int dir, int sd, double alpha)
{
    const double a = sd == 0 ? alpha : -alpha;
    int all = 7;
    for (int c = 0; c < 4; ++c) {
        double v[5], lo = 0, hi = 0, mag = 0;
        for (int k = 0; k < 5; ++k) {
            v[k] = split_flux(K, C, dir, cell_of(sd, k), c, a);
            lo = k ? fmin(lo, v[k]) : v[k];
            hi = k ? fmax(hi, v[k]) : v[k];
            mag = fmax(mag, fabs(v[k]));
        }
        if (hi - lo <= 1e-12 * mag) continue;
        all &= teno_flags64(v[0], v[1], v[2], v[3], v[4], K->P.teno_eps, K->P.teno_ct);
    }
    return all;
}

// Plain FP32 TENO5 flags of one side for every component (3 bits each): split fluxes minus
// those of the far field, formed in FP64 and rounded to FP32.
__device__ __forceinline__ int side_teno32(const KConst* K, const FaceCells& C, int dir, int sd, double alpha)
{
    const double a = sd == 0 ? alpha : -alpha;
    const double* Finf = dir == 0 ? K->Fx_inf : K->Fy_inf;
    int pat = 0;
    for (int c = 0; c < 4; ++c) {
        float v[5];
        for (int k = 0; k < 5; ++k) {
            const int s = cell_of(sd, k);
            const double dF = split_flux(K, C, dir, s, c, 0.0) * 2.0 - Finf[c];
            const double dq = C.q[s][c] - K->P.q_inf[c];
            v[k] = (float)(0.5 * fma(a, dq, dF));
        }
        pat |= teno_flags32(v[0], v[1], v[2], v[3], v[4], 1e-30f, (float)K->P.teno_ct) << (3 * c);
    }
    return pat;
}

// ---------------------------------------------------------------------------------------
// Learned flags: one wave per 64 faces of one direction.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_flags2d(const KConst* __restrict__ K, FlagArgs A)
{
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    const int dir = blockIdx.y;
    __shared__ float feat[128][16];
    __shared__ float zs[128][4];
    const long long f = (long long)blockIdx.x * 64 + lane;
    int i = 0, j = 0;
    const bool valid = face_origin(K, dir, f, i, j);
    FaceCells C;
    if (valid) {
        load_face(K, A.Q, A.step, dir, i, j, C);
        side_features(C, 0, feat[2 * lane]);
        side_features(C, 1, feat[2 * lane + 1]);
    } else {
        for (int k = 0; k < 15; ++k) feat[2 * lane][k] = feat[2 * lane + 1][k] = 0.f;
    }
    feat[2 * lane][15] = feat[2 * lane + 1][15] = 0.f;
    __syncthreads();
    // network on 8 tiles of 16 samples (weights as A, features as B operands)
    const float* master = A.M.master;
    const unsigned short* wb = A.M.wbf;
    s4_t w1[2];
    s8_t w2[2], w3;
    for (int m = 0; m < 2; ++m) {
        const int h = 16 * m + r;
        for (int jj = 0; jj < 4; ++jj) {
            const int in = 4 * g + jj;
            w1[m][jj] = (short)(in < MLP_NIN ? wb[MLP_W1 + in * MLP_NH + h] : 0);
        }
        for (int jj = 0; jj < 8; ++jj) {
            const int pi = jj < 4 ? 4 * g + jj : 16 + 4 * g + (jj - 4);
            w2[m][jj] = (short)wb[MLP_W2 + pi * MLP_NH + h];
        }
    }
    for (int jj = 0; jj < 8; ++jj) {
        const int pi = jj < 4 ? 4 * g + jj : 16 + 4 * g + (jj - 4);
        w3[jj] = (short)(r < MLP_NOUT ? wb[MLP_W3 + pi * MLP_NOUT + r] : 0);
    }
    const f4_t zero = {0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 8; ++t) {
        const int sl = 16 * t + r;
        s4_t x;
        for (int jj = 0; jj < 4; ++jj) x[jj] = (short)bf16_bits(feat[sl][4 * g + jj]);
        f4_t a1[2], a2[2];
        s8_t h1, h2;
        for (int m = 0; m < 2; ++m) {
            a1[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1[m], x, zero, 0, 0, 0);
            for (int v = 0; v < 4; ++v) a1[m][v] += master[MLP_B1 + 16 * m + 4 * g + v];
        }
        for (int v = 0; v < 4; ++v) {
            h1[v] = (short)bf16_bits(fmaxf(a1[0][v], 0.f));
            h1[4 + v] = (short)bf16_bits(fmaxf(a1[1][v], 0.f));
        }
        for (int m = 0; m < 2; ++m) {
            a2[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8_t, w2[m]), __builtin_bit_cast(b8_t, h1),
                                                            zero, 0, 0, 0);
            for (int v = 0; v < 4; ++v) a2[m][v] += master[MLP_B2 + 16 * m + 4 * g + v];
        }
        for (int v = 0; v < 4; ++v) {
            h2[v] = (short)bf16_bits(fmaxf(a2[0][v], 0.f));
            h2[4 + v] = (short)bf16_bits(fmaxf(a2[1][v], 0.f));
        }
        const f4_t z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8_t, w3), __builtin_bit_cast(b8_t, h2),
                                                               zero, 0, 0, 0);
        if (g == 0)
            for (int v = 0; v < MLP_NOUT; ++v) zs[sl][v] = z[v] + master[MLP_B3 + v];
    }
    __syncthreads();
    if (!valid) return;
    const double alpha = __longlong_as_double((long long)A.alpha_bits[dir]);
    unsigned word = 0;
    int nfall = 0;
    for (int sd = 0; sd < 2; ++sd) {
        const float* z = zs[2 * lane + sd];
        int bits = 0;
        float conf = 1.0f;
        for (int v = 0; v < MLP_NOUT; ++v) {
            if (z[v] > 0.f) bits |= 1 << v;
            conf = fminf(conf, fabsf(tanhf(0.5f * z[v])));   // |2 sigmoid(z) - 1|
        }
        int pat;
        if (bits == 0 || conf < A.conf_threshold) {
            pat = side_teno32(K, C, dir, sd, alpha);
            ++nfall;
        } else {
            pat = bits | bits << 3 | bits << 6 | bits << 9;
        }
        word |= (unsigned)pat << (16 * sd);
    }
    (dir == 0 ? A.flags_x : A.flags_y)[f] = word;
    if (A.counters) {
        atomicAdd(&A.counters[0], 2ull);
        if (nfall) atomicAdd(&A.counters[1], (unsigned long long)nfall);
    }
}

// ---------------------------------------------------------------------------------------
// Harvest: features and labels of selected face sides, written in face order.
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
    int lab[2] = {7, 7};
    bool sel[2] = {false, false};
    const double alpha = __longlong_as_double((long long)H.alpha_bits[dir]);
    if (valid) {
        load_face(K, H.Q, H.step, dir, i, j, C);
        for (int sd = 0; sd < 2; ++sd) {
            lab[sd] = side_label(K, C, dir, sd, alpha);
            const long long gid = 2 * ((dir == 0 ? 0 : nfx) + f) + sd;
            sel[sd] = select_side(H, gid, lab[sd]);
        }
    }
    const int mine = (int)sel[0] + (int)sel[1];
    // ordered prefix of the block (thread order = face order)
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    if (pass == 0) {
        if (threadIdx.x == blockDim.x - 1) H.block_count[blk] = before + incl;
        return;
    }
    long long pos = H.block_offset[blk] + before + incl - mine;
    for (int sd = 0; sd < 2; ++sd) {
        if (!sel[sd]) continue;
        if (pos < H.max_out) {
            float ft[15];
            side_features(C, sd, ft);
            for (int k = 0; k < 15; ++k) H.feats[pos * 16 + k] = ft[k];
            H.feats[pos * 16 + 15] = 0.f;
            H.labels[pos] = (unsigned char)lab[sd];
        }
        ++pos;
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

}  // namespace

int launch_flags2d(const KConst* K, const Grid& G, const FlagArgs& A, hipStream_t s)
{
    const long long nfx = (long long)(G.n[0] + 1) * G.n[1], nfy = (long long)G.n[0] * (G.n[1] + 1);
    const long long nf = nfx > nfy ? nfx : nfy;
    hipLaunchKernelGGL(k_flags2d, dim3((unsigned)((nf + 63) / 64), 2), dim3(64), 0, s, K, A);
    return (int)hipGetLastError();
}

long long harvest2d_blocks(const Grid& G)
{
    const long long nfx = (long long)(G.n[0] + 1) * G.n[1], nfy = (long long)G.n[0] * (G.n[1] + 1);
    const long long nf = nfx > nfy ? nfx : nfy;
    return 2 * ((nf + 255) / 256);
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
