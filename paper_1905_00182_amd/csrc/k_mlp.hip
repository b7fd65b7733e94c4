// BF16 MFMA kernels of the learned TENO5 sub-stencil selector: a 15 -> 32 -> 32 -> 3 network
// per face side (ReLU hidden layers, logits out), trained with binary cross-entropy and Adam.
//
// Layout trick: every layer is computed transposed, H^T = W^T X^T, with the weights as the A
// operand and the activations as the B operand of v_mfma_f32_16x16x{16,32}_bf16 (16 samples
// per tile).  The accumulator of a 16x16 tile holds, in lane l, rows 4(l/16)+v and column
// l%16 -- exactly the lane layout the next layer's B operand needs, once the two 16-row tiles
// of a 32-wide layer are interleaved as k-slot 8g+j -> unit (j<4 ? 4g+j : 16+4g+j-4); the A
// operand (weights) is loaded with the same permutation.  So activations never move between
// lanes in the forward pass or in the back-propagation of the deltas.  Weight gradients sum
// over samples, which needs samples along k: they go through a per-wave LDS transpose.
//
// Rounding points (shared with the FP64 reference): features, weights, hidden activations
// and back-propagated deltas are rounded to bf16 (nearest, ties to even); biases,
// accumulation, losses and gradient sums are FP32.
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
__device__ __forceinline__ float bf16_value(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ f4_t mma16(s4_t a, s4_t b, f4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mma32(s8_t a, s8_t b, f4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8_t, a), __builtin_bit_cast(b8_t, b), c, 0,
                                                   0, 0);
}

// hidden unit of k-slot 8g+j of a 32-wide layer (the interleave of two accumulator tiles)
__device__ __forceinline__ int perm32(int g, int j) { return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4); }

// Weight operands of one wave (A operands, loaded once).
struct Weights {
    s4_t w1[2];    // layer 1, M-tiles of hidden units, k = inputs (16x16x16)
    s8_t w2[2];    // layer 2, M-tiles of output units, k = permuted input units
    s8_t w3;       // layer 3, rows = 3 logits (padded to 16)
    s4_t w3t[2];   // backward through layer 3: M-tiles of hidden units, k = logits
    s8_t w2t[2];   // backward through layer 2: M-tiles of input units, k = permuted output units
};

__device__ __forceinline__ void load_weights(const unsigned short* __restrict__ wb, int lane, bool backward, Weights& W)
{
    const int r = lane & 15, g = lane >> 4;
    for (int m = 0; m < 2; ++m) {
        const int h = 16 * m + r;
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * g + j;
            W.w1[m][j] = (short)(i < MLP_NIN ? wb[MLP_W1 + i * MLP_NH + h] : 0);
        }
        for (int j = 0; j < 8; ++j) W.w2[m][j] = (short)wb[MLP_W2 + perm32(g, j) * MLP_NH + h];
    }
    for (int j = 0; j < 8; ++j) W.w3[j] = (short)(r < MLP_NOUT ? wb[MLP_W3 + perm32(g, j) * MLP_NOUT + r] : 0);
    if (backward) {
        for (int m = 0; m < 2; ++m) {
            const int h = 16 * m + r;
            for (int j = 0; j < 4; ++j) {
                const int o = 4 * g + j;
                W.w3t[m][j] = (short)(o < MLP_NOUT ? wb[MLP_W3 + h * MLP_NOUT + o] : 0);
            }
            for (int j = 0; j < 8; ++j) W.w2t[m][j] = (short)wb[MLP_W2 + h * MLP_NH + perm32(g, j)];
        }
    }
}

// Forward pass of one 16-sample tile.  x: this lane's four features (inputs 4g..4g+3) of
// sample l%16, as bf16 bits.  Outputs: z (logits in lanes 0..15, v < 3), pre-activation signs
// and bf16 activations (for the backward pass).
struct Fwd {
    f4_t a1[2], a2[2];
    s8_t h1, h2;      // bf16 activations as the next layer's B operand
    f4_t z;
};

__device__ __forceinline__ void forward_tile(const Weights& W, const float* __restrict__ master, s4_t x, int lane, Fwd& F)
{
    const int g = lane >> 4;
    const f4_t zero = {0.f, 0.f, 0.f, 0.f};
    for (int m = 0; m < 2; ++m) {
        F.a1[m] = mma16(W.w1[m], x, zero);
        for (int v = 0; v < 4; ++v) F.a1[m][v] += master[MLP_B1 + 16 * m + 4 * g + v];
    }
    for (int v = 0; v < 4; ++v) {
        F.h1[v] = (short)bf16_bits(fmaxf(F.a1[0][v], 0.f));
        F.h1[4 + v] = (short)bf16_bits(fmaxf(F.a1[1][v], 0.f));
    }
    for (int m = 0; m < 2; ++m) {
        F.a2[m] = mma32(W.w2[m], F.h1, zero);
        for (int v = 0; v < 4; ++v) F.a2[m][v] += master[MLP_B2 + 16 * m + 4 * g + v];
    }
    for (int v = 0; v < 4; ++v) {
        F.h2[v] = (short)bf16_bits(fmaxf(F.a2[0][v], 0.f));
        F.h2[4 + v] = (short)bf16_bits(fmaxf(F.a2[1][v], 0.f));
    }
    F.z = mma32(W.w3, F.h2, zero);
    if (g == 0)
        for (int v = 0; v < MLP_NOUT; ++v) F.z[v] += master[MLP_B3 + v];
}

// Features of sample s (row of feats [n][16]) for this lane's inputs 4g..4g+3, as bf16.
__device__ __forceinline__ s4_t load_x(const float* __restrict__ feats, long long n, long long s, int lane)
{
    s4_t x = {0, 0, 0, 0};
    if (s < n) {
        const int g = lane >> 4;
        for (int j = 0; j < 4; ++j) x[j] = (short)bf16_bits(feats[s * 16 + 4 * g + j]);
    }
    return x;
}

__global__ __launch_bounds__(64) void k_mlp_forward(MLPArgs M, const float* __restrict__ feats, long long n,
                                                    float* __restrict__ logits)
{
    const int lane = threadIdx.x;
    Weights W;
    load_weights(M.wbf, lane, false, W);
    for (long long base = (long long)blockIdx.x * 16; base < n; base += (long long)gridDim.x * 16) {
        const long long s = base + (lane & 15);
        Fwd F;
        forward_tile(W, M.master, load_x(feats, n, s, lane), lane, F);
        if (lane < 16 && s < n)
            for (int v = 0; v < MLP_NOUT; ++v) logits[s * MLP_NOUT + v] = F.z[v];
    }
}

// One wave takes chunks of 32 samples: two forward/backward tiles, then the weight-gradient
// tiles over the chunk (k = samples) from an LDS transpose.  Per-wave partial sums go to
// partial[wave][NPARAM] and loss_part[wave]; k_mlp_reduce adds them in wave order.
__global__ __launch_bounds__(64) void k_mlp_grad(MLPArgs M, const float* __restrict__ feats,
                                                 const unsigned char* __restrict__ labels, long long n,
                                                 float* __restrict__ partial, float* __restrict__ loss_part)
{
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    __shared__ unsigned short Lx[32][16], Lh1[32][32], Lh2[32][32], Ldz[32][16], Ld2[32][32], Ld1[32][32];
    Weights W;
    load_weights(M.wbf, lane, true, W);
    const float scale = 1.0f / (3.0f * (float)n);
    const f4_t zero = {0.f, 0.f, 0.f, 0.f};
    f4_t gw1[2] = {zero, zero}, gw2[2][2] = {{zero, zero}, {zero, zero}}, gw3[2] = {zero, zero};
    float gb1[2][4] = {}, gb2[2][4] = {}, gb3[4] = {}, loss = 0.f;
    for (long long base = (long long)blockIdx.x * 32; base < n; base += (long long)gridDim.x * 32) {
        for (int t = 0; t < 2; ++t) {
            const long long s = base + 16 * t + r;
            const bool valid = s < n;
            const int sl = 16 * t + r;
            const s4_t x = load_x(feats, n, s, lane);
            Fwd F;
            forward_tile(W, M.master, x, lane, F);
            // output deltas (lanes 0..15 hold the three logits of sample s)
            float dz[4] = {0.f, 0.f, 0.f, 0.f};
            if (g == 0 && valid) {
                const int lab = labels[s];
                for (int v = 0; v < MLP_NOUT; ++v) {
                    const float z = F.z[v], y = (float)((lab >> v) & 1);
                    const float sg = 1.0f / (1.0f + __expf(-z));
                    dz[v] = (sg - y) * scale;
                    loss += fmaxf(z, 0.f) - z * y + __logf(1.0f + __expf(-fabsf(z)));
                    gb3[v] += dz[v];
                }
            }
            s4_t bz = {0, 0, 0, 0};
            for (int v = 0; v < 4; ++v) bz[v] = (short)bf16_bits(dz[v]);
            // back through layer 3 and the second ReLU
            s8_t b2;
            float d2[2][4];
            for (int m = 0; m < 2; ++m) {
                const f4_t dh = mma16(W.w3t[m], bz, zero);
                for (int v = 0; v < 4; ++v) {
                    d2[m][v] = F.a2[m][v] > 0.f ? dh[v] : 0.f;
                    gb2[m][v] += d2[m][v];
                }
            }
            for (int v = 0; v < 4; ++v) {
                b2[v] = (short)bf16_bits(d2[0][v]);
                b2[4 + v] = (short)bf16_bits(d2[1][v]);
            }
            // back through layer 2 and the first ReLU
            float d1[2][4];
            for (int m = 0; m < 2; ++m) {
                const f4_t dh = mma32(W.w2t[m], b2, zero);
                for (int v = 0; v < 4; ++v) {
                    d1[m][v] = F.a1[m][v] > 0.f ? dh[v] : 0.f;
                    gb1[m][v] += d1[m][v];
                }
            }
            // stage the tile in LDS as [sample][unit] for the weight gradients
            for (int j = 0; j < 4; ++j) Lx[sl][4 * g + j] = (unsigned short)x[j];
            for (int v = 0; v < 4; ++v) {
                Lh1[sl][4 * g + v] = (unsigned short)F.h1[v];
                Lh1[sl][16 + 4 * g + v] = (unsigned short)F.h1[4 + v];
                Lh2[sl][4 * g + v] = (unsigned short)F.h2[v];
                Lh2[sl][16 + 4 * g + v] = (unsigned short)F.h2[4 + v];
                Ld2[sl][4 * g + v] = (unsigned short)b2[v];
                Ld2[sl][16 + 4 * g + v] = (unsigned short)b2[4 + v];
                Ld1[sl][4 * g + v] = bf16_bits(d1[0][v]);
                Ld1[sl][16 + 4 * g + v] = bf16_bits(d1[1][v]);
                Ldz[sl][4 * g + v] = (unsigned short)bz[v];
            }
        }
        __syncthreads();
        // weight gradients over the 32 samples of the chunk: k-slot 8g+j = sample
        s8_t ax, ah1[2], ah2[2], bd1[2], bd2[2], bdz;
        for (int j = 0; j < 8; ++j) {
            const int sl = 8 * g + j;
            ax[j] = (short)Lx[sl][r];
            bdz[j] = (short)Ldz[sl][r];
            for (int m = 0; m < 2; ++m) {
                ah1[m][j] = (short)Lh1[sl][16 * m + r];
                ah2[m][j] = (short)Lh2[sl][16 * m + r];
                bd1[m][j] = (short)Ld1[sl][16 * m + r];
                bd2[m][j] = (short)Ld2[sl][16 * m + r];
            }
        }
        __syncthreads();
        for (int nt = 0; nt < 2; ++nt) gw1[nt] = mma32(ax, bd1[nt], gw1[nt]);
        for (int mt = 0; mt < 2; ++mt) {
            for (int nt = 0; nt < 2; ++nt) gw2[mt][nt] = mma32(ah1[mt], bd2[nt], gw2[mt][nt]);
            gw3[mt] = mma32(ah2[mt], bdz, gw3[mt]);
        }
    }
    // per-wave partial gradient in the natural parameter layout
    float* P = partial + (long long)blockIdx.x * MLP_NPARAM;
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * g + v;
        for (int nt = 0; nt < 2; ++nt)
            if (i < MLP_NIN) P[MLP_W1 + i * MLP_NH + 16 * nt + r] = gw1[nt][v];
        for (int mt = 0; mt < 2; ++mt) {
            const int ii = 16 * mt + 4 * g + v;
            for (int nt = 0; nt < 2; ++nt) P[MLP_W2 + ii * MLP_NH + 16 * nt + r] = gw2[mt][nt][v];
            if (r < MLP_NOUT) P[MLP_W3 + ii * MLP_NOUT + r] = gw3[mt][v];
        }
    }
    // bias sums: add the 16 sample columns of each lane group
    for (int off = 1; off < 16; off <<= 1)
        for (int v = 0; v < 4; ++v) {
            gb1[0][v] += __shfl_xor(gb1[0][v], off, 64);
            gb1[1][v] += __shfl_xor(gb1[1][v], off, 64);
            gb2[0][v] += __shfl_xor(gb2[0][v], off, 64);
            gb2[1][v] += __shfl_xor(gb2[1][v], off, 64);
            gb3[v] += __shfl_xor(gb3[v], off, 64);
        }
    for (int off = 1; off < 64; off <<= 1) loss += __shfl_xor(loss, off, 64);
    if (r == 0) {
        for (int m = 0; m < 2; ++m)
            for (int v = 0; v < 4; ++v) {
                P[MLP_B1 + 16 * m + 4 * g + v] = gb1[m][v];
                P[MLP_B2 + 16 * m + 4 * g + v] = gb2[m][v];
            }
        if (g == 0)
            for (int v = 0; v < MLP_NOUT; ++v) P[MLP_B3 + v] = gb3[v];
    }
    if (lane == 0) loss_part[blockIdx.x] = loss;
}

// grad[p] = sum over waves of partial[w][p] in wave order; loss = sum of the wave losses / 3n.
__global__ void k_mlp_reduce(const float* __restrict__ partial, const float* __restrict__ loss_part, int nwaves,
                             long long n, float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPARAM) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += partial[(long long)w * MLP_NPARAM + p];
        grad[p] = s;
    }
    if (p == 0 && loss) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += loss_part[w];
        *loss = s / (3.0f * (float)n);
    }
}

// Adam on the FP32 master weights; refreshes their bf16 copies.
__global__ void k_mlp_adam(MLPArgs M, const float* __restrict__ grad, float lr, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float g = grad[p];
    const float m = 0.9f * M.m[p] + 0.1f * g;
    const float v = 0.999f * M.v[p] + 0.001f * g * g;
    M.m[p] = m;
    M.v[p] = v;
    const float w = M.master[p] - lr * (m * c1) / (sqrtf(v * c2) + 1e-8f);
    M.master[p] = w;
    M.wbf[p] = bf16_bits(w);
}

__global__ void k_mlp_round(MLPArgs M)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPARAM) M.wbf[p] = bf16_bits(M.master[p]);
}

}  // namespace

int launch_mlp_forward(const MLPArgs& M, const float* feats, long long n, float* logits, hipStream_t s)
{
    if (n <= 0) return 0;
    long long tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)(tiles < 4096 ? tiles : 4096);
    hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(64), 0, s, M, feats, n, logits);
    return (int)hipGetLastError();
}

int mlp_grad_waves(long long n)
{
    const long long chunks = (n + 31) / 32;
    return (int)(chunks < 512 ? chunks : 512);
}

int launch_mlp_grad(const MLPArgs& M, const float* feats, const unsigned char* labels, long long n, float* partial,
                    float* loss_part, float* grad, float* loss, hipStream_t s)
{
    if (n <= 0) return 0;
    const int waves = mlp_grad_waves(n);
    hipLaunchKernelGGL(k_mlp_grad, dim3(waves), dim3(64), 0, s, M, feats, labels, n, partial, loss_part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, partial, loss_part, waves, n,
                       grad, loss);
    return (int)hipGetLastError();
}

int launch_mlp_adam(const MLPArgs& M, const float* grad, float lr, int t, hipStream_t s)
{
    const float c1 = 1.0f / (1.0f - powf(0.9f, (float)t));
    const float c2 = 1.0f / (1.0f - powf(0.999f, (float)t));
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, M, grad, lr, c1, c2);
    return (int)hipGetLastError();
}

int launch_mlp_round(const MLPArgs& M, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_round, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, M);
    return (int)hipGetLastError();
}

}  // namespace fsa
