// Learned TENO5 sub-stencil selector: parameter layout and launchers.
#pragma once

#include "fsa_impl.hpp"

namespace fsa {

// 15 -> 32 -> 32 -> 3; flat parameters W1[15][32], b1[32], W2[32][32], b2[32], W3[32][3], b3[3]
constexpr int MLP_NIN = 15, MLP_NH = 32, MLP_NOUT = 3;
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_NIN * MLP_NH;     // 480
constexpr int MLP_W2 = MLP_B1 + MLP_NH;               // 512
constexpr int MLP_B2 = MLP_W2 + MLP_NH * MLP_NH;      // 1536
constexpr int MLP_W3 = MLP_B2 + MLP_NH;               // 1568
constexpr int MLP_B3 = MLP_W3 + MLP_NH * MLP_NOUT;    // 1664
constexpr int MLP_NPARAM = MLP_B3 + MLP_NOUT;         // 1667

struct MLPArgs {
    float* master;         // FP32 parameters (biases are read from here)
    unsigned short* wbf;   // bf16 copies of the parameters (weights are read from here)
    float* m;              // Adam moments
    float* v;
};

// Learned flags of every face of a 2D state (see k_faces2d.hip).
struct FlagArgs {
    const double* Q;
    long long step;
    const unsigned long long* alpha_bits;  // global LF speeds of Q
    MLPArgs M;
    float zthr;                            // confidence min_k |2 sigma(z_k) - 1| >= c  <=>
                                           // min_k |z_k| >= ln((1 + c) / (1 - c))
    unsigned* flags_x;                     // [(nx+1) ny]: side 0 pattern | side 1 pattern << 16
    unsigned* flags_y;                     // [nx (ny+1)]
    unsigned long long* counters;          // accumulated per block [flags2d_blocks][3]: face sides,
                                           // fallback sides, significant sides
    const float* qrange;                   // if set: deviation ranges of Q per stage-kernel strip and
    int qr_ty, qr_ncolx, qr_w;             // segment (rows per segment, strips per row of segments,
                                           // columns per strip)
};

struct HarvestArgs {
    const double* Q;
    long long step;
    const unsigned long long* alpha_bits;
    double keep_rate;                      // fraction of all-kept sides written
    unsigned long long seed;
    long long max_out;
    float* feats;                          // [max_out][16]
    unsigned char* labels;                 // [max_out]
    int* block_count;
    long long* block_offset;
    long long* total;                      // selected sides (may exceed max_out)
};

long long flags2d_blocks(const Grid& G);
int launch_flags2d(const KConst* K, const Grid& G, const FlagArgs& A, hipStream_t s);
long long harvest2d_blocks(const Grid& G);
// 3D: the faces of the three directions; blocks of both passes (3 x faces / 256).
long long harvest3d_blocks(const Grid& G);
int launch_harvest3d(const KConst* K, const Grid& G, const HarvestArgs& H, hipStream_t s);
int launch_harvest2d(const KConst* K, const Grid& G, const HarvestArgs& H, hipStream_t s);

int launch_mlp_forward(const MLPArgs& M, const float* feats, long long n, float* logits, hipStream_t s);
int mlp_grad_waves(long long n);
int launch_mlp_grad(const MLPArgs& M, const float* feats, const unsigned char* labels, long long n, float* partial,
                    float* loss_part, float* grad, float* loss, hipStream_t s);
int launch_mlp_adam(const MLPArgs& M, const float* grad, float lr, int t, hipStream_t s);
int launch_mlp_round(const MLPArgs& M, hipStream_t s);

}  // namespace fsa
