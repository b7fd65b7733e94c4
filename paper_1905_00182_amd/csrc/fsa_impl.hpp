// Internal interfaces between the C-ABI layer (fsa_api.hip) and the kernel launchers.
#pragma once

#include "fsa_dev.hpp"

namespace fsa {

// Arguments of the fused right-hand-side / stage kernels.
struct StageArgs {
    const double* Qs;                      // state the right-hand side is evaluated on
    const double* Qn;                      // step-start state (used only when ca != 0; 2D: loaded
                                           // in every stage, so never null there)
    double* out;                           // L (mode_rhs) or ca Qn + cb (Qs + dt L)
    const unsigned long long* alpha_bits;  // global LF speeds of Qs, as bit patterns [3]
    const double* fwin;                    // IB force density on the window box [dim][cells]
    int wlo[3];                            // window box origin (cell indices)
    int wn[3];                             // window box extent
    double ca, cb, dt;
    int mode_rhs;
    int ty;                                // rows (2D) per wave segment
    unsigned long long* alpha_part;        // if set: per wave, NaN-propagating max of |u_d| + c of
                                           // the output, [wave][3] (reduced by launch_alpha_final)
    long long step;                        // step counter (inflow-noise counter)
    double t;                              // time of the stage (periodic pressure source)
    const unsigned* flags_x;               // learned form: keep patterns of the x faces
    const unsigned* flags_y;               // and of the y faces
    float* qrange;                         // learned form, if set (with alpha_part): per strip and
                                           // segment [segment][strip][8], the least and the largest
                                           // FP32 deviation of rho, u, v, p of the cells written
    const double* ghosts;                  // 2D: inflow ghost table of this step (required when a
                                           // side is an inflow; see launch_inflow_ghosts2d)
    int nrbc;                              // bit 2d+s: side s of direction d is non-reflecting; the
                                           // stage kernels leave out the convective term along d
                                           // at its boundary cells (launch_nrbc adds its
                                           // characteristic form)
    unsigned* dbg_x;                       // if set (FP64 TENO5 only): the keep pattern of every
    unsigned* dbg_y;                       // x, y (and z) face this launch reconstructs, bits
    unsigned* dbg_z;                       // 3c+k (side +) and 16+3c+k (side -), face layout of
                                           // launch_stage2d / launch_stage3d
    int arow0, arow1;                      // layers along the last direction (y in 2D, z in 3D)
                                           // whose cells enter the wave-speed partials
};

// Arguments of the per-stage immersed-boundary kernel.
struct IBArgs {
    const double* Qs;
    int nm;
    const double* X;       // [dim][nm]
    const double* dV;      // [nm]
    const double* U;       // [dim][nm]
    int motion;            // 0 static, 1 rotating, 2 external
    double omega;
    double* xi;            // penalty integral (stage value)
    double* xi_out;        // its update (== xi: in place; ib_stage_fused launches need another
                           // buffer, which then holds the new value)
    double* xi_n;          // penalty integral at the step start
    double* F;             // penalty force [dim][nm]
    int stage;             // 0: right-hand side only; 1..3: SSP-RK3 stage
    double ca, cb, dt;
    double alpha, beta;    // penalty constants
    double* fwin;          // out: spread force density on the window box
    int wlo[3], wn[3];
    const int* cell_start; // CSR window cell -> markers (increasing marker index)
    const int* cell_marker;
    const double* cell_w;  // per CSR entry: W(cell) dV_k / h^dim
    const int* mj0;        // per marker: first support cell per direction [nm][3]
    const double* mw;      // per marker: one-dimensional weights [nm][dim][4]
    // optional: a wave-speed reduction (as launch_alpha_final) carried out by one extra
    // block of the window launch; part == nullptr for none
    const unsigned long long* alpha_part;
    long long alpha_n;
    unsigned long long* alpha_bits;
};

int launch_stage2d(const KConst* K, const Grid& G, int scheme, int precision, const StageArgs& A, hipStream_t s);
// Non-reflecting side `side` (0 low, 1 high) of direction d: at its boundary cells, out +=
// cb dt C (mode_rhs: out += C), C the characteristic form of the convective term along d of
// A.Qs (see fsa.h).  One launch per side; sides sharing a corner cell run one after another.
int launch_nrbc(const KConst* K, const Grid& G, int d, int side, const StageArgs& A, hipStream_t s);
// 2D inflow ghost states of steps step0 .. step0 + nsteps - 1 (the far field with the
// seeded perturbation, the values the boundary rule gives the four ghost layers of every
// inflow side) into g, one table of inflow_ghosts2d_elems per step, each
// [component][side][depth - 1][position along the side] with the position stride
// max(nx, ny); sides that are not inflows are left unwritten.
long long inflow_ghosts2d_elems(const Grid& G);
bool has_inflow(const Grid& G);
int launch_inflow_ghosts2d(const KConst* K, const Grid& G, long long step0, int nsteps, double* g, hipStream_t s);
long long stage2d_waves(const Grid& G, int ty);
// 3D: stress pass into `stress` ([9][(nx+4)(ny+4)(nz+4)] of T = double, or float in the
// precision form), face-flux passes into `faces` (faces3d_elems of T; variables = 1:
// characteristic-wise, FP64 only), then the stage pass; one wave-speed partial per block of
// the stage pass.
int launch_stage3d(const KConst* K, const Grid& G, int scheme, int precision, int variables, const StageArgs& A,
                   void* stress, void* faces, hipStream_t s);
// 2D in three passes (the characteristic-wise reconstruction, FP64): stress pass into
// `stress` (pass2d_stress_elems doubles; skipped without viscosity), characteristic-wise
// face-flux passes into `faces` (pass2d_face_elems doubles), then the stage pass; one
// wave-speed partial per block of the stage pass (pass2d_blocks).
int launch_pass2d(const KConst* K, const Grid& G, int scheme, int terms, double mu, const StageArgs& A,
                  double* stress, double* faces, hipStream_t s);
long long pass2d_stress_elems(const Grid& G);
// Blocks of one domain on one GPU: a list of contiguous double runs copied in one launch
// (entries in device memory, max_count the longest run), and the NaN-propagating maximum of
// nb wave-speed slots written into nb others.
struct CopyEntry {
    const double* src;
    double* dst;
    long long count;
};
int launch_copy_list(const CopyEntry* d_list, int n, long long max_count, hipStream_t s);
int launch_amax_blocks(unsigned long long* const* d_in, unsigned long long* const* d_out, int nb, hipStream_t s);
long long pass2d_face_elems(const Grid& G);
long long pass2d_blocks(const Grid& G);
long long stress3d_elems(const Grid& G);
long long faces3d_elems(const Grid& G);
long long stage3d_blocks(const Grid& G);
int stage2d_ncolx(int nx);
int stage2d_strip_width();
// Wave speeds max over cells of |u_d| + c of Q into bits[3]: per-block partials in part
// (ALPHA_MAX_BLOCKS x 3), then launch_alpha_final.  No same-address atomics.
constexpr int ALPHA_MAX_BLOCKS = 2048;
// Blocks (partials) launch_alpha uses for grid G: one per 256 cells, at most ALPHA_MAX_BLOCKS.
long long alpha_blocks(const Grid& G);
int launch_alpha(const Grid& G, const Phys& P, const double* Q, unsigned long long* part, unsigned long long* bits,
                 hipStream_t s);
// The same over the layers row0 .. row1 - 1 along the last direction only.
int launch_alpha_rows(const Grid& G, const Phys& P, const double* Q, int row0, int row1, unsigned long long* part,
                      unsigned long long* bits, hipStream_t s);
// bits[d] = NaN-propagating max over n partials part[k * 3 + d] (d < 3).
int launch_alpha_final(const unsigned long long* part, long long n, unsigned long long* bits, hipStream_t s);
int launch_ib_stage(const Grid& G, const Phys& P, const IBArgs& A, hipStream_t s);
// Whether launch_ib_stage takes the one-launch form (which writes the integral's update to a
// buffer other than xi).
bool ib_stage_fused(const Grid& G, int nm);
// Field totals out[m] = sum_cells q_m h^dim (deterministic order; part: totals_part_size doubles)
// and the dilatation div u at every cell.
int totals_part_size(int nq);
int launch_totals(const Grid& G, int nq, const double* Q, double* part, double* out, hipStream_t s);
int launch_dilatation(const Grid& G, const Phys& P, const double* Q, long long step, double* out, hipStream_t s);
// A marker placement: the staged arrays (device copies of one host block) are put in place
// and the per-marker and per-entry weights computed from them.
struct WindowUpdate {
    const double* sX;         // staged positions [dim][nm]
    const double* sU;         // staged velocities [dim][nm]
    const int* s_start;       // staged CSR window cell -> markers: starts [wcells + 1]
    const int* s_marker;      // markers per entry [nent] (increasing per cell)
    const int* s_cell;        // window cell per entry [nent]
    int nm;
    long long wcells, nent;
    int wlo[3], wn[3];
    const double* dV;         // [nm]
    double* X;                // out: positions, velocities, CSR lists
    double* U;
    int* cell_start;
    int* cell_marker;
    int* mj0;                 // out: per marker first support cell [nm][3]
    double* mw;               // out: per marker one-dimensional weights [nm][dim][4]
    double* cell_w;           // out: per entry W(cell) dV_k / h^dim
};
int launch_ib_place(const Grid& G, const WindowUpdate& W, hipStream_t s);
// n16 16-byte words from src (host memory visible to the device, e.g. coherent pinned) to dst.
int launch_stage_in(const void* src, void* dst, long long n16, hipStream_t s);
int launch_interp(const Grid& G, int npts, const double* X, const double* field, int ncomp, double* out,
                  hipStream_t s);
int launch_spread(const Grid& G, const IBArgs& A, const double* F, int ncomp, double* field, double scale,
                  hipStream_t s);
int launch_probe_dp(const Grid& G, const Phys& P, int np, const double* Xp, const double* Q, double* dp,
                    hipStream_t s);

}  // namespace fsa
