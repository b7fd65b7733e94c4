// C-ABI entry points (include/fsa.h): argument checking, device buffers, and the enqueue
// order of the kernels for one right-hand side and one SSP-RK3 step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "fsa.h"
#include "fsa_impl.hpp"
#include "fsa_mlp.hpp"

using namespace fsa;

// steps of inflow ghost tables formed per launch
constexpr int GHOST_STEPS = 16;

struct fsa_ctx {
    fsa_desc d;
    Grid G;
    Phys P;
    KConst* dK = nullptr;                // device copy of the constants
    hipStream_t stream = nullptr;
    int device = 0;
    int nq = 0;
    long long ncell = 0;
    int ty = 16;                         // rows per wave segment of the 2D stage kernel
    double* Qa = nullptr;                // RK stage buffers
    double* Qb = nullptr;
    unsigned long long* abits = nullptr; // alpha slots: [4][3]
    unsigned long long* apart = nullptr; // per-block / per-wave partial maxima [apart_n][3]
    unsigned char* stress3d = nullptr;   // 3D: tau and b with two ghost layers, [9][ext cells] of T;
                                         // 2D characteristic-wise: [5][ext cells] of double
    unsigned char* faces3d = nullptr;    // 3D: face fluxes of the three directions, [5][faces] of T
    double* tot_part = nullptr;          // diagnostics: per-block partial totals
    double* tot_out = nullptr;
    long long apart_n = 0;
    long long fin_n = 0;                 // deferred wave-speed reduction: partials in apart, and
    unsigned long long* fin_bits = nullptr;  // the slot it writes (0: none pending)
    unsigned long long* h_abits = nullptr;  // pinned mirror of the last step's slots
    hipEvent_t ev_alpha = nullptr;
    bool alpha_pending = false;
    int nonfinite = 0;
    int last_slot = 0;                   // slot holding the wave speeds of the last state
    const double* advanced = nullptr;    // the state the last step call left (slot 0 holds its
                                         // wave speeds; null: none, or slot 0 reused since)
    // markers
    int nm = 0;
    int motion = 0;
    double omega = 0.0;
    double *X = nullptr, *dV = nullptr, *U = nullptr, *xi = nullptr, *xi_n = nullptr, *F = nullptr;
    double* xi2 = nullptr;               // the other penalty-integral buffer (one-launch IB stages
                                         // write the update there; the two then swap)
    std::vector<double> hX;
    int wlo[3] = {0, 0, 0}, wn[3] = {0, 0, 0};
    long long wcells = 0;
    double* fwin = nullptr;
    int* cell_start = nullptr;
    int* cell_marker = nullptr;
    double* cell_w = nullptr;            // per CSR entry spreading weight
    int* mj0 = nullptr;                  // per marker support origin
    double* mw = nullptr;                // per marker one-dimensional weights
    long long cap_wcells = 0;            // window capacities in the workspace (desc.max_window_cells,
    long long cap_entries = 0;           // 4^dim entries per marker)
    int cap_markers = 0;                 // desc.max_markers, desc.max_probes
    int cap_probes = 0;
    char* h_stage = nullptr;             // coherent pinned staging of marker placements, two
    const char* h_stage_dev = nullptr;   // halves used in turn (and its device-side address)
    char* d_stage = nullptr;             // its device twin (same size and layout)
    size_t stage_bytes = 0;              // bytes per half (the device twin holds one)
    int stage_idx = 0;                   // the half the next placement fills
    hipEvent_t ev_stage[2] = {nullptr, nullptr};  // recorded after the launch that read a half
    bool stage_pending[2] = {false, false};
    // probes
    int np = 0;
    double* Xp = nullptr;
    double t = 0.0;
    long long step = 0;
    // learned selector
    float* mlp_master = nullptr;
    unsigned short* mlp_wbf = nullptr;
    float* mlp_m = nullptr;
    float* mlp_v = nullptr;
    float* mlp_grad = nullptr;
    float* mlp_partial = nullptr;
    float* mlp_loss_part = nullptr;
    int mlp_t = 0;
    bool mlp_ready = false;
    double conf_threshold = 0.8;
    unsigned* flags_x = nullptr;
    unsigned* flags_y = nullptr;
    unsigned long long* counters = nullptr;
    float* qrange = nullptr;             // learned form: deviation ranges of the last stage output
    double* ghosts = nullptr;            // 2D with an inflow side: inflow ghost tables of
    long long ghosts_step = -1;          // steps ghosts_step .. + GHOST_STEPS - 1 (-1: none)
    const double* qrange_of = nullptr;   // the buffer they describe (null: none valid)
    int qrange_ty = 0;                   // rows per segment they were taken with
    int arow0 = 0, arow1 = 0;            // layers along the last direction whose cells enter the
                                         // wave speeds (all of them; a block: its own layers)
    bool quiet_tiles = true;             // flags passes may skip quiet tiles (FSA_NO_QUIET_TILES=1:
                                         // never; tests compare the two)
    int* hv_count = nullptr;
    long long* hv_offset = nullptr;
    long long* hv_total = nullptr;
    unsigned* dbg_bits = nullptr;        // test read-out of the TENO5 keep patterns (or null)
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> tev;   // pairs (start, stop) per timed launch
    size_t tused = 0;
    std::string err;
};

namespace {

int fail(fsa_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

int hipcheck(fsa_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return FSA_OK;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return fail(c, FSA_EDEVICE, buf);
}

#define HIPCHK(ctx, expr)                                          \
    do {                                                           \
        int rc_ = hipcheck((ctx), (expr), #expr);                  \
        if (rc_ != FSA_OK) return rc_;                             \
    } while (0)

// Bump allocation of the context's device buffers from the caller's workspace, 256-byte
// aligned (base null: only the byte count).
struct Carve {
    char* base;
    size_t off;
    template <class T>
    T* take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

// Bytes of one marker placement staged for the device: X and U, the CSR starts and, per
// entry, its marker and window cell.
size_t stage_need(int dim, long long nm, long long wcells, long long nent)
{
    const size_t bx = sizeof(double) * (size_t)dim * (size_t)nm, bs = sizeof(int) * (size_t)(wcells + 1),
                 bm = sizeof(int) * (size_t)nent;
    return (2 * bx + bs + 2 * bm + 15) / 16 * 16;
}

// Every device buffer of context c (its desc, grid and capacities set) in the workspace at
// base; returns the bytes used.  The layout depends on the descriptor only.
size_t carve(fsa_ctx* c, char* base)
{
    Carve W{base, 0};
    const fsa_desc& d = c->d;
    const int dim = d.dim;
    const Grid& G = c->G;
    const size_t nq = (size_t)(dim + 2), nc = (size_t)G.ncell;
    c->dK = W.take<KConst>(1);
    c->Qa = W.take<double>(nq * nc);
    c->Qb = W.take<double>(nq * nc);
    c->abits = W.take<unsigned long long>(12);
    const bool pass2d = dim == 2 && d.variables == FSA_CHARACTERISTIC;
    c->apart_n = std::max<long long>(ALPHA_MAX_BLOCKS, dim == 3 ? stage3d_blocks(G) : stage2d_waves(G, 4));
    if (pass2d) c->apart_n = std::max(c->apart_n, pass2d_blocks(G));
    c->apart = W.take<unsigned long long>(3 * (size_t)c->apart_n);
    c->ghosts = (dim == 2 && has_inflow(G)) ? W.take<double>((size_t)GHOST_STEPS * inflow_ghosts2d_elems(G)) : nullptr;
    if (dim == 3) {
        const size_t tsize = d.precision == FSA_MIXED32 ? sizeof(float) : sizeof(double);
        c->stress3d = W.take<unsigned char>((size_t)stress3d_elems(G) * tsize);
        c->faces3d = W.take<unsigned char>((size_t)faces3d_elems(G) * tsize);
    } else if (pass2d) {
        c->stress3d = W.take<unsigned char>((size_t)pass2d_stress_elems(G) * sizeof(double));
        c->faces3d = W.take<unsigned char>((size_t)pass2d_face_elems(G) * sizeof(double));
    }
    c->tot_part = W.take<double>((size_t)totals_part_size((int)nq));
    c->tot_out = W.take<double>(5);
    // the selector network (any context may run or train it)
    c->mlp_master = W.take<float>(MLP_NPARAM);
    c->mlp_wbf = W.take<unsigned short>(MLP_NPARAM);
    c->mlp_m = W.take<float>(MLP_NPARAM);
    c->mlp_v = W.take<float>(MLP_NPARAM);
    c->mlp_grad = W.take<float>(MLP_NPARAM);
    c->mlp_partial = W.take<float>((size_t)512 * MLP_NPARAM);
    c->mlp_loss_part = W.take<float>(512);
    if (dim == 2) {
        c->counters = W.take<unsigned long long>(3 * (size_t)flags2d_blocks(G));
        c->qrange = W.take<float>(8 * (size_t)stage2d_waves(G, 4));
    }
    {
        const size_t nb = (size_t)(dim == 2 ? harvest2d_blocks(G) : harvest3d_blocks(G));
        c->hv_count = W.take<int>(nb);
        c->hv_offset = W.take<long long>(nb);
        c->hv_total = W.take<long long>(1);
    }
    if (d.precision == FSA_LEARNED32) {
        c->flags_x = W.take<unsigned>((size_t)(G.n[0] + 1) * G.n[1]);
        c->flags_y = W.take<unsigned>((size_t)G.n[0] * (G.n[1] + 1));
    }
    // markers, their window and the device twin of the placement staging
    const size_t cm = (size_t)c->cap_markers, ln = (size_t)dim * cm;
    c->X = W.take<double>(ln);
    c->U = W.take<double>(ln);
    c->xi = W.take<double>(ln);
    c->xi2 = W.take<double>(ln);
    c->xi_n = W.take<double>(ln);
    c->F = W.take<double>(ln);
    c->dV = W.take<double>(cm);
    c->mj0 = W.take<int>(3 * cm);
    c->mw = W.take<double>(ln * 4);
    c->fwin = W.take<double>((size_t)dim * (size_t)c->cap_wcells);
    c->cell_start = W.take<int>((size_t)c->cap_wcells + 1);
    c->cell_marker = W.take<int>((size_t)c->cap_entries);
    c->cell_w = W.take<double>((size_t)c->cap_entries);
    c->stage_bytes = cm ? stage_need(dim, (long long)cm, c->cap_wcells, c->cap_entries) : 0;
    c->d_stage = W.take<char>(c->stage_bytes);
    c->Xp = W.take<double>((size_t)dim * (size_t)c->cap_probes);
    return W.off + 256;   // (room to align the base up)
}

int validate(const fsa_desc* d, std::string& why)
{
    if (!d) { why = "desc is NULL"; return FSA_EINVAL; }
    if (d->dim != 2 && d->dim != 3) { why = "dim must be 2 or 3"; return FSA_EINVAL; }
    for (int k = 0; k < d->dim; ++k)
        if (d->n[k] < 1) { why = "n must be positive"; return FSA_EINVAL; }
    if (d->dim == 2 && d->n[2] != 1) { why = "n[2] must be 1 in 2D"; return FSA_EINVAL; }
    const double nc = (double)d->n[0] * d->n[1] * (d->dim == 3 ? d->n[2] : 1);
    if (nc * (d->dim + 2) > 9.0e18 || nc > 2.0e9) { why = "grid too large"; return FSA_EINVAL; }
    if (!(d->h > 0.0) || !std::isfinite(d->h)) { why = "h must be positive"; return FSA_EINVAL; }
    for (int k = 0; k < 3; ++k)
        for (int s = 0; s < 2; ++s) {
            if (k >= d->dim) continue;
            if (d->bc[k][s] < FSA_BC_PERIODIC || d->bc[k][s] > FSA_BC_NONREFLECT) { why = "bad bc"; return FSA_EINVAL; }
            if (d->bc[k][s] == FSA_BC_NONREFLECT && d->n[k] < 3) {
                why = "a non-reflecting side needs at least 3 cells along its normal";
                return FSA_EINVAL;
            }
            if ((d->bc[k][0] == FSA_BC_PERIODIC) != (d->bc[k][1] == FSA_BC_PERIODIC)) {
                why = "periodic must be set on both sides";
                return FSA_EINVAL;
            }
            if (d->sponge_width[k][s] < 0.0) { why = "negative sponge width"; return FSA_EINVAL; }
        }
    if (!(d->gamma > 1.0)) { why = "gamma must exceed 1"; return FSA_EINVAL; }
    if (d->mu < 0.0) { why = "mu must be non-negative"; return FSA_EINVAL; }
    if (d->scheme != FSA_WENO5JS && d->scheme != FSA_TENO5) { why = "bad scheme"; return FSA_EINVAL; }
    if (d->precision != FSA_FP64 && d->precision != FSA_MIXED32 && d->precision != FSA_LEARNED32) {
        why = "bad precision";
        return FSA_EINVAL;
    }
    if (d->dim == 3 && d->precision == FSA_LEARNED32) { why = "the learned form is built for 2D"; return FSA_EUNSUPPORTED; }
    if (d->variables != FSA_COMPONENT && d->variables != FSA_CHARACTERISTIC) { why = "bad variables"; return FSA_EINVAL; }
    for (int k = 0; k < d->dim; ++k) {
        if (d->global_n[k] == 0) {
            if (d->origin[k] != 0) { why = "origin without global_n"; return FSA_EINVAL; }
            continue;
        }
        if (d->global_n[k] < 1 || d->origin[k] < -FSA_HALO || d->origin[k] + d->n[k] > d->global_n[k] + FSA_HALO) {
            why = "the block must lie within global_n (up to FSA_HALO cells beyond, for a wrapped halo)";
            return FSA_EINVAL;
        }
    }
    if (d->variables == FSA_CHARACTERISTIC && d->precision != FSA_FP64) {
        why = "the characteristic-wise reconstruction is built in FP64";
        return FSA_EUNSUPPORTED;
    }
    if (d->selector_stride != 0 && d->selector_stride != 1 && d->selector_stride != 3) {
        why = "selector_stride must be 0, 1 or 3";
        return FSA_EINVAL;
    }
    if (!(d->prim_inf[0] > 0.0) || !(d->prim_inf[4] > 0.0)) { why = "far field must have rho, p > 0"; return FSA_EINVAL; }
    if (!std::isfinite(d->src_amp) || !std::isfinite(d->src_b) || !std::isfinite(d->src_omega) ||
        !std::isfinite(d->src_x[0]) || !std::isfinite(d->src_x[1]) || !std::isfinite(d->src_x[2])) {
        why = "non-finite source parameters";
        return FSA_EINVAL;
    }
    if (d->src_amp != 0.0 && d->dim != 3) { why = "the periodic pressure source is built for 3D"; return FSA_EUNSUPPORTED; }
    return FSA_OK;
}

void build_consts(fsa_ctx* c)
{
#pragma clang fp contract(off)
    const fsa_desc& d = c->d;
    Grid& G = c->G;
    G.dim = d.dim;
    for (int k = 0; k < 3; ++k) {
        G.n[k] = k < d.dim ? d.n[k] : 1;
        G.lo[k] = d.lo[k];
        G.bc[k][0] = d.bc[k][0];
        G.bc[k][1] = d.bc[k][1];
    }
    G.ncell = (long long)G.n[0] * G.n[1] * G.n[2];
    for (int k = 0; k < 3; ++k) {
        const bool placed = k < d.dim && d.global_n[k] > 0;
        G.org[k] = placed ? d.origin[k] : 0;
        G.gn[k] = placed ? d.global_n[k] : G.n[k];
    }
    G.gncell = (long long)G.gn[0] * G.gn[1] * G.gn[2];
    G.h = d.h;
    G.inv_h = 1.0 / d.h;
    Phys& P = c->P;
    P.gamma = d.gamma;
    P.gm1 = d.gamma - 1.0;
    P.inv_gm1 = 1.0 / (d.gamma - 1.0);
    P.mu = d.mu;
    for (int k = 0; k < 5; ++k) P.prim_inf[k] = d.prim_inf[k];
    {
        const double rho = d.prim_inf[0];
        double ke = 0.0;
        P.q_inf[0] = rho;
        for (int a = 0; a < d.dim; ++a) {
            P.q_inf[1 + a] = rho * d.prim_inf[1 + a];
            ke += d.prim_inf[1 + a] * d.prim_inf[1 + a];
        }
        P.q_inf[d.dim + 1] = d.prim_inf[4] / (d.gamma - 1.0) + 0.5 * rho * ke;
        for (int a = d.dim + 2; a < 5; ++a) P.q_inf[a] = 0.0;
    }
    P.inflow_amp = d.inflow_amp;
    P.seed = d.seed;
    for (int k = 0; k < 3; ++k)
        for (int s = 0; s < 2; ++s) {
            P.sw[k][s] = k < d.dim ? d.sponge_width[k][s] : 0.0;
            P.inv_sw[k][s] = P.sw[k][s] > 0.0 ? 1.0 / P.sw[k][s] : 0.0;
        }
    P.e_inf = d.prim_inf[4] / P.gm1;
    P.sigma = d.sponge_sigma;
    P.weno_eps = d.weno_eps;
    P.teno_ct = d.teno_ct;
    P.teno_eps = d.teno_eps;
    P.terms = d.terms;
    P.src_amp = d.src_amp;
    P.src_bl2 = d.src_b * std::log(2.0);
    P.src_omega = d.src_omega;
    for (int k = 0; k < 3; ++k) P.src_x[k] = d.src_x[k];
}

// Physical fluxes of the far-field state per direction (the precision form stores split
// fluxes relative to these).
void far_field_fluxes(const fsa_ctx* c, KConst& k)
{
#pragma clang fp contract(off)
    const int dim = c->d.dim;
    const double* q = c->P.q_inf;
    const double rho = c->d.prim_inf[0], p = c->d.prim_inf[4];
    double* F[3] = {k.Fx_inf, k.Fy_inf, k.Fz_inf};
    for (int d = 0; d < 3; ++d) {
        for (int m = 0; m < 5; ++m) F[d][m] = 0.0;
        if (d >= dim) continue;
        const double ud = q[1 + d] / rho;
        F[d][0] = q[1 + d];
        for (int a = 0; a < dim; ++a) F[d][1 + a] = q[1 + a] * ud + (a == d ? p : 0.0);
        F[d][dim + 1] = (q[dim + 1] + p) * ud;
    }
    const double cinf = std::sqrt(c->d.gamma * p / rho);
    k.sig[0] = 1e-8 * rho;
    k.sig[1] = 1e-8 * cinf;
    k.sig[2] = 1e-8 * rho * cinf * cinf;
}

// Rows per wave segment of the 2D stage kernel.  The best value depends on how the waves
// fill the chip (occupancy, tail of the last wave round), which no simple model predicts, so
// it is measured: on the first launch of a context every candidate is timed on the caller's
// data as an SSP-RK3 stage into a scratch buffer, and the fastest is kept.  The
// segmentation changes no result: every face is computed from the same inputs whichever
// segment computes it.  FSA_STAGE_TY fixes the value instead (tuning runs, tests).
int env_ty()
{
    if (const char* e = std::getenv("FSA_STAGE_TY")) {
        const int v = std::atoi(e);
        if (v >= 4 && v <= 4096) return v;
    }
    return 0;
}

bool support_inside(const fsa_ctx* c, int n, const double* X)
{
    for (int k = 0; k < n; ++k)
        for (int d = 0; d < c->d.dim; ++d) {
            const double x = X[(size_t)d * n + k];
            if (!std::isfinite(x)) return false;
            const double r0 = (x - c->d.lo[d]) / c->d.h - 0.5;
            const double j0 = std::floor(r0) - 1.0 - (double)c->G.org[d];   // (local cell index)
            if (j0 < 0.0 || j0 + 3.0 > (double)(c->G.n[d] - 1)) return false;
        }
    return true;
}

IBArgs ib_args(const fsa_ctx* c);
int tune_ty(fsa_ctx* c, const StageArgs& S0);
int enqueue_flags(fsa_ctx* c, const double* Qs, const unsigned long long* bits, unsigned* fx, unsigned* fy);

// Window box over all marker supports (c->hX) and the CSR list window cell -> markers (in
// marker order): index bookkeeping only, on the host.
int window_lists(fsa_ctx* c, int* wlo, int* wn, std::vector<int>& count, std::vector<int>& marker,
                 std::vector<int>& ecell)
{
    const int dim = c->d.dim, n = c->nm;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    std::vector<int> j0((size_t)n * 3, 0);
    for (int k = 0; k < 3; ++k) { wlo[k] = 0; wn[k] = 1; }
    for (int d = 0; d < dim; ++d) {
        lo[d] = 1 << 30;
        hi[d] = -(1 << 30);
        for (int k = 0; k < n; ++k) {
            const double r0 = (c->hX[(size_t)d * n + k] - c->d.lo[d]) / c->d.h - 0.5;
            const int j = (int)std::floor(r0) - 1 - c->G.org[d];   // (local cell index)
            j0[(size_t)k * 3 + d] = j;
            lo[d] = std::min(lo[d], j);
            hi[d] = std::max(hi[d], j + 3);
        }
        wlo[d] = lo[d];
        wn[d] = hi[d] - lo[d] + 1;
    }
    const long long wcells = (long long)wn[0] * wn[1] * wn[2];
    if (wcells > (1ll << 26)) return fail(c, FSA_EINVAL, "marker supports span too large a box");
    count.assign((size_t)wcells + 1, 0);
    const int mz = dim == 3 ? 4 : 1;
    auto cell_of = [&](int k, int dx, int dy, int dz) {
        const long long i = j0[(size_t)k * 3] + dx - wlo[0];
        const long long j = j0[(size_t)k * 3 + 1] + dy - wlo[1];
        const long long l = dim == 3 ? j0[(size_t)k * 3 + 2] + dz - wlo[2] : 0;
        return (l * wn[1] + j) * wn[0] + i;
    };
    for (int k = 0; k < n; ++k)
        for (int dz = 0; dz < mz; ++dz)
            for (int dy = 0; dy < 4; ++dy)
                for (int dx = 0; dx < 4; ++dx) count[(size_t)cell_of(k, dx, dy, dz) + 1]++;
    for (long long w = 0; w < wcells; ++w) count[(size_t)w + 1] += count[(size_t)w];
    std::vector<int> fillp(count.begin(), count.end() - 1);
    marker.assign((size_t)count[(size_t)wcells], 0);
    ecell.assign(marker.size(), 0);
    for (int k = 0; k < n; ++k)
        for (int dz = 0; dz < mz; ++dz)
            for (int dy = 0; dy < 4; ++dy)
                for (int dx = 0; dx < 4; ++dx) {
                    const long long w = cell_of(k, dx, dy, dz);
                    const int e = fillp[(size_t)w]++;
                    marker[(size_t)e] = k;
                    ecell[(size_t)e] = (int)w;
                }
    return FSA_OK;
}

// Marker positions X (c->hX holds the same) and velocities U (null: zero): the window box
// and its lists on the host, then one copy of a pinned staging block (X, U and the lists)
// into its device twin and one launch that puts them in place and computes the weights, both
// on the library's stream after the work already enqueued there.  The staging block has two
// halves used in turn; the host waits only for the copy that read the half it is about to
// fill (two placements back).  The window must fit the workspace's capacities.
int update_window_async(fsa_ctx* c, const double* X, const double* U)
{
    const int dim = c->d.dim, n = c->nm;
    int wlo[3], wn[3];
    std::vector<int> count, marker, ecell;
    int rc = window_lists(c, wlo, wn, count, marker, ecell);
    if (rc != FSA_OK) return rc;
    const long long wcells = (long long)wn[0] * wn[1] * wn[2], nent = (long long)marker.size();
    if (wcells > c->cap_wcells)
        return fail(c, FSA_EINVAL, "the markers' supports span " + std::to_string(wcells) +
                                       " cells, more than desc.max_window_cells (" + std::to_string(c->cap_wcells) + ")");
    if (nent > c->cap_entries) return fail(c, FSA_EINVAL, "more support entries than the workspace holds");
    const size_t bx = sizeof(double) * (size_t)dim * n, bs = sizeof(int) * count.size(),
                 bm = sizeof(int) * marker.size(), need = stage_need(dim, n, wcells, nent);
    if (need > c->stage_bytes || !c->h_stage) return fail(c, FSA_EINVAL, "marker staging exceeds its capacity");
    // the half this placement fills: the launch that read it last time must have ended
    const int half = c->stage_idx;
    c->stage_idx ^= 1;
    if (c->stage_pending[half]) {
        HIPCHK(c, hipEventSynchronize(c->ev_stage[half]));
        c->stage_pending[half] = false;
    }
    char* h = c->h_stage + half * c->stage_bytes;
    std::memcpy(h, X, bx);
    if (U) std::memcpy(h + bx, U, bx);
    else std::memset(h + bx, 0, bx);
    std::memcpy(h + 2 * bx, count.data(), bs);
    std::memcpy(h + 2 * bx + bs, marker.data(), bm);
    std::memcpy(h + 2 * bx + bs + bm, ecell.data(), bm);
    // (a copy kernel reading the coherent host block: a copy engine transfer would cost the
    // stream more than ten microseconds of waiting per placement)
    int e = launch_stage_in(c->h_stage_dev + half * c->stage_bytes, c->d_stage, (long long)(need / 16), c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "staging copy launch");
    HIPCHK(c, hipEventRecord(c->ev_stage[half], c->stream));
    c->stage_pending[half] = true;
    for (int k = 0; k < 3; ++k) {
        c->wlo[k] = wlo[k];
        c->wn[k] = wn[k];
    }
    c->wcells = wcells;
    WindowUpdate W;
    const char* d = c->d_stage;
    W.sX = (const double*)d;
    W.sU = (const double*)(d + bx);
    W.s_start = (const int*)(d + 2 * bx);
    W.s_marker = (const int*)(d + 2 * bx + bs);
    W.s_cell = (const int*)(d + 2 * bx + bs + bm);
    W.nm = n;
    W.wcells = wcells;
    W.nent = nent;
    for (int k = 0; k < 3; ++k) {
        W.wlo[k] = wlo[k];
        W.wn[k] = wn[k];
    }
    W.dV = c->dV;
    W.X = c->X;
    W.U = c->U;
    W.cell_start = c->cell_start;
    W.cell_marker = c->cell_marker;
    W.mj0 = c->mj0;
    W.mw = c->mw;
    W.cell_w = c->cell_w;
    e = launch_ib_place(c->G, W, c->stream);
    return e ? hipcheck(c, (hipError_t)e, "IB placement launch") : FSA_OK;
}

// First placement of the markers (c->hX, U; null U: zero), synchronously, with the window's
// force buffer cleared.
int build_window(fsa_ctx* c, const double* U)
{
    const int dim = c->d.dim, n = c->nm;
    c->wcells = 0;
    for (int k = 0; k < 3; ++k) { c->wlo[k] = 0; c->wn[k] = 1; }
    if (n == 0) { c->wn[0] = c->wn[1] = c->wn[2] = 0; return FSA_OK; }
    int rc;
    if ((rc = update_window_async(c, c->hX.data(), U)) != FSA_OK) return rc;
    HIPCHK(c, hipMemsetAsync(c->fwin, 0, sizeof(double) * (size_t)dim * c->cap_wcells, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->stage_pending[0] = c->stage_pending[1] = false;
    return FSA_OK;
}

IBArgs ib_args(const fsa_ctx* c)
{
    IBArgs A;
    std::memset(&A, 0, sizeof A);
    A.nm = c->nm;
    A.X = c->X;
    A.dV = c->dV;
    A.U = c->U;
    A.motion = c->motion;
    A.omega = c->omega;
    A.xi = c->xi;
    A.xi_out = c->xi;
    A.xi_n = c->xi_n;
    A.F = c->F;
    A.alpha = c->d.ib_alpha;
    A.beta = c->d.ib_beta;
    A.fwin = c->fwin;
    for (int k = 0; k < 3; ++k) {
        A.wlo[k] = c->wlo[k];
        A.wn[k] = c->wn[k];
    }
    A.cell_start = c->cell_start;
    A.cell_marker = c->cell_marker;
    A.cell_w = c->cell_w;
    A.mj0 = c->mj0;
    A.mw = c->mw;
    return A;
}

bool ib_active(const fsa_ctx* c) { return (c->d.terms & FSA_TERM_IB) && c->nm > 0; }

// Non-reflecting sides as a bit mask (bit 2d+s), 0 for none.
int nrbc_mask(const fsa_ctx* c)
{
    int m = 0;
    for (int d = 0; d < c->d.dim; ++d)
        for (int s = 0; s < 2; ++s)
            if (c->d.bc[d][s] == FSA_BC_NONREFLECT) m |= 1 << (2 * d + s);
    return m;
}

// After a stage kernel with non-reflecting sides: their characteristic terms, then the
// wave speeds of the corrected output into slot acc (the stage kernel took none).
int finish_nrbc(fsa_ctx* c, const StageArgs& S, int acc)
{
    for (int d = 0; d < c->d.dim; ++d)
        for (int side = 0; side < 2; ++side)
            if ((S.nrbc >> (2 * d + side)) & 1 && (c->d.terms & (FSA_TERM_CONV_X << d))) {
                int e = launch_nrbc(c->dK, c->G, d, side, S, c->stream);
                if (e) return hipcheck(c, (hipError_t)e, "non-reflecting boundary launch");
            }
    if (acc >= 0) {
        int e = launch_alpha_rows(c->G, c->P, S.out, S.arow0, S.arow1, c->apart, c->abits + 3 * acc, c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "alpha reduction launch");
    }
    return FSA_OK;
}

// One right-hand-side evaluation on Qs: (optionally) the wave-speed reduction of Qs into
// slot `in`, the penalty step, and the fused stencil/update kernel, which reads slot `in`,
// writes the wave speeds of its output into slot `acc` (per-wave partials, then a one-block
// reduction; slots of three doubles in abits; -1 = none).
// Next pair of timing events of the context (created on first use).
int timing_pair(fsa_ctx* c, hipEvent_t& t0, hipEvent_t& t1)
{
    if (c->tused + 2 > c->tev.size()) {
        for (int k = 0; k < 2; ++k) {
            hipEvent_t ev;
            HIPCHK(c, hipEventCreate(&ev));
            c->tev.push_back(ev);
        }
    }
    t0 = c->tev[c->tused];
    t1 = c->tev[c->tused + 1];
    c->tused += 2;
    return FSA_OK;
}

// A stage's wave-speed partials are reduced into its output slot by the next launch that
// can carry the reduction (the next stage's IB window launch), or on their own: before the
// next stage's kernels when there is no IB step, and at the end of a call.
void defer_alpha_final(fsa_ctx* c, long long n, int slot)
{
    c->fin_n = n;
    c->fin_bits = c->abits + 3 * slot;
}

int flush_alpha_final(fsa_ctx* c)
{
    if (c->fin_n <= 0) return FSA_OK;
    const int e = launch_alpha_final(c->apart, c->fin_n, c->fin_bits, c->stream);
    c->fin_n = 0;
    return e ? hipcheck(c, (hipError_t)e, "wave-speed reduction launch") : FSA_OK;
}

int enqueue_stage(fsa_ctx* c, const double* Qs, const double* Qn, double* out, int in, int acc, bool reduce,
                  int stage, double ca, double cb, double dt, int mode_rhs)
{
    unsigned long long* bits = c->abits + 3 * in;
    int e;
    if (reduce) {
        if ((e = flush_alpha_final(c)) != FSA_OK) return e;   // (apart is reused below)
        e = launch_alpha(c->G, c->P, Qs, c->apart, bits, c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "alpha reduction launch");
    }
    if (ib_active(c)) {
        IBArgs A = ib_args(c);
        A.Qs = Qs;
        A.stage = stage;
        A.ca = ca;
        A.cb = cb;
        A.dt = dt;
        // the previous stage's wave-speed reduction rides on the window launch when its
        // partials are few (2D: one per wave); the 3D stage's many block partials keep the
        // wider standalone reduction
        const bool carry = c->fin_n > 0 && c->fin_n <= 16384;
        A.alpha_part = carry ? c->apart : nullptr;
        A.alpha_n = carry ? c->fin_n : 0;
        A.alpha_bits = c->fin_bits;
        const bool swap_xi = stage > 0 && ib_stage_fused(c->G, c->nm);
        if (swap_xi) A.xi_out = c->xi2;
        e = launch_ib_stage(c->G, c->P, A, c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "IB stage launch");
        if (swap_xi) std::swap(c->xi, c->xi2);   // (stream-ordered: later launches read the new one)
        if (carry) c->fin_n = 0;
    }
    if ((e = flush_alpha_final(c)) != FSA_OK) return e;
    if (c->d.precision == FSA_LEARNED32) {
        if (!c->mlp_ready) return fail(c, FSA_ESTATE, "learned form without a network (fsa_mlp_set)");
        // stage 0 = a lone right-hand side; stages 2 and 3 reuse the first stage's patterns
        // when the selector stride is 3
        if (stage <= 1 || c->d.selector_stride != 3) {
            int rc = enqueue_flags(c, Qs, bits, c->flags_x, c->flags_y);
            if (rc != FSA_OK) return rc;
        }
    }
    StageArgs S;
    std::memset(&S, 0, sizeof S);
    S.Qs = Qs;
    S.Qn = Qn ? Qn : Qs;   // (right-hand-side mode: read but not used)
    S.out = out;
    S.flags_x = c->flags_x;
    S.flags_y = c->flags_y;
    S.alpha_bits = bits;
    S.nrbc = nrbc_mask(c);
    // (non-reflecting sides: the wave speeds come from the corrected output, finish_nrbc)
    S.alpha_part = (acc >= 0 && !S.nrbc) ? c->apart : nullptr;
    S.fwin = ib_active(c) ? c->fwin : nullptr;
    for (int k = 0; k < 3; ++k) {
        S.wlo[k] = c->wlo[k];
        S.wn[k] = c->wn[k];
    }
    S.ca = ca;
    S.cb = cb;
    S.dt = dt;
    S.mode_rhs = mode_rhs;
    S.step = c->step;
    S.arow0 = c->arow0;
    S.arow1 = c->arow1;
    if (c->dbg_bits) {
        const long long nx = c->G.n[0], ny = c->G.n[1], nz = c->G.n[2];
        const long long fx = (nx + 1) * ny * nz, fy = nx * (ny + 1) * nz, fz = c->G.dim == 3 ? nx * ny * (nz + 1) : 0;
        unsigned* b = c->dbg_bits + (stage > 0 ? stage - 1 : 0) * (fx + fy + fz);
        S.dbg_x = b;
        S.dbg_y = b + fx;
        S.dbg_z = c->G.dim == 3 ? b + fx + fy : nullptr;
    }
    // stage times of SSP-RK3 (t, t + dt, t + dt/2; a lone right-hand side at t)
    S.t = c->t + (stage == 2 ? dt : (stage == 3 ? 0.5 * dt : 0.0));
    if (c->G.dim == 3) {
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (c->timing) {
            int rc = timing_pair(c, t0, t1);
            if (rc != FSA_OK) return rc;
            HIPCHK(c, hipEventRecord(t0, c->stream));
        }
        e = launch_stage3d(c->dK, c->G, c->d.scheme, c->d.precision, c->d.variables, S, c->stress3d, c->faces3d,
                           c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "3D stage launch");
        if (t1) HIPCHK(c, hipEventRecord(t1, c->stream));
        if (S.nrbc) return finish_nrbc(c, S, acc);
        if (acc >= 0) defer_alpha_final(c, stage3d_blocks(c->G), acc);
        return FSA_OK;
    }
    if (c->d.variables == FSA_CHARACTERISTIC) {
        // 2D characteristic-wise: stress, face and stage passes (ghosts resolved where read)
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (c->timing) {
            int rc = timing_pair(c, t0, t1);
            if (rc != FSA_OK) return rc;
            HIPCHK(c, hipEventRecord(t0, c->stream));
        }
        e = launch_pass2d(c->dK, c->G, c->d.scheme, c->d.terms, c->d.mu, S, static_cast<double*>((void*)c->stress3d),
                          static_cast<double*>((void*)c->faces3d), c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "2D pass launch");
        if (t1) HIPCHK(c, hipEventRecord(t1, c->stream));
        if (S.nrbc) return finish_nrbc(c, S, acc);
        if (acc >= 0) defer_alpha_final(c, pass2d_blocks(c->G), acc);
        return FSA_OK;
    }
    if (c->ghosts && (c->ghosts_step < 0 || c->step < c->ghosts_step || c->step >= c->ghosts_step + GHOST_STEPS)) {
        // inflow ghost tables of this step and the next ones (stream-ordered: stages that
        // read the previous tables were enqueued before)
        e = launch_inflow_ghosts2d(c->dK, c->G, c->step, GHOST_STEPS, c->ghosts, c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "inflow ghost launch");
        c->ghosts_step = c->step;
    }
    S.ghosts = c->ghosts ? c->ghosts + (c->step - c->ghosts_step) * inflow_ghosts2d_elems(c->G) : nullptr;
    if (c->ty == 0) {
        if (int rf = flush_alpha_final(c)) return rf;   // (the timing launches write the partials)
        int rc = tune_ty(c, S);
        if (rc != FSA_OK) return rc;
    }
    S.ty = c->ty;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (c->timing) {
        int rc = timing_pair(c, t0, t1);
        if (rc != FSA_OK) return rc;
        HIPCHK(c, hipEventRecord(t0, c->stream));
    }
    // learned form: the stage output's deviation ranges, for the next flags pass (only from a
    // stage whose output a flags pass reads: with the selector once per step, the last one)
    S.qrange = (c->d.precision == FSA_LEARNED32 && acc >= 0 && !S.nrbc && (c->d.selector_stride != 3 || stage == 3))
                   ? c->qrange
                   : nullptr;
    e = launch_stage2d(c->dK, c->G, c->d.scheme, c->d.precision, S, c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "stage kernel launch");
    if (t1) HIPCHK(c, hipEventRecord(t1, c->stream));
    c->qrange_of = S.qrange ? out : nullptr;
    c->qrange_ty = S.ty;
    if (S.nrbc) return finish_nrbc(c, S, acc);
    if (acc >= 0) defer_alpha_final(c, stage2d_waves(c->G, S.ty), acc);
    return FSA_OK;
}

// Time the candidate segment heights on this launch's inputs (right-hand-side mode into the
// second stage buffer, which no caller-visible state lives in at this point) and keep the
// fastest.
int tune_ty(fsa_ctx* c, const StageArgs& S0)
{
    // fixed candidates, plus for one to four rounds of waves the shortest segment whose wave
    // count fits that many rounds of the device's wave slots (two waves per SIMD, four SIMDs
    // per compute unit): the halo rows are paid once per segment, so the fewest segments that
    // still fill the rounds are the natural candidates
    std::vector<int> cand = {8, 10, 12, 14, 16, 19, 22, 25, 28, 32, 37, 44, 52, 64};
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
            const long long slots = 8ll * cus, strips = stage2d_ncolx(c->G.n[0]);
            for (int rounds = 1; rounds <= 4; ++rounds) {
                const long long segs = rounds * slots / strips;
                if (segs < 1) continue;
                const long long ty = (c->G.n[1] + segs - 1) / segs;
                if (ty >= 4 && ty <= 4096 && std::find(cand.begin(), cand.end(), (int)ty) == cand.end())
                    cand.push_back((int)ty);
            }
        }
    }
    // timed as an SSP-RK3 middle stage (step-start state read, combination, wave-speed
    // partials), the work the height is chosen for; the output goes to a scratch buffer and
    // the partials are overwritten by the real launch
    StageArgs S = S0;
    S.dbg_x = S.dbg_y = S.dbg_z = nullptr;
    S.mode_rhs = 0;
    S.Qn = S0.Qs;
    S.ca = 0.75;
    S.cb = 0.25;
    S.out = c->Qb;
    S.alpha_part = c->apart;
    S.qrange = nullptr;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // each candidate's time is the least of six samples after a warm-up pass, a sample being
    // three back-to-back launches (as the stages run; single launches of ~0.3 ms vary by a few
    // percent, as much as neighbouring candidates differ)
    std::vector<float> tmin(cand.size(), 1e30f);
    for (int rep = 0; rep < 7; ++rep)
        for (size_t k = 0; k < cand.size(); ++k) {
            const int ty = cand[k];
            if (ty > 2 * c->G.n[1] && ty != cand[0]) continue;
            S.ty = ty;
            HIPCHK(c, hipEventRecord(e0, c->stream));
            for (int l = 0; l < 3; ++l) {
                int e = launch_stage2d(c->dK, c->G, c->d.scheme, c->d.precision, S, c->stream);
                if (e) return hipcheck(c, (hipError_t)e, "stage kernel launch (tuning)");
            }
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) tmin[k] = std::min(tmin[k], ms);   // the first pass warms caches and clocks
        }
    // the tallest segments (fewest halo rows) among the candidates within 1% of the fastest:
    // closer than that, the order of two candidates changes from run to run
    float best_ms = 1e30f;
    for (size_t k = 0; k < cand.size(); ++k) best_ms = std::min(best_ms, tmin[k]);
    int best = -1;
    for (size_t k = 0; k < cand.size(); ++k)
        if (tmin[k] < 1e29f && tmin[k] <= 1.01f * best_ms && cand[k] > best) best = cand[k];
    if (best < 0) best = 16;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->ty = best;
    return FSA_OK;
}

MLPArgs mlp_args(const fsa_ctx* c)
{
    MLPArgs M;
    M.master = c->mlp_master;
    M.wbf = c->mlp_wbf;
    M.m = c->mlp_m;
    M.v = c->mlp_v;
    return M;
}

// Learned keep patterns of the faces of Qs (the learned form's per-stage pass).
int enqueue_flags(fsa_ctx* c, const double* Qs, const unsigned long long* bits, unsigned* fx, unsigned* fy)
{
    FlagArgs F;
    std::memset(&F, 0, sizeof F);
    F.Q = Qs;
    F.step = c->step;
    F.alpha_bits = bits;
    F.M = mlp_args(c);
    // min_k |2 sigma(z_k) - 1| >= c  <=>  min_k |z_k| >= 2 atanh(c) = ln((1 + c) / (1 - c))
    F.zthr = c->conf_threshold >= 1.0 ? INFINITY : (float)std::log((1.0 + c->conf_threshold) / (1.0 - c->conf_threshold));
    F.flags_x = fx;
    F.flags_y = fy;
    F.counters = c->counters;
    // tiles of a quiet region skip the state when Qs is the output of the last learned stage
    if (c->quiet_tiles && c->qrange_of != nullptr && c->qrange_of == Qs && fx == c->flags_x) {
        F.qrange = c->qrange;
        F.qr_ty = c->qrange_ty;
        F.qr_ncolx = stage2d_ncolx(c->G.n[0]);
        F.qr_w = stage2d_strip_width();
    }
    int e = launch_flags2d(c->dK, c->G, F, c->stream);
    return e ? hipcheck(c, (hipError_t)e, "flags launch") : FSA_OK;
}

bool bits_finite(unsigned long long b)
{
    double v;
    std::memcpy(&v, &b, sizeof v);
    return std::isfinite(v);
}

// Check the wave speeds of the previous step (nan_check only).
int check_previous(fsa_ctx* c)
{
    if (!c->d.nan_check || !c->alpha_pending) return c->nonfinite ? FSA_ENONFINITE : FSA_OK;
    HIPCHK(c, hipEventSynchronize(c->ev_alpha));
    c->alpha_pending = false;
    for (int k = 0; k < 9; ++k) {
        const int d = k % 3;
        if (d < c->d.dim && !bits_finite(c->h_abits[k])) c->nonfinite = 1;
    }
    if (c->nonfinite) return fail(c, FSA_ENONFINITE, "non-finite wave speed in the state");
    return FSA_OK;
}

// Scratch of fsa_alpha_noalloc: the per-block partial maxima of the wave-speed reduction
// (three per block, at most ALPHA_MAX_BLOCKS blocks), in a static device array instead of a
// context's workspace.  Each GPU holds its own copy at its own address, taken once per device
// with hipGetSymbolAddress; host code passes that address, never the array's name.
constexpr long long NOALLOC_PARTIALS = 3ll * ALPHA_MAX_BLOCKS;
static __device__ __align__(256) unsigned long long scratch[NOALLOC_PARTIALS];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on the current device (taken on the first call there).
hipError_t scratch_address(unsigned long long** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned long long*)g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t fsa_abi_version(void) { return FSA_ABI_VERSION; }

const char* fsa_status_str(int32_t s)
{
    switch (s) {
        case FSA_OK: return "ok";
        case FSA_EINVAL: return "invalid argument";
        case FSA_ENOMEM: return "out of device memory";
        case FSA_EDEVICE: return "device error";
        case FSA_ENONFINITE: return "non-finite state";
        case FSA_ESTATE: return "bad state";
        case FSA_EUNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* fsa_last_error(const fsa_ctx* c) { return c ? c->err.c_str() : "no context"; }

}  // extern "C"

namespace {

// Context fields that follow from the descriptor alone (grid, constants, capacities).
void plan(fsa_ctx* c, const fsa_desc* desc)
{
    c->d = *desc;
    c->nq = desc->dim + 2;
    build_consts(c);
    c->ncell = c->G.ncell;
    const int dim = desc->dim;
    c->cap_markers = desc->max_markers;
    c->cap_probes = desc->max_probes;
    c->cap_entries = (long long)desc->max_markers * (dim == 3 ? 64 : 16);
    c->cap_wcells = desc->max_markers == 0 ? 0
                    : (desc->max_window_cells > 0 ? std::min<long long>(desc->max_window_cells, c->ncell) : c->ncell);
}

int validate_caps(const fsa_desc* d, std::string& why)
{
    if (d->max_markers < 0 || d->max_probes < 0 || d->max_window_cells < 0) {
        why = "negative capacity";
        return FSA_EINVAL;
    }
    return FSA_OK;
}

}  // namespace

extern "C" {

int32_t fsa_workspace_bytes(const fsa_desc* desc, size_t* bytes)
{
    if (!bytes) return FSA_EINVAL;
    *bytes = 0;
    std::string why;
    int rc = validate(desc, why);
    if (rc == FSA_OK) rc = validate_caps(desc, why);
    if (rc != FSA_OK) {
        std::fprintf(stderr, "fsa_workspace_bytes: %s\n", why.c_str());
        return rc;
    }
    fsa_ctx* c = new (std::nothrow) fsa_ctx();
    if (!c) return FSA_ENOMEM;
    plan(c, desc);
    *bytes = carve(c, nullptr);
    delete c;
    return FSA_OK;
}

int32_t fsa_init(const fsa_desc* desc, void* d_workspace, size_t ws_bytes, void* hip_stream, fsa_ctx** out)
{
    if (!out) return FSA_EINVAL;
    *out = nullptr;
    std::string why;
    int rc = validate(desc, why);
    if (rc == FSA_OK) rc = validate_caps(desc, why);
    if (rc != FSA_OK) {
        std::fprintf(stderr, "fsa_init: %s\n", why.c_str());
        return rc;
    }
    fsa_ctx* c = new (std::nothrow) fsa_ctx();
    if (!c) return FSA_ENOMEM;
    plan(c, desc);
    const size_t need = carve(c, nullptr);
    if (!d_workspace || ws_bytes < need) {
        std::fprintf(stderr, "fsa_init: the workspace needs %zu bytes (fsa_workspace_bytes), got %zu\n", need,
                     d_workspace ? ws_bytes : (size_t)0);
        delete c;
        return FSA_EINVAL;
    }
    c->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&c->device);
    c->ty = env_ty();
    if (const char* e = std::getenv("FSA_NO_QUIET_TILES")) c->quiet_tiles = std::atoi(e) == 0;
    char* base = (char*)(((uintptr_t)d_workspace + 255) & ~(uintptr_t)255);
    carve(c, base);
    c->arow0 = 0;
    c->arow1 = c->G.n[c->G.dim - 1];
    {
        KConst hk;
        std::memset(&hk, 0, sizeof hk);
        hk.G = c->G;
        hk.P = c->P;
        hk.inv12h = 1.0 / (12.0 * c->G.h);
        hk.teno_tall = teno_all_kept_bound(c->P.teno_ct);
        far_field_fluxes(c, hk);
        if (hipMemcpyAsync(c->dK, &hk, sizeof hk, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipMemsetAsync(c->abits, 0, 12 * sizeof(unsigned long long), c->stream) != hipSuccess ||
            (c->counters && hipMemsetAsync(c->counters, 0, 3 * (size_t)flags2d_blocks(c->G) * sizeof(unsigned long long),
                                           c->stream) != hipSuccess) ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            (void)hipGetLastError();
            fsa_destroy(c);
            return FSA_EDEVICE;
        }
    }
    // pinned host memory: wave-speed read-back and the two halves of the marker staging
    if (hipHostMalloc((void**)&c->h_abits, 12 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_alpha, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_stage[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_stage[1], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        fsa_destroy(c);
        return FSA_ENOMEM;
    }
    if (c->stage_bytes) {
        void* hd = nullptr;
        if (hipHostMalloc((void**)&c->h_stage, 2 * c->stage_bytes, hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer(&hd, c->h_stage, 0) != hipSuccess) {
            (void)hipGetLastError();
            fsa_destroy(c);
            return FSA_ENOMEM;
        }
        c->h_stage_dev = (const char*)hd;
    }
    *out = c;
    return FSA_OK;
}

int32_t fsa_destroy(fsa_ctx* c)
{
    if (!c) return FSA_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->h_abits) (void)hipHostFree(c->h_abits);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    for (hipEvent_t ev : c->ev_stage)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : c->tev) (void)hipEventDestroy(ev);
    if (c->ev_alpha) (void)hipEventDestroy(c->ev_alpha);
    delete c;
    return FSA_OK;
}

int32_t fsa_set_markers(fsa_ctx* c, int32_t n, const double* X, const double* dV, const double* U, int32_t motion,
                        double omega)
{
    if (!c) return FSA_EINVAL;
    if (n < 0 || (n > 0 && (!X || !dV))) return fail(c, FSA_EINVAL, "bad marker arrays");
    if (motion < FSA_STATIC || motion > FSA_EXTERNAL) return fail(c, FSA_EINVAL, "bad motion");
    if (n > c->cap_markers)
        return fail(c, FSA_EINVAL, "more markers (" + std::to_string(n) + ") than desc.max_markers (" +
                                       std::to_string(c->cap_markers) + ")");
    if (n > 0 && !support_inside(c, n, X)) return fail(c, FSA_EINVAL, "a marker support leaves the grid");
    HIPCHK(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    c->stage_pending[0] = c->stage_pending[1] = false;   // (the stream is idle: earlier staging copies are done)
    const int dim = c->d.dim;
    c->nm = n;
    c->motion = motion;
    c->omega = omega;
    c->hX.assign(X ? X : nullptr, X ? X + (size_t)dim * n : nullptr);
    const size_t ln = (size_t)dim * n;
    if (ln) {
        HIPCHK(c, hipMemsetAsync(c->U, 0, sizeof(double) * ln, c->stream));
        HIPCHK(c, hipMemsetAsync(c->xi, 0, sizeof(double) * ln, c->stream));
        HIPCHK(c, hipMemsetAsync(c->xi2, 0, sizeof(double) * ln, c->stream));
        HIPCHK(c, hipMemsetAsync(c->xi_n, 0, sizeof(double) * ln, c->stream));
        HIPCHK(c, hipMemsetAsync(c->F, 0, sizeof(double) * ln, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->dV, dV, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return build_window(c, U);   // (X and U go to the device with the window lists)
}

int32_t fsa_set_marker_kinematics(fsa_ctx* c, const double* X, const double* U)
{
    if (!c) return FSA_EINVAL;
    if (c->nm == 0 || c->motion != FSA_EXTERNAL) return fail(c, FSA_ESTATE, "markers are not EXTERNAL");
    if (!X) return fail(c, FSA_EINVAL, "X is NULL");
    if (!support_inside(c, c->nm, X)) return fail(c, FSA_EINVAL, "a marker support leaves the grid");
    const int dim = c->d.dim, n = c->nm;
    c->hX.assign(X, X + (size_t)dim * n);
    return update_window_async(c, X, U);   // (stream-ordered: the host does not wait for the device)
}

int32_t fsa_set_probes(fsa_ctx* c, int32_t n, const double* Xp)
{
    if (!c) return FSA_EINVAL;
    if (n < 0 || (n > 0 && !Xp)) return fail(c, FSA_EINVAL, "bad probe array");
    if (n > 0 && !support_inside(c, n, Xp)) return fail(c, FSA_EINVAL, "a probe support leaves the grid");
    if (n > c->cap_probes)
        return fail(c, FSA_EINVAL, "more probes (" + std::to_string(n) + ") than desc.max_probes (" +
                                       std::to_string(c->cap_probes) + ")");
    HIPCHK(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    c->np = n;
    if (n > 0) {
        HIPCHK(c, hipMemcpyAsync(c->Xp, Xp, sizeof(double) * c->d.dim * n, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return FSA_OK;
}

int32_t fsa_alpha(fsa_ctx* c, const double* d_Q, double* alpha)
{
    if (!c || !d_Q || !alpha) return FSA_EINVAL;
    if (int rf = flush_alpha_final(c)) return rf;
    unsigned long long* bits = c->abits + 9;
    int e = launch_alpha(c->G, c->P, d_Q, c->apart, bits, c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "alpha launch");
    unsigned long long hb[3];
    HIPCHK(c, hipMemcpyAsync(hb, bits, sizeof hb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int d = 0; d < 3; ++d) {
        if (d < c->d.dim) std::memcpy(&alpha[d], &hb[d], sizeof(double));
        else alpha[d] = 0.0;
    }
    return FSA_OK;
}

int32_t fsa_alpha_noalloc(const fsa_desc* desc, const double* d_Q, double* d_alpha, void* hip_stream)
{
    std::string why;
    if (!d_Q || !d_alpha) return FSA_EINVAL;
    if (validate(desc, why) != FSA_OK) {
        std::fprintf(stderr, "fsa_alpha_noalloc: %s\n", why.c_str());
        return FSA_EINVAL;
    }
    fsa_ctx tmp;                       // (grid and gas constants only: no buffers)
    tmp.d = *desc;
    build_consts(&tmp);
    long long blocks = alpha_blocks(tmp.G);
    if (3 * blocks > NOALLOC_PARTIALS) {
        std::fprintf(stderr, "fsa_alpha_noalloc: %lld partials exceed the static scratch of %lld\n", 3 * blocks,
                     NOALLOC_PARTIALS);
        return FSA_EINVAL;
    }
    unsigned long long* part = nullptr;
    if (scratch_address(&part) != hipSuccess) {
        (void)hipGetLastError();
        return FSA_EDEVICE;
    }
    int e = launch_alpha(tmp.G, tmp.P, d_Q, part, (unsigned long long*)d_alpha, (hipStream_t)hip_stream);
    return e ? FSA_EDEVICE : FSA_OK;
}

int32_t fsa_rhs(fsa_ctx* c, const double* d_Q, double* d_L)
{
    if (!c || !d_Q || !d_L) return FSA_EINVAL;
    if ((const void*)d_Q == (const void*)d_L) return fail(c, FSA_EINVAL, "d_L aliases d_Q");
    c->advanced = nullptr;    // (the wave-speed reduction below reuses the step calls' slot 0)
    c->qrange_of = nullptr;   // d_Q may have changed since the ranges were taken
    return enqueue_stage(c, d_Q, nullptr, d_L, 0, -1, true, 0, 0.0, 1.0, 0.0, 1);
}

namespace {

int rk3_run(fsa_ctx* c, double* d_Q, double dt, int32_t nsteps, bool resume)
{
    if (!c || !d_Q) return FSA_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, FSA_EINVAL, "dt must be positive");
    if (nsteps < 1) return fail(c, FSA_EINVAL, "nsteps must be positive");
    if (resume && c->advanced != d_Q)
        return fail(c, FSA_ESTATE, "resume: d_Q is not the state the previous step call left");
    int rc = check_previous(c);
    if (rc != FSA_OK) return rc;
    c->advanced = nullptr;
    if (!resume) c->qrange_of = nullptr;   // d_Q may have changed since the last call
    static const double CA[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double CB[3] = {1.0, 0.25, 2.0 / 3.0};
    // the wave speeds of every stage input come from the kernel that wrote it, except for
    // the first stage of the call, which reduces d_Q into slot 0
    for (int n = 0; n < nsteps; ++n) {
        for (int s = 0; s < 3; ++s) {
            const int g = 3 * n + s;
            const double* Qs = s == 0 ? d_Q : (s == 1 ? c->Qa : c->Qb);
            double* out = s == 0 ? c->Qa : (s == 1 ? c->Qb : d_Q);
            if ((rc = enqueue_stage(c, Qs, d_Q, out, g % 3, (g + 1) % 3, g == 0 && !resume, s + 1, CA[s],
                                    CB[s], dt, 0)) != FSA_OK)
                return rc;
        }
        c->t += dt;
        c->step += 1;
    }
    // the last stage's reduction stays pending: the next step call's first IB launch carries
    // it (as between the steps of one call), and every other reader of the partials or the
    // slots flushes it first
    c->last_slot = (3 * nsteps) % 3;
    if (c->d.nan_check) {
        if ((rc = flush_alpha_final(c)) != FSA_OK) return rc;
        HIPCHK(c, hipMemcpyAsync(c->h_abits, c->abits, 9 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipEventRecord(c->ev_alpha, c->stream));
        c->alpha_pending = true;
    }
    c->advanced = d_Q;   // (slot 0 holds, or the pending reduction writes, its wave speeds)
    return FSA_OK;
}

}  // namespace

int32_t fsa_rk3_steps(fsa_ctx* c, double* d_Q, double dt, int32_t nsteps) { return rk3_run(c, d_Q, dt, nsteps, false); }
int32_t fsa_rk3_steps_resume(fsa_ctx* c, double* d_Q, double dt, int32_t nsteps)
{
    return rk3_run(c, d_Q, dt, nsteps, true);
}
int32_t fsa_rk3_step(fsa_ctx* c, double* d_Q, double dt) { return fsa_rk3_steps(c, d_Q, dt, 1); }

int32_t fsa_ib_interp(fsa_ctx* c, const double* d_field, int32_t ncomp, double* d_out)
{
    if (!c || !d_field || !d_out || ncomp < 1) return FSA_EINVAL;
    int e = launch_interp(c->G, c->nm, c->X, d_field, ncomp, d_out, c->stream);
    return e ? hipcheck(c, (hipError_t)e, "interp launch") : FSA_OK;
}

int32_t fsa_ib_spread(fsa_ctx* c, const double* d_F, int32_t ncomp, double* d_field, double scale)
{
    if (!c || !d_F || !d_field || ncomp < 1) return FSA_EINVAL;
    if (c->nm == 0) return FSA_OK;
    IBArgs A = ib_args(c);
    int e = launch_spread(c->G, A, d_F, ncomp, d_field, scale, c->stream);
    return e ? hipcheck(c, (hipError_t)e, "spread launch") : FSA_OK;
}

int32_t fsa_probe_dp(fsa_ctx* c, const double* d_Q, double* d_dp)
{
    if (!c || !d_Q || !d_dp) return FSA_EINVAL;
    int e = launch_probe_dp(c->G, c->P, c->np, c->Xp, d_Q, d_dp, c->stream);
    return e ? hipcheck(c, (hipError_t)e, "probe launch") : FSA_OK;
}

int32_t fsa_marker_info(const fsa_ctx* c, int32_t* n, int32_t* motion, int32_t* dim)
{
    if (!c) return FSA_EINVAL;
    if (n) *n = c->nm;
    if (motion) *motion = c->motion;
    if (dim) *dim = c->d.dim;
    return FSA_OK;
}

int32_t fsa_marker_force(fsa_ctx* c, double* h_F)
{
    if (!c || !h_F) return FSA_EINVAL;
    if (c->nm == 0) return FSA_OK;
    HIPCHK(c, hipMemcpyAsync(h_F, c->F, sizeof(double) * c->d.dim * c->nm, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FSA_OK;
}

int32_t fsa_get_state(fsa_ctx* c, double* h_xi, double* t, int64_t* step)
{
    if (!c) return FSA_EINVAL;
    if (h_xi && c->nm > 0) {
        HIPCHK(c, hipMemcpyAsync(h_xi, c->xi, sizeof(double) * c->d.dim * c->nm, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (t) *t = c->t;
    if (step) *step = c->step;
    return FSA_OK;
}

int32_t fsa_set_state(fsa_ctx* c, const double* h_xi, double t, int64_t step)
{
    if (!c) return FSA_EINVAL;
    if (step < 0) return fail(c, FSA_EINVAL, "negative step");
    if (h_xi && c->nm > 0) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipMemcpy(c->xi, h_xi, sizeof(double) * c->d.dim * c->nm, hipMemcpyHostToDevice));
    }
    c->t = t;
    c->step = step;
    return FSA_OK;
}

int32_t fsa_mlp_set(fsa_ctx* c, const float* h_params, int32_t nparams, double conf_threshold)
{
    if (!c || !h_params) return FSA_EINVAL;
    if (nparams != MLP_NPARAM) return fail(c, FSA_EINVAL, "the network has 1667 parameters");
    if (!(conf_threshold >= 0.0 && conf_threshold <= 1.0)) return fail(c, FSA_EINVAL, "threshold outside [0, 1]");
    HIPCHK(c, hipMemcpyAsync(c->mlp_master, h_params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->mlp_m, 0, sizeof(float) * MLP_NPARAM, c->stream));
    HIPCHK(c, hipMemsetAsync(c->mlp_v, 0, sizeof(float) * MLP_NPARAM, c->stream));
    int e = launch_mlp_round(mlp_args(c), c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "mlp round launch");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->mlp_t = 0;
    c->conf_threshold = conf_threshold;
    c->mlp_ready = true;
    return FSA_OK;
}

int32_t fsa_set_mlp(fsa_ctx* c, const uint16_t* h_bf16_params, int32_t nparams, double conf_threshold)
{
    if (!c || !h_bf16_params) return FSA_EINVAL;
    if (nparams != MLP_NPARAM) return fail(c, FSA_EINVAL, "the network has 1667 parameters");
    // BF16 -> FP32 is exact (the BF16 bits are the FP32 value's upper half), and rounding
    // that FP32 value back to BF16 returns it unchanged
    std::vector<float> f(MLP_NPARAM);
    for (int k = 0; k < MLP_NPARAM; ++k) {
        const uint32_t bits = (uint32_t)h_bf16_params[k] << 16;
        std::memcpy(&f[k], &bits, sizeof(float));
    }
    return fsa_mlp_set(c, f.data(), nparams, conf_threshold);
}

int32_t fsa_mlp_get(fsa_ctx* c, float* h_params, int32_t nparams)
{
    if (!c || !h_params || nparams != MLP_NPARAM) return FSA_EINVAL;
    if (!c->mlp_ready) return fail(c, FSA_ESTATE, "no network set");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(h_params, c->mlp_master, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
    return FSA_OK;
}

int32_t fsa_mlp_forward(fsa_ctx* c, const float* d_feats, int64_t n, float* d_logits)
{
    if (!c || !d_feats || !d_logits || n < 0) return FSA_EINVAL;
    if (!c->mlp_ready) return fail(c, FSA_ESTATE, "no network set");
    int e = launch_mlp_forward(mlp_args(c), d_feats, n, d_logits, c->stream);
    return e ? hipcheck(c, (hipError_t)e, "mlp forward launch") : FSA_OK;
}

int32_t fsa_mlp_grad(fsa_ctx* c, const float* d_feats, const uint8_t* d_labels, int64_t n, float* d_grad,
                     float* d_loss)
{
    if (!c || !d_feats || !d_labels || !d_grad || n < 1) return FSA_EINVAL;
    if (!c->mlp_ready) return fail(c, FSA_ESTATE, "no network set");
    int e = launch_mlp_grad(mlp_args(c), d_feats, d_labels, n, c->mlp_partial, c->mlp_loss_part, d_grad, d_loss,
                            c->stream);
    return e ? hipcheck(c, (hipError_t)e, "mlp grad launch") : FSA_OK;
}

int32_t fsa_mlp_train_step(fsa_ctx* c, const float* d_feats, const uint8_t* d_labels, int64_t n, float lr,
                           float* d_loss)
{
    if (!c || !d_feats || !d_labels || n < 1 || !(lr > 0.0f)) return FSA_EINVAL;
    if (!c->mlp_ready) return fail(c, FSA_ESTATE, "no network set");
    int e = launch_mlp_grad(mlp_args(c), d_feats, d_labels, n, c->mlp_partial, c->mlp_loss_part, c->mlp_grad, d_loss,
                            c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "mlp grad launch");
    c->mlp_t += 1;
    e = launch_mlp_adam(mlp_args(c), c->mlp_grad, lr, c->mlp_t, c->stream);
    return e ? hipcheck(c, (hipError_t)e, "adam launch") : FSA_OK;
}

int32_t fsa_harvest(fsa_ctx* c, const double* d_Q, double keep_rate, uint64_t seed, int64_t max_out, float* d_feats,
                    uint8_t* d_labels, int64_t* h_count)
{
    if (!c || !d_Q || !h_count || max_out < 0 || (max_out > 0 && (!d_feats || !d_labels))) return FSA_EINVAL;
    if (!(keep_rate >= 0.0 && keep_rate <= 1.0)) return fail(c, FSA_EINVAL, "keep_rate outside [0, 1]");
    if (int rf = flush_alpha_final(c)) return rf;
    unsigned long long* bits = c->abits + 9;
    int e = launch_alpha(c->G, c->P, d_Q, c->apart, bits, c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "alpha launch");
    HarvestArgs H;
    std::memset(&H, 0, sizeof H);
    H.Q = d_Q;
    H.step = c->step;
    H.alpha_bits = bits;
    H.keep_rate = keep_rate;
    H.seed = seed;
    H.max_out = max_out;
    H.feats = d_feats;
    H.labels = d_labels;
    H.block_count = c->hv_count;
    H.block_offset = c->hv_offset;
    H.total = c->hv_total;
    e = c->G.dim == 3 ? launch_harvest3d(c->dK, c->G, H, c->stream) : launch_harvest2d(c->dK, c->G, H, c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "harvest launch");
    long long tot = 0;
    HIPCHK(c, hipMemcpyAsync(&tot, c->hv_total, sizeof tot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *h_count = tot;
    return FSA_OK;
}

int32_t fsa_face_flags(fsa_ctx* c, const double* d_Q, uint32_t* d_flags_x, uint32_t* d_flags_y)
{
    if (!c || !d_Q || !d_flags_x || !d_flags_y) return FSA_EINVAL;
    if (c->d.dim != 2) return fail(c, FSA_EUNSUPPORTED, "learned flags are built for 2D");
    if (!c->mlp_ready) return fail(c, FSA_ESTATE, "no network set");
    if (int rf = flush_alpha_final(c)) return rf;
    unsigned long long* bits = c->abits + 9;
    int e = launch_alpha(c->G, c->P, d_Q, c->apart, bits, c->stream);
    if (e) return hipcheck(c, (hipError_t)e, "alpha launch");
    return enqueue_flags(c, d_Q, bits, d_flags_x, d_flags_y);
}

int32_t fsa_diagnostics(fsa_ctx* c, const double* d_Q, double* h_totals, double* d_dilatation)
{
    if (!c || !d_Q || (!h_totals && !d_dilatation)) return FSA_EINVAL;
    int e;
    if (d_dilatation) {
        e = launch_dilatation(c->G, c->P, d_Q, c->step, d_dilatation, c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "dilatation launch");
    }
    if (h_totals) {
        e = launch_totals(c->G, c->nq, d_Q, c->tot_part, c->tot_out, c->stream);
        if (e) return hipcheck(c, (hipError_t)e, "totals launch");
        HIPCHK(c, hipMemcpyAsync(h_totals, c->tot_out, sizeof(double) * c->nq, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return FSA_OK;
}

int32_t fsa_debug_teno_bits(fsa_ctx* c, uint32_t* d_bits)
{
    if (!c) return FSA_EINVAL;
    if (d_bits && (c->d.scheme != FSA_TENO5 || c->d.precision != FSA_FP64 || c->d.variables != FSA_COMPONENT))
        return fail(c, FSA_EUNSUPPORTED, "the keep-pattern read-out is built for component-wise FP64 TENO5");
    c->dbg_bits = d_bits;
    return FSA_OK;
}

int32_t fsa_timing_enable(fsa_ctx* c, int32_t on)
{
    if (!c) return FSA_EINVAL;
    c->timing = on != 0;
    return FSA_OK;
}

int32_t fsa_timing_read(fsa_ctx* c, double* ms, int64_t* launches)
{
    if (!c || !ms || !launches) return FSA_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double total = 0.0;
    for (size_t k = 0; k + 1 < c->tused; k += 2) {
        float e = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&e, c->tev[k], c->tev[k + 1]));
        total += e;
    }
    *ms = total;
    *launches = (int64_t)(c->tused / 2);
    c->tused = 0;
    return FSA_OK;
}

int32_t fsa_sync(fsa_ctx* c)
{
    if (!c) return FSA_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_previous(c);
}

int32_t fsa_stats_get(fsa_ctx* c, fsa_stats* out)
{
    if (!c || !out) return FSA_EINVAL;
    unsigned long long hb[3];
    if (int rf = flush_alpha_final(c)) return rf;
    HIPCHK(c, hipMemcpyAsync(hb, c->abits + 3 * c->last_slot, sizeof hb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memset(out, 0, sizeof *out);
    for (int d = 0; d < 3; ++d) {
        if (d < c->d.dim) std::memcpy(&out->alpha[d], &hb[d], sizeof(double));
        if (d < c->d.dim && !bits_finite(hb[d])) c->nonfinite = 1;
    }
    out->t = c->t;
    out->step = c->step;
    out->nonfinite = c->nonfinite;
    out->n_markers = c->nm;
    out->n_probes = c->np;
    out->window_cells = (int32_t)c->wcells;
    out->rows_per_wave = c->ty;
    if (c->counters && c->mlp_ready) {
        const long long nb = flags2d_blocks(c->G);
        std::vector<unsigned long long> hc((size_t)(3 * nb));
        HIPCHK(c, hipMemcpy(hc.data(), c->counters, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        unsigned long long tot[3] = {0ull, 0ull, 0ull};
        for (long long b = 0; b < nb; ++b)
            for (int k = 0; k < 3; ++k) tot[k] += hc[(size_t)(3 * b + k)];
        out->learned_sides = (int64_t)tot[0];
        out->fallback_sides = (int64_t)tot[1];
        out->significant_sides = (int64_t)tot[2];
    }
    return FSA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Several blocks of one domain on one GPU (fsa_mb_*, see fsa.h): slabs along the last
// direction, each an ordinary context over its layers plus FSA_HALO halo layers per
// neighbour, stepped stage by stage with explicit halo copies and the cross-block maximum of
// the wave speeds after every stage.
// ---------------------------------------------------------------------------------------
struct fsa_mb {
    fsa_desc whole;
    int nb = 0, dir = 0, nq = 0;
    long long plane = 0;                     // cells of one layer across the slab direction
    bool periodic = false;
    hipStream_t stream = nullptr;            // the caller's: copies, wave speeds, joins
    std::vector<hipStream_t> bstream;        // one per block (default priority): the blocks'
    std::vector<hipEvent_t> bev;             // stages run side by side, joined by events
    hipEvent_t ev_main = nullptr;
    std::vector<fsa_ctx*> blk;
    std::vector<int> first, count, hlo, hhi;
    std::vector<fsa_desc> bdesc;
    std::vector<size_t> ws_off, q_off;       // workspace offsets of each block's context and state
    size_t copy_off = 0, slot_off = 0, total = 0;
    std::vector<double*> Q;                  // each block's state (own layers and halos)
    CopyEntry* d_copy[3] = {nullptr, nullptr, nullptr};   // halo copies of stage outputs Qa, Qb, Q
    int ncopy = 0;
    long long copy_max = 0;
    unsigned long long** d_slot_in = nullptr;   // per block: slot 1, its own maximum
    unsigned long long** d_slot_out = nullptr;  // per block: slot 0, the global maximum
    std::vector<std::vector<int>> marker_of;    // per block: global indices of its markers
    std::vector<int> owner, owner_idx;          // per marker: a block holding it, its index there
    int nm = 0;
    int motion = FSA_STATIC;
    double omega = 0.0;
    std::vector<double> dV;                     // every marker's quadrature weight
    bool markers_bad = false;                   // a marker call failed part-way: the blocks' sets
                                                // no longer match marker_of until fsa_mb_set_markers
    std::string err;
};

namespace {

int mb_fail(fsa_mb* m, int code, const std::string& msg)
{
    m->err = msg;
    return code;
}

// The blocks of desc in nb slabs and their descriptors and workspace layout (device
// pointers are not touched).
int mb_plan(fsa_mb* m, const fsa_desc* desc, int nb, std::string& why)
{
    int rc = validate(desc, why);
    if (rc == FSA_OK) rc = validate_caps(desc, why);
    if (rc != FSA_OK) return rc;
    for (int k = 0; k < 3; ++k)
        if (desc->origin[k] != 0 || desc->global_n[k] != 0) {
            why = "the whole domain's origin and global_n must be zero";
            return FSA_EINVAL;
        }
    if (nb < 1) { why = "nblocks must be positive"; return FSA_EINVAL; }
    m->whole = *desc;
    m->nb = nb;
    m->dir = desc->dim - 1;
    m->nq = desc->dim + 2;
    m->periodic = desc->bc[m->dir][0] == FSA_BC_PERIODIC;
    m->plane = desc->dim == 3 ? (long long)desc->n[0] * desc->n[1] : (long long)desc->n[0];
    const int N = desc->n[m->dir];
    m->first.assign(nb, 0);
    m->count.assign(nb, 0);
    m->hlo.assign(nb, 0);
    m->hhi.assign(nb, 0);
    m->bdesc.assign(nb, *desc);
    m->ws_off.assign(nb, 0);
    m->q_off.assign(nb, 0);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        const size_t at = off;
        off += std::max<size_t>(bytes, 1);
        return at;
    };
    int at = 0;
    for (int b = 0; b < nb; ++b) {
        m->first[b] = at;
        m->count[b] = N / nb + (b < N % nb ? 1 : 0);
        at += m->count[b];
        m->hlo[b] = (b > 0 || m->periodic) ? FSA_HALO : 0;
        m->hhi[b] = (b < nb - 1 || m->periodic) ? FSA_HALO : 0;
        if ((m->hlo[b] || m->hhi[b]) && m->count[b] < FSA_HALO) {
            why = "a block is thinner than FSA_HALO layers";
            return FSA_EINVAL;
        }
        fsa_desc& d = m->bdesc[b];
        d.n[m->dir] = m->hlo[b] + m->count[b] + m->hhi[b];
        for (int k = 0; k < desc->dim; ++k) d.global_n[k] = desc->n[k];
        d.origin[m->dir] = m->first[b] - m->hlo[b];
        if (m->hlo[b]) d.bc[m->dir][0] = FSA_BC_EXTRAP;
        if (m->hhi[b]) d.bc[m->dir][1] = FSA_BC_EXTRAP;
        size_t wb = 0;
        if ((rc = fsa_workspace_bytes(&d, &wb)) != FSA_OK) {
            why = "a block's descriptor is invalid";
            return rc;
        }
        m->ws_off[b] = take(wb);
        long long cells = m->plane * d.n[m->dir];
        m->q_off[b] = take(sizeof(double) * (size_t)m->nq * (size_t)cells);
    }
    const int nif = m->periodic ? nb : nb - 1;   // interfaces
    m->ncopy = 2 * m->nq * nif;
    m->copy_max = FSA_HALO * m->plane;
    m->copy_off = take(3 * sizeof(CopyEntry) * (size_t)std::max(m->ncopy, 1));
    m->slot_off = take(2 * sizeof(unsigned long long*) * (size_t)nb);
    m->total = off + 256;   // (room to align the base up)
    return FSA_OK;
}

// Copy list refreshing every halo from the neighbours' own layers, for stage buffers bufs[b].
std::vector<CopyEntry> mb_copies(const fsa_mb* m, const std::vector<double*>& bufs)
{
    std::vector<CopyEntry> e;
    const int H = FSA_HALO;
    const long long P = m->plane;
    auto cells = [&](int b) { return P * (long long)(m->hlo[b] + m->count[b] + m->hhi[b]); };
    for (int b = 0; b < m->nb; ++b) {
        const int up = b + 1 < m->nb ? b + 1 : (m->periodic ? 0 : -1);
        if (up < 0) continue;
        for (int c = 0; c < m->nq; ++c) {
            // b's upper halo <- up's first own layers; up's lower halo <- b's last own layers
            e.push_back({bufs[up] + c * cells(up) + (long long)m->hlo[up] * P,
                         bufs[b] + c * cells(b) + (long long)(m->hlo[b] + m->count[b]) * P, H * P});
            e.push_back({bufs[b] + c * cells(b) + (long long)(m->hlo[b] + m->count[b] - H) * P,
                         bufs[up] + c * cells(up), H * P});
        }
    }
    return e;
}

// Wave speeds of the own layers of every block's bufs[b], their maximum into every block's
// slot 0 (the start of a step call; between stages the stage kernels' partials serve).
int mb_alpha(fsa_mb* m, const std::vector<const double*>& bufs)
{
    for (int b = 0; b < m->nb; ++b) {
        fsa_ctx* c = m->blk[b];
        const int e = launch_alpha_rows(c->G, c->P, bufs[b], c->arow0, c->arow1, c->apart, c->abits + 3, m->stream);
        if (e) return mb_fail(m, FSA_EDEVICE, "wave-speed launch failed");
    }
    if (launch_amax_blocks(m->d_slot_in, m->d_slot_out, m->nb, m->stream))
        return mb_fail(m, FSA_EDEVICE, "cross-block maximum launch failed");
    return FSA_OK;
}

}  // namespace

extern "C" {

int32_t fsa_mb_workspace_bytes(const fsa_desc* desc, int32_t nblocks, size_t* bytes)
{
    if (!bytes) return FSA_EINVAL;
    *bytes = 0;
    fsa_mb m;
    std::string why;
    const int rc = mb_plan(&m, desc, nblocks, why);
    if (rc != FSA_OK) {
        std::fprintf(stderr, "fsa_mb_workspace_bytes: %s\n", why.c_str());
        return rc;
    }
    *bytes = m.total;
    return FSA_OK;
}

int32_t fsa_mb_init(const fsa_desc* desc, int32_t nblocks, void* d_workspace, size_t ws_bytes, void* hip_stream,
                    fsa_mb** out)
{
    if (!out) return FSA_EINVAL;
    *out = nullptr;
    fsa_mb* m = new (std::nothrow) fsa_mb();
    if (!m) return FSA_ENOMEM;
    std::string why;
    int rc = mb_plan(m, desc, nblocks, why);
    if (rc == FSA_OK && (!d_workspace || ws_bytes < m->total)) {
        why = "the workspace is smaller than fsa_mb_workspace_bytes";
        rc = FSA_EINVAL;
    }
    if (rc != FSA_OK) {
        std::fprintf(stderr, "fsa_mb_init: %s\n", why.c_str());
        delete m;
        return rc;
    }
    m->stream = (hipStream_t)hip_stream;
    char* base = (char*)(((uintptr_t)d_workspace + 255) & ~(uintptr_t)255);
    m->blk.assign(m->nb, nullptr);
    m->Q.assign(m->nb, nullptr);
    m->bstream.assign(m->nb, nullptr);
    m->bev.assign(m->nb, nullptr);
    if (hipEventCreateWithFlags(&m->ev_main, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        fsa_mb_destroy(m);
        return FSA_ENOMEM;
    }
    for (int b = 0; b < m->nb; ++b) {
        if (hipStreamCreateWithFlags(&m->bstream[b], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&m->bev[b], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            fsa_mb_destroy(m);
            return FSA_ENOMEM;
        }
        size_t wb = 0;
        fsa_workspace_bytes(&m->bdesc[b], &wb);
        if ((rc = fsa_init(&m->bdesc[b], base + m->ws_off[b], wb, m->bstream[b], &m->blk[b])) != FSA_OK) {
            fsa_mb_destroy(m);
            return rc;
        }
        m->Q[b] = reinterpret_cast<double*>(base + m->q_off[b]);
        // wave speeds from the block's own layers only; no quiet-tile skipping in the learned
        // form (the stage kernel's deviation ranges would include the halo layers' output
        // before the copies refresh them)
        m->blk[b]->arow0 = m->hlo[b];
        m->blk[b]->arow1 = m->hlo[b] + m->count[b];
        m->blk[b]->quiet_tiles = false;
    }
    // halo copy tables of the three stage outputs and the slot pointer lists
    for (int s = 0; s < 3; ++s) {
        std::vector<double*> bufs(m->nb);
        for (int b = 0; b < m->nb; ++b) bufs[b] = s == 0 ? m->blk[b]->Qa : (s == 1 ? m->blk[b]->Qb : m->Q[b]);
        const std::vector<CopyEntry> e = mb_copies(m, bufs);
        m->d_copy[s] = reinterpret_cast<CopyEntry*>(base + m->copy_off) + (size_t)s * std::max(m->ncopy, 1);
        if (!e.empty() && hipMemcpy(m->d_copy[s], e.data(), sizeof(CopyEntry) * e.size(), hipMemcpyHostToDevice) !=
                              hipSuccess) {
            fsa_mb_destroy(m);
            return FSA_EDEVICE;
        }
    }
    std::vector<unsigned long long*> slots(2 * (size_t)m->nb);
    for (int b = 0; b < m->nb; ++b) {
        slots[b] = m->blk[b]->abits + 3;
        slots[(size_t)m->nb + b] = m->blk[b]->abits;
    }
    m->d_slot_in = reinterpret_cast<unsigned long long**>(base + m->slot_off);
    m->d_slot_out = m->d_slot_in + m->nb;
    if (hipMemcpy(m->d_slot_in, slots.data(), sizeof(unsigned long long*) * slots.size(), hipMemcpyHostToDevice) !=
        hipSuccess) {
        fsa_mb_destroy(m);
        return FSA_EDEVICE;
    }
    m->marker_of.assign(m->nb, {});
    *out = m;
    return FSA_OK;
}

int32_t fsa_mb_destroy(fsa_mb* m)
{
    if (!m) return FSA_OK;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    for (fsa_ctx* c : m->blk) fsa_destroy(c);
    for (hipStream_t st : m->bstream)
        if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : m->bev)
        if (ev) (void)hipEventDestroy(ev);
    if (m->ev_main) (void)hipEventDestroy(m->ev_main);
    delete m;
    return FSA_OK;
}

const char* fsa_mb_last_error(const fsa_mb* m) { return m ? m->err.c_str() : "null block set"; }

int32_t fsa_mb_block_info(const fsa_mb* m, int32_t b, int32_t* first, int32_t* count, int32_t* halo_lo,
                          int32_t* halo_hi)
{
    if (!m || b < 0 || b >= m->nb) return FSA_EINVAL;
    if (first) *first = m->first[b];
    if (count) *count = m->count[b];
    if (halo_lo) *halo_lo = m->hlo[b];
    if (halo_hi) *halo_hi = m->hhi[b];
    return FSA_OK;
}

// The blocks whose own layers the support of each marker reaches, in the markers' global
// order (validating that every support lies inside the whole grid).
int mb_partition(fsa_mb* m, int n, const double* X, std::vector<std::vector<int>>& lists)
{
    const fsa_desc& w = m->whole;
    std::vector<int> j0(n);
    for (int k = 0; k < n; ++k)
        for (int d = 0; d < w.dim; ++d) {
            const double x = X[(size_t)d * n + k];
            if (!std::isfinite(x)) return mb_fail(m, FSA_EINVAL, "non-finite marker position");
            const double j = std::floor((x - w.lo[d]) / w.h - 0.5) - 1.0;
            if (j < 0.0 || j + 3.0 > (double)(w.n[d] - 1)) return mb_fail(m, FSA_EINVAL, "a marker support leaves the grid");
            if (d == m->dir) j0[k] = (int)j;
        }
    lists.assign(m->nb, {});
    for (int b = 0; b < m->nb; ++b) {
        const int lo = m->first[b], hi = m->first[b] + m->count[b] - 1;
        for (int k = 0; k < n; ++k)
            if (j0[k] + 3 >= lo && j0[k] <= hi) lists[b].push_back(k);
    }
    return FSA_OK;
}

// Block b's slice of the markers' host arrays ([dim][n]) for its list.
void mb_slice(const fsa_mb* m, const std::vector<int>& list, int n, const double* A, std::vector<double>& out)
{
    const int dim = m->whole.dim, nbk = (int)list.size();
    out.assign((size_t)dim * nbk, 0.0);
    if (!A) return;
    for (int i = 0; i < nbk; ++i)
        for (int d = 0; d < dim; ++d) out[(size_t)d * nbk + i] = A[(size_t)d * n + list[i]];
}

void mb_owners(fsa_mb* m)
{
    m->owner.assign(m->nm, -1);
    m->owner_idx.assign(m->nm, -1);
    for (int b = 0; b < m->nb; ++b)
        for (int i = 0; i < (int)m->marker_of[b].size(); ++i) {
            const int k = m->marker_of[b][i];
            if (m->owner[k] < 0) {
                m->owner[k] = b;
                m->owner_idx[k] = i;
            }
        }
}

int32_t fsa_mb_set_markers(fsa_mb* m, int32_t n, const double* X, const double* dV, const double* U, int32_t motion,
                           double omega)
{
    if (!m || n < 0 || (n > 0 && (!X || !dV))) return FSA_EINVAL;
    if (motion < FSA_STATIC || motion > FSA_EXTERNAL) return mb_fail(m, FSA_EINVAL, "bad motion");
    std::vector<std::vector<int>> lists;
    if (int rc = mb_partition(m, n, X, lists)) return rc;
    m->markers_bad = true;
    m->nm = n;
    m->motion = motion;
    m->omega = omega;
    m->dV.assign(dV ? dV : nullptr, dV ? dV + n : nullptr);
    for (int b = 0; b < m->nb; ++b) {
        m->marker_of[b] = lists[b];
        const int nbk = (int)lists[b].size();
        std::vector<double> Xb, Ub, dVb(nbk);
        mb_slice(m, lists[b], n, X, Xb);
        mb_slice(m, lists[b], n, U, Ub);
        for (int i = 0; i < nbk; ++i) dVb[i] = dV[lists[b][i]];
        const int rc = fsa_set_markers(m->blk[b], nbk, Xb.data(), dVb.data(), U ? Ub.data() : nullptr, motion, omega);
        if (rc != FSA_OK) return mb_fail(m, rc, std::string("block marker set: ") + fsa_last_error(m->blk[b]));
    }
    mb_owners(m);
    m->markers_bad = false;
    return FSA_OK;
}

int32_t fsa_mb_set_marker_kinematics(fsa_mb* m, const double* X, const double* U)
{
    if (!m || !X) return FSA_EINVAL;
    if (m->markers_bad) return mb_fail(m, FSA_ESTATE, "the markers are undefined after a failed call: set them again");
    if (m->nm == 0 || m->motion != FSA_EXTERNAL) return mb_fail(m, FSA_ESTATE, "markers are not EXTERNAL");
    const int n = m->nm, dim = m->whole.dim;
    std::vector<std::vector<int>> lists;
    if (int rc = mb_partition(m, n, X, lists)) return rc;
    bool moved = false;
    for (int b = 0; b < m->nb; ++b) moved = moved || lists[b] != m->marker_of[b];
    // the penalty integral of every marker, from a block holding it, when a marker's supports
    // reach another set of blocks now (every holder keeps the same values)
    std::vector<double> xi;
    if (moved) {
        xi.assign((size_t)dim * n, 0.0);
        for (int b = 0; b < m->nb; ++b) {
            const std::vector<int>& old = m->marker_of[b];
            if (old.empty()) continue;
            std::vector<double> xb((size_t)dim * old.size());
            if (int rc = fsa_get_state(m->blk[b], xb.data(), nullptr, nullptr)) return mb_fail(m, rc, "block state");
            for (int i = 0; i < (int)old.size(); ++i)
                for (int d = 0; d < dim; ++d) xi[(size_t)d * n + old[i]] = xb[(size_t)d * old.size() + i];
        }
    }
    m->markers_bad = true;
    for (int b = 0; b < m->nb; ++b) {
        std::vector<double> Xb, Ub;
        mb_slice(m, lists[b], n, X, Xb);
        mb_slice(m, lists[b], n, U, Ub);
        int rc = FSA_OK;
        if (lists[b] == m->marker_of[b]) {
            if (!lists[b].empty()) rc = fsa_set_marker_kinematics(m->blk[b], Xb.data(), U ? Ub.data() : nullptr);
        } else {
            const int nbk = (int)lists[b].size();
            std::vector<double> dVb(nbk), xb;
            for (int i = 0; i < nbk; ++i) dVb[i] = m->dV[lists[b][i]];
            mb_slice(m, lists[b], n, xi.data(), xb);
            double t = 0.0;
            int64_t step = 0;
            rc = fsa_get_state(m->blk[b], nullptr, &t, &step);
            if (rc == FSA_OK)
                rc = fsa_set_markers(m->blk[b], nbk, Xb.data(), dVb.data(), U ? Ub.data() : nullptr, FSA_EXTERNAL, 0.0);
            if (rc == FSA_OK) rc = fsa_set_state(m->blk[b], nbk ? xb.data() : nullptr, t, step);
            m->marker_of[b] = lists[b];
        }
        if (rc != FSA_OK) return mb_fail(m, rc, std::string("block kinematics: ") + fsa_last_error(m->blk[b]));
    }
    mb_owners(m);
    m->markers_bad = false;
    return FSA_OK;
}

int32_t fsa_mb_scatter(fsa_mb* m, const double* d_Q)
{
    if (!m || !d_Q) return FSA_EINVAL;
    const int N = m->whole.n[m->dir];
    const long long P = m->plane, whole_cells = P * N;
    for (int b = 0; b < m->nb; ++b) {
        const int nl = m->hlo[b] + m->count[b] + m->hhi[b];
        const long long bcells = P * nl;
        // runs of local layers whose global layers are consecutive (halos may wrap)
        int L = 0;
        while (L < nl) {
            const int g0 = ((m->first[b] - m->hlo[b] + L) % N + N) % N;
            const int len = std::min(nl - L, N - g0);
            for (int c = 0; c < m->nq; ++c)
                if (hipMemcpyAsync(m->Q[b] + c * bcells + (long long)L * P, d_Q + c * whole_cells + (long long)g0 * P,
                                   sizeof(double) * (size_t)(len * P), hipMemcpyDeviceToDevice, m->stream) != hipSuccess)
                    return mb_fail(m, FSA_EDEVICE, "scatter copy failed");
            L += len;
        }
        // a fresh start: time, step and penalty integral zero
        fsa_ctx* c = m->blk[b];
        if (c->nm > 0) {
            std::vector<double> zero((size_t)c->d.dim * c->nm, 0.0);
            const int rc = fsa_set_state(c, zero.data(), 0.0, 0);
            if (rc != FSA_OK) return mb_fail(m, rc, std::string("block state: ") + fsa_last_error(c));
        } else {
            c->t = 0.0;
            c->step = 0;
        }
    }
    return FSA_OK;
}

int32_t fsa_mb_gather(const fsa_mb* m, double* d_Q)
{
    if (!m || !d_Q) return FSA_EINVAL;
    const long long P = m->plane, whole_cells = P * m->whole.n[m->dir];
    for (int b = 0; b < m->nb; ++b) {
        const long long bcells = P * (m->hlo[b] + m->count[b] + m->hhi[b]);
        for (int c = 0; c < m->nq; ++c)
            if (hipMemcpyAsync(d_Q + c * whole_cells + (long long)m->first[b] * P,
                               m->Q[b] + c * bcells + (long long)m->hlo[b] * P, sizeof(double) * (size_t)(m->count[b] * P),
                               hipMemcpyDeviceToDevice, m->stream) != hipSuccess)
                return FSA_EDEVICE;
    }
    return FSA_OK;
}

int32_t fsa_mb_rk3_steps(fsa_mb* m, double dt, int32_t nsteps)
{
    if (!m) return FSA_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return mb_fail(m, FSA_EINVAL, "dt must be positive");
    if (nsteps < 1) return mb_fail(m, FSA_EINVAL, "nsteps must be positive");
    if (m->markers_bad) return mb_fail(m, FSA_ESTATE, "the markers are undefined after a failed call: set them again");
    static const double CA[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double CB[3] = {1.0, 0.25, 2.0 / 3.0};
    std::vector<const double*> bufs(m->nb);
    for (int b = 0; b < m->nb; ++b) {
        m->blk[b]->advanced = nullptr;
        bufs[b] = m->Q[b];
    }
    int rc = mb_alpha(m, bufs);   // the states' wave speeds
    if (rc != FSA_OK) return rc;
    for (int n = 0; n < nsteps; ++n) {
        for (int s = 0; s < 3; ++s) {
            // the blocks' stages side by side on their streams, after the caller's stream
            // (copies, wave speeds), which then waits for all of them
            if (hipEventRecord(m->ev_main, m->stream) != hipSuccess) return mb_fail(m, FSA_EDEVICE, "event record");
            for (int b = 0; b < m->nb; ++b) {
                fsa_ctx* c = m->blk[b];
                if (hipStreamWaitEvent(m->bstream[b], m->ev_main, 0) != hipSuccess)
                    return mb_fail(m, FSA_EDEVICE, "stream wait");
                const double* Qs = s == 0 ? m->Q[b] : (s == 1 ? c->Qa : c->Qb);
                double* out = s == 0 ? c->Qa : (s == 1 ? c->Qb : m->Q[b]);
                // the stage kernel's wave-speed partials of the block's own layers, reduced into
                // its slot 1 on its stream
                if ((rc = enqueue_stage(c, Qs, m->Q[b], out, 0, 1, false, s + 1, CA[s], CB[s], dt, 0)) != FSA_OK ||
                    (rc = flush_alpha_final(c)) != FSA_OK)
                    return mb_fail(m, rc, std::string("block stage: ") + fsa_last_error(c));
                bufs[b] = out;
                if (hipEventRecord(m->bev[b], m->bstream[b]) != hipSuccess ||
                    hipStreamWaitEvent(m->stream, m->bev[b], 0) != hipSuccess)
                    return mb_fail(m, FSA_EDEVICE, "stream join");
            }
            if (launch_copy_list(m->d_copy[s], m->ncopy, m->copy_max, m->stream) ||
                launch_amax_blocks(m->d_slot_in, m->d_slot_out, m->nb, m->stream))
                return mb_fail(m, FSA_EDEVICE, "halo copy or cross-block maximum launch failed");
        }
        for (fsa_ctx* c : m->blk) {
            c->t += dt;
            c->step += 1;
        }
    }
    return FSA_OK;
}

int32_t fsa_mb_marker_force(fsa_mb* m, double* h_F)
{
    if (!m || !h_F) return FSA_EINVAL;
    if (m->markers_bad) return mb_fail(m, FSA_ESTATE, "the markers are undefined after a failed call: set them again");
    const int dim = m->whole.dim;
    for (int b = 0; b < m->nb; ++b) {
        const int nbk = (int)m->marker_of[b].size();
        if (nbk == 0) continue;
        std::vector<double> F((size_t)dim * nbk);
        const int rc = fsa_marker_force(m->blk[b], F.data());
        if (rc != FSA_OK) return mb_fail(m, rc, "block marker force");
        for (int i = 0; i < nbk; ++i) {
            const int k = m->marker_of[b][i];
            if (m->owner[k] != b) continue;
            for (int d = 0; d < dim; ++d) h_F[(size_t)d * m->nm + k] = F[(size_t)d * nbk + i];
        }
    }
    return FSA_OK;
}

}  // extern "C"
