// Fused 2D right-hand side / SSP-RK3 stage kernel for gfx950.
//
// One wave64 owns a column strip of 64 consecutive x cells (56 outputs plus a 4-cell halo
// on each side) and marches along y over a segment of rows.  Per front row it loads the
// state once, forms the y-split fluxes f+-_y and the velocities, and keeps them in register
// windows (five rows, slot = row mod 5 fixed at compile time by unrolling the march by 5),
// so every y-face is reconstructed exactly once.  x-neighbours come from the neighbouring
// lanes of the same wave through DPP wave shifts.  The viscous stress (Sec. 2, Eqs. (5)-(6),
// fourth-order central differences applied twice) lags the front by two rows, the output
// row by four.  The output row combines, in this order, the x and y convective terms, the
// viscous term and the sources (penalty-IB force from the window array, sponge), and
// writes either L(Q) or the SSP-RK3 combination a Qn + b (Qs + dt L); it also accumulates
// the global Lax-Friedrichs speeds of what it writes for the next stage.
//
// Boundary ghosts are resolved once per lane for x and once per row (a wave-uniform value)
// for y; only inflow ghosts take the slow path.  Each state value is loaded from memory once
// per wave: the output row is read back from a lane-private LDS ring of the last five front
// rows.  Constants live in a device-side block and are read where they are used.
//
// Arithmetic type T of the reconstruction and viscous fluxes: double (the FP64 method) or
// float (the precision form).  In the precision form the windows hold, in FP32, the split
// fluxes minus those of the far-field state, formed in FP64 before rounding; the far-field
// part cancels exactly in the flux difference, so FP32 only ever carries deviations.  The
// state, the sources, the RK3 combination and the wave speeds stay FP64.
#include <algorithm>
#include <type_traits>

#include "fsa_impl.hpp"

namespace fsa {

namespace {

constexpr int HALO = 4;
constexpr int WAVE = 64;
constexpr int OUTW = WAVE - 2 * HALO;   // 56 output columns per wave

// Lane shifts across the whole wave with DPP: wave_shr:1 gives lane i the value of lane i-1,
// wave_shl:1 the value of lane i+1 (bound_ctrl: lanes without a source read 0, so no old
// value has to be set up first; only halo lanes read it).
constexpr int DPP_WAVE_SHR1 = 0x138;
constexpr int DPP_WAVE_SHL1 = 0x130;

template <int CTRL>
__device__ __forceinline__ double dpp(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <class T>
__device__ __forceinline__ T lo1(T x) { return dpp<DPP_WAVE_SHR1>(x); }
template <class T>
__device__ __forceinline__ T up1(T x) { return dpp<DPP_WAVE_SHL1>(x); }

// Fourth-order central first derivative from the values at offsets -2..+2 (times 1/(12h)).
template <class T>
__device__ __forceinline__ T d1(T gm2, T gm1, T gp1, T gp2, T inv12h)
{
    return (T(8) * (gp1 - gm1) - (gp2 - gm2)) * inv12h;
}

template <class T>
__device__ __forceinline__ T d1_lanes(T g, T inv12h)
{
    const T l1 = lo1(g), u1 = up1(g);
    return d1(lo1(l1), l1, u1, up1(u1), inv12h);
}

template <int SCHEME>
__device__ __forceinline__ double recon(double a, double b, double c, double d, double e, const Recon& R,
                                        const Recon32&)
{
    return recon5<SCHEME>(a, b, c, d, e, R);
}
template <int SCHEME>
__device__ __forceinline__ float recon(float a, float b, float c, float d, float e, const Recon&, const Recon32& R)
{
    return recon5f<SCHEME>(a, b, c, d, e, R);
}

// Face value of one side: the scheme's own weights, or (learned form) the keep-pattern row
// given by its coefficients.
template <int SCHEME, class T>
__device__ __forceinline__ T recon_side(T a, T b, T c, T d, T e, const Recon& R, const Recon32& R32,
                                        const float (&coef)[5])
{
    if constexpr (SCHEME == LEARNED) {
        (void)R;
        (void)R32;
        return keep_sum(coef, a, b, c, d, e);
    } else {
        (void)coef;
        return recon<SCHEME>(a, b, c, d, e, R, R32);
    }
}

// Learned form: the keep-pattern rows of both sides of components C0, C0+1 of one face word,
// all read before any is used so that the LDS reads overlap.
template <int SCHEME, int C0>
__device__ __forceinline__ void face_rows(unsigned word, bool all_kept, const float (*rows)[8], float (&cp)[4][5],
                                          float (&cm)[4][5])
{
    if constexpr (SCHEME == LEARNED) {
#pragma unroll
        for (int c = C0; c < C0 + 2; ++c) {
            const int bp = all_kept ? 7 : (int)(word >> (3 * c)) & 7;
            const int bm = all_kept ? 7 : (int)(word >> (16 + 3 * c)) & 7;
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                cp[c][j] = rows[bp][j];
                cm[c][j] = rows[bm][j];
            }
        }
    } else {
        (void)word;
        (void)all_kept;
        (void)rows;
        (void)cp;
        (void)cm;
    }
}

template <class T>
constexpr bool F64v = std::is_same<T, double>::value;

// Learned form: a face word (both sides) in which every component keeps every sub-stencil.
constexpr unsigned ALL_KEPT2 = 0x0FFF0FFFu;

// True when the learned form's face words of the whole wave keep everything: the faces then
// take the all-kept table row at a compile-time index (no lookup waits on the word).
template <int SCHEME>
__device__ __forceinline__ bool wave_all_kept(unsigned word)
{
    if constexpr (SCHEME == LEARNED) return __ballot(word != ALL_KEPT2) == 0ull;
    else return false;
}

template <int SCHEME, class T, bool DBG = false, bool NR = false>
struct Column2D {
    static constexpr bool F64 = std::is_same<T, double>::value;
    // Rows of loads in flight ahead of their use: the FP32 forms have less arithmetic per row
    // to cover memory latency with, and the registers for a second row.
    static constexpr int PF = F64 ? 1 : 2;
    const KConst* __restrict__ K;   // grid and physics constants (device memory)
    const double* __restrict__ Qs;
    const double* Qn;               // may alias out (last stage writes in place)
    double* out;
    const double* __restrict__ fwin;
    const unsigned* __restrict__ flags_x;
    const unsigned* __restrict__ flags_y;
    long long ncell;
    int nx, ny, bcy0, bcy1;
    double sigma;                   // sponge sigma_max (0 when the sponge term is off)
    // far-field constants used per row, read once at kernel start: a load from the constant
    // block inside the march waits for every LDS access in flight (FP32 forms; the FP64
    // kernel has no registers to spare and reads them where they are used)
    double qinf[4], Fxinf[4], Fyinf[4], rinf, uinf, vinf, pinf, gamma;
    int wlo0, wlo1, wn0, wn1;
    double ax, ay, inv_h, gm1, ca, cb, dt;
    T inv_hT, inv12h, mu;
    Recon R;
    Recon32 R32;
    int mode_rhs, terms;
    int j0, j1;
    int xr;                         // resolved x index of this lane
    int i;                          // x index of this lane (a ghost index in the halo)
    bool x_inflow;                  // this lane is an inflow ghost column
    bool xg_wave;                   // some lane of this wave is (wave-uniform)
    const double* ghosts;           // inflow ghost states of the step, [c][side][depth-1][along]
    long long gcs;                  // their component stride
    int gna;                        // their position stride
    int gxo;                        // x inflow ghost lanes: offset of their side and depth
    bool out_lane;
    bool want_alpha;
    float* qrange;                  // learned form: deviation ranges of the output (or null)
    float (*rng)[WAVE];             // LDS [8][lane]: this lane's least / largest output deviations
    double sg_x;                    // sponge rate sigma * eta^3 of this lane's column
    double sg_rows;                 // sponge rate of row sg_base + lane
    int sg_base;
    unsigned long long amax_x, amax_y;
    int ar0, ar1;                   // rows whose cells enter the wave-speed maximum
    long long step;
    // register windows, slot = (row - first front row) mod 5
    T fp[5][4], fm[5][4];
    T uw[5], vw[5];                 // velocities (minus the far-field velocity in FP32)
    T txy[5], tyy[5];               // stresses used in y derivatives stay in registers
    T (*vring)[3][WAVE];            // LDS: tau_xx, b_x, b_y of the last five stress rows, [slot][.][lane]
    T fy_prev[4], cy_queue[4];
    double qf[PF][4];               // prefetched state of the next PF front rows
    unsigned wy_pf[PF], wx_pf[PF];  // learned form: prefetched keep patterns of the next PF steps
    double qn_pf[PF][4];            // step-start state of the next PF output rows (stages 2 and 3)
    double fw_pf[PF][2];            // penalty-IB force window values of the next PF output rows
    bool ib_on;                     // the force window is present and overlaps this strip
    double (*ring)[4][WAVE];        // LDS: the last five front rows of this wave, [slot][comp][lane]
    int lane;
    bool nrbc_x;                    // this lane's cell is the boundary cell of a non-reflecting
                                    // x side (its x convective term is left to launch_nrbc)
    int nrbc;                       // the non-reflecting sides (StageArgs::nrbc)
    unsigned* dbg_x;                // DBG (FP64 TENO5 only): the keep patterns of every x face
    unsigned* dbg_y;                // [ny][nx+1] and y face [ny+1][nx] this stage decides

    // State of (this lane, row j): interior and periodic/zero-gradient ghosts are loads of
    // their resolved cell; inflow ghosts (an x ghost lane's column, or a whole y ghost row)
    // are loads from the step's ghost table.  Every lane's q is one load per component, so
    // no write ever lands on a register a load in flight will fill (such a write would wait
    // for all loads in flight, the prefetches included).  Waves without inflow ghosts take
    // the plain path (a wave-uniform branch).
    __device__ __forceinline__ void load_row(int j, double* q) const
    {
        int inflow = 0, side = 0, depth = 0;
        const int jr = resolve_index(j, ny, bcy0, bcy1, 1, inflow, side, depth);
        if (xg_wave || inflow) {
            // an x inflow side comes first, as in the boundary rule (x, then y)
            const bool g = x_inflow || inflow;
            const long long o = x_inflow ? (long long)gxo + jr
                                         : (inflow ? (long long)(side * HALO + depth - 1) * gna + xr
                                                   : (long long)jr * nx + xr);
            const double* p = (g ? ghosts : Qs) + o;
            const long long cs = g ? gcs : ncell;
#pragma unroll
            for (int c = 0; c < 4; ++c) q[c] = p[c * cs];
        } else {
            const double* p = Qs + (long long)jr * nx + xr;
#pragma unroll
            for (int c = 0; c < 4; ++c) q[c] = p[c * ncell];
        }
    }

    // Split fluxes f+- = (F +- alpha Q)/2 of component c of one direction, as stored in the
    // windows (relative to the far field in FP32).
    __device__ __forceinline__ void split(int c, double q, double F, double Finf, double alpha, T& fplus,
                                          T& fminus) const
    {
        if (F64) {
            fminus = (T)(0.5 * fma(-alpha, q, F));
            fplus = (T)(0.5 * fma(alpha, q, F));
        } else {
            const double dq = q - qinf[c], dF = F - Finf;
            fminus = (T)(0.5 * fma(-alpha, dq, dF));
            fplus = (T)(0.5 * fma(alpha, dq, dF));
        }
    }

    // Learned form: keep patterns of the y face (R-3)+1/2 and the x face right of this lane
    // in output row R-4, the faces step R reconstructs (rows clamped into range; the loads
    // of steps that do not use them are harmless).
    __device__ __forceinline__ void load_patterns(int R, int slot)
    {
        if constexpr (SCHEME == LEARNED) {
            const int jy = min(max(R - 2, 0), ny), jx = min(max(R - 4, 0), ny - 1);
            wy_pf[slot] = flags_y[(long long)jy * nx + xr];
            wx_pf[slot] = flags_x[(long long)jx * (nx + 1) + min(max(i + 1, 0), nx)];
        }
    }

    // Step-start state Qn of output row r for this lane (issued PF steps before it is used,
    // so the load latency hides behind rows of work).  Rows outside the segment and halo
    // lanes load an in-range cell whose value is not used (a cache hit on a row the wave
    // loads anyway), so the load needs no lane mask.  Issued in every stage, also where the
    // combination does not read it (Qn is then the stage input): four loads that always
    // follow the front-row load let the wait for that load, one step later, leave the
    // younger loads and the stores in flight; with an issue that depended on the stage, the
    // wait would have to assume none follow and drain everything.
    __device__ __forceinline__ void load_qn(int r, int slot)
    {
        const long long o = (long long)min(max(r, j0), j1) * nx + xr;
#pragma unroll
        for (int c = 0; c < 4; ++c) qn_pf[slot][c] = Qn[c * ncell + o];
    }

    // Force-window values (f_x, f_y) of output row r at this lane's column, issued PF steps
    // before use like the other loads (a load used at once would wait for every load in
    // flight, the prefetches included).  Rows outside the window give zero; lanes outside it
    // load an in-range cell and are masked where the values are used.
    __device__ __forceinline__ void load_fwin(int r, int slot)
    {
        fw_pf[slot][0] = fw_pf[slot][1] = 0.0;
        const int wj = r - wlo1;
        if (ib_on && wj >= 0 && wj < wn1) {
            const long long wc = (long long)wj * wn0 + min(max(i - wlo0, 0), wn0 - 1);
            fw_pf[slot][0] = fwin[wc];
            fw_pf[slot][1] = fwin[(long long)wn0 * wn1 + wc];
        }
    }

    __device__ __forceinline__ double q_inf(int c) const { return F64 ? K->P.q_inf[c] : qinf[c]; }
    // gamma (FP64: formed as (gamma - 1) + 1, which is exact, gamma - 1 being exact for
    // gamma > 1: no scalar load inside the march)
    __device__ __forceinline__ double gam() const { return F64 ? gm1 + 1.0 : gamma; }

    // Sponge rate sigma * eta^3 (zero when the sponge term is off).
    __device__ __forceinline__ double sponge_rate(double eta) const { return sigma * (eta * eta * eta); }

    // Sponge rate sigma * eta_y^3 of row r.  Each lane holds the rate of one of 64
    // consecutive rows, refilled when r leaves them (r increases by one per call; called with
    // all lanes active), and the row's value is a lane read instead of the profile arithmetic
    // and its constant-block loads (scalar loads in the march wait for every LDS access in
    // flight).
    __device__ __forceinline__ double sponge_row(int r)
    {
        if (r - sg_base >= WAVE) {
            sg_base = r;
            sg_rows = sponge_rate(K->eta_dir(1, r + lane));
        }
        const int k = r - sg_base;
        const long long b = __double_as_longlong(sg_rows);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
        return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    }

    template <int K5>
    __device__ __forceinline__ void step_row(int Rw)
    {
        constexpr int S0 = K5 % 5;          // row Rw (and row Rw-5 before it is overwritten)
        constexpr int S1 = (K5 + 4) % 5;    // row Rw-1
        constexpr int S2 = (K5 + 3) % 5;    // row Rw-2
        constexpr int S3 = (K5 + 2) % 5;    // row Rw-3
        constexpr int S4 = (K5 + 1) % 5;    // row Rw-4
        const bool do_out = Rw >= j0 + 4;
        const int r = Rw - 4;

        // state of the output row, kept in LDS since it was the front row four steps ago
        // (each lane reads back only what it wrote, so no barrier is involved)
        double qr[4] = {0.0, 0.0, 0.0, 0.0};
        if (do_out) {
#pragma unroll
            for (int c = 0; c < 4; ++c) qr[c] = ring[S4][c][lane];
        }

        // ---- front row Rw (prefetched in the previous step): velocity and y-split fluxes
        const double q[4] = {qf[0][0], qf[0][1], qf[0][2], qf[0][3]};
#pragma unroll
        for (int c = 0; c < 4; ++c) ring[S0][c][lane] = q[c];
        const unsigned word_y = wy_pf[0], word_x = wx_pf[0];
        const double qn[4] = {qn_pf[0][0], qn_pf[0][1], qn_pf[0][2], qn_pf[0][3]};
        const double fw[2] = {fw_pf[0][0], fw_pf[0][1]};
#pragma unroll
        for (int s = 0; s + 1 < PF; ++s) {
            wy_pf[s] = wy_pf[s + 1];
            wx_pf[s] = wx_pf[s + 1];
            fw_pf[s][0] = fw_pf[s + 1][0];
            fw_pf[s][1] = fw_pf[s + 1][1];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                qf[s][c] = qf[s + 1][c];
                qn_pf[s][c] = qn_pf[s + 1][c];
            }
        }
        load_row(Rw + PF, qf[PF - 1]);
        load_patterns(Rw + PF, PF - 1);
        load_qn(Rw - 4 + PF, PF - 1);
        load_fwin(Rw - 4 + PF, PF - 1);
        const double inv_rho = rcp_nr(q[0]);
        const double u = q[1] * inv_rho, v = q[2] * inv_rho;
        const double p = gm1 * (q[3] - 0.5 * fma(q[1], u, q[2] * v));
        T fpr[4];
        {
            const double F[4] = {q[2], q[1] * v, fma(q[2], v, p), (q[3] + p) * v};
#pragma unroll
            for (int c = 0; c < 4; ++c) split(c, q[c], F[c], Fyinf[c], ay, fpr[c], fm[S0][c]);
        }
        if (F64) {
            uw[S0] = (T)u;
            vw[S0] = (T)v;
        } else {
            uw[S0] = (T)(u - uinf);
            vw[S0] = (T)(v - vinf);
        }

        // ---- y face (Rw-3)+1/2: f+ rows Rw-5..Rw-1, f- rows Rw..Rw-4
        T cy_new[4] = {T(0), T(0), T(0), T(0)};
        if ((terms & T_CONVY) && Rw >= j0 + 2 && Rw <= j1 + 3) {
            auto yface = [&](auto all_kept) {
                float cp[4][5], cm[4][5];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c == 0) face_rows<SCHEME, 0>(word_y, all_kept, R32.rows, cp, cm);
                    if (c == 2) face_rows<SCHEME, 2>(word_y, all_kept, R32.rows, cp, cm);
                    const T fh =
                        recon_side<SCHEME, T>(fp[S0][c], fp[S4][c], fp[S3][c], fp[S2][c], fp[S1][c], R, R32, cp[c]) +
                        recon_side<SCHEME, T>(fm[S0][c], fm[S1][c], fm[S2][c], fm[S3][c], fm[S4][c], R, R32, cm[c]);
                    cy_new[c] = -(fh - fy_prev[c]) * inv_hT;
                    fy_prev[c] = fh;
                }
                if constexpr (DBG) {
                    // the decisions recon5 took above, on the same values: face (Rw-3)+1/2 is
                    // y face Rw-2
                    unsigned word = 0u;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        word |= (unsigned)teno_keep5(fp[S0][c], fp[S4][c], fp[S3][c], fp[S2][c], fp[S1][c], R) << (3 * c);
                        word |= (unsigned)teno_keep5(fm[S0][c], fm[S1][c], fm[S2][c], fm[S3][c], fm[S4][c], R)
                                << (16 + 3 * c);
                    }
                    if (out_lane) dbg_y[(long long)(Rw - 2) * nx + i] = word;
                }
            };
            if (wave_all_kept<SCHEME>(word_y)) yface(std::true_type{});
            else yface(std::false_type{});
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) fp[S0][c] = fpr[c];

        // ---- stress at row Rw-2 (velocities of rows Rw-4..Rw in the window)
        if ((terms & T_VISC) && Rw >= j0) {
            const T uc = uw[S2], vc = vw[S2];
            const T dudx = d1_lanes(uc, inv12h), dvdx = d1_lanes(vc, inv12h);
            const T dudy = d1(uw[S4], uw[S3], uw[S1], uw[S0], inv12h);
            const T dvdy = d1(vw[S4], vw[S3], vw[S1], vw[S0], inv12h);
            const T div = dudx + dvdy;
            const T sxx = mu * fma(T(-2.0 / 3.0), div, dudx + dudx);
            const T syy = mu * fma(T(-2.0 / 3.0), div, dvdy + dvdy);
            const T sxy = mu * (dudy + dvdx);
            vring[S2][0][lane] = sxx;
            txy[S2] = sxy;
            tyy[S2] = syy;
            const T uf = F64 ? uc : uc + (T)uinf;
            const T vf = F64 ? vc : vc + (T)vinf;
            vring[S2][1][lane] = fma(uf, sxx, vf * sxy);
            vring[S2][2][lane] = fma(uf, sxy, vf * syy);
        }

        // ---- output row r = Rw-4
        if (do_out) {
            // (a wave-uniform point: the lane table of sponge rates is refilled by every lane)
            const double sg_y = sponge_row(r);
            double ur, vr;
            if (F64) {
                ur = (double)uw[S4];
                vr = (double)vw[S4];
            } else {
                const double ir = rcp_nr(qr[0]);
                ur = qr[1] * ir;
                vr = qr[2] * ir;
            }
            double L[4] = {0.0, 0.0, 0.0, 0.0};
            if (terms & T_CONVX) {
                const double pr = gm1 * (qr[3] - 0.5 * fma(qr[1], ur, qr[2] * vr));
                const double F[4] = {qr[1], fma(qr[1], ur, pr), qr[2] * ur, (qr[3] + pr) * ur};
                auto xface = [&](auto all_kept) {
                    float cp[4][5], cm[4][5];
                    unsigned dword = 0u;
                    (void)dword;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (c == 0) face_rows<SCHEME, 0>(word_x, all_kept, R32.rows, cp, cm);
                        if (c == 2) face_rows<SCHEME, 2>(word_x, all_kept, R32.rows, cp, cm);
                        T fpx, fmx;
                        split(c, qr[c], F[c], Fxinf[c], ax, fpx, fmx);
                        const T pl1 = lo1(fpx), pu1 = up1(fpx);
                        const T ml1 = lo1(fmx), mu1 = up1(fmx), mu2 = up1(mu1);
                        const T fh = recon_side<SCHEME, T>(lo1(pl1), pl1, fpx, pu1, up1(pu1), R, R32, cp[c]) +
                                     recon_side<SCHEME, T>(up1(mu2), mu2, mu1, fmx, ml1, R, R32, cm[c]);
                        L[c] = (double)(-(fh - lo1(fh)) * inv_hT);
                        if constexpr (DBG) {
                            // x face i+1 (right of this lane) of row r, decided above on the same
                            // values
                            dword |= (unsigned)teno_keep5(lo1(pl1), pl1, fpx, pu1, up1(pu1), R) << (3 * c);
                            dword |= (unsigned)teno_keep5(up1(mu2), mu2, mu1, fmx, ml1, R) << (16 + 3 * c);
                        }
                    }
                    if constexpr (DBG) {
                        if ((out_lane || lane == HALO - 1) && i >= -1 && i + 1 <= nx)
                            dbg_x[(long long)r * (nx + 1) + i + 1] = dword;
                    }
                };
                if (wave_all_kept<SCHEME>(word_x)) xface(std::true_type{});
                else xface(std::false_type{});
                if constexpr (NR) {
                    if (nrbc_x) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) L[c] = 0.0;
                    }
                }
            }
            if ((terms & T_CONVY) && !(NR && (((nrbc & 4) && r == 0) || ((nrbc & 8) && r == ny - 1)))) {
#pragma unroll
                for (int c = 0; c < 4; ++c) L[c] += (double)cy_queue[c];
            }
            if (terms & T_VISC) {
                // rows r-2..r+2 sit in slots S1, S0, S4, S3, S2
                // tau_xx, b_x of row r and b_y of rows r-2..r+2 from the wave's LDS ring (each
                // lane reads back only what it wrote)
                const T vx = d1_lanes(vring[S4][0][lane], inv12h) + d1(txy[S1], txy[S0], txy[S3], txy[S2], inv12h);
                const T vy = d1_lanes(txy[S4], inv12h) + d1(tyy[S1], tyy[S0], tyy[S3], tyy[S2], inv12h);
                const T ve = d1_lanes(vring[S4][1][lane], inv12h) +
                             d1(vring[S1][2][lane], vring[S0][2][lane], vring[S3][2][lane], vring[S2][2][lane], inv12h);
                L[1] += (double)vx;
                L[2] += (double)vy;
                L[3] += (double)ve;
            }
            // Sources, the stage combination and the wave speeds.  FP32 forms: formed on every
            // lane (the halo lanes' values are discarded), so that only the stores and the
            // wave-speed maximum depend on the lane and the tail of the row is one scheduling
            // region.  FP64: on the output lanes only (its registers are all taken; the
            // branch keeps the halo lanes' values from being live).  A zero force or sponge
            // rate adds exact zeros.
            if (!F64 || out_lane) {
                const bool in_w = ib_on && (unsigned)(i - wlo0) < (unsigned)wn0;
                const double f0 = in_w ? fw[0] : 0.0, f1 = in_w ? fw[1] : 0.0;
                // sigma * max(eta_x, eta_y)^3 = max of the two rates (a monotone function of
                // eta, rounded the same way for both; zero without a sponge)
                const double sg = fmax(sg_x, sg_y);
                double s[4] = {0.0, f0, f1, fma(f0, ur, f1 * vr)};
                // (FP64: only where the rate is not zero, where the term adds exact zeros, so
                // that the far-field state is read from the constant block in sponge waves only)
                if (!F64 || sg != 0.0) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) s[c] = fma(-sg, qr[c] - q_inf(c), s[c]);
                }
                double val[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const double l = L[c] + s[c];
                    const double stage = fma(dt, l, qr[c]);
                    val[c] = mode_rhs ? l : ((ca == 0.0) ? stage : fma(ca, qn[c], cb * stage));
                }
                if (out_lane) {
                    const long long o = (long long)r * nx + i;
#pragma unroll
                    for (int c = 0; c < 4; ++c) out[c * ncell + o] = val[c];
                }
                if (want_alpha) {
                    const double ir = rcp_nr(val[0]);
                    const double un = val[1] * ir, vn = val[2] * ir;
                    const double pn = gm1 * (val[3] - 0.5 * fma(val[1], un, val[2] * vn));
                    const double cn = sqrt(gam() * pn * ir);
                    const unsigned long long sx = (unsigned long long)__double_as_longlong(fabs(un) + cn);
                    const unsigned long long sy = (unsigned long long)__double_as_longlong(fabs(vn) + cn);
                    const bool ain = out_lane && r >= ar0 && r < ar1;
                    amax_x = ain ? max_bits(amax_x, sx) : amax_x;
                    amax_y = ain ? max_bits(amax_y, sy) : amax_y;
                    if constexpr (SCHEME == LEARNED) {
                        // the FP32 deviations the next flags pass forms from this output (same
                        // expressions), for its test of tiles whose stencils are all
                        // insignificant
                        const float d[4] = {(float)(val[0] - rinf), (float)(un - uinf), (float)(vn - vinf),
                                            (float)(pn - pinf)};
                        if (qrange && out_lane) {
                            // LDS min / max without a returned value: nothing waits on them
#pragma unroll
                            for (int m = 0; m < 4; ++m) {
                                __hip_atomic_fetch_min(&rng[2 * m][lane], d[m], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                                __hip_atomic_fetch_max(&rng[2 * m + 1][lane], d[m], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                            }
                        }
                    }
                }
            }
        }
        if ((terms & T_CONVY) && Rw >= j0 + 3 && Rw <= j1 + 3) {
#pragma unroll
            for (int c = 0; c < 4; ++c) cy_queue[c] = cy_new[c];
        }
    }
};

// Wave issue priority (0 lowest .. 3), set with the immediate the instruction takes.
__device__ __forceinline__ void set_issue_priority(int p)
{
    switch (p) {
    case 3: __builtin_amdgcn_s_setprio(3); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    default: __builtin_amdgcn_s_setprio(0); break;
    }
}

// NR: the instantiation for contexts with non-reflecting sides (StageArgs::nrbc).
template <int SCHEME, class T, bool DBG = false, bool NR = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_stage2d(
    const KConst* __restrict__ K, StageArgs A)
{
    __shared__ __attribute__((aligned(16))) KeepRows<T> keep_rows;
    if (SCHEME != WENO5JS) {
        init_keep_rows<T>(keep_rows, threadIdx.x);
        __syncthreads();
    }
    Column2D<SCHEME, T, DBG, NR> C;
    C.K = K;
    C.dbg_x = A.dbg_x;
    C.dbg_y = A.dbg_y;
    C.Qs = A.Qs;
    C.Qn = A.Qn;
    C.out = A.out;
    C.fwin = A.fwin;
    C.flags_x = A.flags_x;
    C.flags_y = A.flags_y;
    C.ncell = K->G.ncell;
    C.nx = K->G.n[0];
    C.ny = K->G.n[1];
    C.bcy0 = K->G.bc[1][0];
    C.bcy1 = K->G.bc[1][1];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        C.qinf[c] = K->P.q_inf[c];
        C.Fxinf[c] = K->Fx_inf[c];
        C.Fyinf[c] = K->Fy_inf[c];
    }
    C.rinf = K->P.prim_inf[0];
    C.uinf = K->P.prim_inf[1];
    C.vinf = K->P.prim_inf[2];
    C.pinf = K->P.prim_inf[4];
    C.gamma = K->P.gamma;
    C.sigma = (K->P.terms & T_SPONGE) ? K->P.sigma : 0.0;
    C.wlo0 = A.wlo[0];
    C.wlo1 = A.wlo[1];
    C.wn0 = A.wn[0];
    C.wn1 = A.wn[1];
    C.ax = __longlong_as_double((long long)A.alpha_bits[0]);
    C.ay = __longlong_as_double((long long)A.alpha_bits[1]);
    C.inv_h = K->G.inv_h;
    C.inv_hT = (T)K->G.inv_h;
    C.inv12h = (T)K->inv12h;
    C.mu = (T)K->P.mu;
    C.gm1 = K->P.gm1;
    C.R.eps = SCHEME == WENO5JS ? K->P.weno_eps : K->P.teno_eps;
    C.R.ct = K->P.teno_ct;
    C.R32.eps = SCHEME == WENO5JS ? (float)K->P.weno_eps : 1e-30f;   // FP32 TENO5 epsilon
    C.R32.ct = (float)K->P.teno_ct;
    if constexpr (F64v<T>) {
        C.R.rows = keep_rows;
        C.R32.rows = nullptr;
    } else {
        C.R.rows = nullptr;
        C.R32.rows = keep_rows;
    }
    C.ca = A.ca;
    C.cb = A.cb;
    C.dt = A.dt;
    C.mode_rhs = A.mode_rhs;
    C.terms = K->P.terms;
    C.step = A.step;

    // XCD-aware placement: consecutive workgroups go round-robin to the 8 XCDs, each with its
    // own L2, so the linear workgroup index is remapped to give every XCD one contiguous
    // run of strips (row-major): neighbouring strips, which read each other's halo columns,
    // then share an L2.  Any bijection is correct; this one only serves locality.
    int bx, by;
    {
        const int nb = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
        const int q = nb / 8, rm = nb % 8, xcd = b % 8, k = b / 8;
        const int L = xcd < rm ? xcd * (q + 1) + k : rm * (q + 1) + (xcd - rm) * q + k;
        bx = L % gridDim.x;
        by = L / gridDim.x;
    }
    __shared__ double ring[5][4][WAVE];
    __shared__ T vring[5][3][WAVE];

    const int lane = threadIdx.x;
    C.ring = ring;
    C.vring = vring;
    C.lane = lane;
    const int nx = C.nx, ny = K->G.n[1];
    {
        const int i = bx * OUTW - HALO + lane;
        C.i = min(max(i, -HALO), nx + HALO - 1);
        int inflow = 0, side = 0, depth = 0;
        C.xr = resolve_index(C.i, nx, K->G.bc[0][0], K->G.bc[0][1], 0, inflow, side, depth);
        C.x_inflow = inflow != 0;
        C.ghosts = A.ghosts;
        C.gna = max(nx, K->G.n[1]);
        C.gcs = 4ll * HALO * C.gna;
        C.gxo = C.x_inflow ? (side * HALO + depth - 1) * C.gna : 0;
        C.xg_wave = __ballot(C.x_inflow) != 0ull;
        C.out_lane = lane >= HALO && lane < WAVE - HALO && i < nx;
        C.nrbc = A.nrbc;
        C.nrbc_x = ((A.nrbc & 1) && C.i == 0) || ((A.nrbc & 2) && C.i == nx - 1);
    }
    C.sg_x = C.out_lane ? C.sponge_rate(K->eta_dir(0, C.i)) : 0.0;
    C.sg_rows = 0.0;
    C.sg_base = -(1 << 30);   // the first sponge_row call fills the lane table
    // the force window meets this strip's columns (a wave-uniform test)
    C.ib_on = (C.terms & T_IB) && C.fwin && C.wn0 > 0 && C.wn1 > 0 && bx * OUTW - HALO + WAVE > C.wlo0 &&
              bx * OUTW - HALO < C.wlo0 + C.wn0;
    C.j0 = by * A.ty;
    C.j1 = min(C.j0 + A.ty, ny) - 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) C.fy_prev[c] = C.cy_queue[c] = T(0);
#pragma unroll
    for (int s = 0; s < 5; ++s) {
#pragma unroll
        for (int c = 0; c < 4; ++c) C.fp[s][c] = C.fm[s][c] = T(0);
        C.uw[s] = C.vw[s] = T(0);
        C.txy[s] = C.tyy[s] = T(0);
    }
    C.want_alpha = A.alpha_part != nullptr;
    C.qrange = A.qrange;
    __shared__ float rng[SCHEME == LEARNED ? 8 : 1][WAVE];   // (the other forms keep no ranges)
    C.rng = rng;
    if constexpr (SCHEME == LEARNED) {
#pragma unroll
        for (int m = 0; m < 8; ++m) rng[m][threadIdx.x] = (m & 1) ? -INFINITY : INFINITY;
    }
    C.amax_x = C.amax_y = 0ull;
    C.ar0 = A.arow0;
    C.ar1 = A.arow1;
    const int Rend = C.j1 + HALO;
#pragma unroll
    for (int s = 0; s < C.PF; ++s) {
        C.load_row(C.j0 - HALO + s, C.qf[s]);
        // the row's loads go out before the others, as in the march, so that the wait for
        // them at the loop head can leave the younger loads in flight
        __builtin_amdgcn_sched_barrier(0);
        C.wy_pf[s] = C.wx_pf[s] = 0u;
        C.load_patterns(C.j0 - HALO + s, s);
#pragma unroll
        for (int c = 0; c < 4; ++c) C.qn_pf[s][c] = 0.0;
        C.load_qn(C.j0 - 2 * HALO + s, s);
        C.load_fwin(C.j0 - 2 * HALO + s, s);
    }
    // Issue priority falls with progress: 3 over the first 60% of the segment's rows, then 2,
    // 1, and 0 over about the last 7%.  The two waves sharing a SIMD otherwise run oldest
    // first: the older one finishes well ahead and the other then runs alone, with nothing to
    // hide its latency behind.  When the leading wave's priority drops, the other is issued
    // first until it drops too, so the pair is level again at each step; only within the last
    // level does age decide, hence the short last interval.
    const int nrow = Rend - (C.j0 - HALO) + 1;
    for (int Rw = C.j0 - HALO; Rw <= Rend; Rw += 5) {
        {
            const int done100 = (Rw - (C.j0 - HALO)) * 100;
            set_issue_priority(done100 < 60 * nrow ? 3 : done100 < 80 * nrow ? 2 : done100 < 93 * nrow ? 1 : 0);
        }
        C.template step_row<0>(Rw);
        if (Rw + 1 > Rend) break;
        C.template step_row<1>(Rw + 1);
        if (Rw + 2 > Rend) break;
        C.template step_row<2>(Rw + 2);
        if (Rw + 3 > Rend) break;
        C.template step_row<3>(Rw + 3);
        if (Rw + 4 > Rend) break;
        C.template step_row<4>(Rw + 4);
    }
    if (C.want_alpha) {
        unsigned long long mx = C.amax_x, my = C.amax_y;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            mx = max_bits(mx, __shfl_xor(mx, off, WAVE));
            my = max_bits(my, __shfl_xor(my, off, WAVE));
        }
        if (lane < 3) {
            // one partial per wave (plain stores; launch_alpha_final reduces them)
            const long long wv = (long long)blockIdx.y * gridDim.x + blockIdx.x;
            A.alpha_part[wv * 3 + lane] = lane == 0 ? mx : (lane == 1 ? my : 0ull);
        }
        if constexpr (SCHEME == LEARNED) {
            if (C.qrange) {
                float r[8];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    float a = rng[2 * m][lane], b = rng[2 * m + 1][lane];
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) {
                        a = fminf(a, __shfl_xor(a, off, WAVE));
                        b = fmaxf(b, __shfl_xor(b, off, WAVE));
                    }
                    r[2 * m] = a;
                    r[2 * m + 1] = b;
                }
                // indexed by the strip and segment this wave computed (not its launch slot)
                float v = r[0];
#pragma unroll
                for (int k = 1; k < 8; ++k) v = lane == k ? r[k] : v;
                if (lane < 8) C.qrange[((long long)by * gridDim.x + bx) * 8 + lane] = v;
            }
        }
    }
}

// Inflow ghost tables of steps step0 .. step0 + gridDim.z - 1 (one per z block index, each
// inflow_ghosts2d_elems long): thread (t, side * HALO + depth - 1) forms the state of the
// ghost cell `depth` layers beyond side `side` (0: x-, 1: x+, 2: y-, 3: y+) at position t
// along it, by the boundary rule used everywhere else (indices resolved x first, then y;
// the far field with the seeded perturbation of the resolved cell), bit for bit.
__global__ __launch_bounds__(256) void k_inflow_ghosts2d(const KConst* __restrict__ K, long long step0,
                                                         double* __restrict__ g)
{
    const Grid& G = K->G;
    const int side = blockIdx.y / HALO, depth = blockIdx.y % HALO + 1, dir = side >> 1;
    const int na = max(G.n[0], G.n[1]);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G.n[dir ^ 1] || G.bc[dir][side & 1] != BC_INFLOW) return;
    const int across = (side & 1) ? G.n[dir] - 1 + depth : -depth;
    int inflow = 0, s = 0, d = 0;
    const int ir = resolve_index(dir == 0 ? across : t, G.n[0], G.bc[0][0], G.bc[0][1], 0, inflow, s, d);
    const int jr = resolve_index(dir == 0 ? t : across, G.n[1], G.bc[1][0], G.bc[1][1], 1, inflow, s, d);
    double q[4];
    inflow_state<2>(K->P, step0 + blockIdx.z, G.gncell, G.glin(ir, jr, 0), s, d, q);
    double* gz = g + (long long)blockIdx.z * (16ll * HALO * na);
    const long long o = (long long)(side * HALO + depth - 1) * na + t;
#pragma unroll
    for (int c = 0; c < 4; ++c) gz[c * 4ll * HALO * na + o] = q[c];
}

}  // namespace

int launch_stage2d(const KConst* K, const Grid& G, int scheme, int precision, const StageArgs& A, hipStream_t s)
{
    if (has_inflow(G) && !A.ghosts) return (int)hipErrorInvalidValue;   // inflow sides need the ghost table
    if (!A.Qn) return (int)hipErrorInvalidValue;                          // read in every stage
    const int ncolx = (G.n[0] + OUTW - 1) / OUTW;
    const int nseg = (G.n[1] + A.ty - 1) / A.ty;
    dim3 grid(ncolx, nseg), block(WAVE);
    if (A.nrbc) {
        if (A.dbg_x) return (int)hipErrorInvalidValue;
        if (precision == 2) hipLaunchKernelGGL((k_stage2d<LEARNED, float, false, true>), grid, block, 0, s, K, A);
        else if (precision == 1 && scheme == TENO5)
            hipLaunchKernelGGL((k_stage2d<TENO5, float, false, true>), grid, block, 0, s, K, A);
        else if (precision == 1) hipLaunchKernelGGL((k_stage2d<WENO5JS, float, false, true>), grid, block, 0, s, K, A);
        else if (scheme == TENO5) hipLaunchKernelGGL((k_stage2d<TENO5, double, false, true>), grid, block, 0, s, K, A);
        else hipLaunchKernelGGL((k_stage2d<WENO5JS, double, false, true>), grid, block, 0, s, K, A);
    } else if (precision == 2) {
        hipLaunchKernelGGL((k_stage2d<LEARNED, float>), grid, block, 0, s, K, A);
    } else if (precision == 1) {
        if (scheme == TENO5) hipLaunchKernelGGL((k_stage2d<TENO5, float>), grid, block, 0, s, K, A);
        else hipLaunchKernelGGL((k_stage2d<WENO5JS, float>), grid, block, 0, s, K, A);
    } else if (A.dbg_x) {
        // the FP64 TENO5 kernel that also writes its keep patterns (test read-out)
        if (scheme != TENO5 || !A.dbg_y) return (int)hipErrorInvalidValue;
        hipLaunchKernelGGL((k_stage2d<TENO5, double, true>), grid, block, 0, s, K, A);
    } else {
        if (scheme == TENO5) hipLaunchKernelGGL((k_stage2d<TENO5, double>), grid, block, 0, s, K, A);
        else hipLaunchKernelGGL((k_stage2d<WENO5JS, double>), grid, block, 0, s, K, A);
    }
    return (int)hipGetLastError();
}

bool has_inflow(const Grid& G)
{
    for (int d = 0; d < 2; ++d)
        for (int e = 0; e < 2; ++e)
            if (G.bc[d][e] == BC_INFLOW) return true;
    return false;
}

long long inflow_ghosts2d_elems(const Grid& G) { return 4ll * 4 * HALO * std::max(G.n[0], G.n[1]); }

int launch_inflow_ghosts2d(const KConst* K, const Grid& G, long long step0, int nsteps, double* g, hipStream_t s)
{
    const int na = std::max(G.n[0], G.n[1]);
    if (nsteps < 1 || nsteps > 65535) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_inflow_ghosts2d, dim3((na + 255) / 256, 4 * HALO, nsteps), dim3(256), 0, s, K, step0, g);
    return (int)hipGetLastError();
}

int stage2d_ncolx(int nx) { return (nx + OUTW - 1) / OUTW; }

int stage2d_strip_width() { return OUTW; }

long long stage2d_waves(const Grid& G, int ty)
{
    return (long long)((G.n[0] + OUTW - 1) / OUTW) * ((G.n[1] + ty - 1) / ty);
}

}  // namespace fsa
