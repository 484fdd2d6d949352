// RKL2 super time-stepping stage kernel: the explicit alternative to the
// implicit viscous solve (the paper, Section 2.2, which cites the second-order
// Runge-Kutta-Legendre scheme of Meyer, Balsara and Aslam, 2014; Section 4.1
// counts it among the vectorizable stencil algorithms; Section 5.2 finds it
// the faster choice on GPUs).
//
// One kernel per stage.  With dtL(u) = -(dt / V) * sum_f G_f nu_f (u_c - u_nb)
// (interior faces nu_f = (nu_c + nu_nb)/2, Dirichlet walls nu_f = nu_c with
// u_nb = 0), the kernel writes
//
//     out = a X + b Z + g L0 + Y0 + m dtL(X)
//
// for cell arrays X (read with its 6 neighbours), Z, L0, Y0 (cell only; any of
// the three may be absent, read as zero).  The face conductances are formed
// on the fly from nu and the separable 1-D geometry tables (the r factor of a
// face times its theta factor), so a stage streams X, nu, Z and L0 and writes
// out: 5 words per cell instead of the 9 an assembled-coefficient stencil
// would stream.
//
// Work layout as in the PCG iteration kernel: each wave owns RPW theta rows
// of one phi segment (64/RPW lanes per row, V cells per lane) and marches
// through the r planes of its chunk, holding X and nu of the planes m-1, m,
// m+1 in registers; theta neighbours inside the wave come from lane
// shuffles, the wave's outer rows are loaded, phi neighbours come from lane
// shuffles with the two segment-edge cells loaded.  Chunks alternate their
// march direction so that the halo plane two chunks share is read at the same
// time by both.
#pragma once

#include "kernels.hpp"

namespace mas {

// Cache hints (buffer aux field) per stream: X and nu are re-read as
// neighbours, Z, L0, Y0 and out are touched once per stage.
#ifndef MAS_STS_AUX_XN
#define MAS_STS_AUX_XN 0
#endif
#ifndef MAS_STS_AUX_ZL
#define MAS_STS_AUX_ZL kAuxNT
#endif
#ifndef MAS_STS_AUX_ST
#define MAS_STS_AUX_ST kAuxNT
#endif

#ifndef MAS_STS_ORDER
#define MAS_STS_ORDER 3
#endif

struct StsArgs {
    const double *X, *nu, *Z, *L0, *Y0;  // Z, L0, Y0: read only when the kernel's IN mask says so
    double *out;                          // may alias Z or Y0 (same cell read first)
    double a, b, g, mdt;                  // mdt = m * dt
    Geo geo;
    Dims d;
    int tiles_i, tiles_k, tiles_j, ti, nblk;
};

// Inputs a stage reads besides X and nu (template mask).
constexpr int kStsZ = 1, kStsL0 = 2, kStsY0 = 4;

// Plane factors of cell row (m, j): half the r-face factors of the faces
// m | m+1 (zero at m = nr-1) and m-1 | m (zero at m = 0), the Dirichlet wall
// factor (zero with Neumann walls, whose gw_* are zero) and the stage scale
// m dt / V.  Shared by the one- and two-stage kernels so that both round alike.
struct StsPlane {
    double gq, hRp, hRm, gw, scale;
};

// The table entries of plane m.
struct StsPlaneRaw {
    double gq, gr, grm, vr;  // grm = gr[m - 1], zero at m = 0
    int m;
};

__device__ inline StsPlaneRaw sts_plane_raw(const Geo &g, int m) {
    return StsPlaneRaw{g.gq[m], g.gr[m], (m > 0) ? g.gr[m - 1] : 0.0, g.vr[m], m};
}

__device__ inline StsPlane sts_plane(const Geo &g, const StsPlaneRaw &t, int nr, double vt, double mdt) {
    StsPlane p;
    p.gq = t.gq;
    p.hRp = 0.5 * t.gr * vt;
    p.hRm = (t.m > 0) ? 0.5 * t.grm * vt : 0.0;
    p.gw = (((t.m == 0) ? g.gw_in : 0.0) + ((t.m == nr - 1) ? g.gw_out : 0.0)) * vt;
    p.scale = mdt / (t.vr * vt);
    return p;
}

__device__ inline StsPlane sts_plane(const Geo &g, int m, int nr, double vt, double mdt) {
    return sts_plane(g, sts_plane_raw(g, m), nr, vt, mdt);
}

// sum_f G_f (nu_c + nu_nb)/2 (x_c - x_nb) over the six faces of a cell, the
// halves already folded into the factors (tU, tD, tP: theta-face and
// phi-face factors of the row times the plane's gq).  Wherever two products
// meet in one sum the fused multiply-add is written out, so that every kernel
// using these helpers rounds alike whatever the compiler would contract.
__device__ inline double sts_flux(const StsPlane &p, double tU, double tD, double tP, double xc, double nc,
                                  double xp, double np_, double xm, double nm, double xu, double nu_u,
                                  double xd, double nu_d, double xl, double nl, double xr, double nrr) {
    double f = (p.hRp * (nc + np_)) * (xc - xp);
    f = __builtin_fma(p.hRm * (nc + nm), xc - xm, f);
    f = __builtin_fma(p.gw * nc, xc, f);
    f = __builtin_fma(tU * (nc + nu_u), xc - xu, f);
    f = __builtin_fma(tD * (nc + nu_d), xc - xd, f);
    f = __builtin_fma(tP, __builtin_fma(nc + nl, xc - xl, (nc + nrr) * (xc - xr)), f);
    return f;
}

// One stage's value at a cell: a x + b z + g l + y - scale f.
__device__ inline double sts_combine(double a, double x, double b, double z, double g, double l, double y,
                                     double scale, double f) {
    double o = __builtin_fma(a, x, b * z);
    o = __builtin_fma(g, l, o);
    o = o + y;
    return __builtin_fma(-scale, f, o);
}

#ifndef MAS_STS_WPE
#define MAS_STS_WPE 0
#endif

template <int WPB, int RPW, int V, int IN>
__global__ __launch_bounds__(kWave *WPB)
#if MAS_STS_WPE > 0
__attribute__((amdgpu_waves_per_eu(MAS_STS_WPE, 8)))
#endif
void k_sts_stage(StsArgs a) {
    static_assert(kWave % RPW == 0, "rows per wave");
    constexpr int W = kWave / RPW;  // lanes per row
    constexpr int SEG = W * V;
    constexpr bool HZ = IN & kStsZ, HL = IN & kStsL0, HY = IN & kStsY0;
    using VD = VecT<double, V>;

    const int nr = a.d.nr, nt = a.d.nt, np = a.d.np;
    const int64_t plane = a.d.plane;

    const int L = xcd_remap(blockIdx.x, a.nblk);
    int it, kt, jt;
    tile_coords<MAS_STS_ORDER>(L, a.tiles_i, a.tiles_k, a.tiles_j, it, kt, jt);

    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int rr = lane / W;
    const int lp = lane % W;
    const int j = (jt * WPB + wv) * RPW + rr;
    const int k0 = kt * SEG;
    const int nseg = min(SEG, np - k0);  // a multiple of V
    const int nvl = nseg / V;
    const bool rowok = j < nt;
    const bool act = rowok && lp < nvl;
    const int i0 = it * a.ti;
    const int i1 = min(i0 + a.ti, nr);
    const bool up = (it & 1) == 0;
    const int dir = up ? 1 : -1;
    const int first = up ? i0 : i1 - 1;

    // phi neighbours of the segment (periodic).  In a short segment the first
    // lane past its end loads the cell right of it as if it were its own
    // (the last active lane takes it through the phi shuffle); in a full
    // segment the row's last lane loads it in the same instruction as lane 0
    // loads the cell left of the segment.
    const int64_t colL = (int64_t)j * np + ((k0 == 0) ? np - 1 : k0 - 1);
    const int64_t colR = (int64_t)j * np + ((k0 + nseg == np) ? 0 : k0 + nseg);
    const bool pseudoR = rowok && nvl < W && lp == nvl;
    const bool eL = act && lp == 0;
    const bool eR = act && nvl == W && lp == W - 1;
    const int64_t col = act ? (int64_t)j * np + k0 + lp * V : (pseudoR ? colR : 0);
    const bool ldo = act || pseudoR;
    // theta neighbours: with RPW >= 2 the wave's first row loads row j-1 and
    // its last row row j+1 (one set of registers, never both in one lane);
    // the rows in between come from lane shuffles
    const bool ldU = act && j > 0 && rr == 0;
    const bool ldD = act && j < nt - 1 && rr == RPW - 1;
    const int srcU = (rr > 0) ? lane - W : lane;
    const int srcD = (rr < RPW - 1) ? lane + W : lane;

    // per-row geometry: half the theta-face factors (the 1/2 of the face mean)
    const int jj = rowok ? j : 0;
    const double vt = a.geo.vt[jj];
    const double hU = (rowok && j > 0) ? 0.5 * a.geo.gtt[j - 1] : 0.0;
    const double hD = rowok ? 0.5 * a.geo.gtt[jj] : 0.0;  // zero on the last row
    const double hP = (rowok && !a.geo.np_one) ? 0.5 * a.geo.gpt[jj] : 0.0;

    constexpr uint32_t ES = sizeof(double);
    // the planes this block touches, i0 - 1 .. i1
    const PlaneWin win = plane_win(a.d, i0 - 1, i1 + 1);
    const auto RX = win_rsrc(a.X, win), RN = win_rsrc(a.nu, win), RZ = win_rsrc(a.Z, win, HZ),
               RL = win_rsrc(a.L0, win, HL), RY = win_rsrc(a.Y0, win, HY), RO = win_rsrc(a.out, win);

    auto own_off = [&](int m) -> uint32_t {
        return (ldo && m >= 0 && m < nr) ? (uint32_t)((int64_t)(m - win.lo) * plane + col) * ES : kOOB;
    };
    // planes m - dir (behind) and m (current) of the first step
    VD Xb = bld<double, V, MAS_STS_AUX_XN>(RX, own_off(first - dir));
    VD Nb = bld<double, V, MAS_STS_AUX_XN>(RN, own_off(first - dir));
    VD Xc = bld<double, V, MAS_STS_AUX_XN>(RX, own_off(first));
    VD Nc = bld<double, V, MAS_STS_AUX_XN>(RN, own_off(first));

    VD st{};
    uint32_t st_off = kOOB;
    const int nsteps = i1 - i0;
    for (int s = 0; s < nsteps; ++s) {
        const int m = first + s * dir;
        const int64_t base = (int64_t)(m - win.lo) * plane;
        const uint32_t oo = act ? (uint32_t)(base + col) * ES : kOOB;
        const uint32_t oE = ldU ? (uint32_t)(base + col - np) * ES
                                : (ldD ? (uint32_t)(base + col + np) * ES : kOOB);
        const uint32_t oD = ldD ? (uint32_t)(base + col + np) * ES : kOOB;
        const uint32_t oLR = eL ? (uint32_t)(base + colL) * ES
                                : (eR ? (uint32_t)(base + colR) * ES : kOOB);
        // ---- loads: plane m + dir (ahead) and the rest of plane m
        const VD Xa = bld<double, V, MAS_STS_AUX_XN>(RX, own_off(m + dir));
        const VD Na = bld<double, V, MAS_STS_AUX_XN>(RN, own_off(m + dir));
        // RPW = 1: E holds row j-1, D row j+1; RPW >= 2: E holds whichever the lane needs
        const VD XE = bld<double, V, MAS_STS_AUX_XN>(RX, RPW == 1 ? (ldU ? oE : kOOB) : oE);
        const VD NE = bld<double, V, MAS_STS_AUX_XN>(RN, RPW == 1 ? (ldU ? oE : kOOB) : oE);
        VD XD{}, ND{};
        if constexpr (RPW == 1) {
            XD = bld<double, V, MAS_STS_AUX_XN>(RX, oD);
            ND = bld<double, V, MAS_STS_AUX_XN>(RN, oD);
        }
        const double XS = bld<double, 1>(RX, oLR).v[0];
        const double NS = bld<double, 1>(RN, oLR).v[0];
        VD Zv{}, Lv{}, Yv{};
        if constexpr (HZ) Zv = bld<double, V, MAS_STS_AUX_ZL>(RZ, oo);
        if constexpr (HL) Lv = bld<double, V, MAS_STS_AUX_ZL>(RL, oo);
        if constexpr (HY) Yv = bld<double, V, MAS_STS_AUX_ZL>(RY, oo);
        // ---- store of the previous step (issued after this step's loads)
        bst<double, V, MAS_STS_AUX_ST>(RO, st_off, st);

        // ---- plane factors
        const StsPlane pf = sts_plane(a.geo, m, nr, vt, a.mdt);
        const double tU = pf.gq * hU, tD = pf.gq * hD, tP = pf.gq * hP;
        const VD &Xp = up ? Xa : Xb, &Xm = up ? Xb : Xa;  // planes m+1, m-1
        const VD &Np = up ? Na : Nb, &Nm = up ? Nb : Na;

        const double xl0 = lane_prev(Xc.v[V - 1]), nl0 = lane_prev(Nc.v[V - 1]);
        const double xr0 = lane_next(Xc.v[0]), nr0 = lane_next(Nc.v[0]);
        VD o;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const double xc = Xc.v[e], nc = Nc.v[e];
            double sxu, snu, sxd, snd;
            if constexpr (RPW == 2) {
                sxu = sxd = other_half(xc);
                snu = snd = other_half(nc);
            } else {
                sxu = shfl_lane(xc, srcU);
                snu = shfl_lane(nc, srcU);
                sxd = shfl_lane(xc, srcD);
                snd = shfl_lane(nc, srcD);
            }
            const double xu = (rr == 0) ? XE.v[e] : sxu, nu_u = (rr == 0) ? NE.v[e] : snu;
            double xd, nu_d;
            if constexpr (RPW == 1) {
                xd = XD.v[e];
                nu_d = ND.v[e];
            } else {
                xd = (rr == RPW - 1) ? XE.v[e] : sxd;
                nu_d = (rr == RPW - 1) ? NE.v[e] : snd;
            }
            const double xl = (e > 0) ? Xc.v[e - 1] : ((lp == 0) ? XS : xl0);
            const double nl = (e > 0) ? Nc.v[e - 1] : ((lp == 0) ? NS : nl0);
            const double xr = (e < V - 1) ? Xc.v[e + 1] : (eR ? XS : xr0);
            const double nrr = (e < V - 1) ? Nc.v[e + 1] : (eR ? NS : nr0);
            const double f = sts_flux(pf, tU, tD, tP, xc, nc, Xp.v[e], Np.v[e], Xm.v[e], Nm.v[e], xu, nu_u,
                                      xd, nu_d, xl, nl, xr, nrr);
            o.v[e] = sts_combine(a.a, xc, a.b, Zv.v[e], a.g, Lv.v[e], Yv.v[e], pf.scale, f);
        }
        st = o;
        st_off = oo;
        Xb = Xc;
        Nb = Nc;
        Xc = Xa;
        Nc = Na;
    }
    bst<double, V, MAS_STS_AUX_ST>(RO, st_off, st);
}

// ---------------------------------------------------------------- two stages per launch
// Stages j and j+1 of the recursion in one pass (temporal blocking):
//
//     A = aA X + bA Z + gA L0 + mA dtL(X)              (stage j,   D_j)
//     B = aB A + bB X + gB L0 + Y0 + mB dtL(A)         (stage j+1, D_{j+1})
//
// Stage j+1 at a cell needs stage j at its six neighbours, which need X two
// cells away: each block loads a tile of 2 NW theta rows by 64 phi cells (one
// row per half-wave, two cells per lane), forms A on all of it, and keeps B on
// the inner (2 NW - 4) x 60 cells; the ring of two cells on each side is
// overlap with the neighbour tiles.  Along r the block marches its chunk of
// planes with B one plane behind A, starting and ending one plane outside the
// chunk.  Per cell and pair of stages it streams X, nu, Z, L0 and writes A and
// B: 6 words for two stages instead of 10.  A and B go to buffers other than
// X and Z (neighbour tiles read X and Z on their rings while this one writes).
// The theta neighbours go through LDS, the phi neighbours through DPP lane
// shifts (the shifted-in values at the tile's two outer columns are never
// used), the r neighbours through register queues.  Every value A and B take
// is formed by the same expressions as in k_sts_stage, so a pair equals two
// one-stage launches bit for bit.
//
// IN mask: kPairZ reads Z (else zero); kPairL reads L0 (else L0 is X: the
// stage pair 2, 3, where X = L0); kPairY makes B the last stage: it adds Y0,
// stores B to outB and does not store A.
constexpr int kPairLanes = 32;             // lanes per tile row, two cells each
constexpr int kPairCols = 2 * kPairLanes;  // tile columns
constexpr int kPairOut = kPairCols - 4;    // columns kept
constexpr int kPairZ = 1, kPairL = 2, kPairY = 4;
constexpr int kPairMaxTI = 64;             // most r planes per chunk

struct StsPairArgs {
    const double *X, *nu, *Z, *L0, *Y0;
    double *outA, *outB;
    double aA, bA, gA, mdtA;
    double aB, bB, gB, mdtB;
    Geo geo;
    Dims d;
    int tiles_i, tiles_k, tiles_j, ti, nblk;
};

// Waves per SIMD the pair kernel is compiled for (the fewest with more
// registers ran fastest).
#ifndef MAS_PAIR_WPE
#define MAS_PAIR_WPE 2
#endif

template <int NW, int IN>
__global__ __launch_bounds__(kWave *NW) __attribute__((amdgpu_waves_per_eu(MAS_PAIR_WPE, 8)))
void k_sts_pair(StsPairArgs a) {
    constexpr int R = 2 * NW;  // tile rows
    constexpr int RO = R - 4;  // rows kept
    constexpr bool HZ = (IN & kPairZ) != 0, HL = (IN & kPairL) != 0, HY = (IN & kPairY) != 0;
    using VD = VecT<double, 2>;
    // LDS rings by step index: X of the last two planes, nu and A of the
    // last four.  One barrier per step: step s writes X and nu of its plane
    // before the barrier and A after stage B; stage A at step s reads the
    // plane written before the barrier, stage B the planes of steps s-1 and
    // s-2.  A slot is rewritten only after every thread has passed the
    // barrier that follows its last read.
    __shared__ __attribute__((aligned(16))) double sX[2][R][kPairCols];
    __shared__ __attribute__((aligned(16))) double sN[4][R][kPairCols];
    __shared__ __attribute__((aligned(16))) double sY[4][R][kPairCols];

    const int nr = a.d.nr, nt = a.d.nt, np = a.d.np;
    const int64_t plane = a.d.plane;
    const int Lb = xcd_remap(blockIdx.x, a.nblk);
    int it, kt, jt;
    tile_coords<MAS_STS_ORDER>(Lb, a.tiles_i, a.tiles_k, a.tiles_j, it, kt, jt);

    const int lane = threadIdx.x & (kWave - 1);
    const int rho = threadIdx.x / kPairLanes;  // tile row
    const int c = 2 * (lane & (kPairLanes - 1));
    const int ru = rho > 0 ? rho - 1 : rho, rd = rho < R - 1 ? rho + 1 : rho;
    const int j = jt * RO - 2 + rho;
    const int k0 = kt * kPairOut;
    const int nout = min(kPairOut, np - k0);  // even: np is even
    const bool rowin = j >= 0 && j < nt;
    // the lane's two cells k0 - 2 + c, +1 (periodic; np even keeps them adjacent)
    const bool ld = rowin && c <= nout + 2;
    int k = k0 - 2 + c;
    if (k < 0) k += np;
    else if (k >= np) k -= np;
    const int64_t col = ld ? (int64_t)j * np + k : 0;
    const bool own = rowin && rho >= 2 && rho < R - 2 && c >= 2 && c < nout + 2;

    const int jj = rowin ? j : 0;
    const double vt = a.geo.vt[jj];
    const double hU = (rowin && j > 0) ? 0.5 * a.geo.gtt[j - 1] : 0.0;
    const double hD = rowin ? 0.5 * a.geo.gtt[jj] : 0.0;
    const double hP = (rowin && !a.geo.np_one) ? 0.5 * a.geo.gpt[jj] : 0.0;

    const int i0 = it * a.ti;
    const int i1 = min(i0 + a.ti, nr);
    const int nsteps = i1 - i0 + 2;  // A runs from one plane before the chunk to one after
    // the planes this block may address, i0 - 3 .. i1 + 2 (the outermost
    // two are loaded for a step that never comes)
    const PlaneWin win = plane_win(a.d, i0 - 3, i1 + 3);
    constexpr uint32_t ES = sizeof(double);
    const auto RX = win_rsrc(a.X, win), RN = win_rsrc(a.nu, win), RZ = win_rsrc(a.Z, win, HZ),
               RL = win_rsrc(a.L0, win, HL), RY = win_rsrc(a.Y0, win, HY),
               RA = win_rsrc(a.outA, win, !HY), RB = win_rsrc(a.outB, win);
    auto ldoff = [&](int m) -> uint32_t {
        return (ld && m >= 0 && m < nr) ? (uint32_t)((int64_t)(m - win.lo) * plane + col) * ES : kOOB;
    };
    // Z and L0 enter stage A only, whose values on the outermost tile rows
    // are never used: those rows do not load them
    const bool ldzl = ld && rho >= 1 && rho < R - 1;
    auto zloff = [&](int m) -> uint32_t {
        return (ldzl && m >= 0 && m < nr) ? (uint32_t)((int64_t)(m - win.lo) * plane + col) * ES : kOOB;
    };
    auto ownoff = [&](int m) -> uint32_t {
        return (own && m >= i0 && m < i1) ? (uint32_t)((int64_t)(m - win.lo) * plane + col) * ES : kOOB;
    };
    auto lds2 = [&](const double *row) -> VD { return VD{{row[c], row[c + 1]}}; };

    // The chunk's plane-table entries, planes i0-2 .. i1+1 (clamped into the
    // grid; A is zero outside it), copied to LDS once: read there each step,
    // they put no wait on the vector-memory counter that the loads queued for
    // the next step also count on.
    __shared__ double sG[kPairMaxTI + 4][4];
    auto clampm = [&](int m) { return min(max(m, 0), nr - 1); };
    for (int t = threadIdx.x; t < i1 - i0 + 4; t += kWave * NW) {
        const StsPlaneRaw r = sts_plane_raw(a.geo, clampm(i0 - 2 + t));
        sG[t][0] = r.gq;
        sG[t][1] = r.gr;
        sG[t][2] = r.grm;
        sG[t][3] = r.vr;
    }
    __syncthreads();
    auto table = [&](int m) {
        const int t = m - (i0 - 2);
        return StsPlaneRaw{sG[t][0], sG[t][1], sG[t][2], sG[t][3], clampm(m)};
    };

    // chunks march up (even chunk index) or down
    const bool up = (it & 1) == 0;
    const int dir = up ? 1 : -1;
    const int first = up ? i0 - 1 : i1;
    // register queues: X and nu at planes m - dir (b), m (c), m + dir (a);
    // Z and L0 at m (c); L0 at m - dir (b).  Each step loads X and nu of plane
    // m + 2 dir and Z and L0 of plane m + dir for the next step.
    VD Xb = bld<double, 2, MAS_STS_AUX_XN>(RX, ldoff(first - dir));
    VD Nb = bld<double, 2, MAS_STS_AUX_XN>(RN, ldoff(first - dir));
    VD Xc = bld<double, 2, MAS_STS_AUX_XN>(RX, ldoff(first));
    VD Nc = bld<double, 2, MAS_STS_AUX_XN>(RN, ldoff(first));
    VD Xa = bld<double, 2, MAS_STS_AUX_XN>(RX, ldoff(first + dir));
    VD Na = bld<double, 2, MAS_STS_AUX_XN>(RN, ldoff(first + dir));
    VD Zc{}, Lc{}, Lb_{};
    if constexpr (HZ) Zc = bld<double, 2>(RZ, zloff(first));
    if constexpr (HL) Lc = bld<double, 2>(RL, zloff(first));

    for (int s = 0; s < nsteps; ++s) {
        const int m = first + s * dir;
        const int mb = m - dir;  // plane of stage B
        const int q0 = s & 3, q1 = (s - 1) & 3, q2 = (s - 2) & 3, x0 = s & 1;
        // ---- loads for the next step (and Y0 of this step's B)
        const VD Xn = bld<double, 2, MAS_STS_AUX_XN>(RX, ldoff(m + 2 * dir));
        const VD Nn = bld<double, 2, MAS_STS_AUX_XN>(RN, ldoff(m + 2 * dir));
        VD Zn{}, Ln{}, Yo{};
        if constexpr (HZ) Zn = bld<double, 2>(RZ, zloff(m + dir));
        if constexpr (HL) Ln = bld<double, 2>(RL, zloff(m + dir));
        if constexpr (HY) Yo = bld<double, 2, MAS_STS_AUX_ZL>(RY, s >= 2 ? ownoff(mb) : kOOB);

        // ---- X and nu of plane m to LDS; A of plane mb went there last step
        sX[x0][rho][c] = Xc.v[0];
        sX[x0][rho][c + 1] = Xc.v[1];
        sN[q0][rho][c] = Nc.v[0];
        sN[q0][rho][c + 1] = Nc.v[1];
        __syncthreads();

        // ---- stage A at plane m (zero outside the grid)
        VD Yc{};
        const bool inA = rowin && m >= 0 && m < nr;
        {
            const VD XU = lds2(sX[x0][ru]), XD = lds2(sX[x0][rd]);
            const VD NU = lds2(sN[q0][ru]), ND = lds2(sN[q0][rd]);
            const StsPlane pf = sts_plane(a.geo, table(m), nr, vt, a.mdtA);
            const double tU = pf.gq * hU, tD = pf.gq * hD, tP = pf.gq * hP;
            const VD &Xp = up ? Xa : Xb, &Xm = up ? Xb : Xa;
            const VD &Np = up ? Na : Nb, &Nm = up ? Nb : Na;
            const double xl0 = lane_prev(Xc.v[1]), nl0 = lane_prev(Nc.v[1]);
            const double xr1 = lane_next(Xc.v[0]), nr1 = lane_next(Nc.v[0]);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const double xc = Xc.v[e], nc = Nc.v[e];
                const double xl = e ? Xc.v[0] : xl0, nl = e ? Nc.v[0] : nl0;
                const double xr = e ? xr1 : Xc.v[1], nrr = e ? nr1 : Nc.v[1];
                const double f = sts_flux(pf, tU, tD, tP, xc, nc, Xp.v[e], Np.v[e], Xm.v[e], Nm.v[e], XU.v[e],
                                          NU.v[e], XD.v[e], ND.v[e], xl, nl, xr, nrr);
                const double lv = HL ? Lc.v[e] : xc;
                const double o = sts_combine(a.aA, xc, a.bA, Zc.v[e], a.gA, lv, 0.0, pf.scale, f);
                Yc.v[e] = inA ? o : 0.0;
            }
        }

        // ---- stage B at plane mb (inside the chunk from the third step on):
        // A at mb and its theta neighbours, A and nu at m - 2 dir, and nu's
        // theta neighbours at mb come from the LDS rings, A at m from registers
        if (s >= 2) {
            const VD Yb = lds2(sY[q1][rho]), YU = lds2(sY[q1][ru]), YD = lds2(sY[q1][rd]);
            const VD Yb2 = lds2(sY[q2][rho]), Nbb = lds2(sN[q2][rho]);
            const VD NU = lds2(sN[q1][ru]), ND = lds2(sN[q1][rd]);
            const StsPlane pf = sts_plane(a.geo, table(mb), nr, vt, a.mdtB);
            const double tU = pf.gq * hU, tD = pf.gq * hD, tP = pf.gq * hP;
            const VD &Yp = up ? Yc : Yb2, &Ym = up ? Yb2 : Yc;
            const VD &Np = up ? Nc : Nbb, &Nm = up ? Nbb : Nc;
            const double yl0 = lane_prev(Yb.v[1]), nl0 = lane_prev(Nb.v[1]);
            const double yr1 = lane_next(Yb.v[0]), nr1 = lane_next(Nb.v[0]);
            VD o;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const double yc = Yb.v[e], nc = Nb.v[e];
                const double yl = e ? Yb.v[0] : yl0, nl = e ? Nb.v[0] : nl0;
                const double yr = e ? yr1 : Yb.v[1], nrr = e ? nr1 : Nb.v[1];
                const double f = sts_flux(pf, tU, tD, tP, yc, nc, Yp.v[e], Np.v[e], Ym.v[e], Nm.v[e], YU.v[e],
                                          NU.v[e], YD.v[e], ND.v[e], yl, nl, yr, nrr);
                const double lv = HL ? Lb_.v[e] : Xb.v[e];
                o.v[e] = sts_combine(a.aB, yc, a.bB, Xb.v[e], a.gB, lv, Yo.v[e], pf.scale, f);
            }
            bst<double, 2, MAS_STS_AUX_ST>(RB, ownoff(mb), o);
        }
        sY[q0][rho][c] = Yc.v[0];
        sY[q0][rho][c + 1] = Yc.v[1];
        if constexpr (!HY) bst<double, 2, MAS_STS_AUX_ST>(RA, ownoff(m), Yc);

        Nb = Nc;
        Xb = Xc;
        Lb_ = Lc;
        Nc = Na;
        Xc = Xa;
        Na = Nn;
        Xa = Xn;
        Lc = Ln;
        Zc = Zn;
    }
}

}  // namespace mas
