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
    const uint32_t nbytes = (uint32_t)(a.d.n * (int64_t)ES);
    const auto RX = make_rsrc(a.X, nbytes), RN = make_rsrc(a.nu, nbytes),
               RZ = make_rsrc(a.Z, HZ ? nbytes : 0u), RL = make_rsrc(a.L0, HL ? nbytes : 0u),
               RY = make_rsrc(a.Y0, HY ? nbytes : 0u), RO = make_rsrc(a.out, nbytes);

    auto own_off = [&](int m) -> uint32_t {
        return (ldo && m >= 0 && m < nr) ? (uint32_t)((int64_t)m * plane + col) * ES : kOOB;
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
        const int64_t base = (int64_t)m * plane;
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
        const double gq = a.geo.gq[m];
        const double hRp = 0.5 * a.geo.gr[m] * vt;                    // face m | m+1 (0 at m = nr-1)
        const double hRm = (m > 0) ? 0.5 * a.geo.gr[m - 1] * vt : 0.0;  // face m-1 | m
        const double gw = ((m == 0) ? a.geo.gw_in : 0.0) * vt + ((m == nr - 1) ? a.geo.gw_out : 0.0) * vt;
        const double scale = a.mdt / (a.geo.vr[m] * vt);
        const double tU = gq * hU, tD = gq * hD, tP = gq * hP;
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
            double f = hRp * (nc + Np.v[e]) * (xc - Xp.v[e]);
            f += hRm * (nc + Nm.v[e]) * (xc - Xm.v[e]);
            f += gw * nc * xc;
            f += tU * (nc + nu_u) * (xc - xu);
            f += tD * (nc + nu_d) * (xc - xd);
            f += tP * ((nc + nl) * (xc - xl) + (nc + nrr) * (xc - xr));
            o.v[e] = ((a.a * xc + a.b * Zv.v[e]) + a.g * Lv.v[e] + Yv.v[e]) - scale * f;
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

}  // namespace mas
