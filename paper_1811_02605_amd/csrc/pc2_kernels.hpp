// PC2: block-Jacobi preconditioner with a zero-fill incomplete LU factor per
// block (the paper, Section 2.2; MAS factors one block per MPI rank, and
// Section 4.1 notes that its triangular solves are sequential and that PC1
// performed about as well on GPUs).
//
// Blocks are boxes of kPc2I x kPc2J x kPc2K cells (r, theta, phi) tiling the
// grid from index 0; couplings between blocks and the periodic phi coupling
// are left out.  On the scaled system A^ = W^-1 A W^-1 (unit diagonal,
// A^(c, nb) = -c^) with cells in natural order, ILU(0) of a box with the
// 7-point graph changes only the diagonal:
//     d_c = 1 - sum_{lower neighbours nb in the block} c^_{c,nb}^2 / d_nb,
// and M^-1 r is
//     forward   y_c = (r_c + sum_{lower nb} c^ y_nb) / d_c
//     backward  z_c = y_c + (sum_{upper nb} c^ z_nb) / d_c.
// (The ILU(0) factor of the scaled matrix is the scaled ILU(0) factor of A,
// so PCG on A^ with it has the iterates of PCG on A with the ILU(0) of A.)
// The direction and SpMV step of a PC2 iteration (p = z + beta p, q = A^ p,
// (p, q)) is the PCG iteration kernel run without r, q and x inputs.
//
// Factor: one wave per block, lane k' owns phi offset k', the wave walks the
// block's (r, theta) rows in order and solves each row's phi recurrence
// d_k = s_k - c^2 / d_{k-1} by a prefix scan of 2 x 2 matrices (the maps
// d -> (s d - c^2) / d compose as matrix products).
// Solve: one wave per block, lane k' owns phi offset k' (coalesced rows), and
// the wave walks the block's (r, theta) rows in order.  The r and theta
// terms come from the rows already done (kept in registers); along phi the
// forward sweep is the first-order recurrence y_k = c_k y_{k-1} + b_k with
// c_k = c^p_{k-1,k} / d_k, solved by a prefix scan of the affine maps
// y -> c y + b across the lanes (the backward sweep scans the other way).
#pragma once

#include "kernels.hpp"

namespace mas {

constexpr int kPc2I = 8, kPc2J = 8, kPc2K = 64;
static_assert(kPc2K == kWave, "one lane per phi offset of a block");

// T: the precision of the couplings, the modified diagonal and the PCG
// vectors (double, or float inside double-precision refinement); w and the
// partial sums are double.
template <typename T>
struct Pc2Args {
    const T *cr, *ct, *cp;       // scaled couplings to the +r, +theta, +phi neighbours
    const double *w;
    T *d;                        // modified diagonal (written by the factor kernel)
    T *r, *x, *z;                // solve: r -= alpha q, x += alpha p, z = M^-1 r
    const T *q, *p;
    double *partials;            // [blocks][2]: (r, z), ||W r||^2
    const Ctl *ctl;
    Dims dm;
    int nbi, nbj, nbk;           // blocks per direction
    int update;                  // solve: apply the alpha updates first
};

// Inclusive scan of the affine maps y -> C y + B over the 64 lanes in lane
// order: each lane ends with the composition of its own map after those of
// all lower lanes, i.e. B = y_lane for y_-1 = 0.  DPP moves (GFX9 family):
// row_shr by 1, 2, 4, 8 inside each 16-lane row, then row_bcast:15 (the last
// lane of rows 0 and 2 to rows 1 and 3) and row_bcast:31 (lane 31 to rows 2
// and 3).  A lane that receives nothing gets the identity map (1, 0), which
// composes as a no-op.
template <int CTRL, int ROWS>
__device__ inline double dpp_or(double v, double identity) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v), o = __builtin_bit_cast(uint64_t, identity);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)b,
                                                              CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32),
                                                              (int)(uint32_t)(b >> 32), CTRL, ROWS,
                                                              0xf, false);
    return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

template <int CTRL, int ROWS>
__device__ inline float dpp_or(float v, float identity) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, identity),
                                                                 __builtin_bit_cast(int, v), CTRL,
                                                                 ROWS, 0xf, false));
}

template <int CTRL, int ROWS, typename T>
__device__ inline void affine_step(T &C, T &B) {
    const T Cs = dpp_or<CTRL, ROWS>(C, T(1)), Bs = dpp_or<CTRL, ROWS>(B, T(0));
    B = C * Bs + B;
    C = C * Cs;
}

template <typename T>
__device__ inline T affine_scan(T C, T B) {
    affine_step<0x111, 0xf>(C, B);  // row_shr:1
    affine_step<0x112, 0xf>(C, B);  // row_shr:2
    affine_step<0x114, 0xf>(C, B);  // row_shr:4
    affine_step<0x118, 0xf>(C, B);  // row_shr:8
    affine_step<0x142, 0xa>(C, B);  // row_bcast:15 into rows 1 and 3
    affine_step<0x143, 0xc>(C, B);  // row_bcast:31 into rows 2 and 3
    return B;
}

// Linear-fractional maps d -> (m00 d + m01) / (m10 d + m11) as 2 x 2 matrices
// (projective: a common factor does not change the map).
struct Mob {
    double m00, m01, m10, m11;
};

// Inclusive scan of such maps over the 64 lanes in lane order (the same DPP
// moves as affine_scan; a lane that receives nothing composes with the
// identity).  After the first three steps (products of up to eight maps)
// the product is rescaled by a power of two, exactly, so that the longer
// products of the last three steps neither overflow nor underflow: every
// map [s, -c^2; 1, 0] has entries of magnitude at most 1 (unit diagonal,
// diagonal dominance), so the entries of a product of eight stay within
// [min(s)^8, 2^8].  A power-of-two scale commutes with every rounding here,
// so the result is the same, bit for bit, as with a rescale after every
// step; the map is applied as a ratio, which ignores the scale.
template <int CTRL, int ROWS, bool RESCALE>
__device__ inline void mobius_step(Mob &P) {
    const double q00 = dpp_or<CTRL, ROWS>(P.m00, 1.0), q01 = dpp_or<CTRL, ROWS>(P.m01, 0.0);
    const double q10 = dpp_or<CTRL, ROWS>(P.m10, 0.0), q11 = dpp_or<CTRL, ROWS>(P.m11, 1.0);
    // each entry a sum of two products, the first fused: written out, so
    // that the rounding does not depend on which product the compiler would
    // fuse in a given context
    const double r00 = fma(P.m00, q00, P.m01 * q10), r01 = fma(P.m00, q01, P.m01 * q11);
    const double r10 = fma(P.m10, q00, P.m11 * q10), r11 = fma(P.m10, q01, P.m11 * q11);
    if constexpr (RESCALE) {
        const double m = fmax(fmax(fabs(r00), fabs(r01)), fmax(fabs(r10), fabs(r11)));
        const int ex = (m > 0.0) ? ilogb(m) : 0;
        P = Mob{ldexp(r00, -ex), ldexp(r01, -ex), ldexp(r10, -ex), ldexp(r11, -ex)};
    } else {
        P = Mob{r00, r01, r10, r11};
    }
}

__device__ inline Mob mobius_scan(Mob P) {
    mobius_step<0x111, 0xf, false>(P);  // row_shr:1
    mobius_step<0x112, 0xf, false>(P);  // row_shr:2
    mobius_step<0x114, 0xf, true>(P);   // row_shr:4
    mobius_step<0x118, 0xf, false>(P);  // row_shr:8
    mobius_step<0x142, 0xa, false>(P);  // row_bcast:15 into rows 1 and 3
    mobius_step<0x143, 0xc, false>(P);  // row_bcast:31 into rows 2 and 3
    return P;
}

// d_c for every cell of the block, from the double-precision couplings (a
// single-precision factor is the double one rounded: TOUT = float).  Lanes
// run along phi (coalesced rows) and the wave walks the block's (r, theta)
// rows in order, as the solve does; with the r and theta terms of a row
// known from the rows done, the phi recurrence
//     d_k = s_k - cp_{k-1,k}^2 / d_{k-1},   s_k = 1 - (r and theta terms),
// is the composition of the maps d -> (s_k d - cp^2) / d, solved by a prefix
// scan of their matrices [s_k, -cp^2; 1, 0] (the first lane of a block has
// no phi term: [s_0, 0; 1, 0], which gives d_0 = s_0 from any start).
// Each row's couplings are loaded one plane (eight rows) before it is
// scanned, into one of two register sets that alternate by plane.  Every
// access goes through a buffer resource over one r plane, and whatever is
// not there (the -r coupling of the block's first plane, the -theta one of
// its first row, the -phi one of its first lane, lanes and rows past the
// grid, planes past the block) has bit 31 set in its offset or a resource of
// size zero: it reads zero or is not stored.  The loop body has no branch:
// a missing coupling enters as 0 against a previous d of 1, which leaves s_k
// unchanged bit for bit (1 - 0 * 0 / 1 = 1); lanes past the grid are the
// highest ones, and the scan only moves values to higher lanes, so their
// maps never reach a lane in the grid; planes are taken in pairs, the
// second of an odd last pair storing nothing.  So the compiler waits for
// each plane's loads only where they are used.
struct Pc2Fac {
    double cr, ct, cp;
};
struct Pc2FacPlane {
    __amdgpu_buffer_rsrc_t cr, ct, cp;  // cr over the plane below, ct and cp over this one
};

template <typename TOUT>
__global__ __launch_bounds__(kWave) void k_pc2_factor(Pc2Args<double> a, TOUT *dout) {
    const Dims &dm = a.dm;
    const int blk = blockIdx.x;
    const int bk = blk % a.nbk, bj = (blk / a.nbk) % a.nbj, bi = blk / (a.nbk * a.nbj);
    const int lane = threadIdx.x;
    const int I0 = bi * kPc2I, J0 = bj * kPc2J, k0 = bk * kPc2K;
    const int kn = min(kPc2K, dm.np - k0);
    const bool act = lane < kn;
    const int ni = min(kPc2I, dm.nr - I0), nj = min(kPc2J, dm.nt - J0);
    // an r plane of one array holds fewer than 2^31 / 7 bytes (the grid
    // check keeps seven planes below 2 GiB): byte offsets of its cells stay
    // below bit 31
    const uint32_t pbytes = (uint32_t)(dm.plane * 8);
    const uint32_t lbad = act ? 0u : kOOB;
    const uint32_t pbad = (act && lane > 0) ? 0u : kOOB;
    // this lane's cell of block row jj in a plane, and the bad bit of the row
    auto cell = [&](int jj) -> int { return (J0 + jj) * dm.np + k0 + lane; };
    auto rbad = [&](int jj) -> uint32_t { return (jj < nj ? 0u : kOOB) | lbad; };
    auto plane_rsrc = [&](int ii) {
        const bool in = ii < ni;
        const int m = min(I0 + ii, dm.nr - 1), mb = max(I0 + ii - 1, 0);
        return Pc2FacPlane{make_rsrc(a.cr + (int64_t)mb * dm.plane, (in && ii > 0) ? pbytes : 0u),
                           make_rsrc(a.ct + (int64_t)m * dm.plane, in ? pbytes : 0u),
                           make_rsrc(a.cp + (int64_t)m * dm.plane, in ? pbytes : 0u)};
    };
    auto load = [&](const Pc2FacPlane &R, int jj) {
        const int c = cell(jj);
        const uint32_t bad = rbad(jj);
        Pc2Fac v;
        v.cr = bld<double, 1>(R.cr, ((uint32_t)c * 8u) | bad).v[0];
        v.ct = bld<double, 1>(R.ct, ((uint32_t)(c - dm.np) * 8u) | bad | (jj > 0 ? 0u : kOOB)).v[0];
        v.cp = bld<double, 1>(R.cp, ((uint32_t)(c - 1) * 8u) | bad | pbad).v[0];
        return v;
    };
    double dp[kPc2J];  // d of the previous r plane of the block, per theta row
#pragma unroll
    for (int jj = 0; jj < kPc2J; ++jj) dp[jj] = 1.0;
    // plane ii: rows from `cur`, the rows of plane ii + 1 issued into `nxt`
    auto plane_step = [&](int ii, const Pc2Fac (&cur)[kPc2J], Pc2Fac (&nxt)[kPc2J]) {
        const Pc2FacPlane Rn = plane_rsrc(ii + 1);
        const auto Rd = make_rsrc(dout + (int64_t)min(I0 + ii, dm.nr - 1) * dm.plane,
                                  ii < ni ? (uint32_t)(dm.plane * (int64_t)sizeof(TOUT)) : 0u);
        double drow = 1.0;  // d of the previous theta row
#pragma unroll
        for (int jj = 0; jj < kPc2J; ++jj) {
            const Pc2Fac c = cur[jj];
            nxt[jj] = load(Rn, jj);
            // keeps the loads here: the scheduler would otherwise sink them
            // towards their use a plane later, where they would be waited for
            // right after being issued
            __builtin_amdgcn_sched_barrier(0);
            double sk = 1.0;
            sk -= c.cr * c.cr / dp[jj];  // no -r neighbour in the block: 0
            sk -= c.ct * c.ct / drow;    // no -theta neighbour: 0
            Mob P{sk, -(c.cp * c.cp), 1.0, 0.0};
            P = mobius_scan(P);
            const double dv = (P.m00 + P.m01) / (P.m10 + P.m11);  // the map of d = 1
            bst<TOUT, 1>(Rd, ((uint32_t)cell(jj) * (uint32_t)sizeof(TOUT)) | rbad(jj),
                         VecT<TOUT, 1>{{(TOUT)dv}});
            dp[jj] = dv;
            drow = dv;
        }
    };
    Pc2Fac qa[kPc2J], qb[kPc2J];
    {
        const Pc2FacPlane R0 = plane_rsrc(0);
#pragma unroll
        for (int jj = 0; jj < kPc2J; ++jj) qa[jj] = load(R0, jj);
        // the first plane's rows are waited for here, once per block (an
        // empty statement that takes them as register operands: the
        // compiler waits for their loads before it): the loop is then
        // entered with no loads in flight, and the waits the compiler
        // places in it are those of its own loads, a plane after issue
#pragma unroll
        for (int jj = 0; jj < kPc2J; ++jj)
            asm volatile("" ::"v"(qa[jj].cr), "v"(qa[jj].ct), "v"(qa[jj].cp));
    }
    for (int ii = 0; ii < ni; ii += 2) {
        plane_step(ii, qa, qb);
        plane_step(ii + 1, qb, qa);
    }
}

// z = M^-1 r, first applying r -= alpha q and x += alpha p when a.update;
// per-block partials (r, z) and ||W r||^2.  Each sweep loads the next row's
// inputs before it scans the current row, so a wave keeps one row of loads
// in flight behind its scans.
// With L the strictly lower couplings and D = diag(d), M = (D - L) D^-1 (D - L^T),
// the forward sweep gives y = (D - L)^-1 r and z = (D - L^T)^-1 D y, so
// (r, z) = r^T (D - L^T)^-1 D (D - L)^-1 r = y^T D y: the forward sweep
// accumulates it and the backward sweep need not read r again.
template <typename T>
struct Pc2Fwd {
    T r, q, x, p;
    double w;
    T d, cr, ct, cp;
};
template <typename T>
struct Pc2Bwd {
    T cr, ct, d, y, cp;
};

// PF: rows of loads in flight ahead of the row being scanned.
template <typename T, int PF>
__global__ __launch_bounds__(kWave) void k_pc2_solve(Pc2Args<T> a) {
    static_assert(PF == 1 || PF == 2, "prefetch depth");
    if (a.ctl->flag != FLAG_RUN) return;
    const Dims &dm = a.dm;
    const int blk = blockIdx.x;
    const int bk = blk % a.nbk, bj = (blk / a.nbk) % a.nbj, bi = blk / (a.nbk * a.nbj);
    const int lane = threadIdx.x;
    const int k0 = bk * kPc2K;
    const int kn = min(kPc2K, dm.np - k0);
    const bool act = lane < kn;
    const int k = k0 + (act ? lane : 0);
    const int ni = min(kPc2I, dm.nr - bi * kPc2I), nj = min(kPc2J, dm.nt - bj * kPc2J);
    const bool upd = a.update != 0;
    const T alpha = upd ? (T)a.ctl->alpha : T(0);
    // distinct arrays: lets the compiler issue later rows' loads ahead of
    // earlier rows' stores
    const T *__restrict__ cr = a.cr, *__restrict__ ct = a.ct, *__restrict__ cp = a.cp;
    const double *__restrict__ w = a.w;
    const T *__restrict__ dd = a.d, *__restrict__ q = a.q;
    const T *__restrict__ pp = a.p;
    T *__restrict__ r = a.r, *__restrict__ x = a.x, *__restrict__ z = a.z;
    auto cell = [&](int ii, int jj, int kk) -> int64_t {
        return ((int64_t)(bi * kPc2I + ii) * dm.nt + (bj * kPc2J + jj)) * dm.np + kk;
    };
    auto load_f = [&](int ii, int jj) {
        Pc2Fwd<T> v{0, 0, 0, 0, 0.0, 1, 0, 0, 0};
        if (act && ii < ni && jj < nj) {
            const int64_t c = cell(ii, jj, k);
            v.r = r[c];
            if (upd) {
                v.q = q[c];
                v.x = x[c];
                v.p = pp[c];
            }
            v.w = w[c];
            v.d = dd[c];
            if (ii > 0) v.cr = cr[c - dm.plane];
            if (jj > 0) v.ct = ct[c - dm.np];
            if (lane > 0) v.cp = cp[c - 1];
        }
        return v;
    };
    double rw = 0.0, rz = 0.0;
    T yp[kPc2J];  // previous r plane of the block, one value per theta row
    // forward sweep: y into z
#pragma unroll
    for (int jj = 0; jj < kPc2J; ++jj) yp[jj] = T(0);
    // rows in order t = ii nj + jj; row t + PF is loaded before row t is scanned
    auto load_ft = [&](int t) { return load_f(t / nj, t % nj); };
    Pc2Fwd<T> cur = load_f(0, 0);
    Pc2Fwd<T> ahead{};
    if constexpr (PF == 2) ahead = load_ft(1);
    for (int ii = 0; ii < ni; ++ii) {
        T yrow = T(0);  // previous theta row
#pragma unroll
        for (int jj = 0; jj < kPc2J; ++jj) {
            if (jj < nj) {
                const Pc2Fwd<T> nxt = load_ft(ii * nj + jj + PF);
                T Bc = T(0), Cc = T(0);
                T rc = cur.r;
                if (act) {
                    if (upd) rc -= alpha * cur.q;
                    const double t = cur.w * (double)rc;
                    rw += t * t;
                    T sc = rc;
                    if (ii > 0) sc += cur.cr * yp[jj];
                    if (jj > 0) sc += cur.ct * yrow;
                    const T dinv = T(1) / cur.d;
                    Bc = sc * dinv;
                    Cc = cur.cp * dinv;
                }
                const T y = affine_scan(Cc, Bc);
                if (act) {
                    // (r, M^-1 r) = y^T D y (see below)
                    rz += (double)cur.d * (double)y * (double)y;
                    const int64_t c = cell(ii, jj, k);
                    if (upd) {
                        r[c] = rc;
                        x[c] = cur.x + alpha * cur.p;
                    }
                    z[c] = y;
                }
                yp[jj] = y;
                yrow = y;
                if constexpr (PF == 2) {
                    cur = ahead;
                    ahead = nxt;
                } else {
                    cur = nxt;
                }
            }
        }
    }
    // backward sweep: z in place; lane l takes phi offset kn-1-l, so the
    // recurrence z_k = c_k z_{k+1} + b_k runs up the lanes again
    const int kb = k0 + (act ? kn - 1 - lane : 0);
    auto load_b = [&](int ii, int jj) {
        Pc2Bwd<T> v{0, 0, 1, 0, 0};
        if (act && ii >= 0 && jj >= 0) {
            const int64_t c = cell(ii, jj, kb);
            if (ii < ni - 1) v.cr = cr[c];
            if (jj < nj - 1) v.ct = ct[c];
            v.d = dd[c];
            v.y = z[c];
            if (lane > 0) v.cp = cp[c];
        }
        return v;
    };
#pragma unroll
    for (int jj = 0; jj < kPc2J; ++jj) yp[jj] = T(0);
    // rows in reverse order; row t - PF is loaded before row t is scanned
    // (t < 0 divides to ii = 0, jj < 0 or to ii < 0: no load)
    auto load_bt = [&](int t) { return load_b(t / nj, t % nj); };
    Pc2Bwd<T> bcur = load_b(ni - 1, nj - 1);
    Pc2Bwd<T> bahead{};
    if constexpr (PF == 2) bahead = load_bt(ni * nj - 2);
    for (int ii = ni - 1; ii >= 0; --ii) {
        T zrow = T(0);  // next theta row
#pragma unroll
        for (int jj = kPc2J - 1; jj >= 0; --jj) {
            if (jj < nj) {
                const Pc2Bwd<T> nxt = load_bt(ii * nj + jj - PF);
                T Bc = T(0), Cc = T(0);
                if (act) {
                    T sc = T(0);
                    if (ii < ni - 1) sc += bcur.cr * yp[jj];
                    if (jj < nj - 1) sc += bcur.ct * zrow;
                    const T dinv = T(1) / bcur.d;
                    Bc = bcur.y + sc * dinv;
                    Cc = bcur.cp * dinv;
                }
                const T zc = affine_scan(Cc, Bc);
                if (act) z[cell(ii, jj, kb)] = zc;
                yp[jj] = zc;
                zrow = zc;
                if constexpr (PF == 2) {
                    bcur = bahead;
                    bahead = nxt;
                } else {
                    bcur = nxt;
                }
            }
        }
    }
    __shared__ double lds[2];
    double v2[2] = {rz, rw};
    block_sum_store<2>(v2, a.partials + (int64_t)blockIdx.x * 2, lds);
}

// Several right-hand sides under one operator: the block solve of each, as
// k_pc2_solve, with the couplings, w and the modified diagonal loaded once
// per cell for all of them (T: double, or float inside double-precision
// refinement; w and the partial sums are double).  Right-hand side h's
// partial sums go to partials + 2 h gridDim.x; one whose control block is
// stopped moves no bytes.
template <typename T, int NR>
struct Pc2MultiArgs {
    const T *cr, *ct, *cp;
    const double *w;
    const T *d;
    T *r[NR], *x[NR], *z[NR];
    const T *q[NR], *p[NR];
    double *partials;
    const Ctl *ctl;  // [NR]
    Dims dm;
    int nbi, nbj, nbk;
    int update;
};

template <typename T, int NR>
struct Pc2MFwd {
    double w;
    T d, cr, ct, cp;
    T r[NR], q[NR], x[NR], p[NR];
};
template <typename T, int NR>
struct Pc2MBwd {
    T cr, ct, d, cp;
    T y[NR];
};

template <typename T, int NR>
__global__ __launch_bounds__(kWave) void k_pc2_solve_multi(Pc2MultiArgs<T, NR> a) {
    bool run[NR];
    T alpha[NR];
    bool any = false;
#pragma unroll
    for (int h = 0; h < NR; ++h) {
        run[h] = a.ctl[h].flag == FLAG_RUN;
        any = any || run[h];
        alpha[h] = (a.update != 0 && run[h]) ? (T)a.ctl[h].alpha : T(0);
    }
    if (!any) return;
    const Dims &dm = a.dm;
    const int blk = blockIdx.x;
    const int bk = blk % a.nbk, bj = (blk / a.nbk) % a.nbj, bi = blk / (a.nbk * a.nbj);
    const int lane = threadIdx.x;
    const int k0 = bk * kPc2K;
    const int kn = min(kPc2K, dm.np - k0);
    const bool act = lane < kn;
    const int k = k0 + (act ? lane : 0);
    const int ni = min(kPc2I, dm.nr - bi * kPc2I), nj = min(kPc2J, dm.nt - bj * kPc2J);
    const bool upd = a.update != 0;
    auto cell = [&](int ii, int jj, int kk) -> int64_t {
        return ((int64_t)(bi * kPc2I + ii) * dm.nt + (bj * kPc2J + jj)) * dm.np + kk;
    };
    auto load_f = [&](int ii, int jj) {
        Pc2MFwd<T, NR> v;
        v.w = 0.0;
        v.cr = v.ct = v.cp = T(0);
        v.d = T(1);
#pragma unroll
        for (int h = 0; h < NR; ++h) v.r[h] = v.q[h] = v.x[h] = v.p[h] = T(0);
        if (act && ii < ni && jj < nj) {
            const int64_t c = cell(ii, jj, k);
            v.w = a.w[c];
            v.d = a.d[c];
            if (ii > 0) v.cr = a.cr[c - dm.plane];
            if (jj > 0) v.ct = a.ct[c - dm.np];
            if (lane > 0) v.cp = a.cp[c - 1];
#pragma unroll
            for (int h = 0; h < NR; ++h) {
                if (run[h]) {
                    v.r[h] = a.r[h][c];
                    if (upd) {
                        v.q[h] = a.q[h][c];
                        v.x[h] = a.x[h][c];
                        v.p[h] = a.p[h][c];
                    }
                }
            }
        }
        return v;
    };
    double rw[NR], rz[NR];
    T yp[NR][kPc2J];  // previous r plane of the block, per theta row
#pragma unroll
    for (int h = 0; h < NR; ++h) {
        rw[h] = rz[h] = 0.0;
#pragma unroll
        for (int jj = 0; jj < kPc2J; ++jj) yp[h][jj] = T(0);
    }
    // forward sweep: y into z; row t + 1 is loaded before row t is scanned
    auto load_ft = [&](int t) { return load_f(t / nj, t % nj); };
    Pc2MFwd<T, NR> cur = load_f(0, 0);
    for (int ii = 0; ii < ni; ++ii) {
        T yrow[NR];
#pragma unroll
        for (int h = 0; h < NR; ++h) yrow[h] = T(0);
#pragma unroll
        for (int jj = 0; jj < kPc2J; ++jj) {
            if (jj < nj) {
                const Pc2MFwd<T, NR> nxt = load_ft(ii * nj + jj + 1);
                const T dinv = T(1) / cur.d;
                const int64_t c = cell(ii, jj, k);
#pragma unroll
                for (int h = 0; h < NR; ++h) {
                    if (!run[h]) continue;  // uniform across the wave
                    T Bc = T(0), Cc = T(0);
                    T rc = cur.r[h];
                    if (act) {
                        if (upd) rc -= alpha[h] * cur.q[h];
                        const double t = cur.w * (double)rc;
                        rw[h] += t * t;
                        T sc = rc;
                        if (ii > 0) sc += cur.cr * yp[h][jj];
                        if (jj > 0) sc += cur.ct * yrow[h];
                        Bc = sc * dinv;
                        Cc = cur.cp * dinv;
                    }
                    const T y = affine_scan(Cc, Bc);
                    if (act) {
                        rz[h] += (double)cur.d * (double)y * (double)y;  // (r, M^-1 r) = y^T D y
                        if (upd) {
                            a.r[h][c] = rc;
                            a.x[h][c] = cur.x[h] + alpha[h] * cur.p[h];
                        }
                        a.z[h][c] = y;
                    }
                    yp[h][jj] = y;
                    yrow[h] = y;
                }
                cur = nxt;
            }
        }
    }
    // backward sweep: z in place, lanes reversed (see k_pc2_solve)
    const int kb = k0 + (act ? kn - 1 - lane : 0);
    auto load_b = [&](int ii, int jj) {
        Pc2MBwd<T, NR> v;
        v.cr = v.ct = v.cp = T(0);
        v.d = T(1);
#pragma unroll
        for (int h = 0; h < NR; ++h) v.y[h] = T(0);
        if (act && ii >= 0 && jj >= 0) {
            const int64_t c = cell(ii, jj, kb);
            if (ii < ni - 1) v.cr = a.cr[c];
            if (jj < nj - 1) v.ct = a.ct[c];
            v.d = a.d[c];
            if (lane > 0) v.cp = a.cp[c];
#pragma unroll
            for (int h = 0; h < NR; ++h)
                if (run[h]) v.y[h] = a.z[h][c];
        }
        return v;
    };
    auto load_bt = [&](int t) { return load_b(t / nj, t % nj); };
#pragma unroll
    for (int h = 0; h < NR; ++h)
#pragma unroll
        for (int jj = 0; jj < kPc2J; ++jj) yp[h][jj] = T(0);
    Pc2MBwd<T, NR> bcur = load_b(ni - 1, nj - 1);
    for (int ii = ni - 1; ii >= 0; --ii) {
        T zrow[NR];
#pragma unroll
        for (int h = 0; h < NR; ++h) zrow[h] = T(0);
#pragma unroll
        for (int jj = kPc2J - 1; jj >= 0; --jj) {
            if (jj < nj) {
                const Pc2MBwd<T, NR> nxt = load_bt(ii * nj + jj - 1);
                const T dinv = T(1) / bcur.d;
#pragma unroll
                for (int h = 0; h < NR; ++h) {
                    if (!run[h]) continue;
                    T Bc = T(0), Cc = T(0);
                    if (act) {
                        T sc = T(0);
                        if (ii < ni - 1) sc += bcur.cr * yp[h][jj];
                        if (jj < nj - 1) sc += bcur.ct * zrow[h];
                        Bc = bcur.y[h] + sc * dinv;
                        Cc = bcur.cp * dinv;
                    }
                    const T zc = affine_scan(Cc, Bc);
                    if (act) a.z[h][cell(ii, jj, kb)] = zc;
                    yp[h][jj] = zc;
                    zrow[h] = zc;
                }
                bcur = nxt;
            }
        }
    }
    __shared__ double lds[2];
#pragma unroll
    for (int h = 0; h < NR; ++h) {
        if (!run[h]) continue;  // uniform across the block
        double v2[2] = {rz[h], rw[h]};
        block_sum_store<2>(v2, a.partials + (int64_t)(2 * h) * gridDim.x + (int64_t)blockIdx.x * 2, lds);
        __syncthreads();
    }
}

// After the SpMV: alpha = (r, z) / (p, q) (or a breakdown); (p, q) is the
// first of every `stride` partials.
__global__ __launch_bounds__(kRedThreads) void k_pc2_fin_a(const double *partials, int nblk,
                                                           int stride, Ctl *ctl) {
    if (ctl->flag != FLAG_RUN) return;
    __shared__ double sh[kRedThreads];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kRedThreads) v += partials[(int64_t)b * stride];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double PQ = sh[0];
    ctl->pq = PQ;
    if (!(PQ > 0.0) || !isfinite(PQ)) {
        ctl->flag = FLAG_BREAK;
        ctl->conv_iter = ctl->iter;
        ctl->alpha = 0.0;
        return;
    }
    ctl->alpha = ctl->rr / PQ;
}

// After the preconditioner solve: (r, z), ||W r||^2, stopping test, beta.
// ctl->iter counts finished iterations; is_first marks the solve of the
// initial residual (no iteration finished yet).
__global__ __launch_bounds__(kRedThreads) void k_pc2_fin_b(const double *partials, int nblk,
                                                           Ctl *ctl, int is_first) {
    if (ctl->flag != FLAG_RUN) return;
    __shared__ double sh[kRedThreads * 2];
    double v0 = 0.0, v1 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kRedThreads) {
        v0 += partials[(int64_t)b * 2];
        v1 += partials[(int64_t)b * 2 + 1];
    }
    sh[threadIdx.x * 2] = v0;
    sh[threadIdx.x * 2 + 1] = v1;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[threadIdx.x * 2] += sh[(threadIdx.x + s) * 2];
            sh[threadIdx.x * 2 + 1] += sh[(threadIdx.x + s) * 2 + 1];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double RZ = sh[0], RW = sh[1];
    const int k = is_first ? ctl->iter : ctl->iter + 1;
    ctl->iter = k;
    ctl->rw = RW;
    if (RW <= ctl->tol2 || RW == 0.0) {
        ctl->flag = FLAG_CONV;
        ctl->conv_iter = k;
        return;
    }
    if (k >= ctl->max_iter) {
        ctl->flag = FLAG_MAXIT;
        ctl->conv_iter = k;
        return;
    }
    if (!(RZ > 0.0) || !isfinite(RZ)) {
        ctl->flag = FLAG_BREAK;
        ctl->conv_iter = k;
        return;
    }
    ctl->beta = is_first ? 0.0 : RZ / ctl->rr;
    ctl->rr = RZ;
}

}  // namespace mas
