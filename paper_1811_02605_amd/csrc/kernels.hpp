// Device kernels of the implicit viscous solver (gfx950, wave64).
//
// Storage of the operator (built once per nu, dt):
//   w[c]      = sqrt(A_cc)                                 (double)
//   cr[c]     = -A(c, c+r)     / (w_c w_{c+r})             (0 on the last r plane)
//   ct[c]     = -A(c, c+theta) / (w_c w_{c+theta})         (0 on the last theta row: pole)
//   cp[c]     = -A(c, c+phi)   / (w_c w_{c+phi})           (periodic in phi)
// i.e. the symmetrically scaled operator  A^ = W^-1 A W^-1  with unit diagonal,
// W = diag(w).  Jacobi-preconditioned CG on A x = b produces, in exact
// arithmetic, the same iterates as plain CG on A^ x^ = b^ with x = W^-1 x^,
// b^ = W^-1 b (split preconditioning with M = diag(A) = W^2), so the solver
// iterates on the scaled system and never stores or reads diag(A)^-1.
//
// One PCG iteration is ONE stencil kernel (k_pcg_iter) plus a one-block
// finalize.  Kernel k, for every cell, forms
//     r_k = r_{k-1} - alpha_{k-1} q_{k-1}
//     x_k = x_{k-1} + alpha_{k-1} p_{k-1}
//     p_k = r_k + beta_k p_{k-1}
//     q_k = A^ p_k
// and block partials of (p_k,q_k), (r_k,q_k), (q_k,q_k), (r_k,r_k) and, on
// check iterations, ||W r_k||^2 = ||b - A x_k||^2.  The finalize sets
//     alpha_k = (r_k,r_k)/(p_k,q_k)
//     (r_{k+1},r_{k+1}) = (r_k,r_k) - 2 alpha_k (r_k,q_k) + alpha_k^2 (q_k,q_k)
//     beta_{k+1} = (r_{k+1},r_{k+1}) / (r_k,r_k)
// so the next kernel can build p_{k+1} without another global reduction.
// (r_k,r_k) itself is always the freshly summed value; only one step of
// the expansion is ever used.  q_k at a cell needs p_k at its six
// neighbours; p_k at the in-plane neighbours is recomputed from
// (r, q, p)_{k-1} (one halo row/column around the tile, served from L2),
// the r-neighbours come from marching along r with a register queue.  r, p, q
// are double-buffered between iterations (neighbouring tiles still read the
// old values), x is updated in place (it has no halo).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mas {

constexpr int kWave = 64;
constexpr int kNV = 5;        // partial sums per block of the iteration kernel
constexpr int kRedThreads = 256;

// Device control block of one PCG run (lives in the workspace).
struct Ctl {
    double alpha;      // alpha_{k-1}, applied by the next iteration kernel (0: skip)
    double beta;       // beta_k,      applied by the next iteration kernel (0: p = r)
    double rr;         // (r_k, r_k) of the last finished iteration (scaled variables)
    double rw;         // last checked ||W r||^2 (= ||b - A x||^2)
    double tol2;       // threshold on the checked quantity
    double rr_next;    // (r_{k+1}, r_{k+1}) predicted by the recurrence at the last finalize
    double pq, rq, qq; // last sums (diagnostics)
    double sums[8];    // results of k_reduce
    double wratio;     // ||W r||^2 / (r,r) at the last check (predicts ||W r||^2 from (r,r))
    double alpha_prev; // the alpha the last iteration kernel applied (its x update, when that
                       // kernel left it to the next one or to k_x_catchup)
    int32_t flag;      // 0 running, 1 converged, 2 iteration limit, -2 breakdown
    int32_t iter;      // index of the next iteration kernel
    int32_t max_iter;  // last admissible iteration index
    int32_t mode;      // 0: ||W r||^2 <= tol2 on check iterations; 1: (r,r) <= tol2 every iteration
    int32_t conv_iter; // iteration index at which flag was set
    int32_t check;     // mode 0: the next iteration kernel forms ||W r||^2
    int32_t check_every;  // mode 0: a check at least every check_every iterations
    int32_t pad;
};

enum { FLAG_RUN = 0, FLAG_CONV = 1, FLAG_MAXIT = 2, FLAG_BREAK = -2 };

struct Dims {
    int nr, nt, np;
    int64_t plane;  // nt*np
    int64_t n;      // nr*nt*np
};

// 1-D geometric factors (double, device).  With r_f the radial faces, r_i the
// cell centres (face midpoints), t_f / t_j the same in theta and dphi = 2 pi/np:
//   vr[i]  = (r_{i+1}^3 - r_i^3)/3
//   vt[j]  = (cos t_j - cos t_{j+1}) dphi            V_c = vr[i] vt[j]
//   gr[i]  = r_{f,i+1}^2 / (r_{i+1} - r_i)           +r face: G = gr[i] vt[j]  (i < nr-1)
//   gq[i]  = (r_{f,i+1}^2 - r_{f,i}^2) / (2 r_i)
//   gtt[j] = sin(t_{f,j+1}) dphi / (t_{j+1} - t_j)   +theta face: G = gq[i] gtt[j] (0 at the pole)
//   gpt[j] = (t_{f,j+1} - t_{f,j}) / (sin(t_j) dphi) +phi face:   G = gq[i] gpt[j]
//   gw_in  = r_{f,0}^2/(r_0 - r_{f,0}),  gw_out = r_{f,nr}^2/(r_{f,nr} - r_{nr-1})
//            (Dirichlet walls, times vt[j]; 0 for a Neumann wall)
struct Geo {
    const double *vr, *vt, *gr, *gq, *gtt, *gpt;
    double gw_in, gw_out;
    double dt;
    int np_one;  // 1 if np == 1 (the phi face joins a cell to itself: no coupling)
};

// Element i of a table that stays unchanged while kernels run (the geometric
// factors, written before the first launch).  Read through the constant
// address space, a load at an index that is the same for the whole wave (a
// plane's factors) becomes a scalar load: it does not count against the
// vector-memory counter, so using it does not wait for the vector loads a
// marching kernel keeps in flight.  The compiler also need not prove that no
// store of the kernel writes the table.
template <typename T>
__device__ inline T ld_table(const T *p, int64_t i) {
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum NV values over the block in a fixed order; thread 0 writes them to out.
template <int NV>
__device__ inline void block_sum_store(double (&v)[NV], double *out, double *lds) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int nw = (blockDim.x * blockDim.y) / kWave;
#pragma unroll
    for (int t = 0; t < NV; ++t) v[t] = wave_sum(v[t]);
    if (lane == 0) {
#pragma unroll
        for (int t = 0; t < NV; ++t) lds[wv * NV + t] = v[t];
    }
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        for (int t = 0; t < NV; ++t) {
            double s = 0.0;
            for (int u = 0; u < nw; ++u) s += lds[u * NV + t];
            out[t] = s;
        }
    }
}

// ---------------------------------------------------------------- CG finalize
// Fixed-order sum of the kNV partials of right-hand side c over nblk blocks
// ([nblk][nrhs][kNV]) by the NT threads of one block: thread t adds blocks
// t, t + NT, ... in order, the waves combine by a butterfly, the wave sums
// are added in wave order (bitwise reproducible).  Every thread gets the
// sums.
template <int NT>
__device__ inline void sum_partials(const double *partials, int nblk, int nrhs, int c,
                                    double (&out)[kNV], double *lds) {
    double v[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += NT) {
#pragma unroll
        for (int t = 0; t < kNV; ++t) v[t] += partials[((int64_t)b * nrhs + c) * kNV + t];
    }
#pragma unroll
    for (int t = 0; t < kNV; ++t) v[t] = wave_sum(v[t]);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int t = 0; t < kNV; ++t) lds[wv * kNV + t] = v[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kNV; ++t) {
        double s = 0.0;
        for (int u = 0; u < NT / kWave; ++u) s += lds[u * kNV + t];
        out[t] = s;
    }
    __syncthreads();
}

// Residual check: a kernel forms ||W r||^2 (reading w) periodically, at the
// last admissible iteration, and at every iteration once the value predicted
// from (r, r) and the ratio ||W r||^2/(r, r) of the last check is within
// this factor of the threshold, so the run stops at the first checked
// iteration below it instead of up to check_every - 1 iterations late.
constexpr double kCheckMargin = 4.0;

// The scalar recurrences and stopping tests after PCG iteration kernel k
// (one thread), from the sums S = [(p,q), (r,q), (q,q), (r,r), ||W r||^2]:
//   alpha_k = (r_k,r_k)/(p_k,q_k)
//   (r_{k+1},r_{k+1}) = (r_k,r_k) - 2 alpha_k (r_k,q_k) + alpha_k^2 (q_k,q_k)
//   beta_{k+1} = (r_{k+1},r_{k+1}) / (r_k,r_k)
__device__ inline void pcg_finalize(Ctl *ctl, const double (&S)[kNV]) {
    const double PQ = S[0], RQ = S[1], QQ = S[2], RR = S[3], RW = S[4];
    const int k = ctl->iter;
    ctl->alpha_prev = ctl->alpha;
    ctl->pq = PQ;
    ctl->rq = RQ;
    ctl->qq = QQ;
    bool conv = false;
    if (ctl->mode == 0) {
        if (ctl->check) {
            ctl->rw = RW;
            conv = RW <= ctl->tol2;
            if (RR > 0.0 && isfinite(RW)) ctl->wratio = RW / RR;
        }
    } else {
        conv = RR <= ctl->tol2;
    }
    ctl->rr = RR;
    // an exactly zero scaled residual is an exact solution (W r = 0 as well)
    if (RR == 0.0) conv = true;
    // alpha_k and the predicted (r_{k+1}, r_{k+1}) are recorded even when
    // stopping: a refinement step that keeps the search direction folds the
    // pending alpha_k p_k into the solution and compares the replaced
    // residual with the prediction
    {
        const double al = (PQ > 0.0 && isfinite(PQ)) ? RR / PQ : 0.0;
        ctl->alpha = al;
        ctl->rr_next = RR - 2.0 * al * RQ + al * al * QQ;
    }
    if (conv) {
        ctl->flag = FLAG_CONV;
        ctl->conv_iter = k;
        return;
    }
    if (k >= ctl->max_iter) {
        ctl->flag = FLAG_MAXIT;
        ctl->conv_iter = k;
        return;
    }
    if (!(PQ > 0.0) || !isfinite(PQ) || !isfinite(RR)) {
        ctl->flag = FLAG_BREAK;
        ctl->conv_iter = k;
        return;
    }
    const double alpha = RR / PQ;
    const double rho1 = RR - 2.0 * alpha * RQ + alpha * alpha * QQ;
    ctl->alpha = alpha;
    ctl->beta = (rho1 > 0.0 && RR > 0.0) ? rho1 / RR : 0.0;
    ctl->iter = k + 1;
    if (ctl->mode == 0) {
        const int kn = k + 1;
        ctl->check = (kn % ctl->check_every) == 0 || kn >= ctl->max_iter ||
                     ctl->wratio * rho1 <= kCheckMargin * ctl->tol2;
    }
}

// ---------------------------------------------------------------- iteration kernel
// Right-hand sides one iteration kernel can carry (they share the operator).
constexpr int kMaxRhs = 4;

template <typename T>
struct IterArgs {
    // per right-hand side
    const T *r_in[kMaxRhs], *p_in[kMaxRhs], *q_in[kMaxRhs];
    T *r_out[kMaxRhs], *p_out[kMaxRhs], *q_out[kMaxRhs];
    T *x[kMaxRhs];
    // 1: this launch brings x up to date over two iterations, the previous
    // launch's update (alpha_prev times the p that launch read, still in
    // p_out) and its own; 0: x is not touched (see k_pcg_iter)
    int xstep;
    // Segment-edge records [r, p, cp, q] (see k_pcg_iter): written by every
    // iteration kernel into halo_out, read from halo_in by the next one.
    T *halo_out[kMaxRhs];
    const T *halo_in[kMaxRhs];
    int records;  // 1: the record buffers exist
    // shared
    const T *cr, *ct, *cp;
    const double *w;
    double *partials;  // [nblk][NR][kNV]
    const Ctl *ctl;    // [NR]
    Dims d;
    int tiles_i, tiles_k, tiles_j, ti;  // r chunks, phi segments, theta tiles; r planes per chunk
    int nblk;
};

// Bijective block -> tile remap: consecutive hardware block ids go round-robin
// to the 8 XCDs; give each XCD a contiguous range of tiles so that theta
// neighbours (tile distance tiles_k) share an L2.
__device__ inline int xcd_remap(int b, int nblk) {
    const int q = nblk >> 3, rem = nblk & 7;
    const int x = b & 7, s = b >> 3;
    return x * q + (x < rem ? x : rem) + s;
}

// Tile coordinates (r chunk it, phi segment kt, theta tile jt) of logical
// block L.  Consecutive L run on one XCD at the same time (xcd_remap), so the
// fastest index decides which neighbour tiles share that XCD's L2 while they
// run: order 0 puts r chunks fastest, 1 theta tiles then r chunks, 2 theta
// tiles then phi segments, 3 phi segments then theta tiles, 4 phi segments
// then r chunks.
template <int ORDER>
__device__ inline void tile_coords(int L, int ti, int tk, int tj, int &it, int &kt, int &jt) {
    if constexpr (ORDER == 3) {
        kt = L % tk;
        jt = (L / tk) % tj;
        it = L / (tk * tj);
    } else if constexpr (ORDER == 4) {
        kt = L % tk;
        it = (L / tk) % ti;
        jt = L / (tk * ti);
    } else if constexpr (ORDER == 1) {
        jt = L % tj;
        it = (L / tj) % ti;
        kt = L / (tj * ti);
    } else if constexpr (ORDER == 2) {
        jt = L % tj;
        kt = (L / tj) % tk;
        it = L / (tj * tk);
    } else {
        it = L % ti;
        kt = (L / ti) % tk;
        jt = L / (ti * tk);
    }
}

// Vector of V consecutive phi cells (16-byte accesses for V = 16/sizeof(T)).
template <typename T, int V>
struct VecT {
    T v[V];
};

template <typename T, int V>
__device__ inline VecT<T, V> ldv(const T *__restrict__ p, int64_t c) {
    VecT<T, V> r;
    if constexpr (V == 1) {
        r.v[0] = p[c];
    } else {
        typedef T raw_t __attribute__((ext_vector_type(V)));
        const raw_t t = *reinterpret_cast<const raw_t *>(p + c);
#pragma unroll
        for (int e = 0; e < V; ++e) r.v[e] = t[e];
    }
    return r;
}

// Non-temporal variants for data used once per iteration (streamed).
template <typename T, int V>
__device__ inline VecT<T, V> ldv_nt(const T *__restrict__ p, int64_t c) {
    VecT<T, V> r;
    if constexpr (V == 1) {
        r.v[0] = __builtin_nontemporal_load(p + c);
    } else {
        typedef T raw_t __attribute__((ext_vector_type(V)));
        const raw_t t = __builtin_nontemporal_load(reinterpret_cast<const raw_t *>(p + c));
#pragma unroll
        for (int e = 0; e < V; ++e) r.v[e] = t[e];
    }
    return r;
}

template <typename T, int V>
__device__ inline void stv_nt(T *__restrict__ p, int64_t c, const VecT<T, V> &x) {
    if constexpr (V == 1) {
        __builtin_nontemporal_store(x.v[0], p + c);
    } else {
        typedef T raw_t __attribute__((ext_vector_type(V)));
        raw_t t;
#pragma unroll
        for (int e = 0; e < V; ++e) t[e] = x.v[e];
        __builtin_nontemporal_store(t, reinterpret_cast<raw_t *>(p + c));
    }
}

// Buffer-resource access (range-checked by the hardware): an offset at or
// beyond the resource size reads zeros and drops stores without touching
// memory, which gives masked accesses with no branch.  Offsets are bytes,
// 32-bit: a marching block's resources start at the first r plane it
// touches (PlaneWin), and the host keeps every block's planes below 2^31
// bytes per array, so the grid itself may be any size.
constexpr uint32_t kOOB = 0x80000000u;
constexpr int kAuxNT = 2;  // non-temporal hint in the aux field (gfx94x/gfx950)

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// The r planes lo .. hi-1 (clamped to the grid) of a cell array, as seen by
// one block: offsets are ((m - lo) plane + cell-in-plane) elements.
struct PlaneWin {
    int lo, planes;
    int64_t first;   // first cell of plane lo
    uint32_t cells;  // cells of the window
};

__device__ inline PlaneWin plane_win(const Dims &d, int lo, int hi) {
    lo = max(lo, 0);
    hi = min(hi, d.nr);
    PlaneWin w;
    w.lo = lo;
    w.planes = max(hi - lo, 0);
    w.first = (int64_t)lo * d.plane;
    w.cells = (uint32_t)((int64_t)w.planes * d.plane);
    return w;
}

// Resource over the window of cell array p (null or !on: zero length).
template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t win_rsrc(const T *p, const PlaneWin &w, bool on = true) {
    return (p && on) ? make_rsrc(p + w.first, w.cells * (uint32_t)sizeof(T)) : make_rsrc(p, 0u);
}

// The same planes of an array of per_plane elements per r plane.
template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t win_rsrc(const T *p, const PlaneWin &w, int64_t per_plane,
                                                  bool on) {
    return (p && on) ? make_rsrc(p + (int64_t)w.lo * per_plane,
                                 (uint32_t)((int64_t)w.planes * per_plane * (int64_t)sizeof(T)))
                     : make_rsrc(p, 0u);
}

template <typename T, int V, int AUX = 0>
__device__ inline VecT<T, V> bld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    constexpr int B = (int)sizeof(T) * V;
    static_assert(B == 4 || B == 8 || B == 16 || B == 32, "buffer access size");
    VecT<T, V> out;
    if constexpr (B == 32) {
        const auto t0 = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
        const auto t1 = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, AUX);
        __builtin_memcpy(&out, &t0, 16);
        __builtin_memcpy(reinterpret_cast<char *>(&out) + 16, &t1, 16);
    } else if constexpr (B == 16) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
        __builtin_memcpy(&out, &t, 16);
    } else if constexpr (B == 8) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
        __builtin_memcpy(&out, &t, 8);
    } else {
        const auto t = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX);
        __builtin_memcpy(&out, &t, 4);
    }
    return out;
}

template <typename T, int V, int AUX = 0>
__device__ inline void bst(__amdgpu_buffer_rsrc_t r, uint32_t off, const VecT<T, V> &x) {
    constexpr int B = (int)sizeof(T) * V;
    static_assert(B == 4 || B == 8 || B == 16 || B == 32, "buffer access size");
    if constexpr (B == 32) {
        typedef int i4 __attribute__((ext_vector_type(4)));
        i4 t0, t1;
        __builtin_memcpy(&t0, &x, 16);
        __builtin_memcpy(&t1, reinterpret_cast<const char *>(&x) + 16, 16);
        __builtin_amdgcn_raw_buffer_store_b128(t0, r, off, 0, AUX);
        __builtin_amdgcn_raw_buffer_store_b128(t1, r, off + 16u, 0, AUX);
    } else if constexpr (B == 16) {
        typedef int i4 __attribute__((ext_vector_type(4)));
        i4 t;
        __builtin_memcpy(&t, &x, 16);
        __builtin_amdgcn_raw_buffer_store_b128(t, r, off, 0, AUX);
    } else if constexpr (B == 8) {
        typedef int i2 __attribute__((ext_vector_type(2)));
        i2 t;
        __builtin_memcpy(&t, &x, 8);
        __builtin_amdgcn_raw_buffer_store_b64(t, r, off, 0, AUX);
    } else {
        int t;
        __builtin_memcpy(&t, &x, 4);
        __builtin_amdgcn_raw_buffer_store_b32(t, r, off, 0, AUX);
    }
}

#ifndef MAS_ITER_ORDER
#define MAS_ITER_ORDER 3
#endif
// Block barrier after every plane step for kernels carrying at least this
// many right-hand sides (keeps the block's waves on one plane, so the rows
// they load for each other are requested together).  Measured at one fixed
// placement on the 256 x 320 x 640 grid: three right-hand sides 2438 -> 2401
// us, one right-hand side 948 -> 954 us (so not used there).
#ifndef MAS_ITER_SYNC_MIN_NR
#define MAS_ITER_SYNC_MIN_NR 2
#endif
#ifndef MAS_ITER_NT
#define MAS_ITER_NT 1
#endif
#ifndef MAS_ITER_DEFER
#define MAS_ITER_DEFER 1
#endif
#ifndef MAS_ITER_DEFER_MAX_NR
#define MAS_ITER_DEFER_MAX_NR 1
#endif
#if MAS_ITER_NT
#define MAS_LDS_ ldv_nt
#define MAS_STS_ stv_nt
#else
#define MAS_LDS_ ldv
#define MAS_STS_ stv
#endif

template <typename T, int V>
__device__ inline void stv(T *__restrict__ p, int64_t c, const VecT<T, V> &x) {
    if constexpr (V == 1) {
        p[c] = x.v[0];
    } else {
        typedef T raw_t __attribute__((ext_vector_type(V)));
        raw_t t;
#pragma unroll
        for (int e = 0; e < V; ++e) t[e] = x.v[e];
        *reinterpret_cast<raw_t *>(p + c) = t;
    }
}

__device__ inline double shfl_up1(double v) { return __shfl_up(v, 1, kWave); }
__device__ inline float shfl_up1(float v) { return __shfl_up(v, 1, kWave); }
__device__ inline double shfl_dn1(double v) { return __shfl_down(v, 1, kWave); }
__device__ inline float shfl_dn1(float v) { return __shfl_down(v, 1, kWave); }
__device__ inline double shfl_lane(double v, int src) { return __shfl(v, src, kWave); }
__device__ inline float shfl_lane(float v, int src) { return __shfl(v, src, kWave); }

// Cross-lane moves that stay in the vector ALU (no LDS crossbar, no lgkm
// wait), gfx950:
//   other_half: the value of lane (l + 32) mod 64 (v_permlane32_swap; its
//     first result gives lanes 32-63 the lower half's values, its second
//     gives lanes 0-31 the upper half's);
//   lane_prev / lane_next: the value of lane l-1 / l+1 (DPP wave_shr:1 /
//     wave_shl:1); lane 0 / lane 63 get 0 and their callers never use it.
__device__ inline uint32_t other_half_u32(uint32_t v) {
    const auto pr = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? pr[0] : pr[1];
}
__device__ inline uint32_t lane_prev_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ inline uint32_t lane_next_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}
template <uint32_t (*F)(uint32_t)>
__device__ inline double lanes64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = F((uint32_t)b), hi = F((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}
template <uint32_t (*F)(uint32_t)>
__device__ inline float lanes32(float v) {
    return __builtin_bit_cast(float, F(__builtin_bit_cast(uint32_t, v)));
}
__device__ inline double other_half(double v) { return lanes64<other_half_u32>(v); }
__device__ inline float other_half(float v) { return lanes32<other_half_u32>(v); }
__device__ inline double lane_prev(double v) { return lanes64<lane_prev_u32>(v); }
__device__ inline float lane_prev(float v) { return lanes32<lane_prev_u32>(v); }
__device__ inline double lane_next(double v) { return lanes64<lane_next_u32>(v); }
__device__ inline float lane_next(float v) { return lanes32<lane_next_u32>(v); }

// The scalars one iteration launch applies, per right-hand side.
template <typename T, int NR>
struct IterScalars {
    bool run[NR];               // the right-hand side's run goes on
    T alpha[NR], beta[NR], alpha2[NR];  // alpha, beta and alpha_prev of its control block
    bool check;                 // some running right-hand side forms ||W r||^2
};

template <typename T, int NR>
__device__ inline bool iter_scalars(const Ctl *ctl_all, IterScalars<T, NR> &sc) {
    bool any = false;
    sc.check = false;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        const Ctl *ctl = ctl_all + c;
        sc.run[c] = ctl->flag == FLAG_RUN;
        any = any || sc.run[c];
        // ||W r||^2 is formed when any running right-hand side asks for it
        sc.check = sc.check || (sc.run[c] && ctl->check);
        sc.alpha[c] = (T)ctl->alpha;
        sc.alpha2[c] = (T)ctl->alpha_prev;
        sc.beta[c] = (T)ctl->beta;
    }
    return any;
}

// Each wave owns RPW consecutive theta rows, 64/RPW lanes per row, each lane
// V consecutive phi cells (a segment of SEG = (64/RPW) V cells per row), and
// marches through the r planes of its chunk on its own.
// In-plane neighbours of p_k are recomputed from (r, q, p)_{k-1}:
//   - a theta neighbour inside the wave comes from a cross-lane shuffle of
//     the neighbouring row's p_k; only the wave's first row loads row j-1 and
//     its last row loads row j+1 (served by L1/L2/MALL: they are other
//     waves' own rows);
//   - phi neighbours come from lane shuffles, the two segment-edge cells of
//     every row from two extra lanes' loads.
// Chunks march up (even chunk index) or down (odd), so the halo plane a chunk
// reads is the plane its neighbour chunk reads at the same time.
// Per plane step m, the in-plane part of q_k(m) plus the term of the r
// neighbour already visited is summed into S(m); q_k(m) is completed one
// step later, when p_k of the next plane is known.
// NR right-hand sides share one pass: the couplings (and w) are loaded once
// per cell, each right-hand side keeps its own vectors, scalars and partial
// sums.  A right-hand side whose run has stopped gets zero-length buffer
// resources: its loads return zeros and its stores are dropped, so it moves
// no bytes.
// Segment edges: a phi neighbour outside the segment sits in another tile's
// cache line, and fetching a whole line for one value per row is what costs
// bytes.  So every kernel also writes, per (plane, row, segment), a record
// [r_k, p_k, cp, q_k] for its first cell (side 0) and its last cell (side 1)
// into a small side buffer; with HALO the next kernel takes its neighbours'
// p_k and the coupling across the left edge from those records, which pack
// the edges of a whole row into a few lines.  Without HALO (the first kernel
// of a run, whose input no kernel wrote records for) the edge cells are
// loaded directly.  HALO needs every segment to span at least two lanes.
// x moves in every second launch only (a.xstep): x_{k+1} = (x_{k-1} +
// alpha_{k-1} p_{k-1}) + alpha_k p_k, where p_{k-1} is still in the p_out
// buffer (each cell read by its owner before this launch overwrites it with
// its own p) and alpha_{k-1} is ctl->alpha_prev.  The two fused multiply-adds
// are those two successive launches would do, in the same order, so x is
// bitwise what an update in every launch gives, at 8 instead of 16 bytes of
// x per cell and launch.  A run that stops after a launch without the update
// gets it from k_x_catchup.
// One PCG iteration over this block's tile (the body of k_pcg_iter, also
// run in a loop by k_pcg_persist); writes the block's partial sums.
template <typename T, int NR, int WPB, int RPW, int V, bool HALO>
__device__ __forceinline__ void pcg_iter_body(const IterArgs<T> &a, const IterScalars<T, NR> &sc) {
    static_assert(kWave % RPW == 0, "rows per wave");
    static_assert(NR >= 1 && NR <= kMaxRhs, "right-hand sides");
    constexpr int W = kWave / RPW;  // lanes per row
    constexpr int SEG = W * V;
    using VT = VecT<T, V>;

    bool run[NR];
    T alpha[NR], beta[NR], alpha2[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        run[c] = sc.run[c];
        alpha[c] = sc.alpha[c];
        beta[c] = sc.beta[c];
        alpha2[c] = sc.alpha2[c];
    }
    const bool check = sc.check;

    const int nr = a.d.nr, nt = a.d.nt, np = a.d.np;
    const int64_t plane = a.d.plane;

    const int L = xcd_remap(blockIdx.x, a.nblk);
    int it, kt, jt;
    tile_coords<MAS_ITER_ORDER>(L, a.tiles_i, a.tiles_k, a.tiles_j, it, kt, jt);

    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int rr = lane / W;  // row within the wave
    const int lp = lane % W;  // lane within the row
    const int j = (jt * WPB + wv) * RPW + rr;
    const int k0 = kt * SEG;
    const int nseg = min(SEG, np - k0);  // a multiple of V
    const int nvl = nseg / V;            // lanes per row holding cells
    const bool rowok = j < nt;
    const bool act = rowok && lp < nvl;
    const int i0 = it * a.ti;
    const int i1 = min(i0 + a.ti, nr);
    const bool up = (it & 1) == 0;
    // the planes this block touches, i0 - 1 .. i1
    const PlaneWin win = plane_win(a.d, i0 - 1, i1 + 1);

    // phi neighbours of the segment (periodic): the cell left of k0 and the
    // cell right of the segment end
    const int64_t colL = (int64_t)j * np + ((k0 == 0) ? np - 1 : k0 - 1);
    const int64_t colR = (int64_t)j * np + ((k0 + nseg == np) ? 0 : k0 + nseg);
    // In a short segment the first lane past its end stands in for the cell
    // right of it: it loads that cell's r, q, p as if they were its own, and
    // the last active lane receives p_k there through the phi shuffle.  In a
    // full segment the row's last lane loads that cell in the same
    // instruction as lane 0 loads the cell left of the segment.
    const bool pseudoR = !HALO && rowok && nvl < W && lp == nvl;
    const bool eL = rowok && lp == 0;
    const bool eR = rowok && nvl == W && lp == W - 1;
    // edge records: lane 0 owns side 0, lane nvl-1 side 1 (distinct with HALO)
    const int tk = a.tiles_k;
    const int ktL = (kt == 0) ? tk - 1 : kt - 1, ktR = (kt == tk - 1) ? 0 : kt + 1;
    const bool wside0 = act && lp == 0, wside1 = act && lp == nvl - 1 && nvl > 1;
    const bool wrec = wside0 || wside1;
    auto rec_off = [&](int mm, int kk, int side) -> uint32_t {
        return (uint32_t)(((((int64_t)(mm - win.lo) * nt + j) * tk + kk) * 2 + side) * 4 * (int64_t)sizeof(T));
    };

    // own cells; inactive lanes read nothing (out-of-range offsets)
    const int64_t col = act ? (int64_t)j * np + k0 + lp * V : (pseudoR ? colR : 0);
    const bool hasU = act && j > 0, hasD = act && j < nt - 1;
    // rows j-1 / j+1 are loaded only by the wave's first / last row
    const bool ldU = hasU && rr == 0, ldD = hasD && rr == RPW - 1;
    const int64_t colU = ldU ? col - np : 0;
    const int64_t colD = ldD ? col + np : 0;
    const int srcU = (rr > 0) ? lane - W : lane;
    const int srcD = (rr < RPW - 1) ? lane + W : lane;

    double acc[NR * kNV];
#pragma unroll
    for (int t = 0; t < NR * kNV; ++t) acc[t] = 0.0;
    VT pn1[NR], rn1[NR], S1[NR], cr1{};
#pragma unroll
    for (int c = 0; c < NR; ++c) pn1[c] = rn1[c] = S1[c] = VT{};
    int64_t base1 = 0;
    // results of the previous step, stored only after this step's loads are
    // issued: the in-order vector-memory counter then never makes a load
    // wait for a store to complete (costs 4 V registers per right-hand side)
    constexpr bool kDefer = MAS_ITER_DEFER && NR <= MAS_ITER_DEFER_MAX_NR;
    VT st_r[NR], st_p[NR], st_x[NR], st_q[NR];
    VecT<T, 4> st_h[NR];  // edge record [r, p, cp, q] of the previous plane
    bool st_own = false, st_q_do = false;
    uint32_t st_off = kOOB, st_qoff = kOOB, st_hoff = kOOB;
    T cpw1 = T(0);  // the recording lane's coupling at the previous plane
    int m1 = 0;     // the previous plane

    // Every access goes through a range-checked buffer resource; a lane that
    // does not need an access uses an out-of-range offset (zeros in, stores
    // dropped), so the loop body has no branch around a memory access, the
    // compiler counts outstanding accesses exactly and no load waits for a
    // store to complete.
    constexpr int AN = MAS_ITER_NT ? kAuxNT : 0;
    __amdgpu_buffer_rsrc_t Rr[NR], Rq[NR], Rp[NR], Rx[NR], Rro[NR], Rpo[NR], Rqo[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        // q_in, x and r_out may be null: the kernel then only forms the
        // direction p = r + beta p and q = A^ p (q reads as zero, so r and x
        // are left as they are and move no bytes)
        Rr[c] = win_rsrc(a.r_in[c], win, run[c]);
        Rq[c] = win_rsrc(a.q_in[c], win, run[c]);
        Rp[c] = win_rsrc(a.p_in[c], win, run[c]);
        Rx[c] = win_rsrc(a.x[c], win, run[c] && a.xstep);
        Rro[c] = win_rsrc(a.r_out[c], win, run[c]);
        Rpo[c] = win_rsrc(a.p_out[c], win, run[c]);
        Rqo[c] = win_rsrc(a.q_out[c], win, run[c]);
    }
    __amdgpu_buffer_rsrc_t Rhi[NR], Rho[NR];
    const int64_t rec_plane = (int64_t)nt * tk * 8;  // record elements per plane
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        Rhi[c] = win_rsrc(a.halo_in[c], win, rec_plane, HALO && run[c] && a.records);
        Rho[c] = win_rsrc(a.halo_out[c], win, rec_plane, run[c] && a.records);
    }
    const auto Rcr = win_rsrc(a.cr, win), Rct = win_rsrc(a.ct, win), Rcp = win_rsrc(a.cp, win),
               Rw = win_rsrc(a.w, win, check);
    constexpr uint32_t ES = sizeof(T);
    const int nsteps = i1 - i0 + 2;
    for (int s = 0; s < nsteps; ++s) {
        const int m = up ? i0 - 1 + s : i1 - s;
        const bool indom = (m >= 0) && (m < nr);
        const bool own = (m >= i0) && (m < i1);
        const int64_t base = (int64_t)(indom ? m - win.lo : 0) * plane;
        const bool vin = indom && (act || pseudoR), vown = own && act;
        const uint32_t oc = vin ? (uint32_t)(base + col) * ES : kOOB;
        const uint32_t oo = vown ? (uint32_t)(base + col) * ES : kOOB;
        const uint32_t ocr = (vin && m < i1) ? oc : kOOB;
        const bool vU = own && ldU, vD = own && ldD, vL = own && eL, vR = own && eR;
        const uint32_t oU = vU ? (uint32_t)(base + colU) * ES : kOOB;
        const uint32_t oD = vD ? (uint32_t)(base + colD) * ES : kOOB;
        const uint32_t oL = (!HALO && vL) ? (uint32_t)(base + colL) * ES : kOOB;
        const uint32_t oLR = HALO ? kOOB : (vL ? oL : (vR ? (uint32_t)(base + colR) * ES : kOOB));
        // records: lane 0 reads side 1 of the left segment, lane nvl-1 side 0
        // of the right segment
        const uint32_t oRec = !HALO ? kOOB
                                    : ((own && wside0) ? rec_off(m, ktL, 1)
                                                       : ((own && act && lp == nvl - 1) ? rec_off(m, ktR, 0) : kOOB));
        // ---- loads of plane m, all issued before any use
        // With RPW >= 2 a lane needs row j-1 (first row of the wave) or row
        // j+1 (last row), never both: one set of edge-row registers (E)
        // serves both; with RPW = 1 the D set holds row j+1.
        constexpr bool kSplitUD = RPW == 1;
        constexpr int ND = kSplitUD ? NR : 1;
        const uint32_t oE = kSplitUD ? oU : (vU ? oU : oD);
        VT r[NR], q[NR], p[NR], x[NR], p2[NR], rE[NR], qE[NR], pE[NR], rD[ND], qD[ND], pD[ND];
        T lr[NR], lq[NR], lp_[NR];
        VecT<T, 4> hrec[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            r[c] = bld<T, V>(Rr[c], oc);
            q[c] = bld<T, V>(Rq[c], oc);
            p[c] = bld<T, V>(Rp[c], oc);
        }
        VT cr = bld<T, V, AN>(Rcr, ocr);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            x[c] = bld<T, V, AN>(Rx[c], oo);
            p2[c] = bld<T, V, AN>(Rpo[c], a.xstep ? oo : kOOB);  // p_{k-1}
        }
        VT ct = bld<T, V>(Rct, oo);
        VT cp = bld<T, V, AN>(Rcp, oo);
        // w only on check iterations (otherwise a zero-length resource: zeros, no bytes)
        const VecT<double, V> w = bld<double, V>(Rw, vown ? (uint32_t)(base + col) * 8u : kOOB);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            rE[c] = bld<T, V>(Rr[c], oE);
            qE[c] = bld<T, V>(Rq[c], oE);
            pE[c] = bld<T, V>(Rp[c], oE);
        }
        const VT ctU = bld<T, V>(Rct, oU);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            if constexpr (kSplitUD) {
                rD[c] = bld<T, V>(Rr[c], oD);
                qD[c] = bld<T, V>(Rq[c], oD);
                pD[c] = bld<T, V>(Rp[c], oD);
            }
            if constexpr (HALO) {
                hrec[c] = bld<T, 4>(Rhi[c], oRec);
                lr[c] = hrec[c].v[0];
                lp_[c] = hrec[c].v[1];
                lq[c] = hrec[c].v[3];
            } else {
                lr[c] = bld<T, 1>(Rr[c], oLR).v[0];
                lq[c] = bld<T, 1>(Rq[c], oLR).v[0];
                lp_[c] = bld<T, 1>(Rp[c], oLR).v[0];
            }
        }
        const T lcp = HALO ? T(0) : bld<T, 1>(Rcp, oL).v[0];
        // ---- stores of the previous step
        if constexpr (kDefer) {
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                bst<T, V, AN>(Rro[c], st_own ? st_off : kOOB, st_r[c]);
                bst<T, V, AN>(Rpo[c], st_own ? st_off : kOOB, st_p[c]);
                bst<T, V, AN>(Rx[c], st_own ? st_off : kOOB, st_x[c]);
                bst<T, V, AN>(Rqo[c], st_q_do ? st_qoff : kOOB, st_q[c]);
                bst<T, 4>(Rho[c], st_hoff, st_h[c]);
            }
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (!(vin && m < i1)) cr.v[e] = T(0);
            if (!vown) {
                ct.v[e] = T(0);
                cp.v[e] = T(0);
            }
        }
        // face between the previous plane and this one
        const VT cf = up ? cr1 : cr;
        const int mp = up ? m - 1 : m + 1;
        const bool qdo = mp >= i0 && mp < i1 && act;
        const uint32_t oq = qdo ? (uint32_t)(base1 + col) * ES : kOOB;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            // ---- r_k, p_k, x_k of plane m
            VT rn, pn, xn;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                rn.v[e] = r[c].v[e] - alpha[c] * q[c].v[e];
                pn.v[e] = rn.v[e] + beta[c] * p[c].v[e];
                const T xm = x[c].v[e] + alpha2[c] * p2[c].v[e];
                xn.v[e] = xm + alpha[c] * p[c].v[e];
                if (!vin) pn.v[e] = T(0);
            }
            // (r_k, r_k) and ||W r_k||^2 over the cells this tile owns
            if (vown) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const double rd = (double)rn.v[e], t = w.v[e] * rd;
                    acc[c * kNV + 3] += rd * rd;
                    acc[c * kNV + 4] += t * t;
                }
            }
            // ---- in-plane part of q_k(m) plus the visited r neighbour
            VT S{};
            if (own) {
                VT pU_, pD_, ctU_;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    // theta neighbours: shuffled from the neighbouring row of
                    // the wave, or formed from the loaded row at its edges
                    T sU, sD, sct;
                    if constexpr (RPW == 2) {
                        sU = sD = other_half(pn.v[e]);
                        sct = other_half(ct.v[e]);
                    } else {
                        sU = shfl_lane(pn.v[e], srcU);
                        sD = shfl_lane(pn.v[e], srcD);
                        sct = shfl_lane(ct.v[e], srcU);
                    }
                    const T lU = (rE[c].v[e] - alpha[c] * qE[c].v[e]) + beta[c] * pE[c].v[e];
                    T lD = lU;
                    if constexpr (kSplitUD)
                        lD = (rD[c].v[e] - alpha[c] * qD[c].v[e]) + beta[c] * pD[c].v[e];
                    pU_.v[e] = !hasU ? T(0) : (rr == 0 ? lU : sU);
                    pD_.v[e] = !hasD ? T(0) : (rr == RPW - 1 ? lD : sD);
                    ctU_.v[e] = !hasU ? T(0) : (rr == 0 ? ctU.v[e] : sct);
                }
                // p_k at the loaded edge cell (left for lane 0, right for
                // the last lane of a full segment)
                const T e_edge = (lr[c] - alpha[c] * lq[c]) + beta[c] * lp_[c];
                T left0 = lane_prev(pn.v[V - 1]);
                T right0 = lane_next(pn.v[0]);
                T cpl0 = lane_prev(cp.v[V - 1]);
                if (lp == 0) {
                    left0 = vL ? e_edge : T(0);
                    cpl0 = vL ? (HALO ? hrec[c].v[2] : lcp) : T(0);
                }
                if constexpr (HALO) {
                    if (lp == nvl - 1) right0 = e_edge;
                } else {
                    if (eR) right0 = vR ? e_edge : T(0);
                }
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const T left = (e > 0) ? pn.v[e - 1] : left0;
                    const T right = (e < V - 1) ? pn.v[e + 1] : right0;
                    const T cpl = (e > 0) ? cp.v[e - 1] : cpl0;
                    S.v[e] = ct.v[e] * pD_.v[e] + ctU_.v[e] * pU_.v[e] + cp.v[e] * right +
                             cpl * left + cf.v[e] * pn1[c].v[e];
                }
            }
            // ---- complete q_k of the previous plane
            VT qv;
#pragma unroll
            for (int e = 0; e < V; ++e) qv.v[e] = pn1[c].v[e] - (S1[c].v[e] + cf.v[e] * pn.v[e]);
            if (qdo) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const double pd = (double)pn1[c].v[e], qd = (double)qv.v[e],
                                 rd = (double)rn1[c].v[e];
                    acc[c * kNV + 0] += pd * qd;
                    acc[c * kNV + 1] += rd * qd;
                    acc[c * kNV + 2] += qd * qd;
                }
            }
            // ---- edge record of the previous plane, complete now that q is
            VecT<T, 4> hr;
            hr.v[0] = (lp == 0) ? rn1[c].v[0] : rn1[c].v[V - 1];
            hr.v[1] = (lp == 0) ? pn1[c].v[0] : pn1[c].v[V - 1];
            hr.v[2] = cpw1;
            hr.v[3] = (lp == 0) ? qv.v[0] : qv.v[V - 1];
            // ---- stores
            if constexpr (kDefer) {
                st_r[c] = rn;
                st_p[c] = pn;
                st_x[c] = xn;
                st_q[c] = qv;
                st_h[c] = hr;
            } else {
                bst<T, V, AN>(Rro[c], oo, rn);
                bst<T, V, AN>(Rpo[c], oo, pn);
                bst<T, V, AN>(Rx[c], oo, xn);
                bst<T, V, AN>(Rqo[c], oq, qv);
                bst<T, 4>(Rho[c], (qdo && wrec) ? rec_off(m1, kt, wside0 ? 0 : 1) : kOOB, hr);
            }
            pn1[c] = pn;
            rn1[c] = rn;
            S1[c] = S;
        }
        st_own = vown;
        st_off = oo;
        st_q_do = qdo;
        st_qoff = oq;
        st_hoff = (qdo && wrec) ? rec_off(m1, kt, wside0 ? 0 : 1) : kOOB;
        // the recording lane's coupling of this plane (side 1 needs it)
        cpw1 = (lp == 0) ? cp.v[0] : cp.v[V - 1];
        m1 = m;
        if constexpr (NR >= MAS_ITER_SYNC_MIN_NR) __syncthreads();
        cr1 = cr;
        base1 = base;
    }
    if constexpr (kDefer) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            bst<T, V, AN>(Rro[c], st_own ? st_off : kOOB, st_r[c]);
            bst<T, V, AN>(Rpo[c], st_own ? st_off : kOOB, st_p[c]);
            bst<T, V, AN>(Rx[c], st_own ? st_off : kOOB, st_x[c]);
            bst<T, V, AN>(Rqo[c], st_q_do ? st_qoff : kOOB, st_q[c]);
            bst<T, 4>(Rho[c], st_hoff, st_h[c]);
        }
    }
    __shared__ double sRed[WPB * NR * kNV];
    block_sum_store<NR * kNV>(acc, a.partials + (int64_t)L * NR * kNV, sRed);
}

template <typename T, int NR, int WPB, int RPW, int V, bool HALO>
__global__ __launch_bounds__(kWave *WPB)
#if MAS_ITER_WPE > 0
__attribute__((amdgpu_waves_per_eu(MAS_ITER_WPE, 8)))
#endif
void k_pcg_iter(IterArgs<T> a) {
    IterScalars<T, NR> sc;
    if (!iter_scalars<T, NR>(a.ctl, sc)) return;
    pcg_iter_body<T, NR, WPB, RPW, V, HALO>(a, sc);
}

// One block: the finalize of right-hand side blockIdx.x after an iteration
// kernel (partials [nblk][gridDim.x][kNV]).  A launch of its own: folding it
// into the iteration kernel (the last block to finish sums the partials
// after an agent-scope fence) made that kernel 17% slower on the 52.4M-cell
// grid, the fence writing back the XCD's L2, and gained nothing on small
// grids.
__global__ __launch_bounds__(kRedThreads) void k_finalize(const double *partials, int nblk,
                                                         Ctl *ctl_all) {
    const int c = blockIdx.x, nrhs = gridDim.x;
    Ctl *ctl = ctl_all + c;
    if (ctl->flag != FLAG_RUN) return;
    __shared__ double lds[(kRedThreads / kWave) * kNV];
    double S[kNV];
    sum_partials<kRedThreads>(partials, nblk, nrhs, c, S, lds);
    if (threadIdx.x == 0) pcg_finalize(ctl, S);
}

// ---------------------------------------------------------------- persistent PCG run
// A whole PCG run of NR right-hand sides in one cooperative launch, for
// grids small enough that every block of the iteration kernel is resident
// at once (such a grid spends an iteration on launches and latency, not on
// bandwidth).  Each pass of the loop is one iteration (pcg_iter_body, edge
// cells loaded directly), then a grid barrier, then every block sums the
// partial sums itself, in k_finalize's fixed order, and applies
// pcg_finalize to its own copies of the control blocks (block 0 also writes
// them back): every block takes the same decisions, and the results equal
// those of k_pcg_iter and k_finalize launched per iteration, bit for bit.
// The loop ends when no right-hand side runs any more.  The
// vectors, partial sums and records are double-buffered by parity as
// there, and a block starts iteration k + 1 only after every block has
// finished iteration k, so no block overwrites what another still reads.
struct PersistSync {
    uint32_t bar;  // barrier arrivals, zero at launch
    int32_t err;   // 1: a block gave up waiting at a barrier
};

template <typename T, int NR>
struct PersistArgs {
    IterArgs<T> it;                   // shared fields; buffers and partials set per iteration
    T *r[NR][2], *p[NR][2], *q[NR][2];  // by parity: iteration k reads index k & 1
    double *partials[2];              // by parity, [nblk][NR][kNV] each
    Ctl *ctl;                         // [NR] (k_ctl_init has set them)
    PersistSync *sync;
    int iter0;                        // the run's first iteration index
    int keep_p[NR];                   // the first iteration continues the direction in p[c][iter0 & 1]
    uint64_t wait_ticks;              // longest wait at one barrier, in wall-clock ticks
};

// Grid barrier for co-resident blocks: the block's writes are released at
// agent scope by the arrival, the wait ends once every block of this
// generation has arrived, and an agent-scope acquire makes their writes
// visible.  Returns false, with nothing acquired, if the wait exceeds
// wait_ticks of the wall clock (a block that was never resident would
// otherwise leave the others waiting for good).
__device__ inline bool grid_barrier(PersistSync *sync, uint32_t target, uint64_t wait_ticks) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&sync->bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        int good = 1;
        while (__hip_atomic_load(&sync->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (wall_clock64() - t0 > wait_ticks) {
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

template <typename T, int NR, int WPB, int RPW, int V>
__global__ __launch_bounds__(kWave *WPB) void k_pcg_persist(PersistArgs<T, NR> a) {
    static_assert(kWave * WPB == kRedThreads, "one block sums the partials");
    __shared__ Ctl lc[NR];  // this block's copies of the control blocks
    __shared__ double lds[(kRedThreads / kWave) * kNV];
    if (threadIdx.x < NR) lc[threadIdx.x] = a.ctl[threadIdx.x];
    __syncthreads();
    IterArgs<T> it = a.it;
    for (int k = a.iter0;; ++k) {
        const int cur = k & 1, nxt = cur ^ 1;
        const int s = k - a.iter0;
        IterScalars<T, NR> sc;
        sc.check = false;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            // the first iteration has alpha = 0 (and beta = 0 unless the
            // direction is kept): q (and p) point at r, as in the launched form
            it.r_in[c] = a.r[c][cur];
            it.p_in[c] = (s == 0 && !a.keep_p[c]) ? a.r[c][cur] : a.p[c][cur];
            it.q_in[c] = (s == 0) ? a.r[c][cur] : a.q[c][cur];
            it.r_out[c] = a.r[c][nxt];
            it.p_out[c] = a.p[c][nxt];
            it.q_out[c] = a.q[c][nxt];
            sc.run[c] = lc[c].flag == FLAG_RUN;
            sc.alpha[c] = (T)lc[c].alpha;
            sc.beta[c] = (T)lc[c].beta;
            sc.alpha2[c] = (T)lc[c].alpha_prev;
            sc.check = sc.check || (sc.run[c] && lc[c].check);
        }
        it.partials = a.partials[cur];
        it.xstep = (s >= 2 && (s & 1) == 0) ? 1 : 0;
        pcg_iter_body<T, NR, WPB, RPW, V, false>(it, sc);
        if (!grid_barrier(a.sync, (uint32_t)(s + 1) * gridDim.x, a.wait_ticks)) {
            if (threadIdx.x == 0) __hip_atomic_store(&a.sync->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        bool any = false;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            if (lc[c].flag != FLAG_RUN) continue;  // uniform: every thread reads the same flag
            double S[kNV];
            sum_partials<kRedThreads>(it.partials, it.nblk, NR, c, S, lds);
            if (threadIdx.x == 0) {
                pcg_finalize(&lc[c], S);
                if (blockIdx.x == 0) a.ctl[c] = lc[c];
            }
            __syncthreads();
            any = any || lc[c].flag == FLAG_RUN;
        }
        if (!any) return;
    }
}

__global__ void k_persist_init(PersistSync *sync) {
    if (threadIdx.x == 0) {
        sync->bar = 0u;
        sync->err = 0;
    }
}

// After a run of iteration kernels: a right-hand side whose last launch did
// not move x (an odd launch of the run: a.xstep = 0) gets that launch's
// update here, x += alpha_prev p with p the direction the launch read, the
// same fused multiply-add.  blockIdx.y is the right-hand side; one that
// needs nothing returns at once.
template <typename T>
struct CatchupArgs {
    T *x[kMaxRhs];
    const T *p[kMaxRhs][2];  // the p buffers: iteration kernel k reads p[k & 1]
    const Ctl *ctl;          // [NR]
    int64_t n;
    int iter0;               // the run's first iteration index
};

template <typename T>
__global__ __launch_bounds__(256) void k_x_catchup(CatchupArgs<T> a) {
    const int c = blockIdx.y;
    const Ctl *ctl = a.ctl + c;
    // the last launch that did work (after it the finalize either stopped
    // the run at conv_iter or advanced iter)
    const int last = (ctl->flag == FLAG_RUN) ? ctl->iter - 1 : ctl->conv_iter;
    const int s = last - a.iter0;
    T *x = a.x[c];
    if (s < 1 || (s & 1) == 0 || !x) return;
    const T al = (T)ctl->alpha_prev;
    const T *p = a.p[c][last & 1];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * 256)
        x[i] = x[i] + al * p[i];
}

// Generic fixed-order sum of [nblk][nv] partials into ctl->sums[0:nv].
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double *partials, int nblk, int nv,
                                                       Ctl *ctl) {
    __shared__ double sh[kRedThreads];
    for (int t = 0; t < nv; ++t) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kRedThreads) v += partials[(int64_t)b * nv + t];
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int s = kRedThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) ctl->sums[t] = sh[0];
        __syncthreads();
    }
}

// Reset the control block for a new PCG run (a kernel, not a memset, so it
// is safe inside captured graphs as well).
// flag0 = FLAG_RUN starts the run; another flag leaves this control block
// (one right-hand side of several) stopped from the start.
// check0: the first iteration kernel of the run forms ||W r||^2 (in mode 0
// its ratio to (r, r) starts the prediction of the check); then every
// check_every-th and those near the threshold (pcg_finalize).
__global__ void k_ctl_init(Ctl *ctl, int mode, int iter0, int max_iter, double tol2,
                           double beta0, int flag0, int check0, int check_every) {
    if (threadIdx.x != 0) return;
    ctl->alpha = 0.0;
    ctl->beta = beta0;
    ctl->rr = 0.0;
    ctl->rw = 0.0;
    ctl->tol2 = tol2;
    ctl->wratio = 0.0;
    ctl->flag = flag0;
    ctl->iter = iter0;
    ctl->max_iter = max_iter;
    ctl->mode = mode;
    ctl->conv_iter = -1;
    ctl->check = check0;
    ctl->check_every = check_every > 0 ? check_every : 1;
}

// ---------------------------------------------------------------- simple stencil tiles
// Block (64, 4): 64 phi cells x 4 theta rows, looping over kSimpleR r planes.
constexpr int kSimpleJ = 4;
constexpr int kSimpleR = 16;
constexpr int kSimpleNV = 3;  // most partial sums a simple-tile kernel writes per block

struct SimpleCell {
    int i, j, k;
    int64_t c;
    bool ok;
};

#define MAS_SIMPLE_LOOP(d, ...)                                                    \
    {                                                                              \
        const int k_ = blockIdx.x * kWave + threadIdx.x;                           \
        const int j_ = blockIdx.y * kSimpleJ + threadIdx.y;                        \
        const int ib_ = blockIdx.z * kSimpleR;                                     \
        const int ie_ = min(ib_ + kSimpleR, (d).nr);                               \
        const bool ok_ = (k_ < (d).np) && (j_ < (d).nt);                           \
        for (int i_ = ib_; i_ < ie_; ++i_) {                                       \
            SimpleCell cell{i_, j_, k_, ((int64_t)i_ * (d).nt + j_) * (d).np + k_, \
                            ok_};                                                  \
            __VA_ARGS__                                                            \
        }                                                                          \
    }

__device__ inline int64_t simple_block_id() {
    return ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

// ---------------------------------------------------------------- operator build
// One pass over nu builds the stored operator: w = sqrt(A_cc), the scaled
// couplings c^ to the +r, +theta, +phi neighbours (and their single-
// precision copies), a copy of nu (the explicit stages form conductances
// from it), the validity of nu and z_max = max_c 2 (A_cc - V_c)/V_c, the
// Gershgorin bound of dt times the spectral radius of V^-1 (A - V), kept as
// the bits of a non-negative double so that an integer maximum finds it.
//   A_cc = V_c + sum_f c_f,  c_f = dt nu_f G_f,  nu_f = (nu_a + nu_b)/2
//   (the cell's own nu on a Dirichlet wall), c^_f = c_f / (w_a w_b).
// c^ needs w at the + neighbours, and w needs nu at every neighbour, so a
// coupling reads nu two cells away.  Each block owns a tile of kBuR theta
// rows x kBuC phi cells and marches up its r chunk with a ring of three
// planes of nu in LDS (the tile plus one row and one column on each side,
// and a second row and column on the + sides), forms w one plane ahead on
// the tile grown by one row and one column (the + neighbours' w), and then
// the couplings of the plane behind: every value of nu is fetched from
// memory once per block and every output is written once.  The next plane
// of nu is loaded into registers while the current plane is computed.
constexpr int kBuR = 16;                     // theta rows per tile
constexpr int kBuC = 64;                     // phi cells per tile (one per lane)
constexpr int kBuWaves = 4;                  // each wave owns rows wv, wv + 4, ...
constexpr int kBuThreads = kWave * kBuWaves;
constexpr int kBuPR = kBuR + 3, kBuPC = kBuC + 3;  // nu patch: rows J0-1..J0+R+1, cells k0-1..k0+C+1
constexpr int kBuWR = kBuR + 1, kBuWC = kBuC + 1;  // w patch:  rows J0..J0+R,     cells k0..k0+C
constexpr int kBuLoads = (kBuPR * kBuPC + kBuThreads - 1) / kBuThreads;

struct BuildArgs {
    const double *nu;
    double *w, *cr, *ct, *cp, *nu_copy;
    float *cr32, *ct32, *cp32;  // null unless single-precision copies are kept
    int32_t *bad;
    unsigned long long *zmax_bits;
    Geo geo;
    Dims d;
    int tiles_i, tiles_k, tiles_j, ti, nblk;
};

// Face conductance dt * nu_f * G_f, the single definition used by the build.
__device__ inline double face_c(double dt, double nua, double nub, double g) {
    return dt * (0.5 * (nua + nub)) * g;
}

// Factors of one r plane m and of one theta row j (see struct Geo):
//   P = [vr[m], r- face factor, r+ face factor, gq[m]], where the r- factor
//   is gr[m-1] (or the inner wall's gw_in when m = 0) and the r+ factor
//   gr[m] (gw_out when m = nr - 1);
//   R = [vt[j], gtt[j-1] (0 at the pole), gtt[j] (0 at the pole), gpt[j]].
struct PlaneF {
    double vr, grm, grp, gq;
};
struct RowF {
    double vt, gttm, gttp, gpt;
};

// A_cc at plane m, row j (in the grid), from n(pr, pc, dm) = nu at patch row
// pr, patch column pc, plane m + dm; the cell sits at patch (pr, pc).
// Terms in the order r-, r+, theta-, theta+, phi-, phi+.
template <typename NU>
__device__ inline double build_diag(const Geo &g, const Dims &d, int m, int j, int pr, int pc,
                                    const PlaneF &P, const RowF &R, NU n) {
    const double nc = n(pr, pc, 0);
    double s = P.vr * R.vt;
    if (m > 0) s += face_c(g.dt, nc, n(pr, pc, -1), P.grm * R.vt);
    else s += g.dt * nc * (P.grm * R.vt);
    if (m < d.nr - 1) s += face_c(g.dt, nc, n(pr, pc, 1), P.grp * R.vt);
    else s += g.dt * nc * (P.grp * R.vt);
    if (j > 0) s += face_c(g.dt, nc, n(pr - 1, pc, 0), P.gq * R.gttm);
    if (j < d.nt - 1) s += face_c(g.dt, nc, n(pr + 1, pc, 0), P.gq * R.gttp);
    if (!g.np_one) {
        const double gp = P.gq * R.gpt;
        s += face_c(g.dt, nc, n(pr, pc - 1, 0), gp);
        s += face_c(g.dt, nc, n(pr, pc + 1, 0), gp);
    }
    return s;
}

template <bool F32>
__global__ __launch_bounds__(kBuThreads) void k_build(BuildArgs a) {
    __shared__ double sNu[3][kBuPR][kBuPC];  // nu of planes m, m + 1, m + 2 (ring)
    __shared__ double sIw[kBuWR][kBuWC];     // 1/w of plane m on the grown tile
    __shared__ RowF sR[kBuWR];               // rows J0 .. J0 + R (39.9 KB in all: 4 blocks per CU)
    const Dims d = a.d;
    const Geo &g = a.geo;
    const int nr = d.nr, nt = d.nt, np = d.np;
    const int L = xcd_remap(blockIdx.x, a.nblk);
    int it, kt, jt;
    tile_coords<3>(L, a.tiles_i, a.tiles_k, a.tiles_j, it, kt, jt);
    const int J0 = jt * kBuR, k0 = kt * kBuC;
    const int nseg = min(kBuC, np - k0);
    const int i0 = it * a.ti, i1 = min(i0 + a.ti, nr);
    // nu of planes i0 - 1 .. i1 + 2 is read, planes i0 .. i1 - 1 written
    const PlaneWin win = plane_win(d, i0 - 1, i1 + 3);
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);

    // factors of a plane (uniform: scalar loads, once per plane step) and
    // the table of the tile's rows in LDS (rows outside the grid: zeros,
    // never used)
    auto plane_f = [&](int m) {
        PlaneF P{0.0, 0.0, 0.0, 0.0};
        if (m >= 0 && m < nr) {
            P.vr = g.vr[m];
            P.grm = (m > 0) ? g.gr[m - 1] : g.gw_in;
            P.grp = (m < nr - 1) ? g.gr[m] : g.gw_out;
            P.gq = g.gq[m];
        }
        return P;
    };
    if (tid < kBuWR) {
        const int j = J0 + tid;
        RowF R{0.0, 0.0, 0.0, 0.0};
        if (j < nt) {
            R.vt = g.vt[j];
            R.gttm = (j > 0) ? g.gtt[j - 1] : 0.0;
            R.gttp = g.gtt[j];
            R.gpt = g.gpt[j];
        }
        sR[tid] = R;
    }

    // this thread's elements of the nu patch: offsets inside a plane
    // (-1: outside the grid in theta, read as zero; -2: no element)
    int32_t poff[kBuLoads];
#pragma unroll
    for (int q = 0; q < kBuLoads; ++q) {
        const int e = tid + q * kBuThreads;
        poff[q] = -2;
        if (e < kBuPR * kBuPC) {
            const int pr = e / kBuPC, pc = e % kBuPC;
            const int j = J0 - 1 + pr;
            int k = (k0 - 1 + pc) % np;
            if (k < 0) k += np;
            poff[q] = (j >= 0 && j < nt) ? j * np + k : -1;
        }
    }
    const auto Rnu = win_rsrc(a.nu, win);
    auto load_plane = [&](int m, double (&v)[kBuLoads]) {
#pragma unroll
        for (int q = 0; q < kBuLoads; ++q) {
            const bool ok = m >= 0 && m < nr && poff[q] >= 0;
            v[q] = bld<double, 1>(Rnu, ok ? (uint32_t)(((int64_t)(m - win.lo) * d.plane + poff[q]) * 8) : kOOB).v[0];
        }
    };
    auto store_plane = [&](int m, const double (&v)[kBuLoads]) {
        double *flat = &sNu[((m % 3) + 3) % 3][0][0];
#pragma unroll
        for (int q = 0; q < kBuLoads; ++q)
            if (poff[q] != -2) flat[tid + q * kBuThreads] = v[q];
    };
    auto slot_of = [](int m) { return ((m % 3) + 3) % 3; };

    // A_cc at patch-relative (er, ec) of plane m (the tile grown by one row
    // and one column); own cells also check nu and raise z_max
    int badv = 0;
    double zmax = 0.0;
    auto diag_at = [&](int m, const PlaneF &P, int er, int ec) -> double {
        const int j = J0 + er;
        if (j >= nt) return 1.0;  // outside the grid: never used
        const int s0 = slot_of(m), sm = slot_of(m - 1), sp = slot_of(m + 1);
        auto n = [&](int pr, int pc, int dm) {
            return sNu[dm == 0 ? s0 : (dm < 0 ? sm : sp)][pr][pc];
        };
        const RowF R = sR[er];
        const double s = build_diag(g, d, m, j, er + 1, ec + 1, P, R, n);
        if (er < kBuR && ec < nseg && m >= i0 && m < i1) {
            const double nc = n(er + 1, ec + 1, 0);
            if (!(nc > 0.0) || !isfinite(nc)) badv = 1;
            const double vc = P.vr * R.vt;
            const double z = 2.0 * (s - vc) / vc;
            zmax = (z > zmax) ? z : zmax;  // false for NaN: nu was then flagged bad
        }
        return s;
    };
    constexpr int NQ = kBuR / kBuWaves;
    // w and 1/w of plane m at this thread's cells (rows wv + 4q, column
    // lane) and at its point of the grown border (wave 0: the row below the
    // tile; wave 1: the column right of it)
    double w[NQ], iw[NQ], wn[NQ], iwn[NQ], iwb = 0.0;
    const bool hasb = (wv == 0) || (wv == 1 && lane < kBuWR);
    const int ber = (wv == 0) ? kBuR : lane, bec = (wv == 0) ? lane : kBuC;
    auto w_plane = [&](int m, const PlaneF &P, double (&wo)[NQ], double (&iwo)[NQ]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            wo[q] = sqrt(diag_at(m, P, wv + kBuWaves * q, lane));
            iwo[q] = 1.0 / wo[q];
        }
        if (hasb) iwb = 1.0 / sqrt(diag_at(m, P, ber, bec));
    };
    auto put_iw = [&](const double (&iwo)[NQ]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sIw[wv + kBuWaves * q][lane] = iwo[q];
        if (hasb) sIw[ber][bec] = iwb;
    };

    const auto Rw = win_rsrc(a.w, win), Rcr = win_rsrc(a.cr, win), Rct = win_rsrc(a.ct, win),
               Rcp = win_rsrc(a.cp, win), Rnc = win_rsrc(a.nu_copy, win);
    const auto Rcr32 = win_rsrc(a.cr32, win, F32), Rct32 = win_rsrc(a.ct32, win, F32),
               Rcp32 = win_rsrc(a.cp32, win, F32);

    // prologue: nu of planes i0 - 1, i0, i0 + 1; w of plane i0; nu of i0 + 2
    {
        double v[kBuLoads];
        for (int m = i0 - 1; m <= i0 + 1; ++m) {
            load_plane(m, v);
            store_plane(m, v);
        }
    }
    __syncthreads();
    PlaneF Pm = plane_f(i0);
    w_plane(i0, Pm, w, iw);
    double nxt[kBuLoads];
    load_plane(i0 + 2, nxt);
    __syncthreads();  // plane i0 - 1's slot is reused for plane i0 + 2
    put_iw(iw);
    store_plane(i0 + 2, nxt);
    __syncthreads();

    for (int m = i0; m < i1; ++m) {
        // nu of plane m + 3 in flight while plane m is computed
        load_plane(m + 3, nxt);
        // w of plane m + 1 (kept in registers until the couplings of plane m
        // no longer read 1/w of plane m)
        const PlaneF Pn = plane_f(m + 1);
        w_plane(m + 1, Pn, wn, iwn);
        // couplings of plane m: c^_f = c_f (1/w_c) (1/w_nb)
        const int s0 = slot_of(m), s1 = slot_of(m + 1);
        const PlaneF P = Pm;
        const int c = lane;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int r = wv + kBuWaves * q;
            const int j = J0 + r;
            const bool own = j < nt && c < nseg;
            const RowF R = sR[r];
            const double nc = sNu[s0][r + 1][c + 1];
            double vr = 0.0, vth = 0.0, vp = 0.0;
            if (m < nr - 1) vr = face_c(g.dt, nc, sNu[s1][r + 1][c + 1], P.grp * R.vt) * iw[q] * iwn[q];
            if (j < nt - 1) vth = face_c(g.dt, nc, sNu[s0][r + 2][c + 1], P.gq * R.gttp) * iw[q] * sIw[r + 1][c];
            if (!g.np_one) vp = face_c(g.dt, nc, sNu[s0][r + 1][c + 2], P.gq * R.gpt) * iw[q] * sIw[r][c + 1];
            const uint32_t o = own ? (uint32_t)(((int64_t)(m - win.lo) * d.plane + (int64_t)j * np + k0 + c) * 8) : kOOB;
            bst<double, 1, kAuxNT>(Rw, o, VecT<double, 1>{{w[q]}});
            bst<double, 1, kAuxNT>(Rnc, o, VecT<double, 1>{{nc}});
            bst<double, 1, kAuxNT>(Rcr, o, VecT<double, 1>{{vr}});
            bst<double, 1, kAuxNT>(Rct, o, VecT<double, 1>{{vth}});
            bst<double, 1, kAuxNT>(Rcp, o, VecT<double, 1>{{vp}});
            if constexpr (F32) {
                const uint32_t o4 = own ? o / 2u : kOOB;
                bst<float, 1, kAuxNT>(Rcr32, o4, VecT<float, 1>{{(float)vr}});
                bst<float, 1, kAuxNT>(Rct32, o4, VecT<float, 1>{{(float)vth}});
                bst<float, 1, kAuxNT>(Rcp32, o4, VecT<float, 1>{{(float)vp}});
            }
        }
        __syncthreads();  // every read of plane m's nu slot and of 1/w of plane m is done
        put_iw(iwn);
        store_plane(m + 3, nxt);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            w[q] = wn[q];
            iw[q] = iwn[q];
        }
        Pm = Pn;
        __syncthreads();
    }

    if (badv) atomicOr(a.bad, 1);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(zmax, o, kWave);
        zmax = (t > zmax) ? t : zmax;
    }
    if (lane == 0 && zmax > 0.0)
        atomicMax(a.zmax_bits, (unsigned long long)__double_as_longlong(zmax));
}

// Unscaled entries as the solver uses them: -A(c, nb) = w_c c^ w_nb, A_cc = w_c^2.
__global__ __launch_bounds__(kWave *kSimpleJ) void k_export(const double *w, const double *cr,
                                                            const double *ct, const double *cp,
                                                            Dims d, double *ocr, double *oct,
                                                            double *ocp, double *odiag) {
    MAS_SIMPLE_LOOP(d, {
        if (cell.ok) {
            const int i = cell.i, j = cell.j, k = cell.k;
            const int64_t c = cell.c;
            const double wc = w[c];
            if (ocr) ocr[c] = (i < d.nr - 1) ? wc * cr[c] * w[c + d.plane] : 0.0;
            if (oct) oct[c] = (j < d.nt - 1) ? wc * ct[c] * w[c + d.np] : 0.0;
            if (ocp) ocp[c] = wc * cp[c] * w[c - k + ((k == d.np - 1) ? 0 : k + 1)];
            if (odiag) odiag[c] = wc * wc;
        }
    })
}

// A^ u at one cell (unit diagonal), u read through the functor.
template <typename F>
__device__ inline double scaled_apply(const double *cr, const double *ct, const double *cp, Dims d,
                                      const SimpleCell &cell, F u) {
    const int i = cell.i, j = cell.j, k = cell.k;
    const int64_t c = cell.c;
    double s = 0.0;
    if (i < d.nr - 1) s += cr[c] * u(c + d.plane);
    if (i > 0) s += cr[c - d.plane] * u(c - d.plane);
    if (j < d.nt - 1) s += ct[c] * u(c + d.np);
    if (j > 0) s += ct[c - d.np] * u(c - d.np);
    const int64_t km = c - k + ((k == 0) ? d.np - 1 : k - 1);
    const int64_t kp = c - k + ((k == d.np - 1) ? 0 : k + 1);
    s += cp[c] * u(kp) + cp[km] * u(km);
    return u(c) - s;
}

// y = A x = W A^ W x.
__global__ __launch_bounds__(kWave *kSimpleJ) void k_apply(const double *w, const double *cr,
                                                           const double *ct, const double *cp,
                                                           Dims d, const double *x, double *y) {
    MAS_SIMPLE_LOOP(d, {
        if (cell.ok) {
            const double v = scaled_apply(cr, ct, cp, d, cell,
                                          [&](int64_t c) { return w[c] * x[c]; });
            y[cell.c] = w[cell.c] * v;
        }
    })
}

// r^ = b^ - A^ x^ (double), stored as TOUT; block partials ||W r^||^2 and
// ||r^||^2.  (A^ x^)_c = x^_c - sum_f c^_f x^_nb(f), the terms in the order
// +r, -r, +theta, -theta, then the two phi terms.  Same tiling and march as
// the gradient kernel: x^ of the current and the next plane in LDS with a
// one-cell ring, c^_theta and c^_phi of the current plane in LDS with the
// row above and the cell left of the tile (the couplings of the - faces),
// x^ and c^_r of the plane behind in registers, the next plane's x^ and
// couplings loaded while the current one is computed.
constexpr int kReR = 16, kReC = 64, kReWaves = 4, kReThreads = kWave * kReWaves;
constexpr int kRePR = kReR + 2, kRePC = kReC + 2;  // patch: rows J0-1..J0+R, cells k0-1..k0+C
constexpr int kReLoads = (kRePR * kRePC + kReThreads - 1) / kReThreads;

struct ResArgs {
    const double *bhat, *xhat, *w, *cr, *ct, *cp;
    Dims d;
    double *partials;  // [nblk][2]
    int tiles_i, tiles_k, tiles_j, ti, nblk;
};

template <typename TOUT>
__global__ __launch_bounds__(kReThreads) void k_residual(ResArgs a, TOUT *rout) {
    __shared__ double sX[2][kRePR][kRePC];
    __shared__ double sT[kRePR][kRePC], sP[kRePR][kRePC];  // c^_theta, c^_phi of the plane
    const Dims d = a.d;
    const int nr = d.nr, nt = d.nt, np = d.np;
    const int L = xcd_remap(blockIdx.x, a.nblk);
    int it, kt, jt;
    tile_coords<3>(L, a.tiles_i, a.tiles_k, a.tiles_j, it, kt, jt);
    const int J0 = jt * kReR, k0 = kt * kReC;
    const int nseg = min(kReC, np - k0);
    const int i0 = it * a.ti, i1 = min(i0 + a.ti, nr);
    // planes i0 - 1 .. i1 + 1 are read, planes i0 .. i1 - 1 written
    const PlaneWin win = plane_win(d, i0 - 1, i1 + 2);
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);

    int32_t poff[kReLoads];
#pragma unroll
    for (int q = 0; q < kReLoads; ++q) {
        const int e = tid + q * kReThreads;
        poff[q] = -2;
        if (e < kRePR * kRePC) {
            const int pr = e / kRePC, pc = e % kRePC;
            const int j = J0 - 1 + pr;
            int k = (k0 - 1 + pc) % np;
            if (k < 0) k += np;
            poff[q] = (j >= 0 && j < nt) ? j * np + k : -1;
        }
    }
    const auto RB = win_rsrc(a.bhat, win), RX = win_rsrc(a.xhat, win), RW = win_rsrc(a.w, win),
               RCr = win_rsrc(a.cr, win), RCt = win_rsrc(a.ct, win), RCp = win_rsrc(a.cp, win);
    const auto RO = win_rsrc(rout, win);
    auto poffset = [&](int m, int q) -> uint32_t {
        const bool ok = m >= 0 && m < nr && poff[q] >= 0;
        return ok ? (uint32_t)(((int64_t)(m - win.lo) * d.plane + poff[q]) * 8) : kOOB;
    };
    auto store_x = [&](int m, const double (&v)[kReLoads]) {
        double *f = &sX[m & 1][0][0];
#pragma unroll
        for (int q = 0; q < kReLoads; ++q)
            if (poff[q] != -2) f[tid + q * kReThreads] = v[q];
    };
    auto store_c = [&](const double (&vt)[kReLoads], const double (&vp)[kReLoads]) {
        double *ft = &sT[0][0], *fp = &sP[0][0];
#pragma unroll
        for (int q = 0; q < kReLoads; ++q)
            if (poff[q] != -2) {
                ft[tid + q * kReThreads] = vt[q];
                fp[tid + q * kReThreads] = vp[q];
            }
    };
    constexpr int NQ = kReR / kReWaves;
    auto own_off = [&](int m, int q) -> uint32_t {
        const int j = J0 + wv + kReWaves * q;
        const bool ok = m >= 0 && m < nr && j < nt && lane < nseg;
        return ok ? (uint32_t)(((int64_t)(m - win.lo) * d.plane + (int64_t)j * np + k0 + lane) * 8) : kOOB;
    };
    // own cells of the plane behind: x^ and c^_r (the coupling of the -r face)
    double xb[NQ], crb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        xb[q] = bld<double, 1>(RX, own_off(i0 - 1, q)).v[0];
        crb[q] = bld<double, 1>(RCr, own_off(i0 - 1, q)).v[0];
    }
    {
        double v[kReLoads], vt[kReLoads], vp[kReLoads];
#pragma unroll
        for (int q = 0; q < kReLoads; ++q) {
            v[q] = bld<double, 1>(RX, poffset(i0, q)).v[0];
            vt[q] = bld<double, 1>(RCt, poffset(i0, q)).v[0];
            vp[q] = bld<double, 1>(RCp, poffset(i0, q)).v[0];
        }
        store_x(i0, v);
        store_c(vt, vp);
#pragma unroll
        for (int q = 0; q < kReLoads; ++q) v[q] = bld<double, 1>(RX, poffset(i0 + 1, q)).v[0];
        store_x(i0 + 1, v);
    }
    __syncthreads();

    double acc[2] = {0.0, 0.0};
    double nx[kReLoads], nt_[kReLoads], np_[kReLoads];
    // own cells' b^, w and c^_r, one plane ahead
    double bh[NQ], wo[NQ], cro[NQ], bh1[NQ], wo1[NQ], cro1[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        bh[q] = bld<double, 1>(RB, own_off(i0, q)).v[0];
        wo[q] = bld<double, 1>(RW, own_off(i0, q)).v[0];
        cro[q] = bld<double, 1>(RCr, own_off(i0, q)).v[0];
    }
    for (int m = i0; m < i1; ++m) {
        // next planes in flight: x^ of m + 2, c^_theta and c^_phi of m + 1,
        // the own cells of m + 1
#pragma unroll
        for (int q = 0; q < kReLoads; ++q) {
            nx[q] = bld<double, 1>(RX, poffset(m + 2, q)).v[0];
            nt_[q] = bld<double, 1>(RCt, poffset(m + 1, q)).v[0];
            np_[q] = bld<double, 1>(RCp, poffset(m + 1, q)).v[0];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const uint32_t o1 = (m + 1 < i1) ? own_off(m + 1, q) : kOOB;
            bh1[q] = bld<double, 1>(RB, o1).v[0];
            wo1[q] = bld<double, 1>(RW, o1).v[0];
            cro1[q] = bld<double, 1>(RCr, o1).v[0];
        }
        const int s0 = m & 1, s1 = (m + 1) & 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int r = wv + kReWaves * q;
            const int j = J0 + r;
            const bool own = j < nt && lane < nseg;
            const uint32_t o = own_off(m, q);
            const double wc = wo[q], crc = cro[q];
            const int pr = r + 1, pc = lane + 1;
            const double xc = sX[s0][pr][pc];
            double sum = 0.0;
            if (m < nr - 1) sum += crc * sX[s1][pr][pc];
            if (m > 0) sum += crb[q] * xb[q];
            if (j < nt - 1) sum += sT[pr][pc] * sX[s0][pr + 1][pc];
            if (j > 0) sum += sT[pr - 1][pc] * sX[s0][pr - 1][pc];
            sum += sP[pr][pc] * sX[s0][pr][pc + 1] + sP[pr][pc - 1] * sX[s0][pr][pc - 1];
            const double res = bh[q] - (xc - sum);
            bst<TOUT, 1, kAuxNT>(RO, own ? (uint32_t)(o / 8u * sizeof(TOUT)) : kOOB,
                                 VecT<TOUT, 1>{{(TOUT)res}});
            if (own) {
                const double t = wc * res;
                acc[0] += t * t;
                acc[1] += res * res;
            }
            xb[q] = xc;
            crb[q] = crc;
            bh[q] = bh1[q];
            wo[q] = wo1[q];
            cro[q] = cro1[q];
        }
        __syncthreads();  // every read of plane m's x^ slot and of the couplings is done
        store_x(m + 2, nx);
        store_c(nt_, np_);
        __syncthreads();
    }
    __shared__ double lds[kReWaves * 2];
    block_sum_store<2>(acc, a.partials + 2 * (int64_t)blockIdx.x, lds);
}

// b^ = V src / w (src = rhs) or src / w (src = adjoint seed); x^ = w x0
// (warm start) or 0.  Partials [||b||^2, ||W r^||^2, ||r^||^2] of the
// initial residual when it is known here: from x^ = 0, r^ = b^ exactly, and
// it is written to rout (as TOUT) so that no residual kernel has to form it
// (rout may be null; with a warm start the last two partials are 0).
template <typename TOUT>
__global__ __launch_bounds__(kWave *kSimpleJ) void k_setup(const double *src, int src_is_rhs,
                                                           const double *w, Geo geo, Dims d,
                                                           double *bhat, double *x, int use_x0,
                                                           TOUT *rout, double *partials) {
    static_assert(kSimpleNV >= 3, "partials per simple block");
    __shared__ double lds[kSimpleJ * 3];
    double acc[3] = {0.0, 0.0, 0.0};
    MAS_SIMPLE_LOOP(d, {
        if (cell.ok) {
            const int64_t c = cell.c;
            double b = src[c];
            if (src_is_rhs) b *= geo.vr[cell.i] * geo.vt[cell.j];
            const double wc = w[c];
            const double bh = b / wc;
            bhat[c] = bh;
            x[c] = use_x0 ? wc * x[c] : 0.0;
            acc[0] += b * b;
            if (!use_x0) {
                if (rout) rout[c] = (TOUT)bh;
                const double t = wc * bh;
                acc[1] += t * t;
                acc[2] += bh * bh;
            }
        }
    })
    block_sum_store<3>(acc, partials + 3 * simple_block_id(), lds);
}

// x = x^ / w, in place.
__global__ __launch_bounds__(kWave *kSimpleJ) void k_unscale(const double *w, Dims d, double *x) {
    MAS_SIMPLE_LOOP(d, {
        if (cell.ok) x[cell.c] = x[cell.c] / w[cell.c];
    })
}

// Refinement update x^ += d^ + alpha p (double accumulation of the single-
// precision correction and of the pending step, alpha read from the control
// block; alpha = 0 for a restarted inner solve), then d^ = 0.
__global__ __launch_bounds__(kWave *kSimpleJ) void k_refine_fold(float *dh, const float *p,
                                                                 const Ctl *ctl, Dims d, double *x) {
    const double alpha = ctl->alpha;
    MAS_SIMPLE_LOOP(d, {
        if (cell.ok) {
            x[cell.c] = x[cell.c] + ((double)dh[cell.c] + alpha * (double)p[cell.c]);
            dh[cell.c] = 0.0f;
        }
    })
}

// x^ += d^ (a single-precision correction accumulated in double), then d^ = 0.
__global__ __launch_bounds__(kWave *kSimpleJ) void k_fold(float *dh, Dims d, double *x) {
    MAS_SIMPLE_LOOP(d, {
        if (cell.ok) {
            x[cell.c] = x[cell.c] + (double)dh[cell.c];
            dh[cell.c] = 0.0f;
        }
    })
}

template <typename T>
__global__ __launch_bounds__(kWave *kSimpleJ) void k_fill(T *x, Dims d, T v) {
    MAS_SIMPLE_LOOP(d, {
        if (cell.ok) x[cell.c] = v;
    })
}

// dL/dnu and dL/drhs from the forward solution x and the adjoint lam:
//   dL/drhs_c = V_c lam_c,
//   dL/dnu_c  = -dt sum_{faces f of c} (dG_f/dnu_c) (lam_c - lam_nb)(x_c - x_nb),
// where a face's conductance depends on nu_c with weight 1/2 inside the shell
// (face mean) and 1 on a Dirichlet wall (lam_nb = x_nb = 0 there).
// Each face product (lam_c - lam_nb)(x_c - x_nb) is formed once per side, as
// the oracle forms it.
// Each block owns a tile of kGrR theta rows x kGrC phi cells (a wave owns
// rows wv, wv + 4, ..., one cell per lane) and marches up its r chunk: x and
// lam of the current plane and the next one sit in LDS with a one-cell ring
// around the tile (the in-plane neighbours), the plane behind in the
// registers of the thread that owns the cell.  The two planes after the next
// one are in flight in two register sets while the current one is computed
// (a plane's loads are waited for two plane steps after they are issued, so
// a block keeps two plane patches of requests outstanding).  Every value is
// fetched from memory once per block (the ring from the neighbouring tiles'
// lines, mostly in L2) and every output written once.
constexpr int kGrR = 16, kGrC = 64, kGrWaves = 4, kGrThreads = kWave * kGrWaves;
constexpr int kGrPR = kGrR + 2, kGrPC = kGrC + 2;  // patch: rows J0-1..J0+R, cells k0-1..k0+C
constexpr int kGrLoads = (kGrPR * kGrPC + kGrThreads - 1) / kGrThreads;

struct GradArgs {
    const double *x, *lam;
    double *gnu, *grhs;
    Geo geo;
    Dims d;
    int tiles_i, tiles_k, tiles_j, ti, nblk;
};

__global__ __launch_bounds__(kGrThreads) void k_gradient(GradArgs a) {
    __shared__ double sX[2][kGrPR][kGrPC], sL[2][kGrPR][kGrPC], sNone[2];
    // per tile row: vt, halves of the theta- and phi-face factors
    __shared__ double sRow[kGrR][4];
    const Dims d = a.d;
    const Geo &g = a.geo;
    const int nr = d.nr, nt = d.nt, np = d.np;
    const int L = xcd_remap(blockIdx.x, a.nblk);
    int it, kt, jt;
    tile_coords<3>(L, a.tiles_i, a.tiles_k, a.tiles_j, it, kt, jt);
    const int J0 = jt * kGrR, k0 = kt * kGrC;
    const int nseg = min(kGrC, np - k0);
    const int i0 = it * a.ti, i1 = min(i0 + a.ti, nr);
    // planes i0 - 1 .. i1 are read, planes i0 .. i1 - 1 written
    const PlaneWin win = plane_win(d, i0 - 1, i1 + 1);
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);

    if (tid < kGrR) {
        const int j = J0 + tid;
        const bool ok = j < nt;
        const int jj = ok ? j : 0;
        sRow[tid][0] = g.vt[jj];
        sRow[tid][1] = (ok && j > 0) ? 0.5 * g.gtt[j - 1] : 0.0;
        sRow[tid][2] = (ok && j < nt - 1) ? 0.5 * g.gtt[jj] : 0.0;
        sRow[tid][3] = (ok && !g.np_one) ? 0.5 * g.gpt[jj] : 0.0;
    }

    // this thread's elements of the patch: byte offsets inside a plane, kOOB
    // for an element outside the grid in theta (read as zero) or none (-2 in
    // poff: not stored)
    int32_t poff[kGrLoads];
    uint32_t pb[kGrLoads];
#pragma unroll
    for (int q = 0; q < kGrLoads; ++q) {
        const int e = tid + q * kGrThreads;
        poff[q] = -2;
        if (e < kGrPR * kGrPC) {
            const int pr = e / kGrPC, pc = e % kGrPC;
            const int j = J0 - 1 + pr;
            int k = (k0 - 1 + pc) % np;
            if (k < 0) k += np;
            poff[q] = (j >= 0 && j < nt) ? j * np + k : -1;
        }
        pb[q] = poff[q] >= 0 ? (uint32_t)poff[q] * 8u : kOOB;
    }
    const auto RX = win_rsrc(a.x, win), RL = win_rsrc(a.lam, win), RG = win_rsrc(a.gnu, win),
               RH = win_rsrc(a.grhs, win);
    // planes i0 .. min(i1, nr - 1) are loaded into the patch (plane i1, the
    // +r neighbour of the last plane computed, is the last one used); the
    // prefetch runs past them and loads nothing there.
    // The offset is the plane's part plus the element's, with bit 31 (out of
    // range of every window, which stays below 2^31 bytes) set for a plane
    // or an element that is not loaded: no branch, so the compiler tracks
    // the loads in flight exactly.
    const int m_end = min(i1 + 1, nr);
    auto load_plane = [&](int m, double (&vx)[kGrLoads], double (&vl)[kGrLoads]) {
        const bool pin = m >= 0 && m < m_end;
        const uint32_t base = pin ? (uint32_t)((int64_t)(m - win.lo) * d.plane * 8) : 0u;
        const uint32_t bad = pin ? 0u : kOOB;
#pragma unroll
        for (int q = 0; q < kGrLoads; ++q) {
            const uint32_t o = (pb[q] + base) | bad;
            vx[q] = bld<double, 1>(RX, o).v[0];
            vl[q] = bld<double, 1>(RL, o).v[0];
        }
    };
    // a thread with no element in a patch slot writes a slot of its own
    // that nothing reads (no branch around the write, so the wait for the
    // load it writes stands on every path)
    auto store_plane = [&](int m, const double (&vx)[kGrLoads], const double (&vl)[kGrLoads]) {
        double *fx = &sX[m & 1][0][0], *fl = &sL[m & 1][0][0];
#pragma unroll
        for (int q = 0; q < kGrLoads; ++q) {
            const bool el = poff[q] != -2;
            *(el ? &fx[tid + q * kGrThreads] : &sNone[0]) = vx[q];
            *(el ? &fl[tid + q * kGrThreads] : &sNone[1]) = vl[q];
        }
    };
    constexpr int NQ = kGrR / kGrWaves;
    // own cells: rows wv + 4q, column lane; x and lam of the plane behind
    double xb[NQ], lb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = J0 + wv + kGrWaves * q;
        const bool ok = i0 > 0 && j < nt && lane < nseg;
        const uint32_t o = ok ? (uint32_t)(((int64_t)(i0 - 1 - win.lo) * d.plane + (int64_t)j * np + k0 + lane) * 8) : kOOB;
        xb[q] = bld<double, 1>(RX, o).v[0];
        lb[q] = bld<double, 1>(RL, o).v[0];
    }
    // two register sets, alternating by the parity of the step: planes i0
    // and i0 + 1 go to the patch, plane i0 + 2 waits in the first set
    double ax[kGrLoads], al[kGrLoads], bx[kGrLoads], bl[kGrLoads];
    {
        double vx[kGrLoads], vl[kGrLoads];
        load_plane(i0, vx, vl);
        load_plane(i0 + 1, bx, bl);
        load_plane(i0 + 2, ax, al);
        store_plane(i0, vx, vl);
        store_plane(i0 + 1, bx, bl);
    }
    __syncthreads();

    // plane step m: computes plane m from the patch slots of m and m + 1,
    // then moves plane m + 2 (issued into `ready` at the start of the step
    // before) into the slot plane m leaves; plane m + 3 is issued into
    // `fill` first
    auto step = [&](int m, double (&ready_x)[kGrLoads], double (&ready_l)[kGrLoads],
                    double (&fill_x)[kGrLoads], double (&fill_l)[kGrLoads]) {
        load_plane(m + 3, fill_x, fill_l);
        const int s0 = m & 1, s1 = (m + 1) & 1;
        // plane factors (uniform)
        const double gq = ld_table(g.gq, m);
        const double grp = (m < nr - 1) ? 0.5 * ld_table(g.gr, m) : 0.0;
        const double grm = (m > 0) ? 0.5 * ld_table(g.gr, m - 1) : 0.0;
        const double gw = ((m == 0) ? g.gw_in : 0.0) + ((m == nr - 1) ? g.gw_out : 0.0);
        const double vr = ld_table(g.vr, m);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int r = wv + kGrWaves * q;
            const int j = J0 + r;
            const bool own = j < nt && lane < nseg;
            const double vt = sRow[r][0];
            const double cRp = grp * vt, cRm = grm * vt, cW = gw * vt;
            const double cU = gq * sRow[r][1], cD = gq * sRow[r][2], cP = gq * sRow[r][3];
            const int pr = r + 1, pc = lane + 1;
            const double xc = sX[s0][pr][pc], lc = sL[s0][pr][pc];
            const double Xp = sX[s1][pr][pc], Lp = sL[s1][pr][pc];
            const double xu = sX[s0][pr - 1][pc], lu = sL[s0][pr - 1][pc];
            const double xd = sX[s0][pr + 1][pc], ld = sL[s0][pr + 1][pc];
            const double xl = sX[s0][pr][pc - 1], ll = sL[s0][pr][pc - 1];
            const double xr = sX[s0][pr][pc + 1], lr = sL[s0][pr][pc + 1];
            double t = cW * (lc * xc);
            t += cRp * ((lc - Lp) * (xc - Xp));
            t += cRm * ((lc - lb[q]) * (xc - xb[q]));
            t += cU * ((lc - lu) * (xc - xu));
            t += cD * ((lc - ld) * (xc - xd));
            t += cP * ((lc - ll) * (xc - xl) + (lc - lr) * (xc - xr));
            const uint32_t o = own ? (uint32_t)(((int64_t)(m - win.lo) * d.plane + (int64_t)j * np + k0 + lane) * 8) : kOOB;
            bst<double, 1, kAuxNT>(RG, o, VecT<double, 1>{{-g.dt * t}});
            bst<double, 1, kAuxNT>(RH, o, VecT<double, 1>{{(vr * vt) * lc}});
            xb[q] = xc;
            lb[q] = lc;
        }
        __syncthreads();  // every read of plane m's slot is done
        store_plane(m + 2, ready_x, ready_l);
        __syncthreads();
    };
    for (int m = i0; m < i1; m += 2) {
        step(m, ax, al, bx, bl);
        if (m + 1 < i1) step(m + 1, bx, bl, ax, al);
    }
}

// Streaming copy: each block copies one contiguous chunk of kCopyChunk
// 16-byte elements, each thread keeping kCopyU loads in flight.
constexpr int kCopyU = 4;
constexpr int64_t kCopyChunk = 16384;
__global__ __launch_bounds__(256) void k_copy16(const double2 *__restrict__ src,
                                                double2 *__restrict__ dst, int64_t n16) {
    const int64_t beg = (int64_t)blockIdx.x * kCopyChunk;
    const int64_t end = min(beg + kCopyChunk, n16);
    for (int64_t t0 = beg + threadIdx.x; t0 < end; t0 += 256 * kCopyU) {
        double2 v[kCopyU];
#pragma unroll
        for (int u = 0; u < kCopyU; ++u) {
            const int64_t t = t0 + u * 256;
            if (t < end) v[u] = src[t];
        }
#pragma unroll
        for (int u = 0; u < kCopyU; ++u) {
            const int64_t t = t0 + u * 256;
            if (t < end) dst[t] = v[u];
        }
    }
}

// Streaming probe with a stencil kernel's byte mix: NIN arrays read and
// NOUT written, each block walking one contiguous chunk of kStreamChunk
// cells of every array (as the marching kernels walk their r chunks), two
// cells per lane, non-temporal.  out_t[c] = in_0[c] + ... + in_{NIN-1}[c] +
// t, so no load is dead.
constexpr int64_t kStreamChunk = 16384;
constexpr int kStreamMaxIn = 8, kStreamMaxOut = 4;
struct StreamArgs {
    const double *in[kStreamMaxIn];
    double *out[kStreamMaxOut];
    int64_t n;
};

template <int NIN, int NOUT>
__global__ __launch_bounds__(256) void k_stream(StreamArgs a) {
    const int64_t beg = (int64_t)blockIdx.x * kStreamChunk;
    const int64_t end = min(beg + kStreamChunk, a.n);
    for (int64_t c = beg + 2 * (int64_t)threadIdx.x; c < end; c += 2 * 256) {
        double s0 = 0.0, s1 = 0.0;
        if (c + 1 < end) {
#pragma unroll
            for (int t = 0; t < NIN; ++t) {
                const VecT<double, 2> v = ldv_nt<double, 2>(a.in[t], c);
                s0 += v.v[0];
                s1 += v.v[1];
            }
#pragma unroll
            for (int t = 0; t < NOUT; ++t) stv_nt<double, 2>(a.out[t], c, VecT<double, 2>{{s0 + t, s1 + t}});
        } else {
#pragma unroll
            for (int t = 0; t < NIN; ++t) s0 += a.in[t][c];
#pragma unroll
            for (int t = 0; t < NOUT; ++t) a.out[t][c] = s0 + t;
        }
    }
}

}  // namespace mas
