// Host side of the implicit viscous solver: argument checking, storage and
// workspace layout, the 1-D geometry tables, and the PCG / refinement /
// adjoint drivers that launch the kernels in kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mas.h"
#include "kernels.hpp"
#include "sts_kernels.hpp"
#include "pc2_kernels.hpp"

using namespace mas;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

static int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(MAS_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

#define LAUNCHCHK()                                                                    \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return fail(MAS_EHIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ tile configuration
// Iteration kernel: (64 V) phi cells x kTJ theta rows (one wave each) per
// block, an r chunk of Shape::ti() planes per block; V = 16 bytes / element
// size when np is a multiple of it, else 1.
#ifndef MAS_TJ
#define MAS_TJ 4
#endif
#ifndef MAS_TI
#define MAS_TI 16  // shortest r chunk
#endif
#ifndef MAS_RPW
#define MAS_RPW 2
#endif
static constexpr int kTJ = MAS_TJ;   // waves per block
static constexpr int kRPW = MAS_RPW; // theta rows per wave
static constexpr int kTI = MAS_TI;
#ifndef MAS_MIN_BLOCKS
#define MAS_MIN_BLOCKS 1024
#endif
#ifndef MAS_SMALL_TI
#define MAS_SMALL_TI 1
#endif
static constexpr int64_t kMinBlocks = MAS_MIN_BLOCKS;
static constexpr int kSmallTI = MAS_SMALL_TI;

#ifndef MAS_ITER_VEC
#define MAS_ITER_VEC 16  // bytes per lane, double-precision iteration kernel
#endif
#ifndef MAS_MULTI_VEC
#define MAS_MULTI_VEC 1  // several right-hand sides keep the full vector width
#endif
#ifndef MAS_ITER_VEC_F32
#define MAS_ITER_VEC_F32 16  // bytes per lane, single-precision iteration kernel
#endif
template <typename T>
static constexpr int vec_full() {
    constexpr int bytes = sizeof(T) == 8 ? MAS_ITER_VEC : MAS_ITER_VEC_F32;
    return bytes / (int)sizeof(T) > 0 ? bytes / (int)sizeof(T) : 1;
}
template <typename T>
static inline int vec_width(int np) {
    constexpr int v = vec_full<T>();
    return (np % v == 0) ? v : 1;
}

// Lanes' vector width of the iteration kernel for nrhs right-hand sides.
template <typename T>
static inline int iter_vec(int np, int nrhs) {
    return (nrhs > 1 && !MAS_MULTI_VEC) ? 1 : vec_width<T>(np);
}

static inline int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

// Array stagger.  Arrays of n cells sit at offsets that differ by multiples
// of their length, which at the production sizes is a multiple of 16 MiB
// (256 x 320 x 640 cells: 400 MiB), so element c of every array would share
// the low address bits that pick the HBM channel; a stencil kernel reading
// element c of seven arrays at once then sends them to one channel.  Each array of a
// layout is moved by its own multiple of kStagger bytes, and the workspace
// and the stage arrays start at other multiples than the operator storage.
// 2304 = 9 x 256: sixteen consecutive arrays start in sixteen different
// 256-byte slots of a 4 KiB interleave unit (measured 1-2% faster iteration
// and stage kernels than no stagger).
#ifndef MAS_STAGGER
#define MAS_STAGGER 2304
#endif
static constexpr int64_t kStagger = MAS_STAGGER;
static_assert(kStagger % 256 == 0, "stagger keeps 256-byte alignment");
enum { kPhaseStorage = 0, kPhaseWork = 8, kPhaseSts = 20 };

// Offsets of a layout: small tables packed at 256-byte alignment, arrays of
// the grid's size each staggered (see above).
struct LayoutCursor {
    int64_t off = 0;
    int64_t lead;  // extra stagger before the first array: the layout's phase
    explicit LayoutCursor(int phase) : lead(phase * kStagger) {}
    int64_t take(int64_t bytes) {
        const int64_t o = off;
        off = align256(off + bytes);
        return o;
    }
    int64_t take_array(int64_t bytes) {
        off += kStagger + lead;
        lead = 0;
        return take(bytes);
    }
};

// The marching kernels address one block's r planes through buffer
// resources based at its first plane, with 32-bit byte offsets: the planes a
// block may touch, its chunk plus at most kWinHalo more, stay below
// kWinBytes in every array, which bounds the chunk, not the grid.
constexpr int64_t kWinBytes = (int64_t)1 << 31;
constexpr int kWinHalo = 6;

struct Shape {
    int nr, nt, np;
    int64_t plane, n;
    Dims dims() const { return Dims{nr, nt, np, plane, n}; }
    int tiles_k(int v) const { return (np + (kWave / kRPW) * v - 1) / ((kWave / kRPW) * v); }
    int tiles_j() const { return (nt + kTJ * kRPW - 1) / (kTJ * kRPW); }
    // r planes per chunk: the tiles of one chunk are consecutive logical
    // blocks, and xcd_remap hands each of the 8 XCDs a contiguous eighth of
    // them, so with 8 chunks (or a multiple) every XCD owns whole r slabs
    // and only the planes at slab boundaries are read by two XCDs (256 x 320
    // x 640 cells: 32-plane chunks, 1.4% faster than 16).  At least kTI
    // planes, unless that leaves fewer than kMinBlocks blocks: a small grid
    // is latency-bound (each wave's plane steps run one after another), so
    // its chunks shrink, down to kSmallTI planes, until about kMinBlocks
    // blocks share the work.
    // (a forced chunk, or the rule's, capped by max_chunk)
    int ti(int v, int forced = 0) const {
        const int cap = max_chunk(iter_plane_bytes(v));
        if (forced > 0) return std::min(forced, cap);
        return std::min(chunk_for((int64_t)tiles_k(v) * tiles_j()), cap);
    }
    // the same rule for any marching kernel with `tiles` tiles per plane
    // (arrays of 8-byte elements)
    int chunk_for(int64_t tiles) const {
        const int big = std::max(kTI, (nr + 7) / 8);
        int t;
        if (tiles * ((nr + big - 1) / big) >= kMinBlocks) {
            t = big;
        } else {
            const int64_t want = (tiles * nr + kMinBlocks - 1) / kMinBlocks;
            t = (int)std::min<int64_t>(big, std::max<int64_t>(kSmallTI, want));
        }
        return std::min(t, max_chunk());
    }
    // most r planes per chunk of a kernel whose arrays hold bytes_per_plane
    // bytes per r plane (0: 8-byte cells), from the window bound; at least 1
    // on every grid check_grid accepts
    int max_chunk(int64_t bytes_per_plane = 0) const {
        const int64_t b = bytes_per_plane > 0 ? bytes_per_plane : 8 * plane;
        return (int)std::max<int64_t>(1, std::min<int64_t>(nr, (kWinBytes - 1) / b - kWinHalo));
    }
    // the iteration kernel's largest array per r plane: 8-byte cells or the
    // segment-edge records (8 elements per row and segment)
    int64_t iter_plane_bytes(int v) const {
        return 8 * std::max<int64_t>(plane, (int64_t)nt * tiles_k(v) * 8);
    }
    int tiles_i(int v, int forced = 0) const { return (nr + ti(v, forced) - 1) / ti(v, forced); }
    int64_t nblk_iter(int v, int forced = 0) const {
        return (int64_t)tiles_k(v) * tiles_j() * tiles_i(v, forced);
    }
    // most blocks any launch of the iteration kernel can have (one-plane chunks)
    int64_t nblk_iter_max() const { return nblk_iter(1, 1); }
    // bytes of one segment-edge record buffer of the iteration kernel, and
    // whether the records can be used (every segment spans two lanes)
    int64_t halo_bytes(int v, int64_t es) const { return (int64_t)nr * nt * tiles_k(v) * 2 * 4 * es; }
    bool halo_ok(int v) const {
        const int seg = (kWave / kRPW) * v;
        const int last = np - (tiles_k(v) - 1) * seg;
        return last >= 2 * v;
    }
    dim3 simple_grid() const {
        return dim3((np + kWave - 1) / kWave, (nt + kSimpleJ - 1) / kSimpleJ,
                    (nr + kSimpleR - 1) / kSimpleR);
    }
    int64_t nblk_simple() const {
        dim3 g = simple_grid();
        return (int64_t)g.x * g.y * g.z;
    }
};

// ------------------------------------------------------------------ operator
struct mas_op {
    Shape s;
    int precision;
    int bc_inner, bc_outer;
    double dt;
    Geo geo;            // device pointers into storage + scalars
    double *w;
    double *c64[3];
    float *c32[3];      // null unless built with MAS_FP32_REFINED
    double *nu;         // copy of nu (explicit stages form conductances from it)
    double zmax;        // max_c 2 (A_cc - V_c) / V_c
    hipStream_t build_stream;
};

struct StorageLayout {
    int64_t flags, vr, vt, gr, gq, gtt, gpt, w, c64[3], c32[3], nu, total;
};

static StorageLayout storage_layout(const Shape &s, int precision) {
    StorageLayout L{};
    LayoutCursor cur(kPhaseStorage);
    L.flags = cur.take(256);
    L.vr = cur.take(8 * (int64_t)s.nr);
    L.vt = cur.take(8 * (int64_t)s.nt);
    L.gr = cur.take(8 * (int64_t)s.nr);
    L.gq = cur.take(8 * (int64_t)s.nr);
    L.gtt = cur.take(8 * (int64_t)s.nt);
    L.gpt = cur.take(8 * (int64_t)s.nt);
    L.w = cur.take_array(8 * s.n);
    for (int t = 0; t < 3; ++t) L.c64[t] = cur.take_array(8 * s.n);
    for (int t = 0; t < 3; ++t)
        L.c32[t] = (precision == MAS_FP32_REFINED) ? cur.take_array(4 * s.n) : -1;
    L.nu = cur.take_array(8 * s.n);
    L.total = cur.off;
    return L;
}

static int check_grid(const mas_grid *g, Shape *out) {
    if (!g) return fail(MAS_EINVAL, "grid is NULL");
    if (g->nr < 1 || g->nt < 1 || g->np < 1)
        return fail(MAS_EINVAL, "grid sizes must be >= 1 (got %d x %d x %d)", g->nr, g->nt, g->np);
    if (!g->r_faces || !g->t_faces) return fail(MAS_EINVAL, "face arrays must not be NULL");
    Shape sh{g->nr, g->nt, g->np, (int64_t)g->nt * g->np, (int64_t)g->nr * g->nt * g->np};
    // a one-plane chunk and its halo planes must fit a block's 32-bit window
    // (the records of one-cell segments are the largest per-plane array)
    if ((int64_t)(1 + kWinHalo) * sh.iter_plane_bytes(1) >= kWinBytes)
        return fail(MAS_EINVAL, "theta-phi plane too large: nt*np at most %lld cells",
                    (long long)((kWinBytes - 1) / (8 * (1 + kWinHalo))));
    if ((int64_t)g->nt > 65535LL * kSimpleJ) return fail(MAS_EINVAL, "nt too large");
    if ((int64_t)g->nr > 65535LL * kSimpleR) return fail(MAS_EINVAL, "nr too large");
    if (sh.nblk_iter_max() > INT32_MAX) return fail(MAS_EINVAL, "grid too large");
    if (!(g->r_faces[0] > 0.0) || !std::isfinite(g->r_faces[0]))
        return fail(MAS_EINVAL, "r_faces[0] must be positive and finite");
    for (int i = 0; i < g->nr; ++i)
        if (!(g->r_faces[i + 1] > g->r_faces[i]) || !std::isfinite(g->r_faces[i + 1]))
            return fail(MAS_EINVAL, "r_faces must be strictly increasing and finite (index %d)", i + 1);
    if (g->t_faces[0] != 0.0 || g->t_faces[g->nt] != M_PI)
        return fail(MAS_EINVAL, "t_faces must run from exactly 0 to exactly pi");
    for (int j = 0; j < g->nt; ++j)
        if (!(g->t_faces[j + 1] > g->t_faces[j]))
            return fail(MAS_EINVAL, "t_faces must be strictly increasing (index %d)", j + 1);
    for (int b : {g->bc_inner, g->bc_outer})
        if (b != MAS_BC_DIRICHLET0 && b != MAS_BC_NEUMANN0)
            return fail(MAS_EINVAL, "unknown boundary condition %d", b);
    if (out) *out = sh;
    return MAS_OK;
}

// 1-D geometric factors in double precision (libm), see struct Geo.
struct HostGeo {
    std::vector<double> vr, vt, gr, gq, gtt, gpt;
    double gw_in, gw_out;
};

static HostGeo host_geometry(const mas_grid *g) {
    const int nr = g->nr, nt = g->nt, np = g->np;
    const double *rf = g->r_faces, *tf = g->t_faces;
    const double dphi = 2.0 * M_PI / np;
    HostGeo h;
    h.vr.resize(nr);
    h.gr.resize(nr);
    h.gq.resize(nr);
    h.vt.resize(nt);
    h.gtt.resize(nt);
    h.gpt.resize(nt);
    std::vector<double> rc(nr), tc(nt);
    for (int i = 0; i < nr; ++i) rc[i] = 0.5 * (rf[i] + rf[i + 1]);
    for (int j = 0; j < nt; ++j) tc[j] = 0.5 * (tf[j] + tf[j + 1]);
    for (int i = 0; i < nr; ++i) {
        const double a = rf[i], b = rf[i + 1];
        h.vr[i] = (b - a) * (b * b + b * a + a * a) / 3.0;
        h.gq[i] = (b * b - a * a) / (2.0 * rc[i]);
        h.gr[i] = (i < nr - 1) ? b * b / (rc[i + 1] - rc[i]) : 0.0;
    }
    for (int j = 0; j < nt; ++j) {
        const double a = tf[j], b = tf[j + 1];
        // cos a - cos b without cancellation
        h.vt[j] = 2.0 * std::sin(0.5 * (a + b)) * std::sin(0.5 * (b - a)) * dphi;
        h.gtt[j] = (j < nt - 1) ? std::sin(b) * dphi / (tc[j + 1] - tc[j]) : 0.0;
        h.gpt[j] = (b - a) / (std::sin(tc[j]) * dphi);
    }
    h.gw_in = (g->bc_inner == MAS_BC_DIRICHLET0) ? rf[0] * rf[0] / (rc[0] - rf[0]) : 0.0;
    h.gw_out = (g->bc_outer == MAS_BC_DIRICHLET0) ? rf[nr] * rf[nr] / (rf[nr] - rc[nr - 1]) : 0.0;
    return h;
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" void mas_pcg_default_opts(mas_pcg_opts *o) {
    if (!o) return;
    o->rtol = 1e-10;
    o->max_iters = 100000;
    o->precision = MAS_FP64;
    o->inner_rtol = 1e-5;
    o->max_outer = 20;
    o->check_every = 8;
    o->use_x0 = 0;
    o->max_restarts = 3;
    o->sample_timing = 0;
    o->refine = MAS_REFINE_RELIABLE;
    o->precond = MAS_PC1;
    o->chunk_planes = 0;
    o->launch = MAS_LAUNCH_AUTO;
}

extern "C" int64_t mas_op_storage_bytes(const mas_grid *g, int32_t precision) {
    Shape s;
    int st = check_grid(g, &s);
    if (st != MAS_OK) return st;
    if (precision != MAS_FP64 && precision != MAS_FP32_REFINED)
        return fail(MAS_EINVAL, "unknown precision %d", precision);
    return storage_layout(s, precision).total;
}

extern "C" int mas_op_build(const mas_grid *g, const double *nu, double dt, int32_t precision,
                            void *storage, int64_t storage_bytes, void *hip_stream,
                            mas_op **op_out) {
    g_last_error.clear();
    if (op_out) *op_out = nullptr;
    Shape s;
    int st = check_grid(g, &s);
    if (st != MAS_OK) return st;
    if (!nu || !storage || !op_out) return fail(MAS_EINVAL, "nu, storage and op_out must not be NULL");
    if (precision != MAS_FP64 && precision != MAS_FP32_REFINED)
        return fail(MAS_EINVAL, "unknown precision %d", precision);
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(MAS_EINVAL, "dt must be finite and >= 0");
    if (reinterpret_cast<uintptr_t>(storage) & 255)
        return fail(MAS_EINVAL, "storage must be 256-byte aligned");
    const StorageLayout L = storage_layout(s, precision);
    if (storage_bytes < L.total)
        return fail(MAS_ENOMEM, "storage too small: %lld < %lld bytes", (long long)storage_bytes,
                    (long long)L.total);

    hipStream_t stream = as_stream(hip_stream);
    char *base = static_cast<char *>(storage);
    HostGeo h = host_geometry(g);

    mas_op *op = new (std::nothrow) mas_op();
    if (!op) return fail(MAS_EINVAL, "out of host memory");
    op->s = s;
    op->precision = precision;
    op->bc_inner = g->bc_inner;
    op->bc_outer = g->bc_outer;
    op->dt = dt;
    double *vr = reinterpret_cast<double *>(base + L.vr);
    double *vt = reinterpret_cast<double *>(base + L.vt);
    double *gr = reinterpret_cast<double *>(base + L.gr);
    double *gq = reinterpret_cast<double *>(base + L.gq);
    double *gtt = reinterpret_cast<double *>(base + L.gtt);
    double *gpt = reinterpret_cast<double *>(base + L.gpt);
    op->geo = Geo{vr, vt, gr, gq, gtt, gpt, h.gw_in, h.gw_out, dt, s.np == 1 ? 1 : 0};
    op->w = reinterpret_cast<double *>(base + L.w);
    for (int t = 0; t < 3; ++t) {
        op->c64[t] = reinterpret_cast<double *>(base + L.c64[t]);
        op->c32[t] = (L.c32[t] >= 0) ? reinterpret_cast<float *>(base + L.c32[t]) : nullptr;
    }
    op->nu = reinterpret_cast<double *>(base + L.nu);
    // flags: [0] nu invalid, [2:4] bits of z_max
    int32_t *flags = reinterpret_cast<int32_t *>(base + L.flags);

    auto cleanup_fail = [&](int status) {
        delete op;
        return status;
    };
    // the six tables sit back to back in the storage (vr .. gpt): one upload
    // from a staging buffer that lives until the build has been waited for
    std::vector<char> stage;
    {
        const int64_t span = L.gpt + 8 * (int64_t)s.nt - L.vr;
        stage.assign((size_t)span, 0);
        struct Up {
            int64_t off;
            const std::vector<double> *src;
        } ups[] = {{L.vr, &h.vr}, {L.vt, &h.vt}, {L.gr, &h.gr},
                   {L.gq, &h.gq}, {L.gtt, &h.gtt}, {L.gpt, &h.gpt}};
        for (auto &u : ups)
            std::memcpy(stage.data() + (u.off - L.vr), u.src->data(), 8 * u.src->size());
        hipError_t e = hipMemcpyAsync(vr, stage.data(), (size_t)span, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess)
            return cleanup_fail(fail(MAS_EHIP, "geometry upload failed: %s", hipGetErrorString(e)));
    }
    const Dims d = s.dims();
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(1, 1, 1), dim3(kWave, kSimpleJ), 0, stream, flags,
                       Dims{1, 1, 4, 4, 4}, 0);
    {
        BuildArgs ba{};
        ba.nu = nu;
        ba.w = op->w;
        ba.cr = op->c64[0];
        ba.ct = op->c64[1];
        ba.cp = op->c64[2];
        ba.nu_copy = op->nu;
        ba.cr32 = op->c32[0];
        ba.ct32 = op->c32[1];
        ba.cp32 = op->c32[2];
        ba.bad = flags;
        ba.zmax_bits = reinterpret_cast<unsigned long long *>(flags + 2);
        ba.geo = op->geo;
        ba.d = d;
        ba.tiles_k = (s.np + kBuC - 1) / kBuC;
        ba.tiles_j = (s.nt + kBuR - 1) / kBuR;
        ba.ti = s.chunk_for((int64_t)ba.tiles_k * ba.tiles_j);
        ba.tiles_i = (s.nr + ba.ti - 1) / ba.ti;
        const int64_t nblk = (int64_t)ba.tiles_i * ba.tiles_j * ba.tiles_k;
        if (nblk > INT32_MAX) {
            (void)hipStreamSynchronize(stream);
            return cleanup_fail(fail(MAS_EINVAL, "grid too large for the build kernel"));
        }
        ba.nblk = (int)nblk;
        if (precision == MAS_FP32_REFINED)
            hipLaunchKernelGGL(k_build<true>, dim3((unsigned)nblk), dim3(kBuThreads), 0, stream, ba);
        else
            hipLaunchKernelGGL(k_build<false>, dim3((unsigned)nblk), dim3(kBuThreads), 0, stream, ba);
    }
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(stream);  // the upload may still read the staging buffer
            return cleanup_fail(fail(MAS_EHIP, "build launch failed: %s", hipGetErrorString(e)));
        }
    }
    int32_t fl[4] = {0, 0, 0, 0};
    {
        hipError_t e = hipMemcpyAsync(fl, flags, sizeof fl, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess)
            return cleanup_fail(fail(MAS_EHIP, "build failed: %s", hipGetErrorString(e)));
    }
    if (fl[0]) return cleanup_fail(fail(MAS_EINVAL, "nu must be positive and finite everywhere"));
    std::memcpy(&op->zmax, &fl[2], sizeof(double));
    *op_out = op;
    return MAS_OK;
}

extern "C" void mas_op_destroy(mas_op *op) { delete op; }

extern "C" int mas_op_apply(const mas_op *op, const double *x, double *y, void *hip_stream) {
    if (!op || !x || !y) return fail(MAS_EINVAL, "op, x and y must not be NULL");
    if (x == y) return fail(MAS_EINVAL, "x and y must be distinct");
    hipLaunchKernelGGL(k_apply, op->s.simple_grid(), dim3(kWave, kSimpleJ), 0, as_stream(hip_stream),
                       op->w, op->c64[0], op->c64[1], op->c64[2], op->s.dims(), x, y);
    LAUNCHCHK();
    return MAS_OK;
}

extern "C" int mas_op_export(const mas_op *op, double *cr, double *ct, double *cp, double *diag,
                             void *hip_stream) {
    if (!op) return fail(MAS_EINVAL, "op must not be NULL");
    hipLaunchKernelGGL(k_export, op->s.simple_grid(), dim3(kWave, kSimpleJ), 0,
                       as_stream(hip_stream), op->w, op->c64[0], op->c64[1], op->c64[2],
                       op->s.dims(), cr, ct, cp, diag);
    LAUNCHCHK();
    return MAS_OK;
}

// ------------------------------------------------------------------ workspace
struct WorkLayout {
    int64_t ctl, sync, partials, bhat[kMaxRhs], vec[kMaxRhs][6], halo[kMaxRhs][2], dh[kMaxRhs], total;
    int64_t halo_bytes;  // one record buffer (0: records not used)
};

// nrhs right-hand sides: control blocks and the iteration partials for all of
// them, then b^ and the six PCG vectors of each.
static WorkLayout work_layout(const Shape &s, int precision, int nrhs = 1) {
    WorkLayout L{};
    LayoutCursor cur(kPhaseWork);
    auto take = [&](int64_t bytes) { return cur.take(bytes); };
    auto take_array = [&](int64_t bytes) { return cur.take_array(bytes); };
    // the iteration kernel writes nrhs * kNV partials per block (most blocks
    // with V = 1), the simple-tile kernels up to kSimpleNV
    // (a persistent run keeps two sets, by parity)
    const int64_t nparts = std::max(s.nblk_iter_max() * kNV * nrhs * 2, s.nblk_simple() * kSimpleNV);
    L.ctl = take(sizeof(Ctl) * nrhs);
    L.sync = take(sizeof(PersistSync));
    L.partials = take(8 * nparts);
    const int64_t es = (precision == MAS_FP32_REFINED) ? 4 : 8;
    for (int c = 0; c < kMaxRhs; ++c) {
        L.bhat[c] = -1;
        for (int t = 0; t < 6; ++t) L.vec[c][t] = -1;
    }
    for (int c = 0; c < nrhs; ++c) {
        L.bhat[c] = take_array(8 * s.n);
        for (int t = 0; t < 6; ++t) L.vec[c][t] = take_array(es * s.n);
    }
    // segment-edge records of the iteration kernel, double-buffered
    const int v = (precision == MAS_FP32_REFINED) ? iter_vec<float>(s.np, nrhs)
                                                  : iter_vec<double>(s.np, nrhs);
    L.halo_bytes = s.halo_ok(v) ? s.halo_bytes(v, es) : 0;
    for (int c = 0; c < kMaxRhs; ++c) L.halo[c][0] = L.halo[c][1] = -1;
    if (L.halo_bytes > 0)
        for (int c = 0; c < nrhs; ++c)
            for (int t = 0; t < 2; ++t) L.halo[c][t] = take(L.halo_bytes);
    // refined solves: the single-precision correction of each right-hand side
    for (int c = 0; c < kMaxRhs; ++c)
        L.dh[c] = (precision == MAS_FP32_REFINED && c < nrhs) ? take_array(4 * s.n) : -1;
    L.total = cur.off;
    return L;
}

static int check_opts(const mas_op *op, const mas_pcg_opts *o) {
    if (!(o->rtol >= 0.0)) return fail(MAS_EINVAL, "rtol must be >= 0");
    if (o->max_iters < 0) return fail(MAS_EINVAL, "max_iters must be >= 0");
    if (o->check_every < 1) return fail(MAS_EINVAL, "check_every must be >= 1");
    if (o->precision != MAS_FP64 && o->precision != MAS_FP32_REFINED)
        return fail(MAS_EINVAL, "unknown precision %d", o->precision);
    if (o->precision == MAS_FP32_REFINED) {
        if (!op->c32[0])
            return fail(MAS_EINVAL, "operator was built without single-precision coefficients");
        if (!(o->inner_rtol > 0.0 && o->inner_rtol < 1.0))
            return fail(MAS_EINVAL, "inner_rtol must lie in (0, 1)");
        if (o->max_outer < 1) return fail(MAS_EINVAL, "max_outer must be >= 1");
        if (o->refine != MAS_REFINE_RESTART && o->refine != MAS_REFINE_RELIABLE)
            return fail(MAS_EINVAL, "unknown refinement strategy %d", o->refine);
    }
    if (o->max_restarts < 0) return fail(MAS_EINVAL, "max_restarts must be >= 0");
    if (o->chunk_planes < 0) return fail(MAS_EINVAL, "chunk_planes must be >= 0");
    if (o->precond != MAS_PC1 && o->precond != MAS_PC2)
        return fail(MAS_EINVAL, "unknown preconditioner %d", o->precond);
    if (o->launch != MAS_LAUNCH_AUTO && o->launch != MAS_LAUNCH_PER_ITERATION &&
        o->launch != MAS_LAUNCH_PERSISTENT)
        return fail(MAS_EINVAL, "unknown launch mode %d", o->launch);
    if (o->launch == MAS_LAUNCH_PERSISTENT && (o->precond != MAS_PC1 || o->sample_timing))
        return fail(MAS_EINVAL, "the persistent launch needs PC1 and no sample_timing");
    return MAS_OK;
}

extern "C" int64_t mas_pcg_workspace_bytes(const mas_op *op, const mas_pcg_opts *o) {
    if (!op) return fail(MAS_EINVAL, "op must not be NULL");
    mas_pcg_opts def;
    mas_pcg_default_opts(&def);
    if (!o) o = &def;
    return work_layout(op->s, o->precision).total;
}

extern "C" int64_t mas_pcg_multi_workspace_bytes(const mas_op *op, int32_t nrhs) {
    if (!op) return fail(MAS_EINVAL, "op must not be NULL");
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(MAS_EINVAL, "nrhs must lie in [1, %d]", kMaxRhs);
    // enough for either precision
    return std::max(work_layout(op->s, MAS_FP64, nrhs).total,
                    work_layout(op->s, MAS_FP32_REFINED, nrhs).total);
}

// ------------------------------------------------------------------ drivers
namespace {

struct Pinned {
    int32_t *p = nullptr;
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
};
static thread_local Pinned g_pinned;

static int pinned_buffer(int32_t **out) {
    if (!g_pinned.p) {
        void *p = nullptr;
        HIPCHK(hipHostMalloc(&p, 4096, hipHostMallocDefault));
        g_pinned.p = static_cast<int32_t *>(p);
    }
    *out = g_pinned.p;
    return MAS_OK;
}

struct Ctx {
    const mas_op *op;
    hipStream_t stream;
    Ctl *ctl;  // [nrhs]; ctl[0] also receives k_reduce sums
    double *partials;
    bool timing;
    bool no_alloc = false;  // allocation-free entry point: no pinned buffer, no events
    int chunk = 0;          // r planes per chunk of the iteration kernel (0: automatic)
    PersistSync *sync = nullptr;     // barrier words of the persistent launch
    int launch = MAS_LAUNCH_AUTO;    // requested launch mode of PC1 runs
    int launched = 0;                // mode of the last PC1 run (0: none yet)
    // event samples of the iteration kernel
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_iter;
    ~Ctx() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

// Host copy of control block c (synchronous).
static int read_ctl(Ctx &cx, Ctl *h, int c = 0) {
    HIPCHK(hipMemcpyAsync(h, cx.ctl + c, sizeof(Ctl), hipMemcpyDeviceToHost, cx.stream));
    HIPCHK(hipStreamSynchronize(cx.stream));
    return MAS_OK;
}

// Host polling of the run flags of control blocks ctl[0:n] after each batch
// of launches.  Normally one batch behind: the flags are copied into a pinned
// buffer behind the batch and the host waits for the previous batch's event,
// so the device queue never runs dry.  For the allocation-free entry point
// (no pinned buffer, no events) the flags are copied synchronously after
// each batch.
struct FlagPoll {
    Ctx &cx;
    int32_t *pin = nullptr;
    hipEvent_t done[2] = {nullptr, nullptr};
    int nb = 0;  // batches polled
    explicit FlagPoll(Ctx &c) : cx(c) {}
    ~FlagPoll() {
        for (auto e : done)
            if (e) (void)hipEventDestroy(e);
    }
    int init() {
        if (cx.no_alloc) return MAS_OK;
        int e = pinned_buffer(&pin);
        if (e != MAS_OK) return e;
        HIPCHK(hipEventCreateWithFlags(&done[0], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&done[1], hipEventDisableTiming));
        return MAS_OK;
    }
    // Call after enqueueing a batch; *stop becomes true once every flag seen
    // has left FLAG_RUN.
    int after_batch(int n, bool *stop) {
        if (cx.no_alloc) {
            int32_t fl[kMaxRhs];
            for (int h = 0; h < n; ++h)
                HIPCHK(hipMemcpyAsync(fl + h, &cx.ctl[h].flag, sizeof(int32_t),
                                      hipMemcpyDeviceToHost, cx.stream));
            HIPCHK(hipStreamSynchronize(cx.stream));
            bool any = false;
            for (int h = 0; h < n; ++h) any = any || fl[h] == FLAG_RUN;
            *stop = !any;
            ++nb;
            return MAS_OK;
        }
        int32_t *slot = pin + kMaxRhs * (nb & 1);
        for (int h = 0; h < n; ++h)
            HIPCHK(hipMemcpyAsync(slot + h, &cx.ctl[h].flag, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, cx.stream));
        HIPCHK(hipEventRecord(done[nb & 1], cx.stream));
        if (nb > 0) {
            HIPCHK(hipEventSynchronize(done[(nb - 1) & 1]));
            const int32_t *prev = pin + kMaxRhs * ((nb - 1) & 1);
            bool any = false;
            for (int h = 0; h < n; ++h) any = any || prev[h] == FLAG_RUN;
            if (!any) *stop = true;
        }
        ++nb;
        return MAS_OK;
    }
};

// Sum nv values of the simple-kernel partials into ctl->sums[0:nv] and
// copy them to the host (synchronous).
static int reduce_n(Ctx &cx, int nv, double *out, int nblk = -1) {
    if (nblk < 0) nblk = (int)cx.op->s.nblk_simple();
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, cx.stream, cx.partials, nblk, nv,
                       cx.ctl);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(out, &cx.ctl->sums[0], nv * sizeof(double), hipMemcpyDeviceToHost,
                          cx.stream));
    HIPCHK(hipStreamSynchronize(cx.stream));
    return MAS_OK;
}

// r^ = b^ - A^ x^ in double precision, stored as T into r.
// Returns rw2 = ||W r^||^2 = ||b - A x||^2 and rr2 = ||r^||^2.
template <typename T>
static int residual(Ctx &cx, const double *bhat, const double *xhat, T *r, double *rw2,
                    double *rr2 = nullptr) {
    const mas_op *op = cx.op;
    const Shape &s = op->s;
    ResArgs ra{bhat, xhat, op->w, op->c64[0], op->c64[1], op->c64[2], s.dims(), cx.partials,
               0, 0, 0, 0, 0};
    ra.tiles_k = (s.np + kReC - 1) / kReC;
    ra.tiles_j = (s.nt + kReR - 1) / kReR;
    ra.ti = s.chunk_for((int64_t)ra.tiles_k * ra.tiles_j);
    ra.tiles_i = (s.nr + ra.ti - 1) / ra.ti;
    const int64_t nblk = (int64_t)ra.tiles_i * ra.tiles_j * ra.tiles_k;
    // the partial-sum area of every workspace layout holds at least this
    if (nblk * 2 > std::max(s.nblk_iter_max() * kNV, s.nblk_simple() * kSimpleNV))
        return fail(MAS_EINVAL, "internal: partial-sum area too small for the residual");
    ra.nblk = (int)nblk;
    hipLaunchKernelGGL(k_residual<T>, dim3((unsigned)nblk), dim3(kReThreads), 0, cx.stream, ra, r);
    LAUNCHCHK();
    double sums[2];
    int st = reduce_n(cx, 2, sums, ra.nblk);
    *rw2 = sums[0];
    if (rr2) *rr2 = sums[1];
    return st;
}

// The vectors of the right-hand sides one PCG run carries, and which of them
// run (the others stay stopped and move no bytes).
template <typename T>
struct RhsSet {
    int n = 0;
    T *r[kMaxRhs][2], *p[kMaxRhs][2], *q[kMaxRhs][2];
    T *x[kMaxRhs];
    T *halo[kMaxRhs][2];    // segment-edge record buffers (null: not used)
    bool records = false;
    double tol2[kMaxRhs];
    int max_iter[kMaxRhs];  // last admissible iteration index of each
    bool active[kMaxRhs];
    // the first kernel of a run continues the search direction in
    // p[h][iter0 % 2] with p = r + beta0 p (keep_p), or starts with p = r
    bool keep_p[kMaxRhs] = {false, false, false, false};
    double beta0[kMaxRhs] = {0.0, 0.0, 0.0, 0.0};
};

struct PcgResult {
    int flag[kMaxRhs];
    int last_iter[kMaxRhs];  // index of the last iteration kernel that did work
};

constexpr int64_t kCatchupBlocks = 8192;  // grid-stride blocks of k_x_catchup

// The x update of a run's last launch when that launch left it to the next
// one (see k_pcg_iter); enqueued after every run.
template <typename T, int NR>
static int launch_catchup(Ctx &cx, const RhsSet<T> &v, int iter0) {
    CatchupArgs<T> ca{};
    for (int h = 0; h < NR; ++h) {
        ca.x[h] = v.x[h];
        ca.p[h][0] = v.p[h][0];
        ca.p[h][1] = v.p[h][1];
    }
    ca.ctl = cx.ctl;
    ca.n = cx.op->s.n;
    ca.iter0 = iter0;
    const int64_t cblk = std::min<int64_t>((cx.op->s.n + 255) / 256, kCatchupBlocks);
    hipLaunchKernelGGL(k_x_catchup<T>, dim3((unsigned)cblk, NR), dim3(256), 0, cx.stream, ca);
    LAUNCHCHK();
    return MAS_OK;
}

// Persistent launch (k_pcg_persist): the automatic choice takes it for
// grids of at most kPersistAutoCells cells (latency-bound: a launch per
// iteration costs about 14 us there whatever the size); unless chunk_planes
// is set, its r chunks are as long as it takes to have at most about
// kPersistBlocks blocks, since every block sums every block's partials and
// arrives at the barrier (at 32 x 32 x 64 cells: 64 blocks 13.5 us per
// iteration, 128 blocks 15.0 us, against 14.4 us launched per iteration).
// A block gives up waiting at a grid barrier after kPersistWaitSec seconds.
constexpr int64_t kPersistAutoCells = (int64_t)1 << 17;
constexpr int64_t kPersistBlocks = 64;
constexpr double kPersistWaitSec = 2.0;

// r planes per chunk of a persistent run (cx.chunk when set)
static int persist_chunk(const Ctx &cx, int V) {
    if (cx.chunk > 0) return cx.chunk;
    const Shape &s = cx.op->s;
    const int64_t tiles = (int64_t)s.tiles_k(V) * s.tiles_j();
    const int64_t want = (tiles * s.nr + kPersistBlocks - 1) / kPersistBlocks;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, s.nr));
}

template <typename T, int NR>
static const void *persist_kernel(int V) {
    constexpr int VW = vec_full<T>();
    return (V == VW) ? reinterpret_cast<const void *>(&k_pcg_persist<T, NR, kTJ, kRPW, VW>)
                     : reinterpret_cast<const void *>(&k_pcg_persist<T, NR, kTJ, kRPW, 1>);
}

// Whether a PC1 run of NR right-hand sides goes into one persistent launch
// (1) or a launch per iteration (0); MAS_EINVAL when the persistent launch
// was asked for and is not possible.
template <typename T, int NR>
static int persist_choice(Ctx &cx, const RhsSet<T> &v, int iter0) {
    if (cx.launch == MAS_LAUNCH_PER_ITERATION) return 0;
    const bool forced = cx.launch == MAS_LAUNCH_PERSISTENT;
    auto no = [&](const char *why) { return forced ? fail(MAS_EINVAL, "persistent launch: %s", why) : 0; };
    if (cx.timing) return no("sample_timing is set");
    const Shape &s = cx.op->s;
    if (!forced && s.n > kPersistAutoCells) return 0;
    const int V = iter_vec<T>(s.np, NR);
    const int64_t nblk = s.nblk_iter(V, persist_chunk(cx, V));
    int max_iter = iter0;
    for (int h = 0; h < NR; ++h) max_iter = std::max(max_iter, v.max_iter[h]);
    if ((int64_t)(max_iter - iter0 + 1) * nblk >= ((int64_t)1 << 32))
        return no("max_iters too large for the barrier counter");
    int dev = 0, coop = 0, ncu = 0, per_cu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return no("the device has no cooperative launch");
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel<T, NR>(V), kWave * kTJ, 0));
    if ((int64_t)per_cu * ncu < nblk) return no("the iteration kernel's blocks do not fit on the GPU at once");
    return 1;
}

// A PC1 run of NR right-hand sides in one cooperative launch of
// k_pcg_persist: the same control-block set-up, iterations, stopping and
// results as run_pcg's launches per iteration, bit for bit.
template <typename T, int NR>
static int run_pcg_persist(Ctx &cx, const RhsSet<T> &v, const T *const c[3], int mode, int iter0,
                           int check_every, PcgResult *res) {
    const mas_op *op = cx.op;
    const Shape &s = op->s;
    hipStream_t st = cx.stream;
    bool work = false;
    for (int h = 0; h < NR; ++h) {
        const double beta0 = v.keep_p[h] ? v.beta0[h] : 0.0;
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, cx.ctl + h, mode, iter0,
                           v.max_iter[h], v.tol2[h], beta0, v.active[h] ? FLAG_RUN : FLAG_CONV,
                           mode == 0 ? 1 : 0, check_every);
        work = work || (v.active[h] && v.max_iter[h] >= iter0);
    }
    hipLaunchKernelGGL(k_persist_init, dim3(1), dim3(64), 0, st, cx.sync);
    LAUNCHCHK();
    cx.launched = MAS_LAUNCH_PERSISTENT;
    if (work) {
        PersistArgs<T, NR> pa{};
        IterArgs<T> &a = pa.it;
        a.cr = c[0];
        a.ct = c[1];
        a.cp = c[2];
        a.w = op->w;
        a.ctl = cx.ctl;
        a.d = s.dims();
        const int V = iter_vec<T>(s.np, NR);
        const int ch = persist_chunk(cx, V);
        a.tiles_i = s.tiles_i(V, ch);
        a.tiles_k = s.tiles_k(V);
        a.tiles_j = s.tiles_j();
        a.ti = s.ti(V, ch);
        a.nblk = (int)s.nblk_iter(V, ch);
        a.records = 0;
        for (int h = 0; h < NR; ++h) {
            a.x[h] = v.x[h];
            for (int t = 0; t < 2; ++t) {
                pa.r[h][t] = v.r[h][t];
                pa.p[h][t] = v.p[h][t];
                pa.q[h][t] = v.q[h][t];
            }
            pa.keep_p[h] = v.keep_p[h] ? 1 : 0;
        }
        pa.partials[0] = cx.partials;
        pa.partials[1] = cx.partials + (int64_t)a.nblk * NR * kNV;
        pa.ctl = cx.ctl;
        pa.sync = cx.sync;
        pa.iter0 = iter0;
        int dev = 0, khz = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        pa.wait_ticks = (uint64_t)((double)khz * 1000.0 * kPersistWaitSec);
        void *args[] = {&pa};
        HIPCHK(hipLaunchCooperativeKernel(persist_kernel<T, NR>(V), dim3((unsigned)a.nblk),
                                          dim3(kWave * kTJ), args, 0, st));
    }
    int e = launch_catchup<T, NR>(cx, v, iter0);
    if (e != MAS_OK) return e;
    PersistSync hs{};
    HIPCHK(hipMemcpyAsync(&hs, cx.sync, sizeof hs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hs.err)
        return fail(MAS_EHIP, "persistent PCG run: a block waited more than %g s at a grid barrier",
                    kPersistWaitSec);
    for (int h = 0; h < NR; ++h) {
        Ctl hc;
        e = read_ctl(cx, &hc, h);
        if (e != MAS_OK) return e;
        res->flag[h] = hc.flag;
        res->last_iter[h] = (hc.flag == FLAG_RUN) ? v.max_iter[h] : hc.conv_iter;
    }
    return MAS_OK;
}

// PCG iterations on the scaled system in precision T for NR right-hand sides
// sharing the operator.  Before the call, r[c][iter0 % 2] holds r_{iter0} and
// x[c] holds x_{iter0}.  mode 0 stops on ||W r||^2 <= tol2 (checked on the
// iterations the finalize asks for), mode 1 on (r,r) <= tol2 (every
// iteration).  The first kernel uses alpha = 0 and beta = v.beta0[c]: with
// v.keep_p[c] it continues the search direction in p[c][iter0 % 2]
// (p = r + beta0 p), otherwise it starts afresh (p = r).  x is complete
// when it returns (k_x_catchup after the last launch).
template <typename T, int NR>
static int run_pcg(Ctx &cx, const RhsSet<T> &v, const T *const c[3], int mode, int iter0,
                   int check_every, PcgResult *res) {
    {
        const int pc = persist_choice<T, NR>(cx, v, iter0);
        if (pc < 0) return pc;
        if (pc == 1) return run_pcg_persist<T, NR>(cx, v, c, mode, iter0, check_every, res);
    }
    cx.launched = MAS_LAUNCH_PER_ITERATION;
    const mas_op *op = cx.op;
    const Shape &s = op->s;
    hipStream_t st = cx.stream;
    int max_iter = iter0;
    for (int h = 0; h < NR; ++h) {
        const double beta0 = v.keep_p[h] ? v.beta0[h] : 0.0;
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, cx.ctl + h, mode, iter0,
                           v.max_iter[h], v.tol2[h], beta0, v.active[h] ? FLAG_RUN : FLAG_CONV,
                           mode == 0 ? 1 : 0, check_every);
        if (v.active[h]) max_iter = std::max(max_iter, v.max_iter[h]);
    }
    LAUNCHCHK();
    FlagPoll poll(cx);
    int e = poll.init();
    if (e != MAS_OK) return e;

    IterArgs<T> a{};
    a.cr = c[0];
    a.ct = c[1];
    a.cp = c[2];
    a.w = op->w;
    a.partials = cx.partials;
    a.ctl = cx.ctl;
    a.d = s.dims();
    const int V = iter_vec<T>(s.np, NR);
    a.tiles_i = s.tiles_i(V, cx.chunk);
    a.tiles_k = s.tiles_k(V);
    a.tiles_j = s.tiles_j();
    a.ti = s.ti(V, cx.chunk);
    a.nblk = (int)s.nblk_iter(V, cx.chunk);
    for (int h = 0; h < NR; ++h) a.x[h] = v.x[h];
    a.records = v.records ? 1 : 0;
    const bool use_halo = v.records;
    const dim3 grid((unsigned)a.nblk), block(kWave * kTJ);

    // batches of launches; the host polls the device flags one batch behind
    const int batch = std::max(check_every, 16);
    int k = iter0;
    bool stop = false;
    while (!stop && k <= max_iter) {
        const int kend = std::min(max_iter, k + batch - 1);
        for (; k <= kend; ++k) {
            const int cur = k & 1, nxt = cur ^ 1;
            for (int h = 0; h < NR; ++h) {
                a.r_in[h] = v.r[h][cur];
                // the first kernel of a run has alpha = 0 (and beta = 0 unless
                // the direction is kept): point q (and p) at r, finite
                // values, so that every load stays unconditional
                a.p_in[h] = (k == iter0 && !v.keep_p[h]) ? v.r[h][cur] : v.p[h][cur];
                a.q_in[h] = (k == iter0) ? v.r[h][cur] : v.q[h][cur];
                a.r_out[h] = v.r[h][nxt];
                a.p_out[h] = v.p[h][nxt];
                a.q_out[h] = v.q[h][nxt];
                a.halo_in[h] = v.halo[h][cur];
                a.halo_out[h] = v.halo[h][nxt];
            }
            // the first kernel of a run reads its edge cells directly (no
            // kernel wrote records for its input); later ones read records
            const bool halo = use_halo && k != iter0;
            // x moves in the even launches of the run from the third on (the
            // first applies alpha = 0)
            a.xstep = (k - iter0 >= 2 && ((k - iter0) & 1) == 0) ? 1 : 0;
            // timing samples: 8 consecutive launches of every 16, so that
            // launches with and without the x update and the check launches
            // (every check_every-th) enter in their proportions
            const bool sample = cx.timing && ((k / 8) & 1) == 1 && cx.ev.size() < 512;
            if (sample) {
                hipEvent_t e0, e1;
                HIPCHK(hipEventCreate(&e0));
                HIPCHK(hipEventCreate(&e1));
                cx.ev.push_back(e0);
                cx.ev.push_back(e1);
                cx.ev_iter.push_back(k);
                HIPCHK(hipEventRecord(e0, st));
            }
            constexpr int VW = vec_full<T>();
            auto go = [&](auto vw, auto hl) {
                hipLaunchKernelGGL((k_pcg_iter<T, NR, kTJ, kRPW, decltype(vw)::value,
                                               decltype(hl)::value>),
                                   grid, block, 0, st, a);
            };
            using F = std::false_type;
            using Tr = std::true_type;
            using IW = std::integral_constant<int, VW>;
            using I1 = std::integral_constant<int, 1>;
            if (V == VW)
                halo ? go(IW{}, Tr{}) : go(IW{}, F{});
            else
                halo ? go(I1{}, Tr{}) : go(I1{}, F{});
            if (sample) HIPCHK(hipEventRecord(cx.ev.back(), st));
            hipLaunchKernelGGL(k_finalize, dim3(NR), dim3(kRedThreads), 0, st, cx.partials, a.nblk,
                               cx.ctl);
        }
        LAUNCHCHK();
        e = poll.after_batch(NR, &stop);
        if (e != MAS_OK) return e;
    }
    e = launch_catchup<T, NR>(cx, v, iter0);
    if (e != MAS_OK) return e;
    HIPCHK(hipStreamSynchronize(st));
    for (int h = 0; h < NR; ++h) {
        Ctl hc;
        e = read_ctl(cx, &hc, h);
        if (e != MAS_OK) return e;
        res->flag[h] = hc.flag;
        res->last_iter[h] = (hc.flag == FLAG_RUN) ? v.max_iter[h] : hc.conv_iter;
    }
    return MAS_OK;
}

static void timing_summary(Ctx &cx, int last_iter, mas_pcg_info *info) {
    double tot = 0.0;
    int n = 0;
    for (size_t t = 0; t < cx.ev_iter.size(); ++t) {
        if (cx.ev_iter[t] > last_iter) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, cx.ev[2 * t], cx.ev[2 * t + 1]) == hipSuccess) {
            tot += ms;
            ++n;
        }
    }
    if (n > 0) {
        // running mean over all solves of this call
        const double prev = info->iter_kernel_us * info->iter_kernel_samples;
        info->iter_kernel_samples += n;
        info->iter_kernel_us = (prev + 1000.0 * tot) / info->iter_kernel_samples;
    }
    for (auto ev : cx.ev) (void)hipEventDestroy(ev);
    cx.ev.clear();
    cx.ev_iter.clear();
}

static int status_from_flag(int flag) {
    switch (flag) {
        case FLAG_CONV: return MAS_OK;
        case FLAG_BREAK: return MAS_EBREAKDOWN;
        default: return MAS_ENOTCONV;
    }
}

// ------------------------------------------------------------------ PC2 driver
static int64_t pc2_blocks(const Shape &s, int *nbi, int *nbj, int *nbk) {
    *nbi = (s.nr + kPc2I - 1) / kPc2I;
    *nbj = (s.nt + kPc2J - 1) / kPc2J;
    *nbk = (s.np + kPc2K - 1) / kPc2K;
    return (int64_t)*nbi * *nbj * *nbk;
}

// PCG with the block-Jacobi ILU(0) preconditioner on the scaled system, from
// x (scaled) and r = b^ - A^ x already in r.  Iterations are counted from
// iter0; the run stops on ||W r||^2 <= tol2 (every iteration), at max_iter
// or on a breakdown.  The modified diagonal must already be in d.
// PC2 solve: rows of loads in flight ahead of the scan.  Measured at one
// fixed placement on the 256 x 320 x 640 grid: two rows 1.2% faster than one
// in double precision (2007 vs 2031 us per PC2 iteration), no gain in single
// precision.
#ifndef MAS_PC2_PF64
#define MAS_PC2_PF64 2
#endif
#ifndef MAS_PC2_PF32
#define MAS_PC2_PF32 1
#endif
template <typename T>
static constexpr int pc2_prefetch() {
    return std::is_same<T, float>::value ? MAS_PC2_PF32 : MAS_PC2_PF64;
}

template <typename T>
static int run_pcg_pc2(Ctx &cx, T *r, T *z, T *const p[2], T *q, T *d, T *x, int iter0,
                       int max_iter, double tol2, PcgResult *res) {
    const mas_op *op = cx.op;
    const Shape &s = op->s;
    hipStream_t st = cx.stream;
    int nbi, nbj, nbk;
    const int64_t nb = pc2_blocks(s, &nbi, &nbj, &nbk);
    const T *cc[3];
    if constexpr (std::is_same<T, float>::value) {
        for (int t = 0; t < 3; ++t) cc[t] = op->c32[t];
    } else {
        for (int t = 0; t < 3; ++t) cc[t] = op->c64[t];
    }
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, cx.ctl, 0, iter0, max_iter, tol2, 0.0,
                       (int)FLAG_RUN, 0, 1);
    Pc2Args<T> a{cc[0], cc[1], cc[2], op->w, d, r, x, z, q, nullptr, cx.partials,
                 cx.ctl, s.dims(), nbi, nbj, nbk, 0};
    // z = M^-1 r of the initial residual, (r, z), the stopping test
    hipLaunchKernelGGL((k_pc2_solve<T, pc2_prefetch<T>()>), dim3((unsigned)nb), dim3(kWave), 0, st, a);
    hipLaunchKernelGGL(k_pc2_fin_b, dim3(1), dim3(kRedThreads), 0, st, cx.partials, (int)nb, cx.ctl, 1);
    LAUNCHCHK();
    FlagPoll poll(cx);
    int e = poll.init();
    if (e != MAS_OK) return e;
    // the direction and SpMV step: the PCG iteration kernel with no r, q or
    // x (p = z + beta p, q = A^ p, partial (p, q) first of each block's kNV)
    IterArgs<T> it{};
    it.cr = cc[0];
    it.ct = cc[1];
    it.cp = cc[2];
    it.w = op->w;
    it.partials = cx.partials;
    it.ctl = cx.ctl;
    it.d = s.dims();
    const int V = iter_vec<T>(s.np, 1);
    it.tiles_i = s.tiles_i(V, cx.chunk);
    it.tiles_k = s.tiles_k(V);
    it.tiles_j = s.tiles_j();
    it.ti = s.ti(V, cx.chunk);
    it.nblk = (int)s.nblk_iter(V, cx.chunk);
    it.records = 0;
    constexpr int VW = vec_full<T>();
    const dim3 igrid((unsigned)it.nblk), iblock(kWave * kTJ);
    a.update = 1;
    int k = iter0;
    bool stop = false;
    while (!stop && k < max_iter) {
        const int kend = std::min(max_iter, k + 16);
        for (; k < kend; ++k) {
            // the first direction is z itself (beta = 0): p_old points at z
            const T *p_old = (k == iter0) ? z : p[k & 1];
            T *p_new = p[(k + 1) & 1];
            const bool sample = cx.timing && (k % 16 == 7) && cx.ev.size() < 128;
            if (sample) {
                hipEvent_t e0, e1;
                HIPCHK(hipEventCreate(&e0));
                HIPCHK(hipEventCreate(&e1));
                cx.ev.push_back(e0);
                cx.ev.push_back(e1);
                cx.ev_iter.push_back(k + 1);
                HIPCHK(hipEventRecord(e0, st));
            }
            it.r_in[0] = z;
            it.p_in[0] = p_old;
            it.p_out[0] = p_new;
            it.q_out[0] = q;
            if (V == VW)
                hipLaunchKernelGGL((k_pcg_iter<T, 1, kTJ, kRPW, VW, false>), igrid, iblock,
                                   0, st, it);
            else
                hipLaunchKernelGGL((k_pcg_iter<T, 1, kTJ, kRPW, 1, false>), igrid, iblock,
                                   0, st, it);
            hipLaunchKernelGGL(k_pc2_fin_a, dim3(1), dim3(kRedThreads), 0, st, cx.partials, it.nblk,
                               (int)kNV, cx.ctl);
            a.p = p_new;
            hipLaunchKernelGGL((k_pc2_solve<T, pc2_prefetch<T>()>), dim3((unsigned)nb), dim3(kWave), 0, st, a);
            hipLaunchKernelGGL(k_pc2_fin_b, dim3(1), dim3(kRedThreads), 0, st, cx.partials, (int)nb,
                               cx.ctl, 0);
            if (sample) HIPCHK(hipEventRecord(cx.ev.back(), st));
        }
        LAUNCHCHK();
        e = poll.after_batch(1, &stop);
        if (e != MAS_OK) return e;
    }
    HIPCHK(hipStreamSynchronize(st));
    Ctl h;
    e = read_ctl(cx, &h);
    if (e != MAS_OK) return e;
    res->flag[0] = h.flag;
    res->last_iter[0] = (h.flag == FLAG_RUN) ? max_iter : h.conv_iter;
    return MAS_OK;
}

// PC2-PCG for NR right-hand sides under one operator (FP64): per right-hand
// side its control block, r, z, p (two), q and x; the modified diagonal d and
// the couplings are shared.  The direction and SpMV step of all of them is
// one launch of the several-right-hand-side iteration kernel (couplings read
// once); the block solves and the finalize kernels run per right-hand side.
// Right-hand sides with active[h] false get a stopped control block and move
// no bytes.  All start at iteration iter0.
template <typename T, int NR>
static int run_pcg_pc2_multi(Ctx &cx, T *const r[NR], T *const z[NR], T *const p[NR][2],
                             T *const q[NR], const T *d, T *const x[NR], const bool active[NR],
                             const int max_iter[NR], const double tol2[NR], int iter0,
                             PcgResult *res) {
    const mas_op *op = cx.op;
    const Shape &s = op->s;
    hipStream_t st = cx.stream;
    int nbi, nbj, nbk;
    const int64_t nb = pc2_blocks(s, &nbi, &nbj, &nbk);
    for (int h = 0; h < NR; ++h)
        hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, cx.ctl + h, 0, iter0,
                           active[h] ? max_iter[h] : iter0, tol2[h], 0.0,
                           (int)(active[h] ? FLAG_RUN : FLAG_CONV), 0, 1);
    // the block solves of all right-hand sides in one launch (couplings, w
    // and d read once); right-hand side h's partials at partials + 2 h nb
    const T *cc[3];
    if constexpr (std::is_same<T, float>::value) {
        for (int t = 0; t < 3; ++t) cc[t] = op->c32[t];
    } else {
        for (int t = 0; t < 3; ++t) cc[t] = op->c64[t];
    }
    Pc2MultiArgs<T, NR> a{};
    a.cr = cc[0];
    a.ct = cc[1];
    a.cp = cc[2];
    a.w = op->w;
    a.d = d;
    for (int h = 0; h < NR; ++h) {
        a.r[h] = r[h];
        a.x[h] = x[h];
        a.z[h] = z[h];
        a.q[h] = q[h];
        a.p[h] = nullptr;
    }
    a.partials = cx.partials;
    a.ctl = cx.ctl;
    a.dm = s.dims();
    a.nbi = nbi;
    a.nbj = nbj;
    a.nbk = nbk;
    a.update = 0;
    auto solve_all = [&](int is_first) {
        hipLaunchKernelGGL((k_pc2_solve_multi<T, NR>), dim3((unsigned)nb), dim3(kWave), 0, st, a);
        for (int h = 0; h < NR; ++h)
            hipLaunchKernelGGL(k_pc2_fin_b, dim3(1), dim3(kRedThreads), 0, st,
                               cx.partials + 2 * h * nb, (int)nb, cx.ctl + h, is_first);
    };
    // z = M^-1 r of the initial residuals, (r, z), the stopping tests
    solve_all(1);
    a.update = 1;
    LAUNCHCHK();
    FlagPoll poll(cx);
    int e = poll.init();
    if (e != MAS_OK) return e;
    IterArgs<T> it{};
    it.cr = cc[0];
    it.ct = cc[1];
    it.cp = cc[2];
    it.w = op->w;
    it.partials = cx.partials;
    it.ctl = cx.ctl;
    it.d = s.dims();
    const int V = iter_vec<T>(s.np, NR);
    it.tiles_i = s.tiles_i(V, cx.chunk);
    it.tiles_k = s.tiles_k(V);
    it.tiles_j = s.tiles_j();
    it.ti = s.ti(V, cx.chunk);
    it.nblk = (int)s.nblk_iter(V, cx.chunk);
    it.records = 0;
    constexpr int VW = vec_full<T>();
    const dim3 igrid((unsigned)it.nblk), iblock(kWave * kTJ);
    int kmax = iter0;
    for (int h = 0; h < NR; ++h)
        if (active[h]) kmax = std::max(kmax, max_iter[h]);
    int k = iter0;
    bool stop = false;
    while (!stop && k < kmax) {
        const int kend = std::min(kmax, k + 16);
        for (; k < kend; ++k) {
            const bool sample = cx.timing && (k % 16 == 7) && cx.ev.size() < 128;
            if (sample) {
                hipEvent_t e0, e1;
                HIPCHK(hipEventCreate(&e0));
                HIPCHK(hipEventCreate(&e1));
                cx.ev.push_back(e0);
                cx.ev.push_back(e1);
                cx.ev_iter.push_back(k + 1);
                HIPCHK(hipEventRecord(e0, st));
            }
            for (int h = 0; h < NR; ++h) {
                // the first direction is z itself (beta = 0): p_old points at z
                it.r_in[h] = z[h];
                it.p_in[h] = (k == iter0) ? z[h] : p[h][k & 1];
                it.p_out[h] = p[h][(k + 1) & 1];
                it.q_out[h] = q[h];
            }
            if (V == VW)
                hipLaunchKernelGGL((k_pcg_iter<T, NR, kTJ, kRPW, VW, false>), igrid, iblock,
                                   0, st, it);
            else
                hipLaunchKernelGGL((k_pcg_iter<T, NR, kTJ, kRPW, 1, false>), igrid, iblock,
                                   0, st, it);
            for (int h = 0; h < NR; ++h)
                hipLaunchKernelGGL(k_pc2_fin_a, dim3(1), dim3(kRedThreads), 0, st,
                                   cx.partials + h * kNV, it.nblk, (int)(NR * kNV), cx.ctl + h);
            for (int h = 0; h < NR; ++h) a.p[h] = p[h][(k + 1) & 1];
            solve_all(0);
            if (sample) HIPCHK(hipEventRecord(cx.ev.back(), st));
        }
        LAUNCHCHK();
        e = poll.after_batch(NR, &stop);
        if (e != MAS_OK) return e;
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int h = 0; h < NR; ++h) {
        Ctl hc;
        e = read_ctl(cx, &hc, h);
        if (e != MAS_OK) return e;
        res->flag[h] = hc.flag;
        res->last_iter[h] = (hc.flag == FLAG_RUN) ? max_iter[h] : hc.conv_iter;
    }
    return MAS_OK;
}

// Record buffers of right-hand side h from the workspace layout.
template <typename T>
static void set_halo(RhsSet<T> &v, char *base, const WorkLayout &L, int h = 0) {
    v.records = L.halo_bytes > 0;
    for (int t = 0; t < 2; ++t)
        v.halo[h][t] = L.halo_bytes > 0 ? reinterpret_cast<T *>(base + L.halo[h][t]) : nullptr;
}

// Solve A x = b with b = V src (src_is_rhs) or b = src; result (unscaled) in x.
// no_alloc: the allocation-free entry point's call (no pinned buffer, no
// events; timing samples are refused).
static int solve_core(const mas_op *op, const double *src, int src_is_rhs, double *x,
                      const mas_pcg_opts *o_in, void *work, int64_t work_bytes, void *hip_stream,
                      mas_pcg_info *info_out, bool no_alloc = false) {
    const auto t0 = std::chrono::steady_clock::now();
    mas_pcg_info info{};
    mas_pcg_opts o;
    mas_pcg_default_opts(&o);
    if (o_in) o = *o_in;
    if (!op || !src || !x || !work)
        return fail(MAS_EINVAL, "op, right-hand side, solution and work must not be NULL");
    int st = check_opts(op, &o);
    if (st != MAS_OK) return st;
    if (no_alloc && o.sample_timing)
        return fail(MAS_EINVAL, "sample_timing needs HIP events: not available without allocation");
    if (reinterpret_cast<uintptr_t>(work) & 255)
        return fail(MAS_EINVAL, "work must be 256-byte aligned");
    const Shape &s = op->s;
    const WorkLayout L = work_layout(s, o.precision);
    if (work_bytes < L.total)
        return fail(MAS_ENOMEM, "workspace too small: %lld < %lld bytes", (long long)work_bytes,
                    (long long)L.total);

    if (std::max(s.nblk_iter_max() * kNV, s.nblk_simple() * kSimpleNV) * 8 >
        L.bhat[0] - L.partials)
        return fail(MAS_EINVAL, "internal: partial-sum area too small");
    char *base = static_cast<char *>(work);
    Ctx cx;
    cx.op = op;
    cx.stream = as_stream(hip_stream);
    cx.ctl = reinterpret_cast<Ctl *>(base + L.ctl);
    cx.partials = reinterpret_cast<double *>(base + L.partials);
    double *bhat = reinterpret_cast<double *>(base + L.bhat[0]);
    cx.timing = o.sample_timing != 0;
    cx.no_alloc = no_alloc;
    cx.chunk = o.chunk_planes;
    cx.sync = reinterpret_cast<PersistSync *>(base + L.sync);
    cx.launch = o.launch;
    const Dims d = s.dims();
    const dim3 sgrid = s.simple_grid(), sblock(kWave, kSimpleJ);

    // b^ = W^-1 b, x^ = W x0 or 0, ||b||^2; from x^ = 0 also r^0 = b^ (into
    // the first residual vector, in the working precision) and its norms
    const bool single = o.precision == MAS_FP32_REFINED;
    if (single)
        hipLaunchKernelGGL(k_setup<float>, sgrid, sblock, 0, cx.stream, src, src_is_rhs, op->w,
                           op->geo, d, bhat, x, o.use_x0 ? 1 : 0,
                           reinterpret_cast<float *>(base + L.vec[0][0]), cx.partials);
    else
        hipLaunchKernelGGL(k_setup<double>, sgrid, sblock, 0, cx.stream, src, src_is_rhs, op->w,
                           op->geo, d, bhat, x, o.use_x0 ? 1 : 0,
                           reinterpret_cast<double *>(base + L.vec[0][0]), cx.partials);
    LAUNCHCHK();
    double sums0[3] = {0.0, 0.0, 0.0};
    st = reduce_n(cx, 3, sums0);
    if (st != MAS_OK) return st;
    const double b2 = sums0[0];
    // r^0 into r (the first residual vector): already there from x^ = 0,
    // else b^ - A^ x^ by the residual kernel
    auto initial_residual = [&](auto *r, double *rw2, double *rr2) -> int {
        if (!o.use_x0) {
            *rw2 = sums0[1];
            if (rr2) *rr2 = sums0[2];
            return MAS_OK;
        }
        return residual(cx, bhat, x, r, rw2, rr2);
    };
    const double bnorm = std::sqrt(b2);
    info.bnorm = bnorm;
    if (!std::isfinite(bnorm)) return fail(MAS_EINVAL, "right-hand side is not finite");
    const double tol2 = (o.rtol * bnorm) * (o.rtol * bnorm);
    int status = MAS_OK;

    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_fill<double>, sgrid, sblock, 0, cx.stream, x, d, 0.0);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(cx.stream));
        info.status = MAS_OK;
        info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info_out) *info_out = info;
        return MAS_OK;
    }

    if (o.precond == MAS_PC2 && o.precision == MAS_FP32_REFINED) {
        // Single-precision PC2-PCG inside double-precision refinement: each
        // outer step solves A^ d = r^ (the double-precision residual, rounded)
        // from d = 0 until its recursive residual is inner_rtol below ||W r||
        // (or a quarter of the final tolerance), then x^ += d in double and
        // r^ = b^ - A^ x^ in double.  The factor is the double-precision one,
        // rounded.
        float *r = reinterpret_cast<float *>(base + L.vec[0][0]);
        float *z = reinterpret_cast<float *>(base + L.vec[0][1]);
        float *const p[2] = {reinterpret_cast<float *>(base + L.vec[0][2]),
                             reinterpret_cast<float *>(base + L.vec[0][3])};
        float *q = reinterpret_cast<float *>(base + L.vec[0][4]);
        float *dm = reinterpret_cast<float *>(base + L.vec[0][5]);
        float *dh = reinterpret_cast<float *>(base + L.dh[0]);
        int nbi, nbj, nbk;
        const int64_t nb = pc2_blocks(s, &nbi, &nbj, &nbk);
        if (nb * 2 * 8 > L.bhat[0] - L.partials || s.nblk_simple() * 8 > L.bhat[0] - L.partials)
            return fail(MAS_EINVAL, "internal: partial-sum area too small for PC2");
        if (nb > INT32_MAX) return fail(MAS_EINVAL, "grid too large for PC2");
        Pc2Args<double> fa{op->c64[0], op->c64[1], op->c64[2], op->w, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, nullptr, cx.ctl, d, nbi, nbj, nbk, 0};
        hipLaunchKernelGGL(k_pc2_factor<float>, dim3((unsigned)nb), dim3(kWave), 0, cx.stream, fa, dm);
        hipLaunchKernelGGL(k_fill<float>, sgrid, sblock, 0, cx.stream, dh, d, 0.0f);
        LAUNCHCHK();
        double rw2 = 0.0;
        st = initial_residual(r, &rw2, nullptr);
        if (st != MAS_OK) return st;
        info.rel_resid_true = info.rel_resid_recursive = std::sqrt(rw2) / bnorm;
        status = (rw2 <= tol2) ? MAS_OK : MAS_ENOTCONV;
        const double d2 = o.inner_rtol * o.inner_rtol;
        int used = 0;
        while (status != MAS_OK && info.outer_iters < o.max_outer && used < o.max_iters) {
            const double thr = std::max(d2 * rw2, 0.25 * tol2);
            PcgResult pr{};
            st = run_pcg_pc2<float>(cx, r, z, p, q, dm, dh, 0, o.max_iters - used, thr, &pr);
            if (st != MAS_OK) return st;
            timing_summary(cx, pr.last_iter[0], &info);
            used += pr.last_iter[0];
            info.outer_iters++;
            if (pr.flag[0] == FLAG_BREAK && pr.last_iter[0] == 0) {
                status = MAS_EBREAKDOWN;
                break;
            }
            Ctl h;
            st = read_ctl(cx, &h);
            if (st != MAS_OK) return st;
            info.rel_resid_recursive = std::sqrt(h.rw) / bnorm;
            hipLaunchKernelGGL(k_fold, sgrid, sblock, 0, cx.stream, dh, d, x);
            LAUNCHCHK();
            st = residual<float>(cx, bhat, x, r, &rw2);
            if (st != MAS_OK) return st;
            info.rel_resid_true = std::sqrt(rw2) / bnorm;
            if (rw2 <= tol2) status = MAS_OK;
        }
        info.iters = used;
    } else if (o.precond == MAS_PC2) {
        // vectors: r, z, p[2], q, and the modified diagonal
        double *r = reinterpret_cast<double *>(base + L.vec[0][0]);
        double *z = reinterpret_cast<double *>(base + L.vec[0][1]);
        double *const p[2] = {reinterpret_cast<double *>(base + L.vec[0][2]),
                              reinterpret_cast<double *>(base + L.vec[0][3])};
        double *q = reinterpret_cast<double *>(base + L.vec[0][4]);
        double *dm = reinterpret_cast<double *>(base + L.vec[0][5]);
        int nbi, nbj, nbk;
        const int64_t nb = pc2_blocks(s, &nbi, &nbj, &nbk);
        if (nb * 2 * 8 > L.bhat[0] - L.partials || s.nblk_simple() * 8 > L.bhat[0] - L.partials)
            return fail(MAS_EINVAL, "internal: partial-sum area too small for PC2");
        if (nb > INT32_MAX) return fail(MAS_EINVAL, "grid too large for PC2");
        Pc2Args<double> fa{op->c64[0], op->c64[1], op->c64[2], op->w, dm, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, cx.ctl, d, nbi, nbj, nbk, 0};
        hipLaunchKernelGGL(k_pc2_factor<double>, dim3((unsigned)nb), dim3(kWave), 0, cx.stream, fa, dm);
        LAUNCHCHK();
        double rw2 = 0.0;
        st = initial_residual(r, &rw2, nullptr);
        if (st != MAS_OK) return st;
        info.rel_resid_true = info.rel_resid_recursive = std::sqrt(rw2) / bnorm;
        status = (rw2 <= tol2) ? MAS_OK : MAS_ENOTCONV;
        int iter0 = 0;
        while (status != MAS_OK && iter0 < o.max_iters) {
            PcgResult pr{};
            st = run_pcg_pc2(cx, r, z, p, q, dm, x, iter0, o.max_iters, tol2, &pr);
            if (st != MAS_OK) return st;
            timing_summary(cx, pr.last_iter[0], &info);
            info.iters = pr.last_iter[0];
            Ctl h;
            st = read_ctl(cx, &h);
            if (st != MAS_OK) return st;
            info.rel_resid_recursive = std::sqrt(h.rw) / bnorm;
            st = residual<double>(cx, bhat, x, r, &rw2);
            if (st != MAS_OK) return st;
            info.rel_resid_true = std::sqrt(rw2) / bnorm;
            if (rw2 <= tol2) {
                status = MAS_OK;
                break;
            }
            if (pr.flag[0] == FLAG_BREAK) {
                status = MAS_EBREAKDOWN;
                break;
            }
            if (pr.flag[0] != FLAG_CONV || info.restarts >= o.max_restarts) {
                status = MAS_ENOTCONV;
                break;
            }
            ++info.restarts;
            iter0 = pr.last_iter[0];
        }
    } else if (o.precision == MAS_FP64) {
        RhsSet<double> v;
        v.n = 1;
        for (int t = 0; t < 2; ++t) {
            v.r[0][t] = reinterpret_cast<double *>(base + L.vec[0][t]);
            v.p[0][t] = reinterpret_cast<double *>(base + L.vec[0][2 + t]);
            v.q[0][t] = reinterpret_cast<double *>(base + L.vec[0][4 + t]);
        }
        v.x[0] = x;
        v.tol2[0] = tol2;
        v.max_iter[0] = o.max_iters;
        v.active[0] = true;
        set_halo(v, base, L);
        const double *const c[3] = {op->c64[0], op->c64[1], op->c64[2]};
        double rw2 = 0.0;
        st = initial_residual(v.r[0][0], &rw2, nullptr);
        if (st != MAS_OK) return st;
        info.rel_resid_true = info.rel_resid_recursive = std::sqrt(rw2) / bnorm;
        int iter0 = 0;
        status = MAS_ENOTCONV;
        if (rw2 <= tol2) status = MAS_OK;
        while (status != MAS_OK) {
            if (iter0 > o.max_iters) break;
            PcgResult pr{};
            st = run_pcg<double, 1>(cx, v, c, 0, iter0, o.check_every, &pr);
            if (st != MAS_OK) return st;
            timing_summary(cx, pr.last_iter[0], &info);
            info.iters = pr.last_iter[0];
            Ctl h;
            st = read_ctl(cx, &h);
            if (st != MAS_OK) return st;
            info.rel_resid_recursive = std::sqrt(h.rw) / bnorm;
            // true residual of x_k into the buffer the next iteration reads
            const int nxt = (pr.last_iter[0] + 1) & 1;
            st = residual<double>(cx, bhat, x, v.r[0][nxt], &rw2);
            if (st != MAS_OK) return st;
            info.rel_resid_true = std::sqrt(rw2) / bnorm;
            if (rw2 <= tol2) {
                status = MAS_OK;
                break;
            }
            if (pr.flag[0] == FLAG_BREAK) {
                status = MAS_EBREAKDOWN;
                break;
            }
            if (pr.flag[0] != FLAG_CONV || info.restarts >= o.max_restarts) {
                status = MAS_ENOTCONV;
                break;
            }
            ++info.restarts;
            iter0 = pr.last_iter[0] + 1;
        }
    } else {
        RhsSet<float> v;
        v.n = 1;
        for (int t = 0; t < 2; ++t) {
            v.r[0][t] = reinterpret_cast<float *>(base + L.vec[0][t]);
            v.p[0][t] = reinterpret_cast<float *>(base + L.vec[0][2 + t]);
            v.q[0][t] = reinterpret_cast<float *>(base + L.vec[0][4 + t]);
        }
        float *dh = reinterpret_cast<float *>(base + L.dh[0]);
        v.x[0] = dh;
        v.active[0] = true;
        set_halo(v, base, L);
        float *const *r = v.r[0];
        float *const *p = v.p[0];
        const float *const c[3] = {op->c32[0], op->c32[1], op->c32[2]};
        const bool reliable = o.refine == MAS_REFINE_RELIABLE;
        double rw2 = 0.0, rr2 = 0.0;
        st = initial_residual(r[0], &rw2, &rr2);
        if (st != MAS_OK) return st;
        info.rel_resid_true = std::sqrt(rw2) / bnorm;
        status = (rw2 <= tol2) ? MAS_OK : MAS_ENOTCONV;
        hipLaunchKernelGGL(k_fill<float>, sgrid, sblock, 0, cx.stream, dh, d, 0.0f);
        LAUNCHCHK();
        const double d2 = o.inner_rtol * o.inner_rtol;
        int k0 = 0;          // index of the next iteration kernel
        int used = 0;        // inner iterations taken
        double beta0 = 0.0;  // reliable: beta for the first kernel after a replacement
        while (status != MAS_OK && info.outer_iters < o.max_outer && used < o.max_iters) {
            // Inner stop on the single-precision recursive (scaled) residual:
            // a factor inner_rtol below the last double-precision residual, or
            // low enough that the unscaled residual it predicts meets the
            // tolerance (ratio ||W r||/||r|| taken at the last double-precision
            // residual), whichever comes first: the last step of either
            // strategy then stops near the tolerance instead of a factor
            // inner_rtol below the step before.
            double thr = d2 * rr2;
            if (rw2 > 0.0) thr = std::max(thr, 0.25 * tol2 * (rr2 / rw2));
            v.tol2[0] = thr;
            v.max_iter[0] = k0 + (o.max_iters - used);
            PcgResult pr{};
            v.keep_p[0] = reliable && beta0 > 0.0;
            v.beta0[0] = beta0;
            st = run_pcg<float, 1>(cx, v, c, 1, k0, 1, &pr);
            if (st != MAS_OK) return st;
            timing_summary(cx, pr.last_iter[0], &info);
            const int taken = pr.last_iter[0] - k0 + 1;  // iteration kernels that did work
            used += taken;
            info.outer_iters++;
            if (pr.flag[0] == FLAG_BREAK && taken == 0) {
                status = MAS_EBREAKDOWN;
                break;
            }
            Ctl h;
            st = read_ctl(cx, &h);
            if (st != MAS_OK) return st;
            const int nxt = (pr.last_iter[0] + 1) & 1;
            if (reliable) {
                // x^ += d^ + alpha_K p_K, then replace r by the double-precision
                // residual and continue from the same search direction p_K
                hipLaunchKernelGGL(k_refine_fold, sgrid, sblock, 0, cx.stream, dh, p[nxt], cx.ctl,
                                   d, x);
                LAUNCHCHK();
                const double rr_old = h.rr, rr_pred = h.rr_next;
                st = residual<float>(cx, bhat, x, r[nxt], &rw2, &rr2);
                if (st != MAS_OK) return st;
                // keep the direction only while the replaced residual agrees
                // with the one the recurrence predicted (no drift of the
                // single-precision residual); otherwise restart from r
                const bool keep = pr.flag[0] == FLAG_CONV && rr_old > 0.0 && rr_pred > 0.0 &&
                                  rr2 <= 4.0 * rr_pred;
                beta0 = keep ? rr2 / rr_old : 0.0;
                k0 = pr.last_iter[0] + 1;
            } else {
                // classical refinement: x^ += d^; the next inner solve restarts
                hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, cx.stream, cx.ctl, 1, 0, 0,
                                   0.0, 0.0, (int)FLAG_RUN, 0, 1);  // alpha = 0 for the fold
                hipLaunchKernelGGL(k_refine_fold, sgrid, sblock, 0, cx.stream, dh, p[nxt], cx.ctl,
                                   d, x);
                LAUNCHCHK();
                st = residual<float>(cx, bhat, x, r[0], &rw2, &rr2);
                if (st != MAS_OK) return st;
                k0 = 0;
            }
            info.rel_resid_true = std::sqrt(rw2) / bnorm;
            status = (rw2 <= tol2) ? MAS_OK : MAS_ENOTCONV;
            if (pr.flag[0] == FLAG_BREAK && status != MAS_OK && !reliable) {
                status = MAS_EBREAKDOWN;
                break;
            }
        }
        info.iters = used;
        info.rel_resid_recursive = info.rel_resid_true;
    }

    hipLaunchKernelGGL(k_unscale, sgrid, sblock, 0, cx.stream, op->w, d, x);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(cx.stream));
    info.status = status;
    info.launch = cx.launched;
    info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info_out) *info_out = info;
    if (status == MAS_ENOTCONV)
        fail(status, "tolerance not reached (relative residual %.3e)", info.rel_resid_true);
    if (status == MAS_EBREAKDOWN) fail(status, "PCG breakdown: (p, A p) <= 0 or not finite");
    return status;
}

// nrhs right-hand sides (contiguous, right-hand side h at rhs + h N) solved
// together in double precision: one iteration kernel carries all of them and
// each keeps its own CG scalars, stopping test and restarts.
template <int NR>
static int solve_multi_core(const mas_op *op, const double *rhs, double *x, const mas_pcg_opts &o,
                            char *base, const WorkLayout &L, hipStream_t stream,
                            mas_pcg_info *info) {
    const auto t0 = std::chrono::steady_clock::now();
    const Shape &s = op->s;
    const int64_t n = s.n;
    Ctx cx;
    cx.op = op;
    cx.stream = stream;
    cx.ctl = reinterpret_cast<Ctl *>(base + L.ctl);
    cx.partials = reinterpret_cast<double *>(base + L.partials);
    cx.timing = o.sample_timing != 0;
    cx.chunk = o.chunk_planes;
    cx.sync = reinterpret_cast<PersistSync *>(base + L.sync);
    cx.launch = o.launch;
    const Dims d = s.dims();
    const dim3 sgrid = s.simple_grid(), sblock(kWave, kSimpleJ);
    const double *const c[3] = {op->c64[0], op->c64[1], op->c64[2]};

    RhsSet<double> v;
    v.n = NR;
    double *bhat[NR];
    double bnorm[NR], rw2[NR];
    bool done[NR];
    int kernels[NR];  // iteration kernels that did work for each right-hand side
    for (int h = 0; h < NR; ++h) {
        info[h] = mas_pcg_info{};
        bhat[h] = reinterpret_cast<double *>(base + L.bhat[h]);
        for (int t = 0; t < 2; ++t) {
            v.r[h][t] = reinterpret_cast<double *>(base + L.vec[h][t]);
            v.p[h][t] = reinterpret_cast<double *>(base + L.vec[h][2 + t]);
            v.q[h][t] = reinterpret_cast<double *>(base + L.vec[h][4 + t]);
        }
        v.x[h] = x + h * n;
        kernels[h] = 0;
        set_halo(v, base, L, h);
        // b^ = W^-1 V rhs, x^ = W x0 or 0, ||b||^2 (and r^0 = b^ from x^ = 0)
        hipLaunchKernelGGL(k_setup<double>, sgrid, sblock, 0, stream, rhs + h * n, 1, op->w, op->geo,
                           d, bhat[h], v.x[h], o.use_x0 ? 1 : 0, v.r[h][0], cx.partials);
        LAUNCHCHK();
        double sums0[3] = {0.0, 0.0, 0.0};
        int st = reduce_n(cx, 3, sums0);
        if (st != MAS_OK) return st;
        const double b2 = sums0[0];
        bnorm[h] = std::sqrt(b2);
        info[h].bnorm = bnorm[h];
        if (!std::isfinite(bnorm[h]))
            return fail(MAS_EINVAL, "right-hand side %d is not finite", h);
        v.tol2[h] = (o.rtol * bnorm[h]) * (o.rtol * bnorm[h]);
        done[h] = false;
        info[h].status = MAS_ENOTCONV;
        if (bnorm[h] == 0.0) {
            hipLaunchKernelGGL(k_fill<double>, sgrid, sblock, 0, stream, v.x[h], d, 0.0);
            LAUNCHCHK();
            done[h] = true;
            info[h].status = MAS_OK;
            continue;
        }
        if (o.use_x0) {
            st = residual<double>(cx, bhat[h], v.x[h], v.r[h][0], &rw2[h]);
            if (st != MAS_OK) return st;
        } else {
            rw2[h] = sums0[1];
        }
        info[h].rel_resid_true = info[h].rel_resid_recursive = std::sqrt(rw2[h]) / bnorm[h];
        if (rw2[h] <= v.tol2[h]) {
            done[h] = true;
            info[h].status = MAS_OK;
        }
    }
    if (o.precond == MAS_PC2) {
        // vectors of right-hand side h: r, z, p (two), q; the shared modified
        // diagonal in right-hand side 0's sixth vector
        double *r[NR], *z[NR], *p[NR][2], *q[NR], *xs[NR];
        for (int h = 0; h < NR; ++h) {
            r[h] = reinterpret_cast<double *>(base + L.vec[h][0]);
            z[h] = reinterpret_cast<double *>(base + L.vec[h][1]);
            p[h][0] = reinterpret_cast<double *>(base + L.vec[h][2]);
            p[h][1] = reinterpret_cast<double *>(base + L.vec[h][3]);
            q[h] = reinterpret_cast<double *>(base + L.vec[h][4]);
            xs[h] = v.x[h];
        }
        double *dm = reinterpret_cast<double *>(base + L.vec[0][5]);
        int nbi, nbj, nbk;
        const int64_t nb = pc2_blocks(s, &nbi, &nbj, &nbk);
        if (NR * nb * 2 * 8 > L.bhat[0] - L.partials)
            return fail(MAS_EINVAL, "internal: partial-sum area too small for PC2");
        if (nb > INT32_MAX) return fail(MAS_EINVAL, "grid too large for PC2");
        Pc2Args<double> fa{op->c64[0], op->c64[1], op->c64[2], op->w, dm, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, cx.ctl, d, nbi, nbj, nbk, 0};
        hipLaunchKernelGGL(k_pc2_factor<double>, dim3((unsigned)nb), dim3(kWave), 0, stream, fa, dm);
        LAUNCHCHK();
        int iter0 = 0, restarts = 0;
        for (;;) {
            bool active[NR], any = false;
            int maxit[NR];
            for (int h = 0; h < NR; ++h) {
                active[h] = !done[h] && info[h].iters < o.max_iters;
                maxit[h] = iter0 + (o.max_iters - info[h].iters);
                any = any || active[h];
            }
            if (!any) break;
            PcgResult pr{};
            int st = run_pcg_pc2_multi<double, NR>(cx, r, z, p, q, dm, xs, active, maxit, v.tol2, iter0, &pr);
            if (st != MAS_OK) return st;
            int last = iter0;
            for (int h = 0; h < NR; ++h) {
                if (!active[h]) continue;
                last = std::max(last, pr.last_iter[h]);
                info[h].iters += pr.last_iter[h] - iter0;
                Ctl hc;
                st = read_ctl(cx, &hc, h);
                if (st != MAS_OK) return st;
                info[h].rel_resid_recursive = std::sqrt(hc.rw) / bnorm[h];
                st = residual<double>(cx, bhat[h], v.x[h], r[h], &rw2[h]);
                if (st != MAS_OK) return st;
                info[h].rel_resid_true = std::sqrt(rw2[h]) / bnorm[h];
                if (rw2[h] <= v.tol2[h]) {
                    done[h] = true;
                    info[h].status = MAS_OK;
                } else if (pr.flag[h] == FLAG_BREAK) {
                    done[h] = true;
                    info[h].status = MAS_EBREAKDOWN;
                } else if (pr.flag[h] != FLAG_CONV || restarts >= o.max_restarts) {
                    done[h] = true;
                    info[h].status = MAS_ENOTCONV;
                } else {
                    info[h].restarts++;
                }
            }
            mas_pcg_info tinfo{};
            timing_summary(cx, last, &tinfo);
            for (int h = 0; h < NR; ++h) {
                info[h].iter_kernel_us = tinfo.iter_kernel_us;
                info[h].iter_kernel_samples = tinfo.iter_kernel_samples;
            }
            ++restarts;
            iter0 = last;
        }
    }
    int iter0 = 0;
    int restarts = 0;
    for (; o.precond != MAS_PC2;) {
        bool any = false;
        // as in the single solve, at most max_iters + 1 iteration kernels
        // (the first of a run only forms q = A p) and iters = kernels - 1
        for (int h = 0; h < NR; ++h) {
            v.active[h] = !done[h] && kernels[h] <= o.max_iters;
            v.max_iter[h] = iter0 + (o.max_iters - kernels[h]);
            any = any || v.active[h];
        }
        if (!any) break;
        PcgResult pr{};
        int st = run_pcg<double, NR>(cx, v, c, 0, iter0, o.check_every, &pr);
        if (st != MAS_OK) return st;
        int last = iter0;
        for (int h = 0; h < NR; ++h)
            if (v.active[h]) last = std::max(last, pr.last_iter[h]);
        for (int h = 0; h < NR; ++h) {
            if (!v.active[h]) continue;
            kernels[h] += pr.last_iter[h] - iter0 + 1;
            info[h].iters = kernels[h] - 1;
            Ctl hc;
            st = read_ctl(cx, &hc, h);
            if (st != MAS_OK) return st;
            info[h].rel_resid_recursive = std::sqrt(hc.rw) / bnorm[h];
            // true residual of x_k into the buffer the next run starts from
            st = residual<double>(cx, bhat[h], v.x[h], v.r[h][(last + 1) & 1], &rw2[h]);
            if (st != MAS_OK) return st;
            info[h].rel_resid_true = std::sqrt(rw2[h]) / bnorm[h];
            if (rw2[h] <= v.tol2[h]) {
                done[h] = true;
                info[h].status = MAS_OK;
            } else if (pr.flag[h] == FLAG_BREAK) {
                done[h] = true;
                info[h].status = MAS_EBREAKDOWN;
            } else if (pr.flag[h] != FLAG_CONV || restarts >= o.max_restarts) {
                done[h] = true;
                info[h].status = MAS_ENOTCONV;
            } else {
                info[h].restarts++;
            }
        }
        // the sampled iteration kernels carried every right-hand side
        mas_pcg_info tinfo{};
        timing_summary(cx, last, &tinfo);
        for (int h = 0; h < NR; ++h) {
            const double prev = info[h].iter_kernel_us * info[h].iter_kernel_samples;
            info[h].iter_kernel_samples += tinfo.iter_kernel_samples;
            if (info[h].iter_kernel_samples > 0)
                info[h].iter_kernel_us =
                    (prev + tinfo.iter_kernel_us * tinfo.iter_kernel_samples) /
                    info[h].iter_kernel_samples;
        }
        ++restarts;
        iter0 = last + 1;
    }
    int status = MAS_OK;
    for (int h = 0; h < NR; ++h) {
        hipLaunchKernelGGL(k_unscale, sgrid, sblock, 0, stream, op->w, d, v.x[h]);
        LAUNCHCHK();
        if (info[h].status == MAS_EBREAKDOWN) status = MAS_EBREAKDOWN;
        else if (info[h].status == MAS_ENOTCONV && status == MAS_OK) status = MAS_ENOTCONV;
    }
    HIPCHK(hipStreamSynchronize(stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int h = 0; h < NR; ++h) {
        info[h].seconds = secs;
        info[h].launch = cx.launched;
    }
    return status;
}

// nrhs right-hand sides solved together by the single-precision PCG inside
// double-precision refinement (PC1 with either refinement strategy, or PC2
// restarted at each refinement step), as the single refined solve does for
// each of them: one iteration kernel (PC1), or one SpMV launch and one
// block-solve launch (PC2), carries every right-hand side whose refinement
// step is running; each keeps its own inner threshold, correction d^,
// double-precision residual, refinement count and status.
template <int NR>
static int solve_multi_refined(const mas_op *op, const double *rhs, double *x,
                               const mas_pcg_opts &o, char *base, const WorkLayout &L,
                               hipStream_t stream, mas_pcg_info *info) {
    const auto t0 = std::chrono::steady_clock::now();
    const Shape &s = op->s;
    const int64_t n = s.n;
    Ctx cx;
    cx.op = op;
    cx.stream = stream;
    cx.ctl = reinterpret_cast<Ctl *>(base + L.ctl);
    cx.partials = reinterpret_cast<double *>(base + L.partials);
    cx.timing = o.sample_timing != 0;
    cx.chunk = o.chunk_planes;
    cx.sync = reinterpret_cast<PersistSync *>(base + L.sync);
    cx.launch = o.launch;
    const Dims d = s.dims();
    const dim3 sgrid = s.simple_grid(), sblock(kWave, kSimpleJ);
    const float *const c32[3] = {op->c32[0], op->c32[1], op->c32[2]};
    const bool pc2 = o.precond == MAS_PC2;
    const bool reliable = !pc2 && o.refine == MAS_REFINE_RELIABLE;

    RhsSet<float> v;
    v.n = NR;
    double *bhat[NR], *xh[NR];
    float *dh[NR];
    double bnorm[NR], tol2[NR], rw2[NR], rr2[NR];
    bool done[NR];
    int used[NR];
    for (int h = 0; h < NR; ++h) {
        info[h] = mas_pcg_info{};
        bhat[h] = reinterpret_cast<double *>(base + L.bhat[h]);
        dh[h] = reinterpret_cast<float *>(base + L.dh[h]);
        xh[h] = x + h * n;
        for (int t = 0; t < 2; ++t) {
            v.r[h][t] = reinterpret_cast<float *>(base + L.vec[h][t]);
            v.p[h][t] = reinterpret_cast<float *>(base + L.vec[h][2 + t]);
            v.q[h][t] = reinterpret_cast<float *>(base + L.vec[h][4 + t]);
        }
        v.x[h] = dh[h];
        set_halo(v, base, L, h);
        used[h] = 0;
        // b^, x^ (and r^0 = b^ from x^ = 0), ||b||^2
        hipLaunchKernelGGL(k_setup<float>, sgrid, sblock, 0, stream, rhs + h * n, 1, op->w, op->geo,
                           d, bhat[h], xh[h], o.use_x0 ? 1 : 0, v.r[h][0], cx.partials);
        LAUNCHCHK();
        double sums0[3] = {0.0, 0.0, 0.0};
        int st = reduce_n(cx, 3, sums0);
        if (st != MAS_OK) return st;
        bnorm[h] = std::sqrt(sums0[0]);
        info[h].bnorm = bnorm[h];
        if (!std::isfinite(bnorm[h]))
            return fail(MAS_EINVAL, "right-hand side %d is not finite", h);
        tol2[h] = (o.rtol * bnorm[h]) * (o.rtol * bnorm[h]);
        done[h] = false;
        info[h].status = MAS_ENOTCONV;
        if (bnorm[h] == 0.0) {
            hipLaunchKernelGGL(k_fill<double>, sgrid, sblock, 0, stream, xh[h], d, 0.0);
            LAUNCHCHK();
            done[h] = true;
            info[h].status = MAS_OK;
            continue;
        }
        if (o.use_x0) {
            st = residual<float>(cx, bhat[h], xh[h], v.r[h][0], &rw2[h], &rr2[h]);
            if (st != MAS_OK) return st;
        } else {
            rw2[h] = sums0[1];
            rr2[h] = sums0[2];
        }
        hipLaunchKernelGGL(k_fill<float>, sgrid, sblock, 0, stream, dh[h], d, 0.0f);
        LAUNCHCHK();
        info[h].rel_resid_true = info[h].rel_resid_recursive = std::sqrt(rw2[h]) / bnorm[h];
        if (rw2[h] <= tol2[h]) {
            done[h] = true;
            info[h].status = MAS_OK;
        }
    }

    // PC2: the factor once, the double-precision one rounded; r, z, p (two)
    // and q of right-hand side h in its first five vectors, the modified
    // diagonal in right-hand side 0's sixth
    float *dm = reinterpret_cast<float *>(base + L.vec[0][5]);
    float *pr_[NR], *pz_[NR], *pp_[NR][2], *pq_[NR];
    if (pc2) {
        for (int h = 0; h < NR; ++h) {
            pr_[h] = v.r[h][0];
            pz_[h] = v.r[h][1];
            pp_[h][0] = v.p[h][0];
            pp_[h][1] = v.p[h][1];
            pq_[h] = v.q[h][0];
        }
        int nbi, nbj, nbk;
        const int64_t nb = pc2_blocks(s, &nbi, &nbj, &nbk);
        if (NR * nb * 2 * 8 > L.bhat[0] - L.partials)
            return fail(MAS_EINVAL, "internal: partial-sum area too small for PC2");
        if (nb > INT32_MAX) return fail(MAS_EINVAL, "grid too large for PC2");
        Pc2Args<double> fa{op->c64[0], op->c64[1], op->c64[2], op->w, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, nullptr, cx.ctl, d, nbi, nbj, nbk, 0};
        hipLaunchKernelGGL(k_pc2_factor<float>, dim3((unsigned)nb), dim3(kWave), 0, stream, fa, dm);
        LAUNCHCHK();
    }

    const double d2 = o.inner_rtol * o.inner_rtol;
    for (;;) {
        bool active[NR], any = false;
        int maxit[NR];
        double thr[NR];
        for (int h = 0; h < NR; ++h) {
            active[h] = !done[h] && info[h].outer_iters < o.max_outer && used[h] < o.max_iters;
            any = any || active[h];
            // inner stop: inner_rtol below the last double-precision residual,
            // or low enough that the unscaled residual it predicts meets the
            // tolerance
            if (pc2) {
                thr[h] = std::max(d2 * rw2[h], 0.25 * tol2[h]);
                maxit[h] = o.max_iters - used[h];
            } else {
                thr[h] = d2 * rr2[h];
                if (rw2[h] > 0.0) thr[h] = std::max(thr[h], 0.25 * tol2[h] * (rr2[h] / rw2[h]));
                maxit[h] = o.max_iters - used[h];
            }
            v.tol2[h] = thr[h];
            v.max_iter[h] = maxit[h];
            v.active[h] = active[h];
        }
        if (!any) break;
        PcgResult pr{};
        int st = pc2 ? run_pcg_pc2_multi<float, NR>(cx, pr_, pz_, pp_, pq_, dm, dh, active, maxit,
                                                    thr, 0, &pr)
                     : run_pcg<float, NR>(cx, v, c32, 1, 0, 1, &pr);
        if (st != MAS_OK) return st;
        int last = 0;
        for (int h = 0; h < NR; ++h)
            if (active[h]) last = std::max(last, pr.last_iter[h]);
        mas_pcg_info tinfo{};
        timing_summary(cx, last, &tinfo);
        for (int h = 0; h < NR; ++h) {
            if (!active[h]) continue;
            if (tinfo.iter_kernel_samples > 0) {
                const double prev = info[h].iter_kernel_us * info[h].iter_kernel_samples;
                info[h].iter_kernel_samples += tinfo.iter_kernel_samples;
                info[h].iter_kernel_us = (prev + tinfo.iter_kernel_us * tinfo.iter_kernel_samples) /
                                         info[h].iter_kernel_samples;
            }
            // PC1 counts iteration kernels (the first of a run forms q only);
            // PC2 counts finished iterations
            const int taken = pc2 ? pr.last_iter[h] : pr.last_iter[h] + 1;
            used[h] += taken;
            info[h].outer_iters++;
            if (pr.flag[h] == FLAG_BREAK && taken == 0) {
                done[h] = true;
                info[h].status = MAS_EBREAKDOWN;
                continue;
            }
            Ctl hc;
            st = read_ctl(cx, &hc, h);
            if (st != MAS_OK) return st;
            if (pc2) {
                info[h].rel_resid_recursive = std::sqrt(hc.rw) / bnorm[h];
                hipLaunchKernelGGL(k_fold, sgrid, sblock, 0, stream, dh[h], d, xh[h]);
                LAUNCHCHK();
                st = residual<float>(cx, bhat[h], xh[h], pr_[h], &rw2[h]);
                if (st != MAS_OK) return st;
            } else if (reliable) {
                // x^ += d^ + alpha_K p_K, then the double-precision residual
                // replaces r and the run continues from the direction p_K
                const int nxt = (pr.last_iter[h] + 1) & 1;
                hipLaunchKernelGGL(k_refine_fold, sgrid, sblock, 0, stream, dh[h], v.p[h][nxt],
                                   cx.ctl + h, d, xh[h]);
                LAUNCHCHK();
                const double rr_old = hc.rr, rr_pred = hc.rr_next;
                st = residual<float>(cx, bhat[h], xh[h], v.r[h][nxt], &rw2[h], &rr2[h]);
                if (st != MAS_OK) return st;
                const bool keep = pr.flag[h] == FLAG_CONV && rr_old > 0.0 && rr_pred > 0.0 &&
                                  rr2[h] <= 4.0 * rr_pred;
                v.keep_p[h] = keep;
                v.beta0[h] = keep ? rr2[h] / rr_old : 0.0;
                // the next run starts at iteration 0: its vectors in slot 0
                if (nxt == 1) {
                    std::swap(v.r[h][0], v.r[h][1]);
                    std::swap(v.p[h][0], v.p[h][1]);
                    std::swap(v.q[h][0], v.q[h][1]);
                }
            } else {
                // classical refinement: x^ += d^; the next inner solve restarts
                hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, stream, cx.ctl + h, 1, 0, 0,
                                   0.0, 0.0, (int)FLAG_RUN, 0, 1);  // alpha = 0 for the fold
                hipLaunchKernelGGL(k_refine_fold, sgrid, sblock, 0, stream, dh[h], v.p[h][0],
                                   cx.ctl + h, d, xh[h]);
                LAUNCHCHK();
                st = residual<float>(cx, bhat[h], xh[h], v.r[h][0], &rw2[h], &rr2[h]);
                if (st != MAS_OK) return st;
                v.keep_p[h] = false;
                v.beta0[h] = 0.0;
            }
            info[h].rel_resid_true = std::sqrt(rw2[h]) / bnorm[h];
            if (!pc2) info[h].rel_resid_recursive = info[h].rel_resid_true;
            if (rw2[h] <= tol2[h]) {
                done[h] = true;
                info[h].status = MAS_OK;
            } else if (pr.flag[h] == FLAG_BREAK && !reliable) {
                done[h] = true;
                info[h].status = MAS_EBREAKDOWN;
            }
        }
    }
    int status = MAS_OK;
    for (int h = 0; h < NR; ++h) {
        info[h].iters = used[h];
        hipLaunchKernelGGL(k_unscale, sgrid, sblock, 0, stream, op->w, d, xh[h]);
        LAUNCHCHK();
        if (info[h].status == MAS_EBREAKDOWN) status = MAS_EBREAKDOWN;
        else if (info[h].status == MAS_ENOTCONV && status == MAS_OK) status = MAS_ENOTCONV;
    }
    HIPCHK(hipStreamSynchronize(stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int h = 0; h < NR; ++h) {
        info[h].seconds = secs;
        info[h].launch = cx.launched;
    }
    return status;
}

}  // namespace

extern "C" int mas_pcg_solve(const mas_op *op, const double *rhs, double *x, const mas_pcg_opts *o,
                             void *work, int64_t work_bytes, void *hip_stream, mas_pcg_info *info) {
    g_last_error.clear();
    return solve_core(op, rhs, 1, x, o, work, work_bytes, hip_stream, info);
}

// ------------------------------------------------------------------ allocation-free solve
// The workspace of mas_pcg_solve_noalloc: a static device array, one copy per
// GPU, kept until the process ends.  Host code never uses the array's name
// as an address (on the host it is only a stand-in for the symbol): the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current.
static __device__ __align__(256) unsigned char scratch[MAS_NOALLOC_WORK_BYTES];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static int scratch_of_current_device(void **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MAS_EINVAL, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MAS_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MAS_OK;
}

extern "C" int mas_pcg_solve_noalloc(const mas_op *op, const double *rhs, double *x,
                                     const mas_pcg_opts *o, void *hip_stream, mas_pcg_info *info) {
    g_last_error.clear();
    if (!op) return fail(MAS_EINVAL, "op must not be NULL");
    mas_pcg_opts def;
    mas_pcg_default_opts(&def);
    const mas_pcg_opts *oo = o ? o : &def;
    int st = check_opts(op, oo);
    if (st != MAS_OK) return st;
    const int64_t need = work_layout(op->s, oo->precision).total;
    if (need > (int64_t)MAS_NOALLOC_WORK_BYTES)
        return fail(MAS_ENOMEM, "grid too large for the allocation-free solve: workspace %lld > %lld bytes",
                    (long long)need, (long long)MAS_NOALLOC_WORK_BYTES);
    void *work = nullptr;
    st = scratch_of_current_device(&work);
    if (st != MAS_OK) return st;
    return solve_core(op, rhs, 1, x, oo, work, (int64_t)MAS_NOALLOC_WORK_BYTES, hip_stream, info,
                      true);
}

extern "C" int mas_pcg_solve_multi(const mas_op *op, int32_t nrhs, const double *rhs, double *x,
                                   const mas_pcg_opts *o_in, void *work, int64_t work_bytes,
                                   void *hip_stream, mas_pcg_info *info) {
    g_last_error.clear();
    if (!op || !rhs || !x || !work)
        return fail(MAS_EINVAL, "op, rhs, x and work must not be NULL");
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(MAS_EINVAL, "nrhs must lie in [1, %d]", kMaxRhs);
    mas_pcg_opts o;
    mas_pcg_default_opts(&o);
    if (o_in) o = *o_in;
    int st = check_opts(op, &o);
    if (st != MAS_OK) return st;
    if (reinterpret_cast<uintptr_t>(work) & 255)
        return fail(MAS_EINVAL, "work must be 256-byte aligned");
    const WorkLayout L = work_layout(op->s, o.precision, nrhs);
    if (work_bytes < L.total)
        return fail(MAS_ENOMEM, "workspace too small: %lld < %lld bytes", (long long)work_bytes,
                    (long long)L.total);
    mas_pcg_info local[kMaxRhs];
    char *base = static_cast<char *>(work);
    hipStream_t stream = as_stream(hip_stream);
    if (o.precision == MAS_FP32_REFINED) {
        switch (nrhs) {
            case 1: st = solve_multi_refined<1>(op, rhs, x, o, base, L, stream, local); break;
            case 2: st = solve_multi_refined<2>(op, rhs, x, o, base, L, stream, local); break;
            case 3: st = solve_multi_refined<3>(op, rhs, x, o, base, L, stream, local); break;
            default: st = solve_multi_refined<4>(op, rhs, x, o, base, L, stream, local); break;
        }
    } else {
        switch (nrhs) {
            case 1: st = solve_multi_core<1>(op, rhs, x, o, base, L, stream, local); break;
            case 2: st = solve_multi_core<2>(op, rhs, x, o, base, L, stream, local); break;
            case 3: st = solve_multi_core<3>(op, rhs, x, o, base, L, stream, local); break;
            default: st = solve_multi_core<4>(op, rhs, x, o, base, L, stream, local); break;
        }
    }
    if (info)
        for (int h = 0; h < nrhs; ++h) info[h] = local[h];
    if (st == MAS_ENOTCONV) fail(st, "tolerance not reached for at least one right-hand side");
    if (st == MAS_EBREAKDOWN) fail(st, "PCG breakdown in at least one right-hand side");
    return st;
}

namespace {
struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    int make(hipEvent_t *out) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ev.push_back(e);
        *out = e;
        return MAS_OK;
    }
};
}  // namespace

// The gradient kernel over the whole grid (one launch).
static int gradient_launch(const mas_op *op, const double *x, const double *lambda, double *g_nu,
                           double *g_rhs, hipStream_t stream) {
    const Shape &s = op->s;
    const int64_t tiles_k = (s.np + kGrC - 1) / kGrC;
    const int64_t tiles_j = (s.nt + kGrR - 1) / kGrR;
    const int ti = s.chunk_for(tiles_k * tiles_j);
    const int64_t tiles_i = (s.nr + ti - 1) / ti;
    const int64_t nblk = tiles_i * tiles_k * tiles_j;
    if (nblk > INT32_MAX) return fail(MAS_EINVAL, "grid too large for the gradient kernel");
    GradArgs ga{x, lambda, g_nu, g_rhs, op->geo, s.dims(), (int)tiles_i, (int)tiles_k, (int)tiles_j,
                ti, (int)nblk};
    hipLaunchKernelGGL(k_gradient, dim3((unsigned)nblk), dim3(kGrThreads), 0, stream, ga);
    LAUNCHCHK();
    return MAS_OK;
}

extern "C" int mas_pcg_solve_adjoint(const mas_op *op, const double *x, const double *gx,
                                     double *lambda, double *g_nu, double *g_rhs,
                                     const mas_pcg_opts *o, void *work, int64_t work_bytes,
                                     void *hip_stream, mas_pcg_info *info) {
    g_last_error.clear();
    if (!op || !x || !gx || !lambda || !g_nu)
        return fail(MAS_EINVAL, "op, x, gx, lambda and g_nu must not be NULL");
    int st = solve_core(op, gx, 0, lambda, o, work, work_bytes, hip_stream, info);
    if (st < 0) return st;
    hipStream_t stream = as_stream(hip_stream);
    const bool timing = o && o->sample_timing;
    EventPool pool;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st2;
    if (timing) {
        if ((st2 = pool.make(&e0)) != MAS_OK || (st2 = pool.make(&e1)) != MAS_OK) return st2;
        HIPCHK(hipEventRecord(e0, stream));
    }
    st2 = gradient_launch(op, x, lambda, g_nu, g_rhs, stream);
    if (st2 != MAS_OK) return st2;
    if (timing) HIPCHK(hipEventRecord(e1, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (timing && info) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        info->grad_kernel_us = 1e3 * (double)ms;
    }
    return st;
}

// ------------------------------------------------------------------ RKL2 super time-stepping
#ifndef MAS_STS_WPB
#define MAS_STS_WPB 4
#endif
#ifndef MAS_STS_RPW
#define MAS_STS_RPW 2
#endif
#ifndef MAS_STS_TI
#define MAS_STS_TI 16
#endif
#ifndef MAS_PAIR_NW
#define MAS_PAIR_NW 10
#endif
#ifndef MAS_PAIR_TI
#define MAS_PAIR_TI 32
#endif
static constexpr int kStsWPB = MAS_STS_WPB, kStsRPW = MAS_STS_RPW, kStsTI = MAS_STS_TI;
#ifndef MAS_PAIR_SLAB
#define MAS_PAIR_SLAB 1
#endif
static constexpr int kPairNW = MAS_PAIR_NW, kPairTI = MAS_PAIR_TI;
static_assert(kPairTI >= 1 && kPairTI <= kPairMaxTI, "r planes per chunk of the two-stage kernel");
static constexpr int kStsMaxStages = 1000000;

// Smallest s >= 2 whose stability interval [-(s^2 + s - 2)/2, 0] holds
// [-zmax, 0]; -1 when that needs more than kStsMaxStages.
static int sts_stages_for(double zmax) {
    if (!(zmax <= 0.5 * ((double)kStsMaxStages * kStsMaxStages + kStsMaxStages - 2.0))) return -1;
    auto covers = [&](int s) { return 0.5 * ((double)s * s + s - 2.0) >= zmax; };
    int s = std::max(2, (int)std::ceil(0.5 * (-1.0 + std::sqrt(9.0 + 8.0 * std::max(zmax, 0.0)))));
    while (!covers(s)) ++s;
    while (s > 2 && covers(s - 1)) --s;
    return s;
}

// Coefficients of the s-stage RKL2 recursion (Meyer, Balsara and Aslam,
// 2014), index j = 0..s:
//   w1 = 4/(s^2+s-2), b_0 = b_1 = b_2 = 1/3, b_j = (j^2+j-2)/(2j(j+1)),
//   mt_1 = b_1 w1, and for j >= 2
//   mu_j = (2j-1)/j b_j/b_{j-1}, nu_j = -(j-1)/j b_j/b_{j-2},
//   mt_j = mu_j w1, gt_j = -(1 - b_{j-1}) mt_j.
struct Rkl2 {
    std::vector<double> mu, nu, mt, gt;
};

static Rkl2 rkl2_coefficients(int s) {
    Rkl2 c;
    c.mu.assign(s + 1, 0.0);
    c.nu.assign(s + 1, 0.0);
    c.mt.assign(s + 1, 0.0);
    c.gt.assign(s + 1, 0.0);
    std::vector<double> b(s + 1);
    for (int j = 0; j <= s; ++j)
        b[j] = (j < 3) ? 1.0 / 3.0 : ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
    const double w1 = 4.0 / ((double)s * s + s - 2.0);
    c.mt[1] = b[1] * w1;
    for (int j = 2; j <= s; ++j) {
        c.mu[j] = (2.0 * j - 1.0) / j * b[j] / b[j - 1];
        c.nu[j] = -(j - 1.0) / j * b[j] / b[j - 2];
        c.mt[j] = c.mu[j] * w1;
        c.gt[j] = -(1.0 - b[j - 1]) * c.mt[j];
    }
    return c;
}

// L_0 and four stage arrays: the two-stage kernel writes D_j, D_{j+1} to a
// pair of arrays other than the pair it reads.
struct StsWork {
    int64_t vec[5], total;
};

static StsWork sts_work_layout(const Shape &s) {
    StsWork L{};
    LayoutCursor cur(kPhaseSts);
    for (int t = 0; t < 5; ++t) L.vec[t] = cur.take_array(8 * s.n);
    L.total = cur.off;
    return L;
}

extern "C" void mas_sts_default_opts(mas_sts_opts *o) {
    if (!o) return;
    o->stages = 0;
    o->sample_timing = 0;
    o->single_stage_kernels = 0;
    o->pad_ = 0;
}

extern "C" int32_t mas_sts_stages(const mas_op *op) {
    if (!op) return fail(MAS_EINVAL, "op must not be NULL");
    const int s = sts_stages_for(op->zmax);
    if (s < 0) return fail(MAS_EINVAL, "dt needs more than %d explicit stages", kStsMaxStages);
    return s;
}

extern "C" int64_t mas_sts_workspace_bytes(const mas_op *op) {
    if (!op) return fail(MAS_EINVAL, "op must not be NULL");
    return sts_work_layout(op->s).total;
}

// One stage kernel: out = a X + b Z + g L0 + Y0 + m dtL(X).
static int sts_launch(const mas_op *op, hipStream_t stream, const double *X, const double *Z,
                      const double *L0, const double *Y0, double *out, double a, double b,
                      double g, double m) {
    const Shape &s = op->s;
    const int v = (s.np % 2 == 0) ? 2 : 1;
    const int seg = (kWave / kStsRPW) * v;
    const int ti = std::min(kStsTI, s.max_chunk());
    const int64_t tiles_i = (s.nr + ti - 1) / ti;
    const int64_t tiles_k = (s.np + seg - 1) / seg;
    const int64_t tiles_j = (s.nt + kStsWPB * kStsRPW - 1) / (kStsWPB * kStsRPW);
    const int64_t nblk = tiles_i * tiles_k * tiles_j;
    if (nblk > INT32_MAX) return fail(MAS_EINVAL, "grid too large for the stage kernel");
    StsArgs args{X, op->nu, Z, L0, Y0, out, a, b, g, m * op->dt, op->geo, s.dims(),
                 (int)tiles_i, (int)tiles_k, (int)tiles_j, ti, (int)nblk};
    const int in = (Z ? kStsZ : 0) | (L0 ? kStsL0 : 0) | (Y0 ? kStsY0 : 0);
    const dim3 grid((unsigned)nblk), block(kWave * kStsWPB);
    auto go = [&](auto vtag) {
        constexpr int VV = decltype(vtag)::value;
        switch (in) {
            case 0: hipLaunchKernelGGL((k_sts_stage<kStsWPB, kStsRPW, VV, 0>), grid, block, 0, stream, args); break;
            case kStsY0: hipLaunchKernelGGL((k_sts_stage<kStsWPB, kStsRPW, VV, kStsY0>), grid, block, 0, stream, args); break;
            case kStsL0: hipLaunchKernelGGL((k_sts_stage<kStsWPB, kStsRPW, VV, kStsL0>), grid, block, 0, stream, args); break;
            case kStsL0 | kStsY0: hipLaunchKernelGGL((k_sts_stage<kStsWPB, kStsRPW, VV, kStsL0 | kStsY0>), grid, block, 0, stream, args); break;
            case kStsZ | kStsL0: hipLaunchKernelGGL((k_sts_stage<kStsWPB, kStsRPW, VV, kStsZ | kStsL0>), grid, block, 0, stream, args); break;
            default: hipLaunchKernelGGL((k_sts_stage<kStsWPB, kStsRPW, VV, kStsZ | kStsL0 | kStsY0>), grid, block, 0, stream, args); break;
        }
    };
    if (in != 0 && in != kStsY0 && in != kStsL0 && in != (kStsL0 | kStsY0) &&
        in != (kStsZ | kStsL0) && in != (kStsZ | kStsL0 | kStsY0))
        return fail(MAS_EINVAL, "internal: unsupported stage inputs %d", in);
    if (v == 2)
        go(std::integral_constant<int, 2>{});
    else
        go(std::integral_constant<int, 1>{});
    LAUNCHCHK();
    return MAS_OK;
}

// The two-stage kernel keeps the lane's two cells adjacent across the
// periodic seam only for even np; odd np runs one stage per launch.
static bool sts_pairs_ok(const Shape &s) { return s.np % 2 == 0; }

// Stages j, j+1 in one kernel (k_sts_pair): outA = aA X + bA Z + gA L0 +
// mA dtL(X), outB = aB outA + bB X + gB L0 + Y0 + mB dtL(outA).  L0 == nullptr
// stands for L0 = X; Y0 != nullptr makes B the last stage (outA not written).
static int sts_pair_launch(const mas_op *op, hipStream_t stream, const double *X, const double *Z,
                           const double *L0, const double *Y0, double *outA, double *outB, double aA,
                           double bA, double gA, double mA, double aB, double bB, double gB, double mB) {
    const Shape &s = op->s;
    constexpr int RO = 2 * kPairNW - 4;
    // r chunks: at least kPairTI planes, and long enough that there are at
    // most 8 of them (whole r slabs per XCD, as for the iteration kernel)
    const int ti = std::min(s.max_chunk(), MAS_PAIR_SLAB ? std::min(kPairMaxTI, std::max(kPairTI, (s.nr + 7) / 8))
                                                         : kPairTI);
    const int64_t tiles_i = (s.nr + ti - 1) / ti;
    const int64_t tiles_k = (s.np + kPairOut - 1) / kPairOut;
    const int64_t tiles_j = (s.nt + RO - 1) / RO;
    const int64_t nblk = tiles_i * tiles_k * tiles_j;
    if (nblk > INT32_MAX) return fail(MAS_EINVAL, "grid too large for the stage kernel");
    if (!sts_pairs_ok(s)) return fail(MAS_EINVAL, "internal: two-stage kernel needs an even np");
    StsPairArgs args{X, op->nu, Z, L0, Y0, outA, outB, aA, bA, gA, mA * op->dt, aB, bB, gB, mB * op->dt,
                     op->geo, s.dims(), (int)tiles_i, (int)tiles_k, (int)tiles_j, ti, (int)nblk};
    const int in = (Z ? kPairZ : 0) | (L0 ? kPairL : 0) | (Y0 ? kPairY : 0);
    const dim3 grid((unsigned)nblk), block(kWave * kPairNW);
    switch (in) {
        case 0: hipLaunchKernelGGL((k_sts_pair<kPairNW, 0>), grid, block, 0, stream, args); break;
        case kPairY: hipLaunchKernelGGL((k_sts_pair<kPairNW, kPairY>), grid, block, 0, stream, args); break;
        case kPairZ | kPairL: hipLaunchKernelGGL((k_sts_pair<kPairNW, kPairZ | kPairL>), grid, block, 0, stream, args); break;
        case kPairZ | kPairL | kPairY: hipLaunchKernelGGL((k_sts_pair<kPairNW, kPairZ | kPairL | kPairY>), grid, block, 0, stream, args); break;
        default: return fail(MAS_EINVAL, "internal: unsupported stage-pair inputs %d", in);
    }
    LAUNCHCHK();
    return MAS_OK;
}


// The recursion runs on D_j = Y_j - Y_0 (linearity of L gives
// dtL(Y_{j-1}) = dtL(D_{j-1}) + L_0 with L_0 = dtL(Y_0)):
//   D_1 = mt_1 L_0,
//   D_j = mu_j D_{j-1} + nu_j D_{j-2} + mt_j dtL(D_{j-1}) + (mt_j + gt_j) L_0,
//   u1 = Y_0 + D_s,
// so only the last stage reads Y_0.  D_1 is never stored (stages 2 and 3 read
// L_0 in its place) and D_j overwrites D_{j-2} cell by cell.
extern "C" int mas_sts_step(const mas_op *op, const double *u0, double *u1, const mas_sts_opts *o,
                            void *work, int64_t work_bytes, void *hip_stream, mas_sts_info *info) {
    g_last_error.clear();
    if (info) std::memset(info, 0, sizeof *info);
    auto done = [&](int st) {
        if (info) info->status = st;
        return st;
    };
    if (!op || !u0 || !u1 || !work) return done(fail(MAS_EINVAL, "op, u0, u1 and work must not be NULL"));
    mas_sts_opts def;
    mas_sts_default_opts(&def);
    if (!o) o = &def;
    if (reinterpret_cast<uintptr_t>(work) & 255)
        return done(fail(MAS_EINVAL, "work must be 256-byte aligned"));
    const StsWork L = sts_work_layout(op->s);
    if (work_bytes < L.total)
        return done(fail(MAS_ENOMEM, "workspace too small: %lld < %lld bytes",
                         (long long)work_bytes, (long long)L.total));
    int s = o->stages;
    if (s == 0) {
        s = sts_stages_for(op->zmax);
        if (s < 0) return done(fail(MAS_EINVAL, "dt needs more than %d explicit stages", kStsMaxStages));
    } else if (s < 2 || s > kStsMaxStages) {
        return done(fail(MAS_EINVAL, "stages must be 0 (automatic) or in [2, %d]", kStsMaxStages));
    }
    if (info) {
        info->stages = s;
        info->z_max = op->zmax;
    }
    hipStream_t stream = as_stream(hip_stream);
    char *base = static_cast<char *>(work);
    double *L0 = reinterpret_cast<double *>(base + L.vec[0]);
    double *W[4];
    for (int t = 0; t < 4; ++t) W[t] = reinterpret_cast<double *>(base + L.vec[t + 1]);
    const Rkl2 c = rkl2_coefficients(s);
    const bool pairs = !o->single_stage_kernels && sts_pairs_ok(op->s) && s >= 3;
    if (info) info->stages_per_kernel = pairs ? 2 : 1;

    EventPool pool;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = o->sample_timing != 0;
    if (timing) {
        int st = pool.make(&ev0);
        if (st == MAS_OK) st = pool.make(&ev1);
        if (st != MAS_OK) return done(st);
        if (hipEventRecord(ev0, stream) != hipSuccess)
            return done(fail(MAS_EHIP, "hipEventRecord failed"));
    }
    // The general kernels (stages 4 .. s-1, or the pairs among them) run back
    // to back; one event pair brackets that whole run and its mean is
    // reported (events between single launches would add their own gaps).
    const int ngen = pairs ? std::max(0, (s - 3) / 2 - ((s - 3) % 2 == 0 ? 1 : 0)) : std::max(0, s - 4);
    hipEvent_t eg0 = nullptr, eg1 = nullptr;
    bool gen_timed = false;
    // run one launch; g >= 0 numbers the general kernels
    auto run = [&](int g, auto &&launch) -> int {
        int st2;
        if (timing && g == 0 && ngen > 0) {
            if ((st2 = pool.make(&eg0)) != MAS_OK || (st2 = pool.make(&eg1)) != MAS_OK) return st2;
            if (hipEventRecord(eg0, stream) != hipSuccess) return fail(MAS_EHIP, "hipEventRecord failed");
        }
        if ((st2 = launch()) != MAS_OK) return st2;
        if (timing && g == ngen - 1 && ngen > 0) {
            if (hipEventRecord(eg1, stream) != hipSuccess) return fail(MAS_EHIP, "hipEventRecord failed");
            gen_timed = true;
        }
        return MAS_OK;
    };

    // L_0 = dtL(Y_0)
    int st = sts_launch(op, stream, u0, nullptr, nullptr, nullptr, L0, 0.0, 0.0, 0.0, 1.0);
    if (st != MAS_OK) return done(st);
    // D_2 = (mu_2 mt_1 + mt_2 + gt_2) L_0 + mt_2 mt_1 dtL(L_0)
    const double a2 = c.mu[2] * c.mt[1] + c.mt[2] + c.gt[2], m2 = c.mt[2] * c.mt[1];
    // D_3 = mu_3 D_2 + mt_3 dtL(D_2) + (nu_3 mt_1 + mt_3 + gt_3) L_0
    const double g3 = s >= 3 ? c.nu[3] * c.mt[1] + c.mt[3] + c.gt[3] : 0.0;
    if (!pairs) {
        for (int j = 2; j <= s; ++j) {
            const bool last = j == s;
            double *out = last ? u1 : W[j & 1];
            const double *Y0 = last ? u0 : nullptr;
            st = run(last ? -1 : j - 4, [&] {
                if (j == 2) return sts_launch(op, stream, L0, nullptr, nullptr, Y0, out, a2, 0.0, 0.0, m2);
                if (j == 3) return sts_launch(op, stream, W[0], nullptr, L0, Y0, out, c.mu[3], 0.0, g3, c.mt[3]);
                return sts_launch(op, stream, W[(j - 1) & 1], W[j & 1], L0, Y0, out, c.mu[j], c.nu[j],
                                  c.mt[j] + c.gt[j], c.mt[j]);
            });
            if (st != MAS_OK) return done(st);
        }
    } else {
        // stages 2, 3 (X = L_0), then pairs j, j+1 from j = 4; pair q writes
        // (D_j, D_{j+1}) to W[2 (q%2)], W[2 (q%2) + 1]; an odd stage left at
        // the end runs alone
        st = run(-1, [&] {
            return sts_pair_launch(op, stream, L0, nullptr, nullptr, s == 3 ? u0 : nullptr, W[0],
                                   s == 3 ? u1 : W[1], a2, 0.0, 0.0, m2, c.mu[3], 0.0, g3, c.mt[3]);
        });
        if (st != MAS_OK) return done(st);
        int j = 4, q = 1;
        for (; j + 1 <= s; j += 2, ++q) {
            const bool last = j + 1 == s;
            const double *X = W[2 * ((q - 1) & 1) + 1], *Z = W[2 * ((q - 1) & 1)];
            double *oA = W[2 * (q & 1)], *oB = last ? u1 : W[2 * (q & 1) + 1];
            st = run(last ? -1 : q - 1, [&] {
                return sts_pair_launch(op, stream, X, Z, L0, last ? u0 : nullptr, oA, oB, c.mu[j], c.nu[j],
                                       c.mt[j] + c.gt[j], c.mt[j], c.mu[j + 1], c.nu[j + 1],
                                       c.mt[j + 1] + c.gt[j + 1], c.mt[j + 1]);
            });
            if (st != MAS_OK) return done(st);
        }
        if (j == s) {
            const double *X = W[2 * ((q - 1) & 1) + 1], *Z = W[2 * ((q - 1) & 1)];
            st = sts_launch(op, stream, X, Z, L0, u0, u1, c.mu[s], c.nu[s], c.mt[s] + c.gt[s], c.mt[s]);
            if (st != MAS_OK) return done(st);
        }
    }
    if (timing) {
        if (hipEventRecord(ev1, stream) != hipSuccess || hipEventSynchronize(ev1) != hipSuccess)
            return done(fail(MAS_EHIP, "stage timing failed"));
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess)
            return done(fail(MAS_EHIP, "hipEventElapsedTime failed"));
        float tg = 0.f;
        if (gen_timed && hipEventElapsedTime(&tg, eg0, eg1) != hipSuccess)
            return done(fail(MAS_EHIP, "hipEventElapsedTime failed"));
        if (info) {
            info->step_us = 1e3 * ms;
            info->stage_kernel_samples = gen_timed ? ngen : 0;
            info->stage_kernel_us = gen_timed ? 1e3 * (double)tg / ngen : 0.0;
        }
    }
    return done(MAS_OK);
}

extern "C" int mas_probe_copy(const void *src, void *dst, int64_t bytes, void *hip_stream) {
    if (!src || !dst) return fail(MAS_EINVAL, "src and dst must not be NULL");
    if (bytes < 0 || (bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15) ||
        (reinterpret_cast<uintptr_t>(dst) & 15))
        return fail(MAS_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    const int64_t n16 = bytes / 16;
    if (n16 == 0) return MAS_OK;
    const int64_t blocks = (n16 + kCopyChunk - 1) / kCopyChunk;
    if (blocks > INT32_MAX) return fail(MAS_EINVAL, "copy too large");
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, as_stream(hip_stream),
                       static_cast<const double2 *>(src), static_cast<double2 *>(dst), n16);
    LAUNCHCHK();
    return MAS_OK;
}

// Layout of the streaming probe's arrays in one buffer: nin + nout arrays of
// n doubles, staggered as the library's own arrays are.
static int64_t stream_layout(int64_t n, int nin, int nout, int64_t *off) {
    LayoutCursor cur(kPhaseWork);
    for (int t = 0; t < nin + nout; ++t) off[t] = cur.take_array(8 * n);
    return cur.off;
}

extern "C" int64_t mas_probe_stream_bytes(int64_t n, int32_t nin, int32_t nout) {
    if (n < 1 || nin < 1 || nin > kStreamMaxIn || nout < 1 || nout > kStreamMaxOut)
        return fail(MAS_EINVAL, "need n >= 1, 1 <= nin <= %d, 1 <= nout <= %d", kStreamMaxIn,
                    kStreamMaxOut);
    int64_t off[kStreamMaxIn + kStreamMaxOut];
    return stream_layout(n, nin, nout, off);
}

extern "C" int mas_probe_stream(void *buf, int64_t bytes, int64_t n, int32_t nin, int32_t nout,
                                void *hip_stream) {
    const int64_t need = mas_probe_stream_bytes(n, nin, nout);
    if (need < 0) return (int)need;
    if (!buf || (reinterpret_cast<uintptr_t>(buf) & 255))
        return fail(MAS_EINVAL, "buf must be non-NULL and 256-byte aligned");
    if (bytes < need) return fail(MAS_ENOMEM, "buffer too small: %lld < %lld bytes",
                                  (long long)bytes, (long long)need);
    int64_t off[kStreamMaxIn + kStreamMaxOut];
    stream_layout(n, nin, nout, off);
    StreamArgs a{};
    char *base = static_cast<char *>(buf);
    for (int t = 0; t < nin; ++t) a.in[t] = reinterpret_cast<const double *>(base + off[t]);
    for (int t = 0; t < nout; ++t) a.out[t] = reinterpret_cast<double *>(base + off[nin + t]);
    a.n = n;
    const int64_t blocks = (n + kStreamChunk - 1) / kStreamChunk;
    if (blocks > INT32_MAX) return fail(MAS_EINVAL, "probe too large");
    const dim3 grid((unsigned)blocks), block(256);
    hipStream_t st = as_stream(hip_stream);
    // the byte mixes the library's kernels stream (7 in / 4 out: the PCG
    // iteration; 2 / 2: the gradient; 4 / 1: an RKL2 stage)
    if (nin == 8 && nout == 4) hipLaunchKernelGGL((k_stream<8, 4>), grid, block, 0, st, a);
    else if (nin == 6 && nout == 3) hipLaunchKernelGGL((k_stream<6, 3>), grid, block, 0, st, a);
    else if (nin == 7 && nout == 4) hipLaunchKernelGGL((k_stream<7, 4>), grid, block, 0, st, a);
    else if (nin == 6 && nout == 1) hipLaunchKernelGGL((k_stream<6, 1>), grid, block, 0, st, a);
    else if (nin == 2 && nout == 2) hipLaunchKernelGGL((k_stream<2, 2>), grid, block, 0, st, a);
    else if (nin == 4 && nout == 1) hipLaunchKernelGGL((k_stream<4, 1>), grid, block, 0, st, a);
    else if (nin == 1 && nout == 1) hipLaunchKernelGGL((k_stream<1, 1>), grid, block, 0, st, a);
    else return fail(MAS_EINVAL, "stream probe mixes: 8/4, 6/3, 7/4, 6/1, 2/2, 4/1 or 1/1 (got %d/%d)", nin, nout);
    LAUNCHCHK();
    return MAS_OK;
}

extern "C" const char *mas_status_string(int status) {
    switch (status) {
        case MAS_OK: return "MAS_OK: converged";
        case MAS_ENOTCONV: return "MAS_ENOTCONV: tolerance not reached";
        case MAS_EINVAL: return "MAS_EINVAL: invalid argument";
        case MAS_EBREAKDOWN: return "MAS_EBREAKDOWN: PCG breakdown";
        case MAS_EHIP: return "MAS_EHIP: HIP runtime error";
        case MAS_ENOMEM: return "MAS_ENOMEM: storage or workspace too small";
        default: return "unknown status";
    }
}

extern "C" const char *mas_last_error(void) { return g_last_error.c_str(); }
