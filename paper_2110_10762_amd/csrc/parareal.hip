// Host side of the C ABI declared in include/parareal.h.
//
// Everything numerical runs in the kernels of fine.hpp, coarse.hpp, sync.hpp,
// async.hpp, adjoint.hpp and batched.hpp; this file validates arguments, owns
// the workspace, sequences launches on the caller's stream and reads back the
// per-iteration stop decisions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "parareal.h"
#include "fine.hpp"
#include "sync.hpp"
#include "async.hpp"
#include "adjoint.hpp"
#include "batched.hpp"
#include "implicit.hpp"

using namespace pr;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(PR_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                            \
    } while (0)

extern "C" const char *pr_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ shapes
// 2D: (x points per lane, rows, depth); rows >= SW_MIN_ROWS is a sliding
// window over segments of that many rows, fewer is a register strip.
struct Shape {
    int xp, r, d;
    bool sliding() const { return r >= SW_MIN_ROWS; }
};
static const Shape kShapes2D[] = {{2, 32, 1},  {2, 32, 2},   {2, 32, 4},  {2, 32, 8},  {2, 16, 8},
                                  {2, 24, 12}, {2, 16, 16},  {1, 64, 8},  {2, 16, 4},  {2, 8, 4},
                                  {2, 128, 4}, {3, 128, 4},  {2, 128, 8}, {3, 128, 8}, {4, 128, 8},
                                  {3, 256, 8}, {2, 128, 16}, {3, 96, 8},  {2, 128, 1}, {3, 128, 12},
                                  {2, SW_AUTO_ROWS, 8}, {2, 128, 12}, {2, SW_AUTO_ROWS, 12},
                                  {2, 128, 14}, {2, SW_AUTO_ROWS, 14}};
// 3D: (x points per lane, rows, depth); depth > 1 marches z with that many
// time levels (k_fine3d_tb), depth 1 is the one-step register strip.
static const Shape kShapes3D[] = {{2, 8, 1}, {2, 16, 1}, {1, 16, 1}, {2, 4, 1}, {1, 8, 2}, {1, 6, 3}, {1, 8, 4}};
static const int kDefault2D = 24;        // sliding window (2, auto rows, 14): batches of states
static const int kDefault2DSingle = 4;   // register strip (2, 16, 8): one state (more waves)
static const int kDefault3D = 0;     // (2, 8, 1): one step per slice
static const int kDefault3DTB = 6;   // (1, 8, 4): slices of several steps
static const int kNum2D = sizeof(kShapes2D) / sizeof(kShapes2D[0]);
static const int kNum3D = sizeof(kShapes3D) / sizeof(kShapes3D[0]);

// first table entry matching every given (> 0) parameter, or -1
static int find_shape(int dim, int d, int r, int xp) {
    const Shape *tab = dim == 2 ? kShapes2D : kShapes3D;
    const int cnt = dim == 2 ? kNum2D : (dim == 3 ? kNum3D : 0);
    for (int i = 0; i < cnt; ++i)
        if ((d <= 0 || tab[i].d == d) && (r <= 0 || tab[i].r == r) && (xp <= 0 || tab[i].xp == xp))
            return i;
    return -1;
}

static int r1d_for(int n) {   // registers per lane for a 1D state
    int R = 1;
    while (R * WAVE < n) R *= 2;
    return R;
}
static const int kMax1D = 32 * WAVE;   // 2048 points
static const int SWEEP_BLOCK = SWEEP_THREADS;   // threads per workgroup of the whole-GPU coarse sweeps
static const int kXcds = 8;            // MI355X: accelerator complex dies (each with its own L2)

// ------------------------------------------------------------------ handle
struct Prob {
    pr_config cfg;
    int dim, n, N, m;
    int shape1 = -1;       // fine-kernel shape for single-state runs (serial fine), -1: same
    double nu, T, h, dT, dt, r, s;
    long long npts;
    long long off_state;   // offset of this problem's state in concatenated u0
    long long off_lam;     // offset of lambda_0 in a concatenated iterate
    int shape;             // index into the 2D/3D shape table
    Geom g;
    double cg_tol;
    int cg_maxit, kmax;
    double eps;
    int fine;              // FINE_EXPLICIT, FINE_BACKWARD_EULER or FINE_TRAPEZOIDAL
    bool pcg;              // 2D coarse solves by the preconditioned CG
};

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct pr_problem {
    int device = 0;
    hipStream_t stream = nullptr;
    int ncu = 0;
    std::vector<Prob> P;
    std::vector<Buf> allocs;
    // synchronous workspace (single problem)
    double *v = nullptr, *w = nullptr, *tmp = nullptr, *wn = nullptr, *d0 = nullptr, *d1 = nullptr;
    double *w2 = nullptr;   // 2D preconditioned sync: coarse values of alternate iterations
    double *cg_r = nullptr, *cg_p0 = nullptr, *cg_p1 = nullptr, *red = nullptr;
    double *cg_r1 = nullptr;   // second residual buffer of the 2D one-synchronisation CG
    double *cg_w0 = nullptr, *cg_w1 = nullptr;   // 2D preconditioned CG: u (p and r shared)
    double *inv_tab = nullptr;        // 1D Thomas factors, padded
    double *inv_tab_f = nullptr;      // 1D Thomas factors of an implicit fine step (s = theta r)
    // implicit fine steps on many states (2D/3D): per-team tmp, rhs, CG set
    double *fth_scr = nullptr, *fth_red = nullptr;
    unsigned *fth_ctr = nullptr;
    unsigned long long *fth_its = nullptr;
    int fth_grid = 0;
    unsigned *ctr = nullptr;          // team barrier counters
    Control *ctl = nullptr;
    double *dscal = nullptr;          // device scalars: [0] delta
    unsigned long long *iscal = nullptr;   // device counters: [0] cg iterations
    int sweep_grid = 0;               // cooperative grid for CG sweeps
    int red_slots = 0;
    hipEvent_t ev[6] = {};
    // asynchronous options and workspace
    pr_async_opts aopt{};
    std::vector<int> sched;           // copy of the replay schedule
    std::vector<int> delays;
    std::vector<int> drops, resets;   // failure injection, [N+1] each (empty: none)
    AsyncWork aw{};
    bool aw_ready = false;
    // batched workspace
    BatchWork bw{};
    bool bw_ready = false;
    bool bw_dirty = false;
    // adjoint workspace
    AdjWork jw{};
    bool jw_ready = false;
};

static int dev_alloc(pr_problem *h, void **p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(PR_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    h->allocs.push_back({*p, bytes});
    return PR_OK;
}

static void dev_free(pr_problem *h, void *p) {
    if (!p) return;
    for (size_t i = 0; i < h->allocs.size(); ++i)
        if (h->allocs[i].p == p) {
            (void)hipFree(p);
            h->allocs.erase(h->allocs.begin() + i);
            return;
        }
}

template <typename T>
static int alloc_t(pr_problem *h, T **p, size_t count) {
    void *q = nullptr;
    int rc = dev_alloc(h, &q, count * sizeof(T));
    *p = (T *)q;
    return rc;
}

// ------------------------------------------------------------------ config
static int derive(const pr_config &c, Prob &P) {
    if (c.dim < 1 || c.dim > 3) return fail(PR_EINVAL, "dim must be 1, 2 or 3 (got %d)", c.dim);
    if (c.n < 1) return fail(PR_EINVAL, "n must be >= 1 (got %d)", c.n);
    if (c.dim == 1 && c.n > kMax1D) return fail(PR_EINVAL, "1D supports n <= %d (got %d)", kMax1D, c.n);
    if (c.dim >= 2 && std::pow((double)c.n, c.dim) >= 2147483647.0)
        return fail(PR_EINVAL, "a %dD state must hold fewer than 2^31 points (n = %d)", c.dim, c.n);
    if (!(c.nu > 0) || !std::isfinite(c.nu)) return fail(PR_EINVAL, "nu must be > 0");
    if (!(c.T > 0) || !std::isfinite(c.T)) return fail(PR_EINVAL, "T must be > 0");
    if (c.nslices < 1) return fail(PR_EINVAL, "nslices must be >= 1");
    if (!(c.dt_nominal > 0)) return fail(PR_EINVAL, "dt_nominal must be > 0");
    if (c.coarse == PR_COARSE_THOMAS && c.dim != 1)
        return fail(PR_EINVAL, "the Thomas coarse solver is 1D only");
    if (c.coarse == PR_COARSE_CG && c.dim == 1)
        return fail(PR_EINVAL, "1D problems use the Thomas coarse solver");
    if (c.coarse < 0 || c.coarse > 2) return fail(PR_EINVAL, "unknown coarse solver %d", c.coarse);
    if (c.fine < PR_FINE_EXPLICIT || c.fine > PR_FINE_TRAPEZOIDAL) return fail(PR_EINVAL, "unknown fine propagator %d", c.fine);
    P.cfg = c;
    P.dim = c.dim;
    P.n = c.n;
    P.N = c.nslices;
    P.nu = c.nu;
    P.T = c.T;
    P.h = 1.0 / (c.n + 1);
    P.dT = c.T / c.nslices;
    const double ratio = P.dT / c.dt_nominal;
    if (!(ratio < 1e9)) return fail(PR_EINVAL, "too many fine steps per slice");
    P.m = std::max(1, (int)std::ceil(ratio - 1e-9));
    P.dt = P.dT / P.m;
    P.r = P.nu * P.dt / (P.h * P.h);
    P.s = P.nu * P.dT / (P.h * P.h);
    P.fine = c.fine;
    if (c.cg_precond != 0 && c.cg_precond != -1 && c.cg_precond != PCG_DEGREE)
        return fail(PR_EINVAL, "cg_precond: 0 (default), -1 (none) or %d (got %d)", PCG_DEGREE, c.cg_precond);
    P.pcg = c.dim == 2 && c.cg_precond >= 0;
    if (P.fine == FINE_EXPLICIT && P.r > 0.5 / P.dim * (1.0 + 1e-12))
        return fail(PR_EUNSTABLE, "explicit Euler unstable: r = %.6g > 1/(2d) = %.6g", P.r, 0.5 / P.dim);
    P.g = make_geom(P.dim, P.n);
    P.npts = P.g.npts;
    P.cg_tol = c.cg_tol > 0 ? c.cg_tol : 1e-12;
    P.cg_maxit = c.cg_maxit > 0 ? c.cg_maxit : 10 * c.n + 100;
    P.kmax = (c.kmax <= 0 || c.kmax > c.nslices) ? c.nslices : c.kmax;
    P.eps = c.eps;
    P.shape = P.dim == 2 ? kDefault2D : (P.dim == 3 ? (P.m > 1 ? kDefault3DTB : kDefault3D) : 0);
    P.shape1 = P.dim == 2 ? kDefault2DSingle : -1;
    if (P.dim > 1 && (c.tb_depth > 0 || c.tile_rows > 0 || c.fine_xpts > 0)) {
        P.shape1 = -1;
        const int found = find_shape(P.dim, c.tb_depth, c.tile_rows, c.fine_xpts);
        if (found < 0)
            return fail(PR_EINVAL, "no fine-kernel shape with depth %d, %d rows and %d x points per lane",
                        c.tb_depth, c.tile_rows, c.fine_xpts);
        P.shape = found;
    }
    return PR_OK;
}

// ------------------------------------------------------------------ launches
template <int XP, int R, int D>
static void launch2d(hipStream_t st, const double *src, double *dst, long long ss, long long ds, int n,
                     double r, int steps, int count) {
    constexpr int W = Shape2D<XP, R, D>::W;
    const int nsx = (n + W - 1) / W, nsy = (n + R - 1) / R;
    const long long waves = (long long)nsx * nsy * count;
    const int nblk = (int)((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
    const int grid = 8 * ((nblk + 7) / 8);
    hipLaunchKernelGGL((k_fine2d<XP, R, D>), dim3(grid), dim3(BLOCK), 0, st, src, dst, ss, ds, n, r, steps,
                       nsx, nsy, count, nblk);
}

// Rows per segment for SW_AUTO_ROWS: the segment count whose units fill the
// resident wave slots in the fewest rounds, each round costing the rows a
// wave marches (its segment plus 2D halo rows).
template <int XP, int D>
static int sw_auto_rows(int n, int count, int nsx) {
    static int slots = 0;
    if (slots == 0) {
        int occ = 0, ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_fine2d_sw<XP, D>, BLOCK, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return 128;
        }
        slots = std::max(1, occ * ncu * WAVES_PER_BLOCK);
    }
    int best = n;
    double best_cost = 1e300;
    for (int nseg = 1; nseg <= std::max(1, n / 32); ++nseg) {
        const int seg = (n + nseg - 1) / nseg;
        const long long units = (long long)count * nsx * ((n + seg - 1) / seg);
        const long long rounds = (units + slots - 1) / slots;
        const double cost = (double)rounds * (seg + 2 * D);
        if (cost < best_cost) {
            best_cost = cost;
            best = seg;
        }
    }
    return best;
}

template <int XP, int D>
static void launch2d_sw(hipStream_t st, const double *src, double *dst, long long ss, long long ds, int n,
                        double r, int steps, int count, int ry) {
    const int nsx = sw_strips<XP, D>(n);
    if (ry == SW_AUTO_ROWS) ry = sw_auto_rows<XP, D>(n, count, nsx);
    const int nsy = (n + ry - 1) / ry;
    const long long waves = (long long)nsx * nsy * count;
    const int nblk = (int)((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
    const int grid = 8 * ((nblk + 7) / 8);
    hipLaunchKernelGGL((k_fine2d_sw<XP, D>), dim3(grid), dim3(BLOCK), 0, st, src, dst, ss, ds, n, r, steps, nsx,
                       nsy, ry, count, nblk);
}

static void launch2d_shape(int shape, hipStream_t st, const double *src, double *dst, long long ss,
                           long long ds, int n, double r, int steps, int count) {
    const int ry = kShapes2D[shape].r;
    switch (shape) {
        case 10: launch2d_sw<2, 4>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 11: launch2d_sw<3, 4>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 12: launch2d_sw<2, 8>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 13: launch2d_sw<3, 8>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 14: launch2d_sw<4, 8>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 15: launch2d_sw<3, 8>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 16: launch2d_sw<2, 16>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 17: launch2d_sw<3, 8>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 18: launch2d_sw<2, 1>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 19: launch2d_sw<3, 12>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 20: launch2d_sw<2, 8>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 21:
        case 22: launch2d_sw<2, 12>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        case 23:
        case 24: launch2d_sw<2, 14>(st, src, dst, ss, ds, n, r, steps, count, ry); return;
        default: break;
    }
    switch (shape) {
        case 0: launch2d<2, 32, 1>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 1: launch2d<2, 32, 2>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 2: launch2d<2, 32, 4>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 3: launch2d<2, 32, 8>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 4: launch2d<2, 16, 8>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 5: launch2d<2, 24, 12>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 6: launch2d<2, 16, 16>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 7: launch2d<1, 64, 8>(st, src, dst, ss, ds, n, r, steps, count); break;
        case 8: launch2d<2, 16, 4>(st, src, dst, ss, ds, n, r, steps, count); break;
        default: launch2d<2, 8, 4>(st, src, dst, ss, ds, n, r, steps, count); break;
    }
}

template <int XP, int R>
static void launch3d(hipStream_t st, const double *src, double *dst, long long ss, long long ds, int n,
                     double r, int count) {
    constexpr int W = WAVE * XP - 2;
    const int nsx = (n + W - 1) / W, nsy = (n + R - 1) / R;
    // split z so that a launch has enough waves to fill the chip
    int zc = n;
    while (zc > 8 && (long long)nsx * nsy * count * ((n + zc - 1) / zc) < 8192) zc = (zc + 1) / 2;
    const int nsz = (n + zc - 1) / zc;
    const long long waves = (long long)nsx * nsy * nsz * count;
    const int nblk = (int)((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
    const int grid = 8 * ((nblk + 7) / 8);
    hipLaunchKernelGGL((k_fine3d<XP, R>), dim3(grid), dim3(BLOCK), 0, st, src, dst, ss, ds, n, r, nsx, nsy,
                       nsz, zc, count, nblk);
}

// Planes per z segment of a depth-D pass: the segment count whose units fill
// the GPU's wave slots in whole rounds at the least marched planes (each
// segment recomputes 2D halo planes).
template <int R, int D, int PF>
static int tb3_planes(int n, long long strips) {
    static int slots = 0;
    if (slots == 0) {
        int occ = 0, ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_fine3d_tb<R, D, PF>, BLOCK, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return n;
        }
        slots = std::max(1, occ * ncu * WAVES_PER_BLOCK);
    }
    int best = n;
    double best_cost = 1e300;
    for (int nseg = 1; nseg <= std::max(1, n / 8); ++nseg) {
        const int zc = (n + nseg - 1) / nseg;
        const long long units = strips * ((n + zc - 1) / zc);
        const double cost = (double)((units + slots - 1) / slots) * (zc + 2 * D);
        if (cost < best_cost) {
            best_cost = cost;
            best = zc;
        }
    }
    return best;
}

template <int R, int D, int PF>
static void launch3d_tb(hipStream_t st, const double *src, double *dst, long long ss, long long ds, int n,
                        double r, int steps, int count) {
    const int nsx = (n + WAVE - 2 * D - 1) / (WAVE - 2 * D), nsy = (n + R - 1) / R;
    const int zc = tb3_planes<R, D, PF>(n, (long long)nsx * nsy * count);
    const int nsz = (n + zc - 1) / zc;
    const long long waves = (long long)nsx * nsy * nsz * count;
    const int nblk = (int)((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK);
    const int grid = 8 * ((nblk + 7) / 8);
    hipLaunchKernelGGL((k_fine3d_tb<R, D, PF>), dim3(grid), dim3(BLOCK), 0, st, src, dst, ss, ds, n, r, steps, nsx,
                       nsy, nsz, zc, count, nblk);
}

static void launch3d_shape(int shape, hipStream_t st, const double *src, double *dst, long long ss,
                           long long ds, int n, double r, int steps, int count) {
    switch (shape) {
        case 4: launch3d_tb<8, 2, 2>(st, src, dst, ss, ds, n, r, steps, count); return;
        case 5: launch3d_tb<6, 3, 2>(st, src, dst, ss, ds, n, r, steps, count); return;
        case 6: launch3d_tb<8, 4, 1>(st, src, dst, ss, ds, n, r, steps, count); return;
        default: break;
    }
    switch (shape) {
        case 0: launch3d<2, 8>(st, src, dst, ss, ds, n, r, count); break;
        case 1: launch3d<2, 16>(st, src, dst, ss, ds, n, r, count); break;
        case 2: launch3d<1, 16>(st, src, dst, ss, ds, n, r, count); break;
        default: launch3d<2, 4>(st, src, dst, ss, ds, n, r, count); break;
    }
}

static void launch1d(hipStream_t st, const double *src, double *dst, long long ss, long long ds, int n, double r,
                     int steps, int count) {
    const int R = r1d_for(n);
#define L1(RR) hipLaunchKernelGGL((k_fine1d<RR>), dim3(count), dim3(64), 0, st, src, dst, ss, ds, n, r, steps, count)
    switch (R) {
        case 1: L1(1); break;
        case 2: L1(2); break;
        case 4: L1(4); break;
        case 8: L1(8); break;
        case 16: L1(16); break;
        default: L1(32); break;
    }
#undef L1
}

static int fine_depth(const Prob &P) {
    if (P.dim == 1) return 1 << 30;
    if (P.dim == 2) return kShapes2D[P.shape].d;
    return kShapes3D[P.shape].d;
}

// Passes of at most D steps; the passes ping-pong between dst and tmp so that
// the last one lands in dst.  src is never written.
static int run_fine_theta(pr_problem *h, const Prob &P, const double *src, double *dst, int count, int steps,
                          long long ss, long long ds);

static int run_fine(pr_problem *h, const Prob &P, const double *src, double *dst, double *tmp, int count,
                    int steps, long long ss, long long ds) {
    if (count <= 0 || steps <= 0) return PR_OK;
    if (P.fine != FINE_EXPLICIT) return run_fine_theta(h, P, src, dst, count, steps, ss, ds);
    if (P.dim == 1) {
        launch1d(h->stream, src, dst, ss, ds, P.n, P.r, steps, count);
        HIPCHK(hipGetLastError());
        return PR_OK;
    }
    int shape = P.shape;
    if (count == 1 && P.dim == 2 && P.shape1 >= 0) {
        // a single state: the shape made for one state, unless it needs a scratch buffer there is none of
        const int d1 = kShapes2D[P.shape1].d;
        if ((steps + d1 - 1) / d1 <= 1 || tmp) shape = P.shape1;
    }
    const int D = P.dim == 2 ? kShapes2D[shape].d : kShapes3D[shape].d;
    const int passes = (steps + D - 1) / D;
    if (passes > 1 && !tmp) return fail(PR_EINVAL, "internal: fine pass needs a scratch buffer");
    const double *cur = src;
    long long cs = ss;
    for (int p = 0; p < passes; ++p) {
        const int st = std::min(D, steps - p * D);
        double *tgt = ((passes - 1 - p) % 2 == 0) ? dst : tmp;
        const long long ts = (tgt == dst) ? ds : P.npts;
        if (P.dim == 2)
            launch2d_shape(shape, h->stream, cur, tgt, cs, ts, P.n, P.r, st, count);
        else
            launch3d_shape(shape, h->stream, cur, tgt, cs, ts, P.n, P.r, st, count);
        HIPCHK(hipGetLastError());
        cur = tgt;
        cs = ts;
    }
    return PR_OK;
}

static int zero_words(pr_problem *h, void *p, int nwords) {
    hipLaunchKernelGGL(k_zero_words, dim3((nwords + 255) / 256), dim3(256), 0, h->stream, (unsigned *)p, nwords);
    HIPCHK(hipGetLastError());
    return PR_OK;
}

static int copy_dev(pr_problem *h, const double *src, double *dst, long long n) {
    if (n <= 0 || src == dst) return PR_OK;
    hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, h->stream, src, dst, n);
    HIPCHK(hipGetLastError());
    return PR_OK;
}

static int coop_launch(pr_problem *h, const void *fn, int grid, int block, void **args) {
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, 0, h->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PR_ENORESIDENT, "cooperative launch of %d workgroups failed: %s", grid, hipGetErrorString(e));
    }
    return PR_OK;
}

static int check_control(pr_problem *h) {
    Control c;
    HIPCHK(hipMemcpyAsync(&c, h->ctl, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (c.abort || c.error) return fail(PR_ETIMEOUT, "a bounded device-side wait ran out (error %d)", c.error);
    return PR_OK;
}

static int thomas_table(pr_problem *h, int n, double s, double **tab);

// Implicit fine steps (theta-method) of `count` states: 1D one wave per state
// in registers; 2D/3D a cooperative launch of teams, one per XCD (fewer when
// there are fewer states), each with its own tmp, rhs and CG set.  The CG
// iterations accumulate in h->fth_its.
static int run_fine_theta(pr_problem *h, const Prob &P, const double *src, double *dst, int count, int steps,
                          long long ss, long long ds) {
    int rc;
    if (P.dim == 1) {
        if (!h->inv_tab_f && (rc = thomas_table(h, P.n, theta_of(P.fine) * P.r, &h->inv_tab_f))) return rc;
        const int R = r1d_for(P.n);
#define F1(RR)                                                                                                  \
    hipLaunchKernelGGL((k_fine1d_theta<RR>), dim3(count), dim3(64), 0, h->stream, src, dst, ss, ds, P.n, P.r, \
                       P.fine, h->inv_tab_f, steps, count)
        switch (R) {
            case 1: F1(1); break;
            case 2: F1(2); break;
            case 4: F1(4); break;
            case 8: F1(8); break;
            case 16: F1(16); break;
            default: F1(32); break;
        }
#undef F1
        HIPCHK(hipGetLastError());
        return PR_OK;
    }
    const void *fn = P.dim == 2 ? (const void *)k_fine_theta<2> : (const void *)k_fine_theta<3>;
    const long long stride = (P.npts + 63) / 64 * 64 + 1536;   // per-team vectors, staggered in memory
    if (!h->fth_scr) {
        int occ = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, BLOCK, 0));
        if (occ < 1) return fail(PR_ENORESIDENT, "implicit fine kernel cannot be resident");
        h->fth_grid = (h->ncu * std::min(occ, 4)) / kXcds * kXcds;
        if ((rc = alloc_t(h, &h->fth_scr, (size_t)kXcds * 6 * stride))) return rc;
        if ((rc = alloc_t(h, &h->fth_red, (size_t)6 * h->fth_grid))) return rc;
        if ((rc = alloc_t(h, &h->fth_ctr, (size_t)kXcds * team_counter_words(0)))) return rc;
        if ((rc = alloc_t(h, &h->fth_its, 1))) return rc;
        if ((rc = zero_words(h, h->fth_its, 2))) return rc;
    }
    int nteams = 1;
    while (nteams * 2 <= std::min(count, kXcds)) nteams *= 2;
    if ((rc = zero_words(h, h->fth_ctr, kXcds * team_counter_words(0)))) return rc;
    if ((rc = zero_words(h, h->ctl, sizeof(Control) / 4))) return rc;
    Geom g = P.g;
    int kind = P.fine, maxit = P.cg_maxit;
    double r = P.r, tol = P.cg_tol;
    double *scr = h->fth_scr, *red = h->fth_red;
    unsigned *ctr = h->fth_ctr;
    Control *ctl = h->ctl;
    unsigned long long *its = h->fth_its;
    long long strd = stride;
    void *args[] = {&src, &dst, &ss, &ds, &count, &g, &kind, &r, &steps, &tol, &maxit, &scr, &strd, &ctr, &red,
                    &ctl, &nteams, &its};
    if ((rc = coop_launch(h, fn, h->fth_grid, BLOCK, args))) return rc;
    return check_control(h);
}

static int reset_fine_its(pr_problem *h) {
    return h->fth_its ? zero_words(h, h->fth_its, 2) : PR_OK;
}

static long long read_fine_its(pr_problem *h) {
    unsigned long long v = 0;
    if (h->fth_its && hipMemcpy(&v, h->fth_its, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return -1;
    return (long long)v;
}

static SweepArgs sweep_args(pr_problem *h, const Prob &P, double *lam) {
    SweepArgs a{};
    a.lam = lam;
    a.v = h->v;
    a.w = h->w;
    a.wn = h->wn;
    a.npts = P.npts;
    a.kguard = -1;
    a.delta = h->dscal;
    a.incr = P.cfg.coarse_increment ? 1 : 0;
    a.d0 = h->d0;
    a.d1 = h->d1;
    a.cg_iters = h->iscal;
    a.n = P.n;
    a.s = P.s;
    a.inv_tab = h->inv_tab;
    a.g = P.g;
    a.cg_tol = P.cg_tol;
    a.cg_maxit = P.cg_maxit;
    a.wk = CGWork{h->cg_r, h->cg_p0, h->cg_p1, h->red};
    a.wk2 = CGWork2{{h->cg_r, h->cg_r1}, {h->cg_p0, h->cg_p1}, h->red};
    a.wkp = CGWorkP{{h->cg_r, h->cg_r1}, {h->cg_w0, h->cg_w1}, {h->cg_p0, h->cg_p1}, h->red};
    a.ctr = h->ctr;
    a.ctl = h->ctl;
    return a;
}

static int run_sweep(pr_problem *h, const Prob &P, SweepArgs a) {
    if (P.dim == 1) {
        const int R = r1d_for(P.n);
#define S1(RR) hipLaunchKernelGGL((k_sweep_1d<RR>), dim3(1), dim3(64), 0, h->stream, a)
        switch (R) {
            case 1: S1(1); break;
            case 2: S1(2); break;
            case 4: S1(4); break;
            case 8: S1(8); break;
            case 16: S1(16); break;
            default: S1(32); break;
        }
#undef S1
        HIPCHK(hipGetLastError());
        return PR_OK;
    }
    int rc = zero_words(h, h->ctr, team_counter_words(h->sweep_grid));
    if (rc) return rc;
    rc = zero_words(h, h->ctl, sizeof(Control) / 4);
    if (rc) return rc;
    void *args[] = {&a};
    const void *fn = P.dim == 3 ? (const void *)k_sweep_cg<3>
                                : (P.pcg ? (const void *)k_sweep_cg<2, true> : (const void *)k_sweep_cg<2>);
    return coop_launch(h, fn, h->sweep_grid, sweep_threads(P.dim == 2 && P.pcg), args);
}

// ------------------------------------------------------------------ create / destroy
// Whether the synchronous sweep carries each slice's correction in the
// set-up march of the next slice's solve: the marching solvers (2D
// preconditioned CG, 3D CG) in the literal (not incremental) form, with the
// coarse values of consecutive iterations in alternate buffers.
static bool carries_corrections(const Prob &P) {
    return (P.dim == 3 || (P.dim == 2 && P.pcg)) && !P.cfg.coarse_increment;
}

// The iterate-sized buffers of the synchronous driver: fine outputs v, coarse
// values w (and w2, see carries_corrections) and, when a slice takes several
// fine passes, their ping-pong buffer.
static int alloc_sync_big(pr_problem *h) {
    const Prob &P = h->P[0];
    const size_t all = (size_t)(P.N + 1) * P.npts;
    int rc;
    if (!h->v && (rc = alloc_t(h, &h->v, all))) return rc;
    if (!h->w && (rc = alloc_t(h, &h->w, all))) return rc;
    // optional: without it each slice is corrected in a pass of its own
    if (carries_corrections(P) && !h->w2 && alloc_t(h, &h->w2, all) != PR_OK) h->w2 = nullptr;
    const int passes = (P.m + fine_depth(P) - 1) / fine_depth(P);
    if (P.dim > 1 && passes > 1 && !h->tmp)
        if ((rc = alloc_t(h, &h->tmp, all))) return rc;
    return PR_OK;
}

static int alloc_sync(pr_problem *h) {
    const Prob &P = h->P[0];
    int rc;
    if ((rc = alloc_sync_big(h))) return rc;
    if (P.dim > 1) {
        if ((rc = alloc_t(h, &h->wn, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->cg_r, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->cg_p0, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->cg_p1, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->cg_r1, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->cg_w0, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->cg_w1, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->d0, P.npts))) return rc;
        if ((rc = alloc_t(h, &h->d1, P.npts))) return rc;
    }
    return PR_OK;
}

// Thomas elimination factors of tridiag(-s, 1+2s, -s), padded to 64*R:
// inv_i = 1 / (1 + 2s + s c'_{i-1}), c'_i = -s inv_i, c'_{-1} = 0.
static int thomas_table(pr_problem *h, int n, double s, double **tab) {
    const int R = r1d_for(n);
    std::vector<double> inv(WAVE * R, 0.0);
    double cprev = 0.0;
    for (int i = 0; i < n; ++i) {
        inv[i] = 1.0 / (1.0 + 2.0 * s + s * cprev);
        cprev = -s * inv[i];
    }
    int rc = alloc_t(h, tab, inv.size());
    if (rc) return rc;
    HIPCHK(hipMemcpy(*tab, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice));
    return PR_OK;
}

static int setup_1d(pr_problem *h) {
    const Prob &P = h->P[0];
    int rc = thomas_table(h, P.n, P.s, &h->inv_tab);
    if (rc) return rc;
    if (P.fine != FINE_EXPLICIT) return thomas_table(h, P.n, theta_of(P.fine) * P.r, &h->inv_tab_f);
    return PR_OK;
}

extern "C" int pr_create(const pr_config *cfgs, int nproblems, int device, void *stream, pr_problem **out) {
    if (!out) return fail(PR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfgs || nproblems < 1) return fail(PR_EINVAL, "need at least one config");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(PR_EINVAL, "device %d out of range (%d devices)", device, ndev);
    pr_problem *h = new (std::nothrow) pr_problem();
    if (!h) return fail(PR_ENOMEM, "host allocation failed");
    auto bail = [&](int rc) {
        pr_destroy(h);
        return rc;
    };
    h->device = device;
    h->stream = (hipStream_t)stream;
    if (hipSetDevice(device) != hipSuccess) return bail(fail(PR_EHIP, "hipSetDevice failed"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return bail(fail(PR_EHIP, "device query failed"));
    h->ncu = prop.multiProcessorCount;
    long long off_s = 0, off_l = 0;
    for (int b = 0; b < nproblems; ++b) {
        Prob P;
        int rc = derive(cfgs[b], P);
        if (rc) {
            std::string m = g_err;
            return bail(fail(rc, "config %d: %s", b, m.c_str()));
        }
        if (nproblems > 1 && P.dim != 2) return bail(fail(PR_EINVAL, "batched problems must be 2D"));
        if (nproblems > 1 && P.fine != FINE_EXPLICIT)
            return bail(fail(PR_EINVAL, "batched problems take the explicit fine propagator"));
        P.off_state = off_s;
        P.off_lam = off_l;
        off_s += P.npts;
        off_l += (long long)(P.N + 1) * P.npts;
        h->P.push_back(P);
    }
    for (int i = 0; i < 6; ++i)
        if (hipEventCreate(&h->ev[i]) != hipSuccess) return bail(fail(PR_EHIP, "hipEventCreate failed"));
    int rc;
    if ((rc = alloc_t(h, &h->ctr, 4096))) return bail(rc);
    if ((rc = alloc_t(h, &h->ctl, 1))) return bail(rc);
    if ((rc = alloc_t(h, &h->dscal, 16))) return bail(rc);
    if ((rc = alloc_t(h, &h->iscal, 16))) return bail(rc);
    int occ = 0;
    int occ2 = 0;
    int occ3 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_sweep_cg<3>, SWEEP_BLOCK, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ2, (const void *)k_sweep_cg<2>, SWEEP_BLOCK, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ3, (const void *)k_sweep_cg<2, true>, PCG_THREADS, 0) !=
            hipSuccess ||
        std::min({occ, occ2, occ3}) < 1)
        return bail(fail(PR_EHIP, "occupancy query failed"));
    h->sweep_grid = h->ncu * std::min(occ, 1);
    h->red_slots = 2 * 4096;
    if ((rc = alloc_t(h, &h->red, h->red_slots))) return bail(rc);
    if (nproblems == 1) {
        if ((rc = alloc_sync(h))) return bail(rc);
        if (h->P[0].dim == 1 && (rc = setup_1d(h))) return bail(rc);
    }
    *out = h;
    return PR_OK;
}

extern "C" void pr_destroy(pr_problem *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (auto &b : h->allocs) (void)hipFree(b.p);
    h->allocs.clear();
    for (int i = 0; i < 6; ++i)
        if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    delete h;
}

extern "C" int pr_get_info(const pr_problem *h, int problem, pr_info *out) {
    if (!h || !out) return fail(PR_EINVAL, "NULL argument");
    if (problem < 0 || problem >= (int)h->P.size()) return fail(PR_EINVAL, "problem index out of range");
    const Prob &P = h->P[problem];
    out->m = P.m;
    out->dt = P.dt;
    out->dT = P.dT;
    out->h = P.h;
    out->r = P.r;
    out->s = P.s;
    out->npts = P.npts;
    out->offset = P.off_lam;
    out->sliding = 0;
    out->cg_precond = P.pcg ? PCG_DEGREE : 0;   // a batch takes it when every problem does
    if (P.dim == 2) {
        out->tb_depth = kShapes2D[P.shape].d;
        out->tile_rows = kShapes2D[P.shape].r;
        out->xpts = kShapes2D[P.shape].xp;
        out->sliding = kShapes2D[P.shape].sliding() ? 1 : 0;
    } else if (P.dim == 3) {
        out->tb_depth = kShapes3D[P.shape].d;
        out->tile_rows = kShapes3D[P.shape].r;
        out->xpts = kShapes3D[P.shape].xp;
    } else {
        out->tb_depth = P.m;
        out->tile_rows = 1;
        out->xpts = r1d_for(P.n);
    }
    return PR_OK;
}

extern "C" int pr_fine_shape_count(int dim) { return dim == 2 ? kNum2D : (dim == 3 ? kNum3D : (dim == 1 ? 1 : 0)); }

extern "C" int pr_fine_shape_get(int dim, int index, int *tb_depth, int *tile_rows, int *xpts, int *sliding) {
    if (dim == 2 && index >= 0 && index < kNum2D) {
        if (tb_depth) *tb_depth = kShapes2D[index].d;
        if (tile_rows) *tile_rows = kShapes2D[index].r;
        if (xpts) *xpts = kShapes2D[index].xp;
        if (sliding) *sliding = kShapes2D[index].sliding() ? 1 : 0;
        return PR_OK;
    }
    if (dim == 3 && index >= 0 && index < kNum3D) {
        if (tb_depth) *tb_depth = kShapes3D[index].d;
        if (tile_rows) *tile_rows = kShapes3D[index].r;
        if (xpts) *xpts = kShapes3D[index].xp;
        if (sliding) *sliding = 0;
        return PR_OK;
    }
    return fail(PR_EINVAL, "no shape %d for dim %d", index, dim);
}

extern "C" int pr_set_fine_shape(pr_problem *h, int problem, int tb_depth, int tile_rows, int xpts) {
    if (!h) return fail(PR_EINVAL, "NULL handle");
    if (problem < 0 || problem >= (int)h->P.size()) return fail(PR_EINVAL, "problem index out of range");
    Prob &P = h->P[problem];
    if (P.dim == 1) return PR_OK;
    const int i = find_shape(P.dim, tb_depth, tile_rows, xpts);
    if (i < 0)
        return fail(PR_EINVAL, "no fine-kernel shape with depth %d, %d rows and %d x points per lane", tb_depth,
                    tile_rows, xpts);
    const int old_passes = (P.m + fine_depth(P) - 1) / fine_depth(P);
    P.shape = i;
    P.shape1 = -1;
    const int passes = (P.m + fine_depth(P) - 1) / fine_depth(P);
    if (h->P.size() == 1 && passes > 1 && old_passes <= 1 && !h->tmp) {
        int rc = alloc_t(h, &h->tmp, (size_t)(P.N + 1) * P.npts);
        if (rc) return rc;
    }
    if (h->bw_ready) h->bw_dirty = true;
    return PR_OK;
}

// ------------------------------------------------------------------ helpers for solves
static int need_single(pr_problem *h) {
    if (!h) return fail(PR_EINVAL, "NULL handle");
    if (h->P.size() != 1) return fail(PR_EINVAL, "this call takes a single-problem handle");
    if (hipSetDevice(h->device) != hipSuccess) return fail(PR_EHIP, "hipSetDevice failed");
    return PR_OK;
}

static double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return ms;
}

static void stats_reset(pr_stats *st) {
    if (!st) return;
    st->iters = st->kappa = st->converged = 0;
    st->last_delta = 0;
    st->wall_ms = st->fine_ms = st->coarse_ms = 0;
    st->fine_lups = 0;
    st->cg_iters = st->g_solves = st->g_skipped = 0;
    st->teams = 0;
    st->kernel_ms = 0;
    st->kernel_cg_iters = st->kernel_updates = 0;
    st->copy_retries = st->idle_rounds = 0;
    st->team_fine_ms = st->team_copy_ms = st->team_coarse_ms = st->team_corr_ms = st->team_total_ms = 0;
    st->fine_cg_iters = 0;
}

// ------------------------------------------------------------------ apply entry points
extern "C" int pr_apply_fine(pr_problem *h, const double *in, double *out, int count, int steps) {
    int rc = need_single(h);
    if (rc) return rc;
    const Prob &P = h->P[0];
    if (!in || !out) return fail(PR_EINVAL, "NULL buffer");
    if (count < 0 || count > P.N + 1) return fail(PR_EINVAL, "count must be in [0, N+1]");
    if (steps <= 0) steps = P.m;
    const int passes = (steps + fine_depth(P) - 1) / fine_depth(P);
    if (P.dim > 1 && passes > 1 && !h->tmp) {
        if ((rc = alloc_t(h, &h->tmp, (size_t)(P.N + 1) * P.npts))) return rc;
    }
    if ((rc = run_fine(h, P, in, out, h->tmp, count, steps, P.npts, P.npts))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return PR_OK;
}

extern "C" int pr_apply_coarse(pr_problem *h, const double *in, double *out, int count, long long *cg_iters) {
    int rc = need_single(h);
    if (rc) return rc;
    const Prob &P = h->P[0];
    if (!in || !out) return fail(PR_EINVAL, "NULL buffer");
    if (in == out) return fail(PR_EINVAL, "in and out must not alias");
    if (count < 0 || count > P.N + 1) return fail(PR_EINVAL, "count must be in [0, N+1]");
    if (cg_iters) *cg_iters = 0;
    if (count == 0) return PR_OK;
    if (P.dim == 1) {
        const int R = r1d_for(P.n);
#define T1(RR) hipLaunchKernelGGL((k_thomas<RR>), dim3(count), dim3(64), 0, h->stream, in, out, P.npts, P.n, P.s, h->inv_tab, count)
        switch (R) {
            case 1: T1(1); break;
            case 2: T1(2); break;
            case 4: T1(4); break;
            case 8: T1(8); break;
            case 16: T1(16); break;
            default: T1(32); break;
        }
#undef T1
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->stream));
        return PR_OK;
    }
    if ((rc = zero_words(h, h->ctr, team_counter_words(h->sweep_grid)))) return rc;
    if ((rc = zero_words(h, h->ctl, sizeof(Control) / 4))) return rc;
    if ((rc = zero_words(h, h->iscal, 2))) return rc;
    long long npts = P.npts;
    Geom g = P.g;
    double s = P.s, tol = P.cg_tol;
    int maxit = P.cg_maxit;
    CGWork wk{h->cg_r, h->cg_p0, h->cg_p1, h->red};
    CGWork2 wk2{{h->cg_r, h->cg_r1}, {h->cg_p0, h->cg_p1}, h->red};
    CGWorkP wkp{{h->cg_r, h->cg_r1}, {h->cg_w0, h->cg_w1}, {h->cg_p0, h->cg_p1}, h->red};
    unsigned *ctr = h->ctr;
    Control *ctl = h->ctl;
    unsigned long long *ci = h->iscal;
    void *args[] = {&in, &out, &npts, &count, &g, &s, &tol, &maxit, &wk, &wk2, &wkp, &ctr, &ctl, &ci};
    const void *fn = P.dim == 3 ? (const void *)k_coarse_cg_batch<3>
                                : (P.pcg ? (const void *)k_coarse_cg_batch<2, true> : (const void *)k_coarse_cg_batch<2>);
    if ((rc = coop_launch(h, fn, h->sweep_grid, sweep_threads(P.dim == 2 && P.pcg), args))) return rc;
    if ((rc = check_control(h))) return rc;
    unsigned long long its = 0;
    HIPCHK(hipMemcpy(&its, h->iscal, sizeof its, hipMemcpyDeviceToHost));
    if (cg_iters) *cg_iters = (long long)its;
    return PR_OK;
}

// ------------------------------------------------------------------ coarse propagator without allocation
// pr_apply_coarse_static keeps every scratch buffer of the coarse solve (CG
// vectors, reduction slots, team counters, control words) in this file-scope
// device array.  Each device the library runs on holds its own copy for the
// life of the process; its device address is taken once per device with
// hipGetSymbolAddress (the array's name is not a device address in host code).
constexpr long long kStaticPts = 1ll << 20;          // largest state: 2^20 points
constexpr long long kStaticRed = 2 * 4096;           // reduction slots (doubles)
constexpr long long kStaticCtr = 4096 / 2;           // team counters: 4096 words
constexpr long long kStaticCtl = 8;                  // Control + iteration counter
constexpr long long kStaticDoubles = 6 * kStaticPts + kStaticRed + kStaticCtr + kStaticCtl;
static __device__ __align__(256) double scratch[kStaticDoubles];

static std::mutex g_static_mu;
static double *g_static_ptr[64] = {};
static int g_static_grid[64] = {};

// Device address of `scratch` on `device` (the current device), taken on the
// first call on that device.
static int static_scratch(int device, double **ptr, int *grid) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(PR_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, device));
        int o2 = 0, o3 = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o2, (const void *)k_coarse_cg_batch<2>, SWEEP_BLOCK, 0));
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o3, (const void *)k_coarse_cg_batch<3>, SWEEP_BLOCK, 0));
        int op = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&op, (const void *)k_coarse_cg_batch<2, true>, PCG_THREADS,
                                                            0));
        if (std::min({o2, o3, op}) < 1) return fail(PR_ENORESIDENT, "coarse solver kernel cannot be resident");
        g_static_grid[device] = prop.multiProcessorCount;
        g_static_ptr[device] = (double *)p;
    }
    *ptr = g_static_ptr[device];
    *grid = g_static_grid[device];
    return PR_OK;
}

extern "C" int pr_apply_coarse_static(const pr_config *cfg, int device, void *stream, const double *in,
                                      double *out, int count, long long *cg_iters) {
    if (cg_iters) *cg_iters = 0;
    if (!cfg) return fail(PR_EINVAL, "cfg is NULL");
    Prob P;
    int rc = derive(*cfg, P);
    if (rc) return rc;
    if (P.dim == 1) return fail(PR_EINVAL, "pr_apply_coarse_static solves 2D and 3D problems (CG); 1D has no scratch");
    if (P.npts > kStaticPts)
        return fail(PR_EINVAL, "pr_apply_coarse_static: a state of %lld points exceeds its limit of %lld",
                    (long long)P.npts, kStaticPts);
    if (!in || !out) return fail(PR_EINVAL, "NULL buffer");
    if (in == out) return fail(PR_EINVAL, "in and out must not alias");
    if (count < 0) return fail(PR_EINVAL, "count must be >= 0");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev || device >= 64) return fail(PR_EINVAL, "device %d out of range", device);
    HIPCHK(hipSetDevice(device));
    double *base = nullptr;
    int grid = 0;
    if ((rc = static_scratch(device, &base, &grid))) return rc;
    if (count == 0) return PR_OK;
    hipStream_t st = (hipStream_t)stream;
    double *r0 = base, *r1 = base + kStaticPts, *p0 = base + 2 * kStaticPts, *p1 = base + 3 * kStaticPts;
    double *w0 = base + 4 * kStaticPts, *w1 = base + 5 * kStaticPts;
    double *red = base + 6 * kStaticPts;
    unsigned *ctr = (unsigned *)(red + kStaticRed);
    Control *ctl = (Control *)(red + kStaticRed + kStaticCtr);
    unsigned long long *ci = (unsigned long long *)(red + kStaticRed + kStaticCtr + 2);
    static_assert(sizeof(Control) <= 2 * sizeof(double), "control words fit their slot");
    static_assert(TEAM_CTR_WORDS <= 2 * kStaticCtr, "team counters fit their slot");
    // counters, control words and the iteration count start at zero (a fill
    // kernel, not a memset); the previous call's contents are overwritten
    const int zw = (int)(2 * (kStaticCtr + kStaticCtl));
    hipLaunchKernelGGL(k_zero_words, dim3((zw + 255) / 256), dim3(256), 0, st, ctr, zw);
    HIPCHK(hipGetLastError());
    long long npts = P.npts;
    Geom g = P.g;
    double s = P.s, tol = P.cg_tol;
    int maxit = P.cg_maxit;
    CGWork wk{r0, p0, p1, red};
    CGWork2 wk2{{r0, r1}, {p0, p1}, red};
    CGWorkP wkp{{r0, r1}, {w0, w1}, {p0, p1}, red};
    void *args[] = {&in, &out, &npts, &count, &g, &s, &tol, &maxit, &wk, &wk2, &wkp, &ctr, &ctl, &ci};
    const void *fn = P.dim == 3 ? (const void *)k_coarse_cg_batch<3>
                                : (P.pcg ? (const void *)k_coarse_cg_batch<2, true> : (const void *)k_coarse_cg_batch<2>);
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(sweep_threads(P.dim == 2 && P.pcg)), args, 0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PR_ENORESIDENT, "cooperative launch of %d workgroups failed: %s", grid, hipGetErrorString(e));
    }
    Control c;
    unsigned long long its = 0;
    HIPCHK(hipMemcpyAsync(&c, ctl, sizeof c, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&its, ci, sizeof its, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (c.abort || c.error) return fail(PR_ETIMEOUT, "a bounded device-side wait ran out (error %d)", c.error);
    if (cg_iters) *cg_iters = (long long)its;
    return PR_OK;
}

// ------------------------------------------------------------------ serial fine
extern "C" int pr_solve_fine(pr_problem *h, const double *u0, double *lam, pr_stats *st) {
    int rc = need_single(h);
    if (rc) return rc;
    const Prob &P = h->P[0];
    if (!u0 || !lam) return fail(PR_EINVAL, "NULL buffer");
    stats_reset(st);
    if ((rc = reset_fine_its(h))) return rc;
    HIPCHK(hipEventRecord(h->ev[0], h->stream));
    if ((rc = copy_dev(h, u0, lam, P.npts))) return rc;
    Prob P1 = P;   // single-state runs may use their own tuned shape
    if (P.shape1 >= 0) P1.shape = P.shape1;
    const int passes1 = (P.m + fine_depth(P1) - 1) / fine_depth(P1);
    if (P.dim > 1 && passes1 > 1 && !h->tmp)
        if ((rc = alloc_t(h, &h->tmp, (size_t)(P.N + 1) * P.npts))) return rc;
    for (int i = 1; i <= P.N; ++i)
        if ((rc = run_fine(h, P1, lam + (long long)(i - 1) * P.npts, lam + (long long)i * P.npts, h->tmp, 1, P.m,
                           P.npts, P.npts)))
            return rc;
    HIPCHK(hipEventRecord(h->ev[1], h->stream));
    HIPCHK(hipEventSynchronize(h->ev[1]));
    if (st) {
        st->wall_ms = st->fine_ms = elapsed(h->ev[0], h->ev[1]);
        st->fine_lups = (double)P.N * P.m * (double)P.npts;
        st->converged = 1;
        st->fine_cg_iters = read_fine_its(h);
    }
    return PR_OK;
}

// ------------------------------------------------------------------ synchronous Parareal
static int batched_solve_sync(pr_problem *h, const double *u0, double *lam, pr_stats *st);
static void free_async(pr_problem *h);

extern "C" int pr_solve_sync(pr_problem *h, const double *u0, double *lam, pr_stats *st) {
    if (h && h->P.size() > 1) return batched_solve_sync(h, u0, lam, st);
    int rc = need_single(h);
    if (rc) return rc;
    const Prob &P = h->P[0];
    if (!u0 || !lam) return fail(PR_EINVAL, "NULL buffer");
    if (u0 == lam) return fail(PR_EINVAL, "u0 must not alias lambda_out");
    if (!h->v) {
        // an asynchronous solve released these buffers to fit its own (large
        // 3D iterates): give its workspace back and allocate them again
        if (h->aw_ready) free_async(h);
        if ((rc = alloc_sync_big(h))) return rc;
    }
    stats_reset(st);
    const long long np = P.npts;
    if ((rc = reset_fine_its(h))) return rc;
    HIPCHK(hipEventRecord(h->ev[0], h->stream));
    if ((rc = copy_dev(h, u0, lam, np))) return rc;
    if ((rc = zero_words(h, h->iscal, 2))) return rc;
    // initial coarse sweep (lambda^0, w^0)
    SweepArgs a = sweep_args(h, P, lam);
    a.i0 = 1;
    a.i1 = P.N;
    a.init = 1;
    if ((rc = run_sweep(h, P, a))) return rc;
    HIPCHK(hipEventRecord(h->ev[1], h->stream));
    double fine_ms = 0, coarse_ms = 0, lups = 0;
    long long gs = P.N, gskip = 0;
    int k = 0, conv = 0;
    double delta = 0;
    while (k < P.kmax) {
        ++k;
        // (1) fine propagation of every slice not yet exact: v_i = F(lambda_{i-1}), i = k..N
        HIPCHK(hipEventRecord(h->ev[2], h->stream));
        const int count = P.N - k + 1;
        if ((rc = run_fine(h, P, lam + (long long)(k - 1) * np, h->v + (long long)k * np, h->tmp, count, P.m, np, np)))
            return rc;
        lups += (double)count * P.m * (double)np;
        HIPCHK(hipEventRecord(h->ev[3], h->stream));
        // (2) sequential coarse sweep with the fused correction and change norm
        if ((rc = zero_words(h, h->dscal, 2))) return rc;
        a.i0 = k;
        a.i1 = P.N;
        a.init = 0;
        a.kguard = k;
        if (carries_corrections(P) && h->w2) {   // w^{k-1} read, w^k written (w^0: the initial sweep's, in w)
            a.wo = (k & 1) ? h->w : h->w2;
            a.w = (k & 1) ? h->w2 : h->w;
        }
        if ((rc = run_sweep(h, P, a))) return rc;
        gs += P.N - k;
        gskip += 1;
        HIPCHK(hipEventRecord(h->ev[4], h->stream));
        HIPCHK(hipMemcpyAsync(&delta, h->dscal, sizeof delta, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (P.dim > 1 && (rc = check_control(h))) return rc;
        fine_ms += elapsed(h->ev[2], h->ev[3]);
        coarse_ms += elapsed(h->ev[3], h->ev[4]);
        if (st && st->deltas && k <= st->deltas_cap) st->deltas[k - 1] = delta;
        if (P.eps > 0 && delta < P.eps) {
            conv = 1;
            break;
        }
        if (k == P.N) {
            conv = 1;   // finite termination: lambda^N is the serial fine solution
            break;
        }
    }
    HIPCHK(hipEventRecord(h->ev[5], h->stream));
    HIPCHK(hipEventSynchronize(h->ev[5]));
    coarse_ms += elapsed(h->ev[0], h->ev[1]);
    if (st) {
        unsigned long long its = 0;
        HIPCHK(hipMemcpy(&its, h->iscal, sizeof its, hipMemcpyDeviceToHost));
        st->iters = k;
        st->kappa = k;
        st->converged = conv;
        st->last_delta = delta;
        st->wall_ms = elapsed(h->ev[0], h->ev[5]);
        st->fine_ms = fine_ms;
        st->coarse_ms = coarse_ms;
        st->fine_lups = lups;
        st->cg_iters = (long long)its;
        st->g_solves = gs;
        st->g_skipped = gskip;
        st->fine_cg_iters = read_fine_its(h);
    }
    if (!conv && P.eps > 0) return fail(PR_ENOTCONV, "kmax = %d reached with delta = %.3e", P.kmax, delta);
    return PR_OK;
}

#include "host_async.inc"
#include "host_adjoint.inc"
#include "host_batched.inc"
