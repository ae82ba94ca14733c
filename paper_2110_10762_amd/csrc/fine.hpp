// Fine propagator F: explicit-Euler steps of the (2d+1)-point Laplacian with
// zero Dirichlet ghosts (the accurate per-slice solver of Section 3.1).
//
// Every slice is independent, so one launch advances a batch of states.
// All kernels are wave-granular and barrier-free:
//   1D: one wave per state, the whole state in registers (R points per lane),
//       halos by DPP lane shifts, all steps in one launch.
//   2D: register strips.  A wave owns 64*XP columns by R+2D rows (XP points
//       per lane in x, one register per row), loads them once from HBM, does
//       up to D steps (temporal blocking: the valid region shrinks by one row
//       and column per step), and writes back the inner R x (64*XP - 2D)
//       block.  y-neighbours are other registers of the same lane, x-neighbours
//       come from DPP lane shifts.
//   2D sliding window: a wave owns 64*XP columns and a segment of rows that
//       it marches down, holding two rows per time level (see fine2d_sw).
//   3D: one step per pass; a wave owns an (x, y) strip of 64*XP by R+2 and
//       marches along z with three planes in registers.
// Out-of-domain halo values are loaded from the odd reflection of the state
// (see reflect()), which keeps the ghost values exactly zero without masks.
#pragma once
#include "common.hpp"

namespace pr {

// ------------------------------------------------------------------ 1D
template <int R>
__device__ __forceinline__ void fine1d_regs(double (&c)[R], const double (&rl)[R], int steps) {
    for (int t = 0; t < steps; ++t) {
        const double left_edge = from_lower_lane(c[R - 1]);
        const double right_edge = from_upper_lane(c[0]);
        double prev = left_edge;
#pragma unroll
        for (int e = 0; e < R; ++e) {
            const double cur = c[e];
            const double nxt = (e + 1 < R) ? c[e + 1] : right_edge;
            const double tt = __builtin_fma(-2.0, cur, prev + nxt);
            c[e] = __builtin_fma(rl[e], tt, cur);
            prev = cur;
        }
    }
}

template <int R>
__device__ __forceinline__ void load1d(const double *src, int n, double r, double (&c)[R], double (&rl)[R]) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int p = lane * R + e;
        c[e] = p < n ? src[p] : 0.0;
        rl[e] = p < n ? r : 0.0;   // padding points stay exactly zero
    }
}

template <int R>
__device__ __forceinline__ void store1d(double *dst, int n, const double (&c)[R]) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int p = lane * R + e;
        if (p < n) dst[p] = c[e];
    }
}

// grid: one wave (block of 64) per state
template <int R>
__global__ __launch_bounds__(64) void k_fine1d(const double *__restrict__ src, double *__restrict__ dst,
                                               long long sstride, long long dstride, int n, double r,
                                               int steps, int count) {
    const int st = blockIdx.x;
    if (st >= count) return;
    double c[R], rl[R];
    load1d<R>(src + (long long)st * sstride, n, r, c, rl);
    fine1d_regs<R>(c, rl, steps);
    store1d<R>(dst + (long long)st * dstride, n, c);
}

// ------------------------------------------------------------------ 2D
// left + right neighbour of each of a lane's XP consecutive points of one row
// (lane edges by DPP); every 2D kernel uses this order so they round alike.
template <int XP>
__device__ __forceinline__ void x_neighbour_sums(const double (&cur)[XP], double (&lr)[XP]) {
    if constexpr (XP == 1) {
        lr[0] = from_lower_lane(cur[0]) + from_upper_lane(cur[0]);
    } else {
        lr[0] = from_lower_lane(cur[XP - 1]) + cur[1];
#pragma unroll
        for (int e = 1; e < XP - 1; ++e) lr[e] = cur[e - 1] + cur[e + 1];
        lr[XP - 1] = cur[XP - 2] + from_upper_lane(cur[0]);
    }
}

template <int XP, int R, int D>
struct Shape2D {
    static constexpr int H = R + 2 * D;          // rows held per lane
    static constexpr int W = WAVE * XP - 2 * D;  // useful columns per strip
};

// One strip pass: load, `steps` (<= D) explicit-Euler steps, store.
template <int XP, int R, int D>
__device__ __forceinline__ void fine2d_strip(const double *__restrict__ src, double *__restrict__ dst,
                                             int n, double r, int steps, int sx, int sy) {
    constexpr int H = Shape2D<XP, R, D>::H;
    constexpr int W = Shape2D<XP, R, D>::W;
    const int lane = threadIdx.x & (WAVE - 1);
    const int x0 = sx * W - D;
    const int y0 = sy * R - D;
    double c[XP][H];
    int xi[XP];
    double xs[XP];
#pragma unroll
    for (int e = 0; e < XP; ++e) xi[e] = reflect(x0 + lane * XP + e, n, xs[e]);
#pragma unroll
    for (int j = 0; j < H; ++j) {
        double ys;
        const int yi = reflect(y0 + j, n, ys);
        const double *row = src + (long long)yi * n;
#pragma unroll
        for (int e = 0; e < XP; ++e) c[e][j] = (ys * xs[e]) * row[xi[e]];
    }
    for (int t = 0; t < steps; ++t) {
        double prev[XP];
#pragma unroll
        for (int e = 0; e < XP; ++e) prev[e] = c[e][0];
#pragma unroll
        for (int j = 1; j < H - 1; ++j) {
            double cur[XP], lr[XP];
#pragma unroll
            for (int e = 0; e < XP; ++e) cur[e] = c[e][j];
            x_neighbour_sums<XP>(cur, lr);
#pragma unroll
            for (int e = 0; e < XP; ++e) {
                c[e][j] = euler_update(cur[e], lr[e], prev[e] + c[e][j + 1], 4.0, r);
                prev[e] = cur[e];
            }
        }
    }
#pragma unroll
    for (int j = D; j < D + R; ++j) {
        const int y = y0 + j;
        if (y < n) {
            double *row = dst + (long long)y * n;
#pragma unroll
            for (int e = 0; e < XP; ++e) {
                const int lx = lane * XP + e;
                const int x = x0 + lx;
                if (lx >= D && lx < D + W && x < n) row[x] = c[e][j];
            }
        }
    }
}

// Workgroups are re-indexed so that each XCD (dispatch round-robins blocks
// over the 8 XCDs) receives a contiguous range of strips: vertically
// adjacent strips then share their halo rows through that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nblk) {
    const int per = (nblk + 7) / 8;
    return (b % 8) * per + b / 8;
}

template <int XP, int R, int D>
__global__ __launch_bounds__(BLOCK) void k_fine2d(const double *__restrict__ src, double *__restrict__ dst,
                                                  long long sstride, long long dstride, int n, double r,
                                                  int steps, int nsx, int nsy, int count, int nblk) {
    const int L = xcd_remap(blockIdx.x, nblk);
    if (L >= nblk) return;
    const long long wv = (long long)L * WAVES_PER_BLOCK + wave_id();
    const long long per_state = (long long)nsx * nsy;
    if (wv >= per_state * count) return;
    const int st = (int)(wv / per_state);
    const int rem = (int)(wv - (long long)st * per_state);
    const int sy = rem % nsy;          // vertical neighbours are consecutive waves
    const int sx = rem / nsy;
    fine2d_strip<XP, R, D>(src + st * sstride, dst + st * dstride, n, r, steps, sx, sy);
}

// ---- 2D sliding window
// A wave owns the same 64*XP columns as a register strip (useful width
// W = 64*XP - 2D), but a segment [ya, yb) of output rows that it marches
// through one input row at a time.  For every time level t < D it keeps the
// two most recent rows of that level in registers, so level t+1 of the row
// one behind is formed as soon as level t of the newest row exists, and level
// D leaves for HBM D rows behind the input.  Levels t >= steps (the short last
// pass of a slice) use coefficient 0, which copies the value exactly, so every
// pass runs the same branch-free code.  Only the 2D halo rows of a segment and
// the 2D halo columns of a strip are computed twice.  Odd segments march
// upwards: two neighbouring segments then read their shared halo rows at the
// same time (the second read hits L2).  Addition is commutative, so the
// direction does not change a single bit; the update order is that of the
// register strip.
// Row counts of at least this select the sliding window in shape tables and
// kernel templates (register strips hold at most 64 rows).
constexpr int SW_MIN_ROWS = 96;
// Segment length of a sliding-window shape chosen at each launch from the
// number of states, so that the (strip, segment) units fill the resident
// waves in whole rounds (a launch of 49 states of 1024^2 in 128-row segments
// is 1.15 rounds of the chip's wave slots, so its second round runs 15% full).
constexpr int SW_AUTO_ROWS = 1000;

// Odd reflection of row y (wave-uniform, so scalar work): the interior row
// to read and its sign.
__device__ __forceinline__ int reflect_row(int y, int n, double &ys) {
    const int P = 2 * (n + 1);
    int t = y + 1;
    if (t < 0 || t >= P) {
        t %= P;
        if (t < 0) t += P;
    }
    int yi = t - 1;
    ys = 1.0;
    if (t == 0 || t == n + 1) {
        yi = 0;
        ys = 0.0;
    } else if (t > n) {
        yi = P - t - 1;
        ys = -1.0;
    }
    return __builtin_amdgcn_readfirstlane(yi);
}

// Issues the loads of row yi (no wait: the values are used PF rows later).
// VEC: the lane's XP points are contiguous and 16-byte aligned (an interior
// strip, XP even): XP/2 16-byte loads, so each instruction moves whole lines.
template <int XP, bool VEC>
__device__ __forceinline__ void issue_row2d(const double *__restrict__ src, int n, int yi, const unsigned (&xo)[XP],
                                            double (&v)[XP]) {
    const char *row = reinterpret_cast<const char *>(src + (long long)yi * n);
    if constexpr (VEC) {
#pragma unroll
        for (int e = 0; e < XP; e += 2) {
            const double2 t = *reinterpret_cast<const double2 *>(row + xo[e]);
            v[e] = t.x;
            v[e + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < XP; ++e) v[e] = *reinterpret_cast<const double *>(row + xo[e]);
    }
}

template <int XP, int D>
struct ShapeSW {
    static constexpr int W = WAVE * XP - 2 * D;
    static constexpr int PF = XP >= 4 ? 4 : 8;   // input rows in flight ahead of the window
};

// Strips of a sliding-window pass.  A wave holds C = 64 XP columns; after D
// levels the values in its outer D columns on a side are invalid, unless that
// side lies on the domain boundary: there the lane shift's zero fill is the
// Dirichlet ghost value itself, at every level.  A grid at least C wide takes
// one strip flush with each boundary (C - D owned columns each) and interior
// strips of C - 2D between them (1024 columns: 120 + 7 x 112 + 120, nine
// strips instead of ten); a narrower grid reads the odd extension on both
// sides of every strip.  Every point is computed alike in either layout.
// (C = 64 XP columns per wave, D levels)
__host__ __device__ inline int sw_strip_count(int C, int D, int n) {
    const int W = C - 2 * D, WB = C - D;
    if (n < C) return (n + W - 1) / W;
    if (n <= 2 * WB) return n == C ? 1 : 2;
    return 2 + (n - 2 * WB + W - 1) / W;
}

template <int XP, int D>
__host__ __device__ inline int sw_strips(int n) {
    return sw_strip_count(WAVE * XP, D, n);
}

// First column x0 of strip sx's wave (negative: odd extension) and the lane
// columns [lo, hi) it owns.
template <int XP, int D>
__device__ __forceinline__ void sw_strip(int sx, int n, int &x0, int &lo, int &hi) {
    constexpr int C = WAVE * XP, W = C - 2 * D, WB = C - D;
    if (n < C) {
        x0 = sx * W - D;
        lo = D;
        hi = min(D + W, n - x0);
        return;
    }
    const int ns = sw_strips<XP, D>(n);
    if (ns == 1 || sx == 0) {
        x0 = 0;
        lo = 0;
        hi = ns == 1 ? C : WB;
        return;
    }
    const int start = WB + (sx - 1) * W;   // first owned column
    if (sx == ns - 1) {
        x0 = n - C;
        lo = start - x0;
        hi = C;
        return;
    }
    x0 = start - D;
    lo = D;
    hi = D + W;
}

// PF: input rows in flight ahead of the window (more hides HBM latency, fewer
// saves registers).
template <int XP, int D, int PF, bool VEC>
__device__ __forceinline__ void fine2d_sw_body(const double *__restrict__ src, double *__restrict__ dst, int n,
                                               double r, int steps, int sx, int ya, int yb, bool upward) {
    const int lane = threadIdx.x & (WAVE - 1);
    int x0, lo, hi;
    sw_strip<XP, D>(sx, n, x0, lo, hi);
    unsigned xo[XP];   // byte offsets of the lane's columns (reflected)
    double xs[XP];
    bool own[XP];
#pragma unroll
    for (int e = 0; e < XP; ++e) {
        const int lx = lane * XP + e;
        xo[e] = (unsigned)reflect(x0 + lx, n, xs[e]) * 8u;
        own[e] = lx >= lo && lx < hi;
    }
    double rt[D];
#pragma unroll
    for (int t = 0; t < D; ++t) rt[t] = t < steps ? r : 0.0;
    double w0[D][XP], w1[D][XP];   // level t: the rows two and one behind its newest
#pragma unroll
    for (int t = 0; t < D; ++t)
#pragma unroll
        for (int e = 0; e < XP; ++e) w0[t][e] = w1[t][e] = 0.0;
    // input rows ya-D .. yb+D-1 in march order; raw values and row signs in a ring
    const int dir = upward ? -1 : 1;
    const int first = upward ? yb - 1 + D : ya - D;
    const int nrows = (yb - ya) + 2 * D;
    double pf[PF][XP], ps[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int yi = reflect_row(first + dir * q, n, ps[q]);
        if (q < nrows) {
            issue_row2d<XP, VEC>(src, n, yi, xo, pf[q]);
        } else {
#pragma unroll
            for (int e = 0; e < XP; ++e) pf[q][e] = 0.0;
        }
    }
    for (int kb = 0; kb < nrows; kb += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = kb + q;
            double c[XP];
#pragma unroll
            for (int e = 0; e < XP; ++e) c[e] = (ps[q] * xs[e]) * pf[q][e];
            if (k + PF < nrows) {
                const int yi = reflect_row(first + dir * (k + PF), n, ps[q]);
                issue_row2d<XP, VEC>(src, n, yi, xo, pf[q]);
            }
#pragma unroll
            for (int t = 0; t < D; ++t) {
                double lr[XP];
                x_neighbour_sums<XP>(w1[t], lr);
#pragma unroll
                for (int e = 0; e < XP; ++e) {
                    const double nx = euler_update(w1[t][e], lr[e], w0[t][e] + c[e], 4.0, rt[t]);
                    w0[t][e] = w1[t][e];
                    w1[t][e] = c[e];
                    c[e] = nx;
                }
            }
            const int y = first + dir * (k - D);
            if (k < nrows && y >= ya && y < yb) {
                double *row = dst + (long long)y * n;
                if constexpr (VEC) {   // owned points come in aligned pairs here
#pragma unroll
                    for (int e = 0; e < XP; e += 2)
                        if (own[e]) *reinterpret_cast<double2 *>(row + x0 + lane * XP + e) = make_double2(c[e], c[e + 1]);
                } else {
#pragma unroll
                    for (int e = 0; e < XP; ++e)
                        if (own[e]) row[x0 + lane * XP + e] = c[e];
                }
            }
        }
    }
}

// A strip wholly inside the grid with XP even, n even and the halo even reads
// and writes 16-byte pairs; every other strip goes through the reflection.
// (VEC_OK = false keeps a single copy of the body, for kernels whose size or
// registers matter more than the fine pass.)
template <int XP, int D, int PF = ShapeSW<XP, D>::PF, bool VEC_OK = true>
__device__ __forceinline__ void fine2d_sw(const double *__restrict__ src, double *__restrict__ dst, int n,
                                          double r, int steps, int sx, int ya, int yb, bool upward) {
    if constexpr (VEC_OK && XP % 2 == 0 && D % 2 == 0) {
        int x0, lo, hi;
        sw_strip<XP, D>(sx, n, x0, lo, hi);
        if (x0 >= 0 && x0 + WAVE * XP <= n && (n & 1) == 0) {
            fine2d_sw_body<XP, D, PF, true>(src, dst, n, r, steps, sx, ya, yb, upward);
            return;
        }
    }
    fine2d_sw_body<XP, D, PF, false>(src, dst, n, r, steps, sx, ya, yb, upward);
}

// Output rows [sy*ry, sy*ry + ry) of strip sx.
template <int XP, int D>
__global__ __launch_bounds__(BLOCK) void k_fine2d_sw(const double *__restrict__ src, double *__restrict__ dst,
                                                     long long sstride, long long dstride, int n, double r,
                                                     int steps, int nsx, int nsy, int ry, int count, int nblk) {
    const int L = xcd_remap(blockIdx.x, nblk);
    if (L >= nblk) return;
    const long long wv = (long long)L * WAVES_PER_BLOCK + wave_id();
    const long long per_state = (long long)nsx * nsy;
    if (wv >= per_state * count) return;
    const int st = (int)(wv / per_state);
    const int rem = (int)(wv - (long long)st * per_state);
    const int sx = rem % nsx;   // strips of the same rows side by side: adjacent memory in flight
    const int sy = rem / nsx;
    const int ya = sy * ry;
    fine2d_sw<XP, D>(src + st * sstride, dst + st * dstride, n, r, steps, sx, ya, min(n, ya + ry), sy & 1);
}

// ------------------------------------------------------------------ 3D
template <int XP, int R>
__device__ __forceinline__ void load_plane3d(const double *__restrict__ src, int n, int z, int y0,
                                             const int (&xi)[XP], const double (&xs)[XP],
                                             double (&p)[XP][R + 2]) {
    double zs;
    const int zi = reflect(z, n, zs);
    const double *pl = src + (long long)zi * n * n;
#pragma unroll
    for (int j = 0; j < R + 2; ++j) {
        double ys;
        const int yi = reflect(y0 + j, n, ys);
        const double *row = pl + (long long)yi * n;
#pragma unroll
        for (int e = 0; e < XP; ++e) p[e][j] = (zs * ys * xs[e]) * row[xi[e]];
    }
}

template <int XP, int R>
__device__ __forceinline__ void step_plane3d(double *__restrict__ dst, int n, int z, int y0, int x0,
                                             double r, const double (&pm)[XP][R + 2],
                                             const double (&pc)[XP][R + 2], const double (&pp)[XP][R + 2]) {
    constexpr int W = WAVE * XP - 2;
    const int lane = threadIdx.x & (WAVE - 1);
    if (z >= n) return;
    double *pl = dst + (long long)z * n * n;
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        double lr[XP];
        if constexpr (XP == 1) {
            lr[0] = from_lower_lane(pc[0][j]) + from_upper_lane(pc[0][j]);
        } else {
            lr[0] = from_lower_lane(pc[XP - 1][j]) + pc[1][j];
#pragma unroll
            for (int e = 1; e < XP - 1; ++e) lr[e] = pc[e - 1][j] + pc[e + 1][j];
            lr[XP - 1] = pc[XP - 2][j] + from_upper_lane(pc[0][j]);
        }
        const int y = y0 + j;
#pragma unroll
        for (int e = 0; e < XP; ++e) {
            const double s2 = (pc[e][j - 1] + pc[e][j + 1]) + (pm[e][j] + pp[e][j]);
            const double v = euler_update(pc[e][j], lr[e], s2, 6.0, r);
            const int lx = lane * XP + e;
            const int x = x0 + lx;
            if (y < n && lx >= 1 && lx < 1 + W && x < n) pl[(long long)y * n + x] = v;
        }
    }
}

// One explicit-Euler step of a 3D state, strip (sx, sy) over planes [z0, z1).
template <int XP, int R>
__device__ __forceinline__ void fine3d_strip(const double *__restrict__ src, double *__restrict__ dst,
                                             int n, double r, int sx, int sy, int z0, int z1) {
    constexpr int W = WAVE * XP - 2;
    const int lane = threadIdx.x & (WAVE - 1);
    const int x0 = sx * W - 1;
    const int y0 = sy * R - 1;
    int xi[XP];
    double xs[XP];
#pragma unroll
    for (int e = 0; e < XP; ++e) xi[e] = reflect(x0 + lane * XP + e, n, xs[e]);
    double a[XP][R + 2], b[XP][R + 2], c[XP][R + 2];
    load_plane3d<XP, R>(src, n, z0 - 1, y0, xi, xs, a);
    load_plane3d<XP, R>(src, n, z0, y0, xi, xs, b);
    int z = z0;
    // unrolled by three so that the plane roles rotate without register moves
    while (z < z1) {
        load_plane3d<XP, R>(src, n, z + 1, y0, xi, xs, c);
        step_plane3d<XP, R>(dst, n, z, y0, x0, r, a, b, c);
        if (++z >= z1) break;
        load_plane3d<XP, R>(src, n, z + 1, y0, xi, xs, a);
        step_plane3d<XP, R>(dst, n, z, y0, x0, r, b, c, a);
        if (++z >= z1) break;
        load_plane3d<XP, R>(src, n, z + 1, y0, xi, xs, b);
        step_plane3d<XP, R>(dst, n, z, y0, x0, r, c, a, b);
        ++z;
    }
}

template <int XP, int R>
__global__ __launch_bounds__(BLOCK) void k_fine3d(const double *__restrict__ src, double *__restrict__ dst,
                                                  long long sstride, long long dstride, int n, double r,
                                                  int nsx, int nsy, int nsz, int zc, int count, int nblk) {
    const int L = xcd_remap(blockIdx.x, nblk);
    if (L >= nblk) return;
    const long long wv = (long long)L * WAVES_PER_BLOCK + wave_id();
    const long long per_state = (long long)nsx * nsy * nsz;
    if (wv >= per_state * count) return;
    const int st = (int)(wv / per_state);
    int rem = (int)(wv - (long long)st * per_state);
    const int sy = rem % nsy;
    rem /= nsy;
    const int sz = rem % nsz;
    const int sx = rem / nsz;
    const int z0 = sz * zc;
    const int z1 = min(n, z0 + zc);
    fine3d_strip<XP, R>(src + st * sstride, dst + st * dstride, n, r, sx, sy, z0, z1);
}

// Depth-D pass of a 3D state (temporal blocking along z): strip (sx, sy) of
// W = 64 - 2D columns, one per lane (x-neighbours by DPP), and R rows, over
// planes [z0, z1).  The wave marches up z one input plane at a time and
// holds, for each level, the two most recent planes of the level below
// (R + 2D rows of its column); level l + 1 forms plane k - l - 1 as soon as
// plane k - l of level l exists, so level D reaches HBM D planes behind the
// input.  Level l + 1 is formed on rows [l + 1, R + 2D - l - 1) of the lane's
// column, the rows its successor reads; halo rows, columns and planes are
// recomputed, not exchanged.  Planes, rows and columns outside the grid are
// the odd extension, which every update keeps exactly, so the zero Dirichlet
// values need no masks.  Levels at and beyond `steps` copy (coefficient 0).
// Each point is formed as in k_fine3d, so the two kernels agree bit for bit.
template <int R, int D, int PF>
__device__ __forceinline__ void fine3d_tb_strip(const double *__restrict__ src, double *__restrict__ dst, int n,
                                                double r, int steps, int sx, int sy, int z0, int z1) {
    constexpr int Y = R + 2 * D;   // rows of the lane's column, halo included
    const int lane = threadIdx.x & (WAVE - 1);
    const int x0 = sx * (WAVE - 2 * D) - D;
    double xs;
    const unsigned xo = (unsigned)reflect(x0 + lane, n, xs) * 8u;   // byte offset of the lane's column
    const bool own = lane >= D && lane < WAVE - D && x0 + lane < n;
    const int y0 = sy * R - D;
    int yo[Y];   // reflected row offsets and signs (wave-uniform)
    double ysg[Y];
#pragma unroll
    for (int j = 0; j < Y; ++j) yo[j] = reflect(y0 + j, n, ysg[j]) * n;
    double rt[D];
#pragma unroll
    for (int t = 0; t < D; ++t) rt[t] = t < steps ? r : 0.0;
    double w0[D][Y], w1[D][Y];   // level l: planes two and one behind its newest
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
        for (int j = 0; j < Y; ++j) w0[l][j] = w1[l][j] = 0.0;
    const int nk = (z1 - z0) + 2 * D;   // input planes z0 - D .. z1 + D - 1
    const int k0 = z0 - D;
    const long long nn = (long long)n * n;
    double ring[PF][Y], zsg[PF];
    // row addresses are wave-uniform, the lane offset is 32-bit
    auto issue = [&](int kk, double (&w)[Y], double &sg) {
        const int zi = reflect(kk, n, sg);
        const double *pl = src + zi * nn;
#pragma unroll
        for (int j = 0; j < Y; ++j) w[j] = *reinterpret_cast<const double *>(reinterpret_cast<const char *>(pl + yo[j]) + xo);
    };
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        zsg[q] = 0.0;
#pragma unroll
        for (int j = 0; j < Y; ++j) ring[q][j] = 0.0;
        if (q < nk) issue(k0 + q, ring[q], zsg[q]);
    }
    for (int kb = 0; kb < nk; kb += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int t = kb + q;
            if (t >= nk) break;
            double c[Y];
#pragma unroll
            for (int j = 0; j < Y; ++j) c[j] = (zsg[q] * ysg[j] * xs) * ring[q][j];
            if (t + PF < nk) issue(k0 + t + PF, ring[q], zsg[q]);
            // level l + 1 at plane k - l - 1, row by row in place: row j
            // needs rows j - 1 .. j + 1 of the older plane of level l, so the
            // row below is kept in `below` once its slot has moved on
#pragma unroll
            for (int l = 0; l < D; ++l) {
                double below = w1[l][l];
                w0[l][l] = w1[l][l];
                w1[l][l] = c[l];
#pragma unroll
                for (int j = l + 1; j < Y - l - 1; ++j) {
                    const double cur = w1[l][j];
                    const double lr = from_lower_lane(cur) + from_upper_lane(cur);
                    const double s2 = (below + w1[l][j + 1]) + (w0[l][j] + c[j]);
                    const double v = euler_update(cur, lr, s2, 6.0, rt[l]);
                    w0[l][j] = cur;
                    w1[l][j] = c[j];
                    c[j] = v;
                    below = cur;
                }
                w0[l][Y - l - 1] = w1[l][Y - l - 1];
                w1[l][Y - l - 1] = c[Y - l - 1];
            }
            const int z = k0 + t - D;
            if (z >= z0 && z < z1 && own) {
                double *pl = dst + z * nn;
                const int x = x0 + lane;
#pragma unroll
                for (int j = D; j < Y - D; ++j)
                    if (y0 + j < n) (pl + (long long)(y0 + j) * n)[x] = c[j];
            }
        }
    }
}

// PF: input planes in flight ahead of the march.
template <int R, int D, int PF>
__global__ __launch_bounds__(BLOCK) void k_fine3d_tb(const double *__restrict__ src, double *__restrict__ dst,
                                                     long long sstride, long long dstride, int n, double r,
                                                     int steps, int nsx, int nsy, int nsz, int zc, int count,
                                                     int nblk) {
    const int L = xcd_remap(blockIdx.x, nblk);
    if (L >= nblk) return;
    const long long wv = (long long)L * WAVES_PER_BLOCK + wave_id();
    const long long per_state = (long long)nsx * nsy * nsz;
    if (wv >= per_state * count) return;
    const int st = (int)(wv / per_state);
    int rem = (int)(wv - (long long)st * per_state);
    const int sx = rem % nsx;   // strips of the same rows side by side
    rem /= nsx;
    const int sy = rem % nsy;
    const int sz = rem / nsy;
    const int z0 = sz * zc;
    fine3d_tb_strip<R, D, PF>(src + st * sstride, dst + st * dstride, n, r, steps, sx, sy, z0, min(n, z0 + zc));
}

}  // namespace pr
