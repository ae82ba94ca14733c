// Coarse propagator G: one backward-Euler step of length dT,
//     (I - nu dT L_h) w = x,
// the cheap per-slice solver of Section 3.1 (the paper's experiment uses
// backward Euler as G, Section 5.1).
//   1D: the tridiagonal system is solved by the Thomas algorithm written as
//       two first-order affine recurrences and evaluated by one wave with a
//       log-depth lane scan (the elimination factors are the same for every
//       slice and iteration and are precomputed once on the host).
//   2D/3D: conjugate gradients started from x0 = b, stopped at
//       ||r||_2 <= tol ||b||_2, executed by a team of workgroups with
//       deterministic team reductions.  2D: the Chronopoulos-Gear variant
//       with one barrier per iteration and the products recomputed (48 B per
//       point and iteration).  3D: the textbook recurrences, two barriers per
//       iteration, the search-direction update fused into the matrix-vector
//       product (64 B per point and iteration).
#pragma once
#include "common.hpp"

namespace pr {

// ------------------------------------------------------------------ 1D Thomas
// With a = c = -s, b = 1 + 2s and inv_i = 1 / (b - a c'_{i-1}), c'_i = -s inv_i:
//   forward   d_i = s inv_i d_{i-1} + inv_i x_i        (coefficient 0 at i = 0)
//   backward  w_i = s inv_i w_{i+1} + d_i             (coefficient 0 at i = n-1)
// Each lane holds R consecutive points; a lane's points compose to one affine
// map, and the maps are combined across lanes by a Hillis-Steele scan.
template <int R>
__device__ __forceinline__ void thomas_wave(double (&x)[R], const double (&inv)[R], int n, double s) {
    const int lane = threadIdx.x & (WAVE - 1);
    double fa[R];
    double A = 1.0, B = 0.0;
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int i = lane * R + e;
        fa[e] = (i == 0 || i >= n) ? 0.0 : s * inv[e];
        const double fb = x[e] * inv[e];
        B = __builtin_fma(fa[e], B, fb);
        A = fa[e] * A;
        x[e] = fb;
    }
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const double Ap = __shfl_up(A, o, WAVE);
        const double Bp = __shfl_up(B, o, WAVE);
        if (lane >= o) {
            B = __builtin_fma(A, Bp, B);
            A = A * Ap;
        }
    }
    double d = __shfl_up(B, 1, WAVE);
    if (lane == 0) d = 0.0;
#pragma unroll
    for (int e = 0; e < R; ++e) {
        d = __builtin_fma(fa[e], d, x[e]);
        x[e] = d;
    }
    // backward recurrence, scanned from the top lane down
    double bc[R];
    double C = 1.0, E = 0.0;
#pragma unroll
    for (int e = R - 1; e >= 0; --e) {
        const int i = lane * R + e;
        bc[e] = (i >= n - 1) ? 0.0 : s * inv[e];
        E = __builtin_fma(bc[e], E, x[e]);
        C = bc[e] * C;
    }
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const double Cp = __shfl_down(C, o, WAVE);
        const double Ep = __shfl_down(E, o, WAVE);
        if (lane + o < WAVE) {
            E = __builtin_fma(C, Ep, E);
            C = C * Cp;
        }
    }
    double w = __shfl_down(E, 1, WAVE);
    if (lane == WAVE - 1) w = 0.0;
#pragma unroll
    for (int e = R - 1; e >= 0; --e) {
        w = __builtin_fma(bc[e], w, x[e]);
        x[e] = w;
    }
}

template <int R>
__device__ __forceinline__ void load_inv(const double *tab, double (&inv)[R]) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int e = 0; e < R; ++e) inv[e] = tab[lane * R + e];   // table padded to 64*R
}

template <int R>
__global__ __launch_bounds__(64) void k_thomas(const double *__restrict__ src, double *__restrict__ dst,
                                               long long stride, int n, double s, const double *inv_tab,
                                               int count) {
    const int st = blockIdx.x;
    if (st >= count) return;
    const int lane = threadIdx.x;
    double x[R], inv[R];
    load_inv<R>(inv_tab, inv);
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int p = lane * R + e;
        x[e] = p < n ? src[st * stride + p] : 0.0;
    }
    thomas_wave<R>(x, inv, n, s);
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int p = lane * R + e;
        if (p < n) dst[st * stride + p] = x[e];
    }
}

// ------------------------------------------------------------------ geometry
// A state is split into chunks of 64 consecutive x values of one grid row;
// a team's workgroups own contiguous chunk ranges, its waves stride over them.
struct Geom {
    int dim, n;
    long long npts;
    int cpr;            // chunks per row
    long long nchunks;  // rows * cpr
};

__host__ __device__ inline Geom make_geom(int dim, int n) {
    Geom g;
    g.dim = dim;
    g.n = n;
    long long rows = 1;
    for (int d = 1; d < dim; ++d) rows *= n;
    g.npts = rows * n;
    g.cpr = (n + WAVE - 1) / WAVE;
    g.nchunks = rows * g.cpr;
    return g;
}

struct ChunkRange {
    long long begin, end;
};

__device__ __forceinline__ ChunkRange team_chunks(const Geom &g, int rank, int size) {
    const long long per = (g.nchunks + size - 1) / size;
    ChunkRange cr;
    cr.begin = per * rank;
    cr.end = min(g.nchunks, cr.begin + per);
    return cr;
}

struct Point {
    long long idx;
    int x, y, z;
    bool valid;
};

__device__ __forceinline__ Point chunk_point(const Geom &g, long long c) {
    const int lane = threadIdx.x & (WAVE - 1);
    const long long row = c / g.cpr;
    const int cx = (int)(c - row * g.cpr);
    Point p;
    p.x = cx * WAVE + lane;
    if (g.dim == 3) {
        p.y = (int)(row % g.n);
        p.z = (int)(row / g.n);
    } else {
        p.y = (int)row;
        p.z = 0;
    }
    p.valid = p.x < g.n;
    p.idx = row * g.n + p.x;
    return p;
}

// Streaming passes over a team's chunks visit them U per wave at a time (the
// chunks c, c + nw, ..., c + (U-1)·nw of a wave's stride, in that order), so
// that a wave has the loads of U chunks in flight before it uses any: one
// chunk per memory round trip left a quarter of the GPU at about 1.3 TB/s on
// a plain copy.  Points past the range or the row are invalid; their index is
// 0, a safe address to load from and never stored to.
constexpr int STREAM_U = 4;

template <int U>
__device__ __forceinline__ void chunk_points(const Geom &g, long long c, long long end, int nw, Point (&p)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long cc = c + (long long)u * nw;
        p[u] = chunk_point(g, cc < end ? cc : c);
        p[u].valid = p[u].valid && cc < end;
        if (!p[u].valid) p[u].idx = 0;
    }
}

// Sum of the 2d neighbour values (zero outside the domain), in the order
// ((y-pair [+ z-pair]) + x-pair).  A chunk holds 64 consecutive x values of
// one row, one per lane, so the x-neighbours come from the adjacent lanes by
// DPP; only the chunk's end lanes load across the chunk border.  `center` is
// the lane's own value (0 for lanes past the end of the row); f(j) loads the
// value at index j.
template <typename Fn>
__device__ __forceinline__ double neighbour_sum(const Geom &g, const Point &p, double center, Fn f) {
    const int lane = threadIdx.x & (WAVE - 1);
    const long long n = g.n;
    double xl = from_lower_lane(center);
    double xr = from_upper_lane(center);
    if (lane == 0) xl = p.x > 0 ? f(p.idx - 1) : 0.0;
    if (lane == WAVE - 1) xr = (p.x + 1 < g.n) ? f(p.idx + 1) : 0.0;
    double s2 = 0.0;
    if (g.dim >= 2) {
        const double yu = (p.valid && p.y > 0) ? f(p.idx - n) : 0.0;
        const double yd = (p.valid && p.y + 1 < g.n) ? f(p.idx + n) : 0.0;
        s2 = yu + yd;
        if (g.dim == 3) {
            const double zf = (p.valid && p.z > 0) ? f(p.idx - n * n) : 0.0;
            const double zb = (p.valid && p.z + 1 < g.n) ? f(p.idx + n * n) : 0.0;
            s2 = s2 + (zf + zb);
        }
    }
    return s2 + (xl + xr);
}

// (I - s h^2 L_h) y at a point, given y there and the neighbour sum.
__device__ __forceinline__ double be_point(double yc, double nsum, double twod, double s) {
    const double lap = __builtin_fma(-twod, yc, nsum);
    return __builtin_fma(-s, lap, yc);
}

// Row-segment length of a marching sweep: `strips` columns of waves (times
// planes in 3D) over n rows, shared by `waves` waves, one (strip, segment)
// unit per wave and round.  The shortest segment of at least minseg rows
// whose units all fit in one round; a whole strip when even one segment per
// strip leaves more units than waves.  (Rounding the rows per wave up before
// the segments per strip can leave a few units for a second round, which
// doubles the sweep's critical path.)
__device__ __forceinline__ int march_seg(int n, long long strips, int waves, int minseg) {
    const long long fit = waves / strips;   // segments per strip in one round
    const int seg = fit > 0 ? (int)((n + fit - 1) / fit) : n;
    return max(min(minseg, n), seg);
}

// ------------------------------------------------------------------ CG
struct CGWork {
    double *r, *p0, *p1;   // [npts] each
    double *red;           // [2 * team size] reduction slots
};

// A chunk point for the CG phases: its index (a state holds < 2^31 points)
// and which neighbours exist.  A missing neighbour (outside the domain, or
// any neighbour of a lane past the row end) is read at the point itself and
// masked, so all loads can be issued unconditionally and early.  The edge
// neighbour is the x-neighbour across the chunk border (lane 0: left, lane 63:
// right); the other x-neighbours come by DPP.
struct CPt {
    int c;
    unsigned m;   // bits: valid, up, down, front, back, edge
};
constexpr unsigned CP_VALID = 1, CP_UP = 2, CP_DN = 4, CP_FR = 8, CP_BK = 16, CP_EDGE = 32;

__device__ __forceinline__ CPt cpt_at(const Geom &g, long long chunk) {
    const int lane = threadIdx.x & (WAVE - 1);
    const Point p = chunk_point(g, chunk);
    CPt q;
    q.c = (int)(p.valid ? p.idx : p.idx - p.x);
    unsigned m = 0;
    if (p.valid) {
        m |= CP_VALID;
        if (g.dim >= 2 && p.y > 0) m |= CP_UP;
        if (g.dim >= 2 && p.y + 1 < g.n) m |= CP_DN;
        if (g.dim == 3 && p.z > 0) m |= CP_FR;
        if (g.dim == 3 && p.z + 1 < g.n) m |= CP_BK;
        if ((lane == 0 && p.x > 0) || (lane == WAVE - 1 && p.x + 1 < g.n)) m |= CP_EDGE;
    }
    q.m = m;
    return q;
}

// Loads the value of the point and of its neighbours: v[0] centre, v[1] up,
// v[2] down, v[3] edge, v[4] front, v[5] back (DIM == 3).
template <int DIM, typename Fn>
__device__ __forceinline__ void cpt_load(const CPt &q, int n, Fn f, double (&v)[2 * DIM]) {
    const int lane = threadIdx.x & (WAVE - 1);
    v[0] = f(q.c);
    v[1] = f((q.m & CP_UP) ? q.c - n : q.c);
    v[2] = f((q.m & CP_DN) ? q.c + n : q.c);
    v[3] = f((q.m & CP_EDGE) ? (lane == 0 ? q.c - 1 : q.c + 1) : q.c);
    if constexpr (DIM == 3) {
        v[4] = f((q.m & CP_FR) ? q.c - n * n : q.c);
        v[5] = f((q.m & CP_BK) ? q.c + n * n : q.c);
    }
}

// (I - s h^2 L_h) applied at the point: centre value masked to 0 past the
// row end, neighbour sum in the order of neighbour_sum.
template <int DIM>
__device__ __forceinline__ double cpt_apply(const CPt &q, const double (&v)[2 * DIM], double &center,
                                            double twod, double s) {
    const int lane = threadIdx.x & (WAVE - 1);
    center = (q.m & CP_VALID) ? v[0] : 0.0;
    double xl = from_lower_lane(center);
    double xr = from_upper_lane(center);
    const double ve = (q.m & CP_EDGE) ? v[3] : 0.0;
    if (lane == 0) xl = ve;
    if (lane == WAVE - 1) xr = ve;
    double s2 = ((q.m & CP_UP) ? v[1] : 0.0) + ((q.m & CP_DN) ? v[2] : 0.0);
    if constexpr (DIM == 3) s2 = s2 + (((q.m & CP_FR) ? v[4] : 0.0) + ((q.m & CP_BK) ? v[5] : 0.0));
    return be_point(center, s2 + (xl + xr), twod, s);
}

// ------------------------------------------------------------------ 3D CG phases, marching
// The phases of the two-phase CG below for a team whose waves each own a long
// run of rows: a wave takes a strip of 64 x-values in one z-plane and a
// segment of y-rows and marches down it, keeping three rows of the stencil
// operand in registers and loading, PF rows ahead, the next row of its plane
// and the two rows beside the output row in the planes z - 1 and z + 1.  The
// operand v and the stores per mode:
//   CG3_A: v = r + beta p_old (r when `first`); p = v, sum v.(A v);
//   CG3_B: v = p; x += alpha v, r -= alpha A v (in place), sum r.r;
//   CG3_S: v = b (set-up with x0 = b); x = b, r = b - A b, sums r.r and b.b;
//   CG3_W: v = x0, a given guess (set-up); x = x0, r = b - A x0 with b (vb)
//          read at the output point, sums r.r and b.b;
//   CG3_WC: CG3_W carrying the previous slice's correction: b = v + (wn - wo)
//          from the terms at the output point (vb = the correction's v), also
//          stored into lam, with the largest change |b - lam_old|.
// A v is formed exactly as in the chunk-wise phases (cpt_apply's order).
enum { CG3_A = 0, CG3_B = 1, CG3_S = 2, CG3_W = 3, CG3_WC = 4 };

// The correction of the previous slice, carried by the set-up march of the
// next slice's solve: its right-hand side b = v + (wn - wo) (eq. (pr), the
// terms added in the order of the separate correction pass, so the values
// are the same bits) is formed where the march reads b, and stored into lam
// at the points the wave owns.  v == NULL: no correction.
struct SetupCorr {
    const double *v = nullptr, *wn = nullptr, *wo = nullptr;
    double *lam = nullptr;
};

struct SW3Row {    // raw loads for one step: centre row (with the strip-border
                   // point) and the two side rows, of one or two vectors;
                   // CG3_WC: the correction's terms at the output point
    double ac, ae, am, ap, bc, be, bm, bp, xo, ro;
    double cw, co, cl;
};

template <int MODE>
__device__ __forceinline__ void sw3_issue(const double *__restrict__ va, const double *__restrict__ vb,
                                          const double *__restrict__ x, const double *__restrict__ r, int n, int z,
                                          int k, int ya, int yb, int xcol, bool lv, int eoff, bool eok,
                                          bool use_b, SW3Row &w, const SetupCorr &sc) {
    const long long plane = (long long)n * n;
    const bool kok = k >= 0 && k < n;
    const int y = k - 1;                        // output row of this step
    const bool yok = y >= ya && y < yb;
    const long long base = ((long long)z * n + (kok ? k : 0)) * n + xcol;
    const long long ob = ((long long)z * n + (yok ? y : 0)) * n + xcol;
    const long long ic = (kok && lv) ? base : 0;
    const long long ie = (kok && eok) ? base + eoff : 0;
    const long long im = (yok && lv && z > 0) ? ob - plane : 0;
    const long long ip = (yok && lv && z + 1 < n) ? ob + plane : 0;
    w.ac = va[ic];
    w.ae = va[ie];
    w.am = va[im];
    w.ap = va[ip];
    if (use_b) {
        w.bc = vb[ic];
        w.be = vb[ie];
        w.bm = vb[im];
        w.bp = vb[ip];
    }
    if constexpr (MODE == CG3_B) {
        const long long io = (yok && lv) ? ob : 0;
        w.xo = x[io];
        w.ro = r[io];
    }
    if constexpr (MODE == CG3_W) w.ro = vb[(yok && lv) ? ob : 0];   // b at the output point
    if constexpr (MODE == CG3_WC) {   // b's terms and the old lambda at the output point
        const long long io = (yok && lv) ? ob : 0;
        w.ro = vb[io];
        w.cw = sc.wn[io];
        w.co = sc.wo[io];
        w.cl = sc.lam[io];
    }
}

template <int MODE, int PF>
__device__ __forceinline__ void cg3_sweep_sw(const Geom &g, int rank, int size, double s, double coef,
                                             bool first, const double *__restrict__ va,
                                             const double *__restrict__ vb, double *__restrict__ x,
                                             double *__restrict__ r, double *__restrict__ pout, double &acc0,
                                             double &acc1, const SetupCorr sc = SetupCorr{},
                                             double *dm = nullptr) {
    const int n = g.n;
    double dml = 0.0;   // CG3_WC: largest change of the carried correction
    const int lane = threadIdx.x & (WAVE - 1);
    const bool l0 = lane == 0, l63 = lane == WAVE - 1;
    const int waves = size * nwaves();
    const int wid = rank * nwaves() + wave_id();
    const bool use_b = MODE == CG3_A && !first;
    // y-segments: one (strip, plane, segment) unit per wave, at least 16 rows
    const int seg = march_seg(n, (long long)g.cpr * n, waves, 16);
    const int nseg = (n + seg - 1) / seg;
    const long long units = (long long)g.cpr * n * nseg;
    for (long long u = wid; u < units; u += waves) {
        const int sx = (int)(u % g.cpr);
        const long long rem = u / g.cpr;
        const int z = (int)(rem % n);
        const int ya = (int)(rem / n) * seg;
        const int yb = min(n, ya + seg);
        const int xcol = sx * WAVE + lane;
        const bool lv = xcol < n;
        const bool eok = (l0 && xcol > 0) || (l63 && xcol + 1 < n);
        const int eoff = l0 ? -1 : 1;
        const bool zmok = z > 0, zpok = z + 1 < n;
        const int nrows = yb - ya + 2;   // centre rows ya-1 .. yb
        double vm2 = 0.0, vm1c = 0.0, vm1l = 0.0, vm1r = 0.0;   // v at rows k-2 (centre) and k-1
        SW3Row ring[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q)
            if (q < nrows)
                sw3_issue<MODE>(va, vb, x, r, n, z, ya - 1 + q, ya, yb, xcol, lv, eoff, eok, use_b, ring[q], sc);
        for (int tb = 0; tb < nrows; tb += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int t = tb + q;
                if (t >= nrows) break;
                const int k = ya - 1 + t;
                const SW3Row w = ring[q];
                if (t + PF < nrows)
                    sw3_issue<MODE>(va, vb, x, r, n, z, k + PF, ya, yb, xcol, lv, eoff, eok, use_b, ring[q], sc);
                const bool kok = k >= 0 && k < n;
                const int y = k - 1;
                const bool yok = y >= ya && y < yb;
                // v at row k (centre, strip-border point) and at row y in the planes z -/+ 1
                double vc = (kok && lv) ? w.ac : 0.0;
                double ve = (kok && eok) ? w.ae : 0.0;
                double vmz = (yok && lv && zmok) ? w.am : 0.0;
                double vpz = (yok && lv && zpok) ? w.ap : 0.0;
                if (use_b) {
                    vc = __builtin_fma(coef, (kok && lv) ? w.bc : 0.0, vc);
                    ve = __builtin_fma(coef, (kok && eok) ? w.be : 0.0, ve);
                    vmz = __builtin_fma(coef, (yok && lv && zmok) ? w.bm : 0.0, vmz);
                    vpz = __builtin_fma(coef, (yok && lv && zpok) ? w.bp : 0.0, vpz);
                }
                // lane shifts on every lane, then the strip-border lanes
                const double sl = from_lower_lane(vc), sr = from_upper_lane(vc);
                const double vl = l0 ? ve : sl;
                const double vr = l63 ? ve : sr;
                if (yok) {
                    // A v at (x, y, z): ((up + down) + (front + back)) + (left + right)
                    const double s2 = (vm2 + vc) + (vmz + vpz);
                    const double av = be_point(vm1c, s2 + (vm1l + vm1r), 6.0, s);
                    if (lv) {
                        const long long i = ((long long)z * n + y) * n + xcol;
                        if constexpr (MODE == CG3_A) {
                            pout[i] = vm1c;
                            acc0 = __builtin_fma(vm1c, av, acc0);
                        } else if constexpr (MODE == CG3_B) {
                            x[i] = __builtin_fma(coef, vm1c, w.xo);
                            const double rv = __builtin_fma(-coef, av, w.ro);
                            r[i] = rv;
                            acc0 = __builtin_fma(rv, rv, acc0);
                        } else if constexpr (MODE == CG3_S) {
                            const double rv = vm1c - av;
                            x[i] = vm1c;
                            r[i] = rv;
                            acc0 = __builtin_fma(rv, rv, acc0);
                            acc1 = __builtin_fma(vm1c, vm1c, acc1);
                        } else if constexpr (MODE == CG3_WC) {
                            const double bo = w.ro + (w.cw - w.co);
                            dml = fmax(dml, fabs(bo - w.cl));
                            sc.lam[i] = bo;
                            const double rv = bo - av;
                            x[i] = vm1c;
                            r[i] = rv;
                            acc0 = __builtin_fma(rv, rv, acc0);
                            acc1 = __builtin_fma(bo, bo, acc1);
                        } else {
                            const double rv = w.ro - av;
                            x[i] = vm1c;
                            r[i] = rv;
                            acc0 = __builtin_fma(rv, rv, acc0);
                            acc1 = __builtin_fma(w.ro, w.ro, acc1);
                        }
                    }
                }
                vm2 = vm1c;
                vm1c = vc;
                vm1l = vl;
                vm1r = vr;
            }
        }
    }
    if constexpr (MODE == CG3_WC) *dm = fmax(*dm, dml);
}

// Solves (I - s h^2 L_h) x = b by CG with the team (DIM = 2 or 3; U chunks
// per wave and loop trip, whose loads are all issued before the first is
// used: memory-level parallelism against register use).  Returns
// the iteration count, or -1 if the launch was aborted.  x and b must not
// alias.  All lanes of a wave run every chunk (lanes past the row end carry
// zeros) so that the lane shifts see the whole chunk.
//   abs_thresh2 < 0: x0 = b (or the guess xg, marching 3D set-up only), stop
//                    at ||r||^2 <= tol^2 ||b||^2 (the coarse propagator
//                    applied to a state);
//   abs_thresh2 >= 0: x0 = 0, stop at ||r||^2 <= abs_thresh2 (applied to the
//                    change of a state: a zero right-hand side returns 0).
// Per iteration: phase A forms p = r + beta p_old (recomputed at the
// neighbours from r and p_old), stores p and reduces <p, A p>; phase B
// updates x and r, recomputing A p from the stored p (bit-identical to phase
// A's value) instead of storing it: 64 B of HBM traffic per point.
// SW3 (DIM = 3): the two phases and the set-up from x0 = b march
// (cg3_sweep_sw) instead of visiting chunks.
// SW3 with a guess xg and sc.v given: the set-up carries the previous slice's
// correction (CG3_WC; b unused, the change goes into *dm).
template <int DIM, int U, bool SW3 = false>
__device__ int cg_team_dim(Team &tm, const Geom &g, double s, double tol, int maxit,
                           const double *__restrict__ b, double *__restrict__ x, const CGWork &wk,
                           double abs_thresh2, const double *__restrict__ xg = nullptr,
                           const SetupCorr sc = SetupCorr{}, double *dm = nullptr) {
    static_assert(!SW3 || DIM == 3, "the marching phases are three-dimensional");
    constexpr int V = 2 * DIM;
    __shared__ double lds[MAX_WAVES];
    const double twod = 2.0 * DIM;
    const int n = g.n;
    const ChunkRange cr = team_chunks(g, tm.rank, tm.size);
    const int w = wave_id();
    const long long nw = nwaves();
    double *__restrict__ r = wk.r;
    const bool from_zero = abs_thresh2 >= 0.0;

    double rr_p = 0.0, bb_p = 0.0, unused = 0.0;
    if (SW3 && !from_zero && xg && sc.v)
        cg3_sweep_sw<CG3_WC, 4>(g, tm.rank, tm.size, s, 0.0, true, xg, sc.v, x, r, nullptr, rr_p, bb_p, sc, dm);
    else if (SW3 && !from_zero && xg)
        cg3_sweep_sw<CG3_W, 4>(g, tm.rank, tm.size, s, 0.0, true, xg, b, x, r, nullptr, rr_p, bb_p);
    else if (SW3 && !from_zero)
        cg3_sweep_sw<CG3_S, 4>(g, tm.rank, tm.size, s, 0.0, true, b, nullptr, x, r, nullptr, rr_p, bb_p);
    else
    for (long long c0 = cr.begin + w; c0 < cr.end; c0 += U * nw) {
        CPt q[U];
        bool act[U];
        double v[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long c = c0 + u * nw;
            act[u] = c < cr.end;
            q[u] = cpt_at(g, act[u] ? c : c0);
            if (from_zero) {
                v[u][0] = b[q[u].c];
            } else {
                cpt_load<DIM>(q[u], n, [&](int j) { return b[j]; }, v[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool keep = act[u] && (q[u].m & CP_VALID);
            if (from_zero) {                       // r = b, x = 0
                const double bv = v[u][0];
                if (keep) {
                    x[q[u].c] = 0.0;
                    r[q[u].c] = bv;
                    rr_p = __builtin_fma(bv, bv, rr_p);
                }
            } else {                               // r = b - A b, x = b
                double bv;
                const double ab = cpt_apply<DIM>(q[u], v[u], bv, twod, s);
                const double rv = bv - ab;
                if (keep) {
                    x[q[u].c] = bv;
                    r[q[u].c] = rv;
                    rr_p = __builtin_fma(rv, rv, rr_p);
                    bb_p = __builtin_fma(bv, bv, bb_p);
                }
            }
        }
    }
    double rr, thresh;
    if (from_zero) {
        if (!team_reduce<false>(tm, rr_p, wk.red, rr, lds)) return -1;
        thresh = abs_thresh2 > 0.0 ? abs_thresh2 : tol * tol * rr;
    } else {
        double bb;
        if (!team_reduce<false>(tm, bb_p, wk.red, bb, lds)) return -1;
        if (!team_reduce<false>(tm, rr_p, wk.red, rr, lds)) return -1;
        thresh = tol * tol * bb;
    }

    const double *pold = r;   // first direction: p = r (beta = 0)
    double beta = 0.0;
    double *pcur = wk.p0;
    int it = 0;
    while (it < maxit && rr > thresh) {
        // phase A: p = r + beta p_old (also at the neighbours), <p, A p>
        double pq_p = 0.0;
        if (SW3)
            cg3_sweep_sw<CG3_A, 4>(g, tm.rank, tm.size, s, beta, it == 0, r, pold, nullptr, nullptr, pcur, pq_p,
                                   unused);
        else
        for (long long c0 = cr.begin + w; c0 < cr.end; c0 += U * nw) {
            CPt q[U];
            bool act[U];
            double v[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long c = c0 + u * nw;
                act[u] = c < cr.end;
                q[u] = cpt_at(g, act[u] ? c : c0);
                cpt_load<DIM>(q[u], n, [&](int j) { return __builtin_fma(beta, pold[j], r[j]); }, v[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double pv;
                const double qv = cpt_apply<DIM>(q[u], v[u], pv, twod, s);
                if (act[u] && (q[u].m & CP_VALID)) {
                    pcur[q[u].c] = pv;
                    pq_p = __builtin_fma(pv, qv, pq_p);
                }
            }
        }
        double pq;
        if (!team_reduce<false>(tm, pq_p, wk.red, pq, lds)) return -1;
        const double alpha = rr / pq;
        // phase B: x += alpha p, r -= alpha A p, <r, r>
        double rn_p = 0.0;
        if (SW3)
            cg3_sweep_sw<CG3_B, 4>(g, tm.rank, tm.size, s, alpha, false, pcur, nullptr, x, r, nullptr, rn_p,
                                   unused);
        else
        for (long long c0 = cr.begin + w; c0 < cr.end; c0 += U * nw) {
            CPt q[U];
            bool act[U];
            double v[U][V], xc[U], rc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long c = c0 + u * nw;
                act[u] = c < cr.end;
                q[u] = cpt_at(g, act[u] ? c : c0);
                cpt_load<DIM>(q[u], n, [&](int j) { return pcur[j]; }, v[u]);
                xc[u] = x[q[u].c];
                rc[u] = r[q[u].c];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double pv;
                const double qv = cpt_apply<DIM>(q[u], v[u], pv, twod, s);
                if (act[u] && (q[u].m & CP_VALID)) {
                    x[q[u].c] = __builtin_fma(alpha, pv, xc[u]);
                    const double rv = __builtin_fma(-alpha, qv, rc[u]);
                    r[q[u].c] = rv;
                    rn_p = __builtin_fma(rv, rv, rn_p);
                }
            }
        }
        double rn;
        if (!team_reduce<false>(tm, rn_p, wk.red, rn, lds)) return -1;
        beta = rn / rr;
        rr = rn;
        pold = pcur;
        pcur = (pcur == wk.p0) ? wk.p1 : wk.p0;
        ++it;
    }
    return it;
}

// ------------------------------------------------------------------ 2D CG, one synchronisation per iteration
// The Chronopoulos-Gear form of CG: with w = A r and s = A p, both inner
// products of an iteration, (r, r) and (w, r), can be reduced together, so an
// iteration costs one team barrier instead of two.  Neither w nor s is
// stored: a wave recomputes A p at the point and its four neighbours from p
// (hence p at distance 2), updates r there, and forms w' = A r' at the point.
// Stored state: x, r, p (r and p double-buffered), 48 B of HBM traffic per
// point and iteration; the extra reads of the distance-2 rows hit the
// caches.  Iteration i:
//   p_i = r_i + beta_i p_{i-1},  x_{i+1} = x_i + alpha_i p_i,
//   r_{i+1} = r_i - alpha_i A p_i,  gamma = (r_{i+1}, r_{i+1}),
//   delta = (A r_{i+1}, r_{i+1}),  beta_{i+1} = gamma_{i+1} / gamma_i,
//   alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1} / alpha_i).
// Every value at a point (p, A p, r') is formed by the same operations in
// the same order wherever it is needed, so all copies agree bit for bit.
struct CGWork2 {
    double *r[2], *p[2];   // [npts] each
    double *red;           // [6 * team size] reduction slots
};
// The same vectors, solved with the marching sweep (cg2_sweep_sw below).
struct CGWork2M : CGWork2 {};

// A chunk point of the distance-2 star: its index, the addresses of the
// loads (missing points read the point itself and are masked) and masks.
struct D2Pt {
    int c;                    // the point (the row start for lanes past the row end)
    int u, d, uu, dd;         // rows y-1, y+1, y-2, y+2 at x
    int e1, e2, ue, de;       // lane 0: x-1, x-2, (x-1, y-1), (x-1, y+1); lane 63: the same at x+1, x+2
    unsigned m;
};
constexpr unsigned D2_V = 1, D2_U = 2, D2_D = 4, D2_UU = 8, D2_DD = 16, D2_E1 = 32, D2_E2 = 64, D2_XL = 128,
                   D2_XR = 256;

__device__ __forceinline__ D2Pt d2_at(const Geom &g, long long chunk) {
    const int lane = threadIdx.x & (WAVE - 1);
    const Point p = chunk_point(g, chunk);
    const int n = g.n;
    D2Pt q;
    q.c = (int)(p.valid ? p.idx : p.idx - p.x);
    unsigned m = 0;
    const bool up = p.y > 0, dn = p.y + 1 < n, uu = p.y > 1, dd = p.y + 2 < n;
    if (p.valid) {
        m |= D2_V;
        if (up) m |= D2_U;
        if (dn) m |= D2_D;
        if (uu) m |= D2_UU;
        if (dd) m |= D2_DD;
        if (p.x > 0) m |= D2_XL;
        if (p.x + 1 < n) m |= D2_XR;
    }
    // edge lanes: the neighbours across the chunk border (lane 0 is always
    // valid; lane 63's right neighbours exist only inside the row)
    int e1 = q.c, e2 = q.c;
    if (lane == 0 && p.x > 0) {
        m |= D2_E1 | D2_E2;   // x >= 64
        e1 = q.c - 1;
        e2 = q.c - 2;
    } else if (lane == WAVE - 1 && p.x + 1 < n) {
        m |= D2_E1;
        e1 = q.c + 1;
        if (p.x + 2 < n) {
            m |= D2_E2;
            e2 = q.c + 2;
        }
    }
    q.u = (m & D2_U) ? q.c - n : q.c;
    q.d = (m & D2_D) ? q.c + n : q.c;
    q.uu = (m & D2_UU) ? q.c - 2 * n : q.c;
    q.dd = (m & D2_DD) ? q.c + 2 * n : q.c;
    q.e1 = e1;
    q.e2 = e2;
    q.ue = ((m & D2_E1) && up) ? e1 - n : q.c;
    q.de = ((m & D2_E1) && dn) ? e1 + n : q.c;
    q.m = m;
    return q;
}

// The 13 values of a state on the distance-2 star of a point (zero outside
// the domain): row y at x-2..x+2, rows y-1 and y+1 at x-1..x+1, rows y-2 and
// y+2 at x.
struct Star13 {
    double c, l1, l2, r1, r2;
    double u, ul, ur;
    double d, dl, dr;
    double uu, dd;
};

struct Raw9 {
    double c, u, d, uu, dd, e1, e2, ue, de;
};

__device__ __forceinline__ void d2_load(const D2Pt &q, const double *__restrict__ v, Raw9 &w) {
    w.c = v[q.c];
    w.u = v[q.u];
    w.d = v[q.d];
    w.uu = v[q.uu];
    w.dd = v[q.dd];
    w.e1 = v[q.e1];
    w.e2 = v[q.e2];
    w.ue = v[q.ue];
    w.de = v[q.de];
}

__device__ __forceinline__ Star13 d2_star(const D2Pt &q, const Raw9 &w) {
    const int lane = threadIdx.x & (WAVE - 1);
    const bool l0 = lane == 0, l63 = lane == WAVE - 1;
    const unsigned m = q.m;
    const bool ok = m & D2_V;
    Star13 t;
    t.c = ok ? w.c : 0.0;
    t.u = (m & D2_U) ? w.u : 0.0;      // D2_U etc. imply D2_V
    t.d = (m & D2_D) ? w.d : 0.0;
    t.uu = (m & D2_UU) ? w.uu : 0.0;
    t.dd = (m & D2_DD) ? w.dd : 0.0;
    const double e1 = (m & D2_E1) ? w.e1 : 0.0;
    const double e2 = (m & D2_E2) ? w.e2 : 0.0;
    const double ue = ((m & D2_E1) && (m & D2_U)) ? w.ue : 0.0;
    const double de = ((m & D2_E1) && (m & D2_D)) ? w.de : 0.0;
    const double cl = from_lower_lane(t.c), cr = from_upper_lane(t.c);
    t.l1 = l0 ? e1 : cl;
    t.r1 = l63 ? e1 : cr;
    const double ll = from_lower_lane(t.l1), rr = from_upper_lane(t.r1);
    t.l2 = l0 ? e2 : ll;
    t.r2 = l63 ? e2 : rr;
    const double ul = from_lower_lane(t.u), ur = from_upper_lane(t.u);
    t.ul = l0 ? ue : ul;
    t.ur = l63 ? ue : ur;
    const double dl = from_lower_lane(t.d), dr = from_upper_lane(t.d);
    t.dl = l0 ? de : dl;
    t.dr = l63 ? de : dr;
    return t;
}

// One sweep of the 2D CG: p = r + beta p_old on the star (p = r when
// `first`), A p at the point and its neighbours, r' = r - alpha A p there
// (zero outside the domain), w' = A r' at the point; stores x + alpha p, r'
// and (unless `setup`) p; accumulates (r', r'), (w', r') and (r, r).
// At set-up r is the right-hand side b, first is set and x is taken as 0.
// The loads of a wave's first chunk of a sweep, issued early: between the
// barrier that ends an iteration and the reading of the reduction slots,
// whose round trip they then overlap.
struct Cg2Pre {
    D2Pt q;
    Raw9 wr, wp;
    double xo;
    bool ok;   // the wave has a chunk
};

__device__ __forceinline__ void cg2_preload(const Geom &g, const ChunkRange &cr, bool first, bool setup,
                                            const double *__restrict__ r, const double *__restrict__ pold,
                                            const double *__restrict__ x, Cg2Pre &pre) {
    const long long c = cr.begin + wave_id();
    pre.ok = c < cr.end;
    if (!pre.ok) return;
    pre.q = d2_at(g, c);
    d2_load(pre.q, r, pre.wr);
    if (!first) d2_load(pre.q, pold, pre.wp);
    pre.xo = setup ? 0.0 : x[pre.q.c];
}

// One sweep, one chunk per wave and loop trip; the first chunk's loads come
// from `pre` when it holds them.
__device__ __forceinline__ void cg2_chunk(const D2Pt &q, const Raw9 &wr, const Raw9 &wp, double xo, double s,
                                          double alpha, double beta, bool first, bool setup,
                                          double *__restrict__ x, double *__restrict__ rnew,
                                          double *__restrict__ pnew, double &ga, double &de, double &rr) {
    const Star13 R = d2_star(q, wr);
    Star13 P = R;
    if (!first) {
        const Star13 Po = d2_star(q, wp);
        P.c = __builtin_fma(beta, Po.c, R.c);
        P.l1 = __builtin_fma(beta, Po.l1, R.l1);
        P.l2 = __builtin_fma(beta, Po.l2, R.l2);
        P.r1 = __builtin_fma(beta, Po.r1, R.r1);
        P.r2 = __builtin_fma(beta, Po.r2, R.r2);
        P.u = __builtin_fma(beta, Po.u, R.u);
        P.ul = __builtin_fma(beta, Po.ul, R.ul);
        P.ur = __builtin_fma(beta, Po.ur, R.ur);
        P.d = __builtin_fma(beta, Po.d, R.d);
        P.dl = __builtin_fma(beta, Po.dl, R.dl);
        P.dr = __builtin_fma(beta, Po.dr, R.dr);
        P.uu = __builtin_fma(beta, Po.uu, R.uu);
        P.dd = __builtin_fma(beta, Po.dd, R.dd);
    }
    // A p at the point and its neighbours: (up + down) + (left + right)
    const double ap_c = be_point(P.c, (P.u + P.d) + (P.l1 + P.r1), 4.0, s);
    const double ap_l = be_point(P.l1, (P.ul + P.dl) + (P.l2 + P.c), 4.0, s);
    const double ap_r = be_point(P.r1, (P.ur + P.dr) + (P.c + P.r2), 4.0, s);
    const double ap_u = be_point(P.u, (P.uu + P.c) + (P.ul + P.ur), 4.0, s);
    const double ap_d = be_point(P.d, (P.c + P.dd) + (P.dl + P.dr), 4.0, s);
    const unsigned m = q.m;
    const double rc = (m & D2_V) ? __builtin_fma(-alpha, ap_c, R.c) : 0.0;
    const double rl = (m & D2_XL) ? __builtin_fma(-alpha, ap_l, R.l1) : 0.0;
    const double rrt = (m & D2_XR) ? __builtin_fma(-alpha, ap_r, R.r1) : 0.0;
    const double ru = (m & D2_U) ? __builtin_fma(-alpha, ap_u, R.u) : 0.0;
    const double rd = (m & D2_D) ? __builtin_fma(-alpha, ap_d, R.d) : 0.0;
    const double wn = be_point(rc, (ru + rd) + (rl + rrt), 4.0, s);
    if (m & D2_V) {
        const int i = q.c;
        x[i] = __builtin_fma(alpha, P.c, xo);
        rnew[i] = rc;
        if (!setup) pnew[i] = P.c;
        ga = __builtin_fma(rc, rc, ga);
        de = __builtin_fma(wn, rc, de);
        rr = __builtin_fma(R.c, R.c, rr);
    }
}

__device__ __forceinline__ void cg2_sweep(const Geom &g, const ChunkRange &cr, double s, double alpha, double beta,
                                          bool first, bool setup, const double *__restrict__ r,
                                          const double *__restrict__ pold, double *__restrict__ x,
                                          double *__restrict__ rnew, double *__restrict__ pnew, double &ga,
                                          double &de, double &rr, const Cg2Pre *pre) {
    const long long nw = nwaves();
    long long c = cr.begin + wave_id();
    if (pre && pre->ok) {
        cg2_chunk(pre->q, pre->wr, pre->wp, pre->xo, s, alpha, beta, first, setup, x, rnew, pnew, ga, de, rr);
        c += nw;
    }
    for (; c < cr.end; c += nw) {
        const D2Pt q = d2_at(g, c);
        Raw9 wr, wp;
        d2_load(q, r, wr);
        if (!first) d2_load(q, pold, wp);
        const double xo = setup ? 0.0 : x[q.c];
        cg2_chunk(q, wr, wp, xo, s, alpha, beta, first, setup, x, rnew, pnew, ga, de, rr);
    }
}

// The same sweep for a team whose waves each own a long run of rows: a
// wave takes a strip of 64 columns and a segment of rows and marches down
// it, loading each input row of r and p_old once (4 rows ahead, so their
// loads are in flight together) and keeping the last rows of p, A p and r'
// in registers.  Every value is formed exactly as in cg2_sweep (the same
// operations in the same order); only the order in which the partial sums
// are accumulated differs.
struct SWRow {          // raw loads of one input row: centre and the two edge points
    double rc, r1, r2, pc, p1, p2, xo;
};

__device__ __forceinline__ void sw_issue(const double *__restrict__ r, const double *__restrict__ pold,
                                         const double *__restrict__ x, int n, int k, int xcol, bool lv, int e1off,
                                         int e2off, bool e1ok, bool e2ok, bool first, bool setup, bool xrow,
                                         SWRow &w) {
    const bool rowok = k >= 0 && k < n;
    const int base = rowok ? k * n + xcol : 0;
    const int ic = (rowok && lv) ? base : 0;
    const int i1 = (rowok && e1ok) ? base + e1off : 0;
    const int i2 = (rowok && e2ok) ? base + e2off : 0;
    w.rc = r[ic];
    w.r1 = r[i1];
    w.r2 = r[i2];
    if (!first) {
        w.pc = pold[ic];
        w.p1 = pold[i1];
        w.p2 = pold[i2];
    }
    // x of the output row (two rows behind the input row)
    w.xo = (!setup && xrow && lv) ? x[(k - 2) * n + xcol] : 0.0;
}

template <int PF, int MINSEG>
__device__ __forceinline__ void cg2_sweep_sw(const Geom &g, int rank, int size, double s, double alpha,
                                             double beta, bool first, bool setup, const double *__restrict__ r,
                                             const double *__restrict__ pold, double *__restrict__ x,
                                             double *__restrict__ rnew, double *__restrict__ pnew, double &ga,
                                             double &de, double &rr) {
    const int n = g.n;
    const int lane = threadIdx.x & (WAVE - 1);
    const bool l0 = lane == 0, l63 = lane == WAVE - 1;
    const int waves = size * nwaves();
    const int wid = rank * nwaves() + wave_id();
    // segments of rows: one (strip, segment) unit per wave, at least MINSEG rows
    const int seg = march_seg(n, g.cpr, waves, MINSEG);
    const int nseg = (n + seg - 1) / seg;
    const int units = g.cpr * nseg;
    for (int u = wid; u < units; u += waves) {
        const int sx = u % g.cpr;
        const int ya = (u / g.cpr) * seg;
        const int yb = min(n, ya + seg);
        const int xcol = sx * WAVE + lane;
        const bool lv = xcol < n;
        const bool xl = lv && xcol > 0, xr = xcol + 1 < n;
        // edge points across the strip border (lane 0 is always inside the row)
        const bool e1ok = (l0 && xcol > 0) || (l63 && xcol + 1 < n);
        const bool e2ok = (l0 && xcol > 0) || (l63 && xcol + 2 < n);
        const int e1off = l0 ? -1 : 1, e2off = l0 ? -2 : 2;
        const int nrows = yb - ya + 4;   // input rows ya-2 .. yb+1
        // window: p at rows k-2 (c, l1, r1) and k-1 (c, l1, r1, l2, r2); r at
        // row k-1 (c, l1, r1) and the centre of row k-2; r' at rows k-3
        // (centre) and k-2 (c, l, r)
        double pm2c = 0, pm2l = 0, pm2r = 0, pm1c = 0, pm1l = 0, pm1r = 0, pm1l2 = 0, pm1r2 = 0;
        double rm1c = 0, rm1l = 0, rm1r = 0, rm2c = 0;
        double qm3c = 0, qm2c = 0, qm2l = 0, qm2r = 0;
        SWRow ring[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int k = ya - 2 + q;
            if (q < nrows)
                sw_issue(r, pold, x, n, k, xcol, lv, e1off, e2off, e1ok, e2ok, first, setup,
                         k - 2 >= ya && k - 2 < yb, ring[q]);
        }
        for (int tb = 0; tb < nrows; tb += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int t = tb + q;
                if (t >= nrows) break;
                const int k = ya - 2 + t;
                const bool rowok = k >= 0 && k < n;
                // row k: r and p (masked), then refill the slot
                const SWRow w = ring[q];
                if (t + PF < nrows) {
                    const int kk = k + PF;
                    sw_issue(r, pold, x, n, kk, xcol, lv, e1off, e2off, e1ok, e2ok, first, setup,
                             kk - 2 >= ya && kk - 2 < yb, ring[q]);
                }
                const double Rc = (rowok && lv) ? w.rc : 0.0;
                const double R1 = (rowok && e1ok) ? w.r1 : 0.0;
                const double R2 = (rowok && e2ok) ? w.r2 : 0.0;
                double Pc = Rc, P1 = R1, P2 = R2;
                if (!first) {
                    Pc = __builtin_fma(beta, (rowok && lv) ? w.pc : 0.0, Rc);
                    P1 = __builtin_fma(beta, (rowok && e1ok) ? w.p1 : 0.0, R1);
                    P2 = __builtin_fma(beta, (rowok && e2ok) ? w.p2 : 0.0, R2);
                }
                // lane shifts first, on every lane: a shift evaluated only where
                // the edge test fails would read inactive lanes as zero
                const double sRl = from_lower_lane(Rc), sRr = from_upper_lane(Rc);
                const double sPl = from_lower_lane(Pc), sPr = from_upper_lane(Pc);
                const double Rl = l0 ? R1 : sRl;
                const double Rr = l63 ? R1 : sRr;
                const double Pl = l0 ? P1 : sPl;
                const double Pr = l63 ? P1 : sPr;
                const double sPl2 = from_lower_lane(Pl), sPr2 = from_upper_lane(Pr);
                const double Pl2 = l0 ? P2 : sPl2;
                const double Pr2 = l63 ? P2 : sPr2;
                // row j = k-1: A p at (x, j), (x-1, j), (x+1, j); r' there
                const int j = k - 1;
                const bool jok = j >= 0 && j < n;
                const double apc = be_point(pm1c, (pm2c + Pc) + (pm1l + pm1r), 4.0, s);
                const double apl = be_point(pm1l, (pm2l + Pl) + (pm1l2 + pm1c), 4.0, s);
                const double apr = be_point(pm1r, (pm2r + Pr) + (pm1c + pm1r2), 4.0, s);
                const double qc = (jok && lv) ? __builtin_fma(-alpha, apc, rm1c) : 0.0;
                const double ql = (jok && xl) ? __builtin_fma(-alpha, apl, rm1l) : 0.0;
                const double qr = (jok && xr) ? __builtin_fma(-alpha, apr, rm1r) : 0.0;
                // row y = k-2: A r' at (x, y), stores, partial sums
                const int y = k - 2;
                if (y >= ya && y < yb) {
                    const double wn = be_point(qm2c, (qm3c + qc) + (qm2l + qm2r), 4.0, s);
                    if (lv) {
                        const int i = y * n + xcol;
                        x[i] = __builtin_fma(alpha, pm2c, w.xo);
                        rnew[i] = qm2c;
                        if (!setup) pnew[i] = pm2c;
                        ga = __builtin_fma(qm2c, qm2c, ga);
                        de = __builtin_fma(wn, qm2c, de);
                        rr = __builtin_fma(rm2c, rm2c, rr);
                    }
                }
                // shift the window
                qm3c = qm2c;
                qm2c = qc;
                qm2l = ql;
                qm2r = qr;
                rm2c = rm1c;
                rm1c = Rc;
                rm1l = Rl;
                rm1r = Rr;
                pm2c = pm1c;
                pm2l = pm1l;
                pm2r = pm1r;
                pm1c = Pc;
                pm1l = Pl;
                pm1r = Pr;
                pm1l2 = Pl2;
                pm1r2 = Pr2;
            }
        }
    }
}

// Solves (I - s h^2 L_h) x = b in 2D; same start and stop rules as
// cg_team_dim (abs_thresh2 < 0: x0 = b, relative stop; >= 0: x0 = 0,
// absolute stop).  Returns the iteration count, or -1 if the launch was
// aborted.  x must not alias b or the work vectors.
// SW: the marching sweep (teams that own a whole state with few waves);
// otherwise chunk-wise, with each wave's first chunk of the next sweep loaded
// while the reduction slots are read.
template <bool SW = false, int SWSEG = 16, int SWPF = 4>
__device__ int cg_team_2d_r(Team &tm, const Geom &g, double s, double tol, int maxit,
                            const double *__restrict__ b, double *__restrict__ x, const CGWork2 &wk,
                            double abs_thresh2) {
    const ChunkRange cr = team_chunks(g, tm.rank, tm.size);
    const bool from_zero = abs_thresh2 >= 0.0;
    Cg2Pre pre;
    auto sweep = [&](double alpha, double beta, bool first, bool setup, const double *r, const double *pold,
                     double *rnew, double *pnew, double &ga, double &de, double &rr) {
        if constexpr (SW)
            cg2_sweep_sw<SWPF, SWSEG>(g, tm.rank, tm.size, s, alpha, beta, first, setup, r, pold, x, rnew, pnew, ga,
                                      de, rr);
        else
            cg2_sweep(g, cr, s, alpha, beta, first, setup, r, pold, x, rnew, pnew, ga, de, rr,
                      setup ? nullptr : &pre);
    };
    // set-up: r0 = b - A x0 with x0 = b (alpha = 1) or x0 = 0 (alpha = 0)
    double part[3] = {0.0, 0.0, 0.0}, tot[3];
    sweep(from_zero ? 0.0 : 1.0, 0.0, true, true, b, nullptr, wk.r[0], nullptr, part[0], part[1], part[2]);
    int q = team_reduce_begin<3>(tm, part, wk.red);
    if (q < 0) return -1;
    if constexpr (!SW) cg2_preload(g, cr, true, false, wk.r[0], nullptr, x, pre);
    team_reduce_end<3>(tm, wk.red, q, tot);
    double gamma = tot[0], delta = tot[1];
    const double bb = tot[2];
    const double thresh = from_zero ? (abs_thresh2 > 0.0 ? abs_thresh2 : tol * tol * bb) : tol * tol * bb;
    double alpha = gamma / delta, beta = 0.0;
    int cur = 0;
    int it = 0;
    while (it < maxit && gamma > thresh) {
        double pp[2] = {0.0, 0.0}, tt[2];
        double unused = 0.0;
        sweep(alpha, beta, it == 0, false, wk.r[cur], wk.p[cur], wk.r[cur ^ 1], wk.p[cur ^ 1], pp[0], pp[1],
              unused);
        q = team_reduce_begin<2>(tm, pp, wk.red);
        if (q < 0) return -1;
        // the next sweep reads the vectors just written (p is read from the
        // second iteration on)
        if constexpr (!SW) cg2_preload(g, cr, false, false, wk.r[cur ^ 1], wk.p[cur ^ 1], x, pre);
        team_reduce_end<2>(tm, wk.red, q, tt);
        ++it;
        beta = tt[0] / gamma;
        alpha = tt[0] / (tt[1] - beta * tt[0] / alpha);
        gamma = tt[0];
        cur ^= 1;
    }
    return it;
}

}  // namespace pr
