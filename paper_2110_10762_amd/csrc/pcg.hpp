// Coarse propagator G in 2D by preconditioned conjugate gradients: the
// backward-Euler system (I - s h^2 L_h) x = b (Section 3.1; backward Euler as
// G, Section 5.1) solved by CG with a fixed polynomial preconditioner.
//
// Preconditioner: M^-1 = p(A), the degree-PD polynomial that PD steps of
// Chebyshev acceleration on A z = r from z = 0 produce (Saad, Iterative
// Methods for Sparse Linear Systems, Chebyshev acceleration): with the
// spectrum of A = I - s h^2 L_h inside [1, 1 + 4 d s] (d = 2),
//     1 - lambda p(lambda) = T_{PD+1}((theta - lambda)/delta) / T_{PD+1}(theta/delta),
// theta, delta the centre and half-width of the interval.  p is positive on
// the interval, so M^-1 is symmetric positive definite and CG applies; the
// condition number drops from about 1 + 8 s (132 for the 1024^2 workload) to
// about 3.4 (PD = 6), and the iteration count by about 6x.  Applying p costs
// PD stencil passes with no inner product: it needs no synchronisation.
//
// Iteration (Chronopoulos-Gear form of preconditioned CG: one team barrier
// per iteration, the three inner products reduced together):
//     p_i = u_i + beta_i p_{i-1},   s_i = A p_i
//     x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i
//     u_{i+1} = p(A) r_{i+1},       w_{i+1} = A u_{i+1}
//     gamma = (r_{i+1}, u_{i+1}), delta = (w_{i+1}, u_{i+1}), rho = (r_{i+1}, r_{i+1})
//     beta_{i+1} = gamma_{i+1} / gamma_i
//     alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1} / alpha_i)
// Only r, u, p and x are stored; s = A p and w = A u are formed where they
// are used.  Start and stop as the unpreconditioned solvers: x0 = b and
// ||r||_2 <= tol ||b||_2 (or x0 = 0 and ||r||_2^2 <= abs_thresh2 for the
// increment form), rho being the true recurrence residual of CG.
//
// One sweep does a whole iteration.  A wave takes a strip of 64 columns and
// a segment of rows and marches down it: each input row brings r_i, u_i and
// p_{i-1}, from which p_i is formed at once; a level forming s_i = A p_i and
// r_{i+1}, the PD Chebyshev levels and the level forming w = A u each lag one
// row behind the one before (two rows of the stencil operand and one row of
// the pointwise terms held per level), so the output row, where x, p_i and
// u_{i+1} are formed and stored, is H = PD + 2 rows behind the input.  The
// strip's outer H columns and the segment's H halo rows on either side are
// recomputed, not exchanged.  Out-of-domain rows and columns are read from
// the odd extension of each vector, which every step commutes with, so the
// zero Dirichlet values need no masks (as in the fine kernels).
// HBM traffic per point and iteration: r, u, p, x read, the same four
// written (64 B); the halo re-reads and the output row's second reads of u
// and p hit the caches.
#pragma once
#include "fine.hpp"
#include "coarse.hpp"

namespace pr {

// Chebyshev polynomial degree of the preconditioner, and the shortest row
// segment a wave of the marching sweep takes (the H = degree + 2 halo rows on
// either side of a segment are recomputed).
// Measured on the 1024^2 workload (sync / async solve): degree 4 with
// segments of 16 / 24 rows 495 / 488 ms, degree 6 with 8 / 16 rows 396 / 400
// ms, degree 8 with 16 / 24 rows 477 / 449 ms; segments of 32 rows 696 ms.
constexpr int PCG_DEGREE = 6;
constexpr int PCG_MINSEG_GPU = 8;     // a team spanning the GPU (many waves per state)
constexpr int PCG_MINSEG_TEAM = 16;   // teams of a few XCDs or less

struct CGWorkP {
    double *r[2], *u[2], *p[2];   // [npts] each, read with halos: double-buffered
    double *red;                  // [8 * team size] reduction slots
};
// The same vectors, for a team of a few workgroups (longer row segments).
struct CGWorkPT : CGWorkP {};

// Chebyshev acceleration coefficients on [lo, hi]: level j (1..PD) forms
//   R_j = R_{j-1} - A d_{j-1},  d_j = c1[j-1] d_{j-1} + c2[j-1] R_j,  X_{j+1} = X_j + d_j
// from R_0 = r, d_0 = X_1 = r / theta; p(A) r = X_{PD+1}.
template <int PD>
struct Cheb {
    double inv_theta;
    double c1[PD], c2[PD];
};

template <int PD>
__device__ __forceinline__ Cheb<PD> cheb_coef(double lo, double hi) {
    Cheb<PD> c;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    const double sigma = theta / delta;
    c.inv_theta = 1.0 / theta;
    double rho = 1.0 / sigma;
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        c.c1[k] = rn * rho;
        c.c2[k] = 2.0 * rn / delta;
        rho = rn;
    }
    return c;
}

// Raw loads of one march step: input row (r, u, p_old) and output row (x,
// u, p_old); a set-up that carries the previous slice's correction loads its
// three terms at both rows (cw, co at the input row, ow, oo at the output
// row, beside r and uo) and the old lambda at the output row (ol).
struct PRow {
    double r, u, p, x, uo, po;
    double cw, co, ow, oo, ol;
};


// One iteration of the team's share of the state; accumulates the partial
// sums of (r', u'), (w', u') and (r', r') over the points the wave owns.
// SETUP: the start of a solve in the same march, with rin = b, pin = x0 (b,
// a guess, or null for x0 = 0) and alpha = 1: the first level forms
// r0 = b - A x0, then u0 = p(A) r0 and w0 = A u0; x = x0 is written and
// (b, b) summed into bb.  CORR (with SETUP): when sc is given, b is the
// previous slice's corrected value formed from sc (rin unused), written to
// sc->lam at the owned points, and the largest change |b - lam_old| goes
// into dm.  (sc.v == NULL: no correction; passed by value so that nothing
// of it lives in memory.)
template <int PD, int PF, bool SETUP, bool SKIP, bool CORR = false>
__device__ __forceinline__ void cgp_sweep(const Geom &g, int rank, int size, int minseg, double s,
                                          const Cheb<PD> &cc, double alpha, double beta, bool first,
                                          const double *__restrict__ rin, const double *__restrict__ uin,
                                          const double *__restrict__ pin, double *__restrict__ rout,
                                          double *__restrict__ uout, double *__restrict__ pout,
                                          double *__restrict__ x, double &ga, double &de, double &rr,
                                          double &bb, const SetupCorr sc = SetupCorr{}, double *dm = nullptr) {
    // Rounding exactly as written (no contraction of the remaining products
    // and sums into fused operations): a point's values come out the same
    // bits in every segment and strip that recomputes them, whatever code
    // the compiler makes of the step.
#pragma clang fp contract(off)
    constexpr int H = PD + 2;            // stencil levels between input and output row
    constexpr int W = WAVE - 2 * H;      // columns a strip owns
    const int n = g.n;
    const int lane = threadIdx.x & (WAVE - 1);
    const int waves = size * nwaves();
    const int wid = rank * nwaves() + wave_id();
    const int nsx = (n + W - 1) / W;
    // segments of rows: one (strip, segment) unit per wave, at least minseg rows
    const int seg = march_seg(n, nsx, waves, minseg);
    const int nseg = (n + seg - 1) / seg;
    const int units = nsx * nseg;
    const bool read_p = SETUP ? pin != nullptr : !first;   // p_{-1} = 0; x0 = 0
    const bool corr = CORR && sc.v != nullptr;
    const double *__restrict__ cv = sc.v;
    const double *__restrict__ cwn = sc.wn;
    const double *__restrict__ cwo = sc.wo;
    double *__restrict__ clam = sc.lam;
    double dmax = 0.0;
    for (int un = wid; un < units; un += waves) {
        const int sx = un % nsx;   // strips of the same rows side by side
        const int ya = (un / nsx) * seg;
        const int yb = min(n, ya + seg);
        const int xcol = sx * W - H + lane;
        double xsg;
        const int xi = reflect(xcol, n, xsg);
        const bool own = lane >= H && lane < H + W && xcol < n;
        double pa = 0.0, pb = 0.0, rd = 0.0;   // p_i at rows k-2, k-1; r_i at row k-1
        double w0[PD], w1[PD], Rd[PD], Xd[PD];
#pragma unroll
        for (int j = 0; j < PD; ++j) w0[j] = w1[j] = Rd[j] = Xd[j] = 0.0;
        double ua = 0.0, ub = 0.0;
        double DR[H - 1];   // r_{i+1} of the last H - 1 rows it was formed for, oldest first
#pragma unroll
        for (int j = 0; j < H - 1; ++j) DR[j] = 0.0;
        const int nrows = yb - ya + 2 * H;
        const int k0 = ya - H;
        PRow ring[PF];
        double rsg[PF];
        // Loads of march step kk into a ring slot: input row kk (odd extension)
        // and output row kk - H (clamped into the segment when outside it, so
        // every load is issued unconditionally); row addresses are scalar, the
        // lane offset is 32-bit.
        auto issue = [&](int kk, PRow &w, double &sg) {
            double ys;
            const int yi = reflect_row(kk, n, ys);
            const long long rb = (long long)yi * n;
            const int y = min(max(kk - H, ya), yb - 1);
            const long long ob = (long long)y * n;
            if constexpr (SETUP) {   // x0 at both rows, b at the output row
                // carrying a correction: b's terms at both rows, the old lambda
                // at the output row (both branches write the same fields in the
                // same order, so that the slot stays in registers)
                const double *__restrict__ bsrc = (CORR && corr) ? cv : rin;
                w.r = (bsrc + rb)[xi];
                w.uo = (bsrc + ob)[xi];
                if constexpr (CORR) {
                    if (corr) {
                        w.cw = (cwn + rb)[xi];
                        w.co = (cwo + rb)[xi];
                        w.ow = (cwn + ob)[xi];
                        w.oo = (cwo + ob)[xi];
                        w.ol = (clam + ob)[xi];
                    } else {
                        w.cw = 0.0;
                        w.co = 0.0;
                        w.ow = 0.0;
                        w.oo = 0.0;
                        w.ol = 0.0;
                    }
                }
                w.p = read_p ? (pin + rb)[xi] : 0.0;
                w.x = read_p ? (pin + ob)[xi] : 0.0;
            } else {
                w.r = (rin + rb)[xi];
                w.u = (uin + rb)[xi];
                w.p = read_p ? (pin + rb)[xi] : 0.0;
                w.x = (x + ob)[xi];
                w.uo = (uin + ob)[xi];
                w.po = read_p ? (pin + ob)[xi] : 0.0;
            }
            sg = ys * xsg;
        };
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            ring[q] = PRow{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            rsg[q] = 0.0;
            if (q < nrows) issue(k0 + q, ring[q], rsg[q]);
        }
        // One march step t (input row k = k0 + t, ring slot q).  Level l of the
        // march (1: s = A p, 2 .. H - 1: Chebyshev, H: w = A u) works on row
        // k0 + t - l, and the output rows depend on it only from t >= 2 l
        // on.  SKIP: until then a level skips its arithmetic (a third of the
        // levels' work in a 12-row segment) while its input rows still move
        // through the registers; needed values are unchanged.  (The tests are
        // wave-uniform; a second copy of the step without them for t >= 2 H
        // spills registers, and so do the tests themselves in the kernels
        // whose other phases hold many registers.)
        auto step = [&](const int t, const int q) {
            const int k = k0 + t;
            const double sg = rsg[q];
            // input row k: p_i (set-up: x0) and r_i (set-up: b)
            const double pn = SETUP ? sg * ring[q].p : __builtin_fma(beta, sg * ring[q].p, sg * ring[q].u);
            // (set-up carrying a correction: b = v + (wn - wo) at row k)
            const double rk = (CORR && corr) ? sg * (ring[q].r + (ring[q].cw - ring[q].co)) : sg * ring[q].r;
            // s_i = A p_i and r_{i+1} at row k - 1 (set-up: r0 = b - A x0)
            double rn = 0.0;
            if (!SKIP || t >= 2) {
                const double pl = from_lower_lane(pb), pr = from_upper_lane(pb);
                const double sv = be_point(pb, (pa + pn) + (pl + pr), 4.0, s);
                rn = __builtin_fma(-alpha, sv, rd);
            }
            pa = pb;
            pb = pn;
            rd = rk;
            const double rf = DR[0];   // r_{i+1} at row k - H
#pragma unroll
            for (int j = 0; j + 1 < H - 1; ++j) DR[j] = DR[j + 1];
            DR[H - 2] = rn;
            // Chebyshev levels: level j+1 forms row k-2-j from rows k-3-j..k-1-j of level j
            double dn = rn * cc.inv_theta, Rn = rn, Xn = dn;
#pragma unroll
            for (int j = 0; j < PD; ++j) {
                double dj = 0.0, Rj = 0.0, Xj = 0.0;
                if (!SKIP || t >= 2 * (j + 2)) {
                    const double l = from_lower_lane(w1[j]), r = from_upper_lane(w1[j]);
                    const double ad = be_point(w1[j], (w0[j] + dn) + (l + r), 4.0, s);
                    Rj = Rd[j] - ad;
                    dj = __builtin_fma(cc.c2[j], Rj, cc.c1[j] * w1[j]);
                    Xj = Xd[j] + dj;
                }
                w0[j] = w1[j];
                w1[j] = dn;
                Rd[j] = Rn;
                Xd[j] = Xn;
                dn = dj;
                Rn = Rj;
                Xn = Xj;
            }
            // u = p(A) r' reached row k - 1 - PD; w = A u and the output at row
            // k - H (inside the segment from t = 2 H on)
            if (t >= 2 * H) {
                const double l = from_lower_lane(ub), r = from_upper_lane(ub);
                const double wn = be_point(ub, (ua + Xn) + (l + r), 4.0, s);
                const double un = ub;
                const int y = k - H;
                if (y < yb && own) {
                    const long long i = (long long)y * n + xcol;
                    if constexpr (SETUP) {
                        x[i] = ring[q].x;
                        double bo = ring[q].uo;
                        if (CORR && corr) {
                            bo = ring[q].uo + (ring[q].ow - ring[q].oo);
                            dmax = fmax(dmax, fabs(bo - ring[q].ol));
                            clam[i] = bo;
                        }
                        bb = __builtin_fma(bo, bo, bb);
                    } else {
                        const double pi = __builtin_fma(beta, ring[q].po, ring[q].uo);
                        x[i] = __builtin_fma(alpha, pi, ring[q].x);
                        pout[i] = pi;
                    }
                    rout[i] = rf;
                    uout[i] = un;
                    ga = __builtin_fma(rf, un, ga);
                    de = __builtin_fma(wn, un, de);
                    rr = __builtin_fma(rf, rf, rr);
                }
            }
            ua = ub;
            ub = Xn;
            if (t + PF < nrows) issue(k + PF, ring[q], rsg[q]);
        };
        for (int tb = 0; tb < nrows; tb += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                if (tb + q >= nrows) break;
                step(tb + q, q);
            }
        }
    }
    if (CORR && corr) *dm = fmax(*dm, dmax);
}

// Solves (I - s h^2 L_h) x = b in 2D by the preconditioned CG above; same
// start and stop rules as cg_team_dim (abs_thresh2 < 0: x0 = b, or the guess
// xg when given, relative stop; >= 0: x0 = 0, absolute stop).  Returns the
// iteration count, or -1 if the launch was aborted.  x must not alias b, xg
// or the work vectors.  CORR: with sc given, b is the previous slice's
// corrected value formed in the set-up march (b unused; the change goes into
// *dm; sc.v == NULL: none).
template <int PD, int MINSEG, int PF = 4, bool SKIP = false, bool CORR = false>
__device__ int cg_team_2d_p(Team &tm, const Geom &g, double s, double tol, int maxit,
                            const double *__restrict__ b, double *__restrict__ x, const CGWorkP &wk,
                            double abs_thresh2, const double *__restrict__ xg = nullptr,
                            const SetupCorr sc = SetupCorr{}, double *dm = nullptr) {
    const bool from_zero = abs_thresh2 >= 0.0;
    if (from_zero) xg = nullptr;
    // the spectrum of I - s h^2 L_h lies in (1, 1 + 8 s)
    const Cheb<PD> cc = cheb_coef<PD>(1.0, 1.0 + 8.0 * s);
    // the start in one march: x = x0, r0 = b - A x0, u0 = p(A) r0, the sums
    double part[4] = {0.0, 0.0, 0.0, 0.0}, tot[4];
    // a set-up that can carry a correction loads nine values a row pair:
    // two march steps ahead instead of PF keeps them in registers
    constexpr int PFS = CORR ? 2 : PF;
    cgp_sweep<PD, PFS, true, SKIP, CORR>(g, tm.rank, tm.size, MINSEG, s, cc, 1.0, 0.0, true, b, nullptr,
                                        from_zero ? nullptr : (xg ? xg : b), wk.r[0], wk.u[0], nullptr, x,
                                        part[0], part[1], part[2], part[3], sc, dm);
    if (!team_reduce_n<4>(tm, part, wk.red, tot)) return -1;
    double gamma = tot[0], rho = tot[2];
    const double thresh = from_zero ? (abs_thresh2 > 0.0 ? abs_thresh2 : tol * tol * tot[3]) : tol * tol * tot[3];
    double alpha = gamma / tot[1], beta = 0.0;
    int cur = 0;
    int it = 0;
    while (it < maxit && rho > thresh) {
        double pp[3] = {0.0, 0.0, 0.0}, tt[3], unused = 0.0;
        cgp_sweep<PD, PF, false, SKIP>(g, tm.rank, tm.size, MINSEG, s, cc, alpha, beta, it == 0, wk.r[cur], wk.u[cur],
                                 wk.p[cur], wk.r[cur ^ 1], wk.u[cur ^ 1], wk.p[cur ^ 1], x, pp[0], pp[1], pp[2],
                                 unused);
        if (!team_reduce_n<3>(tm, pp, wk.red, tt)) return -1;
        ++it;
        beta = tt[0] / gamma;
        alpha = tt[0] / (tt[1] - beta * tt[0] / alpha);
        gamma = tt[0];
        rho = tt[2];
        cur ^= 1;
    }
    return it;
}

}  // namespace pr
