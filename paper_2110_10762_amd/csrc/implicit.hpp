// Implicit fine propagators (the paper's experiments integrate each slice with
// implicit schemes, Section 5.1): m steps of the theta-method
//     (I - theta r h^2 L_h) u' = (I + (1 - theta) r h^2 L_h) u,
// theta = 1/2 (trapezoidal rule) or 1 (backward Euler), unconditionally
// stable.  The left-hand matrix is the coarse propagator's with s = theta r,
// so the same solvers serve: the wave-scan Thomas solver in 1D (its own factor
// table), the team CG (x0 = right-hand side, ||res|| <= tol ||rhs||) in 2D/3D.
#pragma once
#include "coarse.hpp"
#include "fine.hpp"

namespace pr {

constexpr int FINE_EXPLICIT = 0, FINE_BACKWARD_EULER = 1, FINE_TRAPEZOIDAL = 2;
__host__ __device__ inline double theta_of(int kind) { return kind == FINE_TRAPEZOIDAL ? 0.5 : 1.0; }

// ------------------------------------------------------------------ 1D
// One wave, the state in registers; rl = (1 - theta) r on the state's points
// and 0 on the padding (the explicit half of the trapezoidal rule).
template <int R>
__device__ __forceinline__ void fine1d_theta_regs(double (&c)[R], const double (&rl)[R], const double (&inv)[R],
                                                  int n, double s, int steps, bool trap) {
    for (int t = 0; t < steps; ++t) {
        if (trap) fine1d_regs<R>(c, rl, 1);
        thomas_wave<R>(c, inv, n, s);
    }
}

// grid: one wave (block of 64) per state
template <int R>
__global__ __launch_bounds__(64) void k_fine1d_theta(const double *__restrict__ src, double *__restrict__ dst,
                                                     long long sstride, long long dstride, int n, double r,
                                                     int kind, const double *inv_tab, int steps, int count) {
    const int st = blockIdx.x;
    if (st >= count) return;
    const double th = theta_of(kind);
    double c[R], rl[R], inv[R];
    load1d<R>(src + (long long)st * sstride, n, (1.0 - th) * r, c, rl);
    load_inv<R>(inv_tab, inv);
    fine1d_theta_regs<R>(c, rl, inv, n, th * r, steps, kind == FINE_TRAPEZOIDAL);
    store1d<R>(dst + (long long)st * dstride, n, c);
}

// ------------------------------------------------------------------ 2D / 3D
// dst = (I - s h^2 L_h) src by the team (s = -(1 - theta) r: the explicit
// half step of the trapezoidal rule), then a team barrier.
template <int DIM>
__device__ bool team_apply_be(Team &tm, const Geom &g, double s, const double *__restrict__ src,
                              double *__restrict__ dst) {
    const ChunkRange cr = team_chunks(g, tm.rank, tm.size);
    const int w = wave_id();
    const long long nw = nwaves();
    for (long long c = cr.begin + w; c < cr.end; c += nw) {
        const CPt q = cpt_at(g, c);
        double v[2 * DIM];
        cpt_load<DIM>(q, g.n, [&](int j) { return src[j]; }, v);
        double center;
        const double y = cpt_apply<DIM>(q, v, center, 2.0 * DIM, s);
        if (q.m & CP_VALID) dst[q.c] = y;
    }
    return team_sync(tm);
}

// `steps` theta-steps of one state by the team, src -> dst, ping-pong through
// tmp so that the last step lands in dst (src is never written); rhs holds the
// trapezoidal right-hand side.  Returns the CG iterations, or -1 if aborted.
// 2D solves take the one-synchronisation CG (wk2): marching when the team's
// waves each get 16 rows of a column strip or more, chunk-wise otherwise (a
// team spanning the whole GPU); ALWAYS_MARCH keeps only the marching form
// (teams of an XCD or less).  3D solves take the two-phase CG (wk).
template <int DIM, int U, bool ALWAYS_MARCH = false>
__device__ __forceinline__ long long team_fine_theta(Team &tm, const Geom &g, int kind, double r, int steps, double tol,
                                     int maxit, const double *src, double *dst, double *tmp, double *rhs,
                                     const CGWork &wk, const CGWork2 &wk2) {
    const double th = theta_of(kind);
    long long its = 0;
    const double *cur = src;
    for (int t = 0; t < steps; ++t) {
        double *tgt = ((steps - 1 - t) % 2 == 0) ? dst : tmp;
        const double *b = cur;
        if (kind == FINE_TRAPEZOIDAL) {
            if (!team_apply_be<DIM>(tm, g, -(1.0 - th) * r, cur, rhs)) return -1;
            b = rhs;
        }
        int it;
        if constexpr (DIM == 2) {
            if (ALWAYS_MARCH || (long long)g.n * g.cpr >= 16LL * tm.size * nwaves())
                it = cg_team_2d_r<true>(tm, g, th * r, tol, maxit, b, tgt, wk2, -1.0);
            else
                it = cg_team_2d_r<false>(tm, g, th * r, tol, maxit, b, tgt, wk2, -1.0);
        } else {
            it = cg_team_dim<DIM, U>(tm, g, th * r, tol, maxit, b, tgt, wk, -1.0);
        }
        if (it < 0 || !team_sync(tm)) return -1;
        its += it;
        cur = tgt;
    }
    return its;
}

// Many states (the synchronous driver's fine sweep, serial runs): one team per
// group of workgroups with equal blockIdx modulo nteams (nteams divides 8, so
// a team stays on the XCDs dispatch gives those blocks); team t takes states
// t, t + nteams, ...  Per team: tmp, rhs and four CG vectors at `stride`
// apart, and 6 * size reduction slots.
template <int DIM>
__global__ __launch_bounds__(BLOCK) void k_fine_theta(const double *src, double *dst, long long sstride,
                                                      long long dstride, int count, Geom g, int kind, double r,
                                                      int steps, double tol, int maxit, double *scr,
                                                      long long stride, unsigned *ctr, double *red, Control *ctl,
                                                      int nteams, unsigned long long *cg_iters) {
    const int team = blockIdx.x % nteams;
    const int size = gridDim.x / nteams;
    Team tm{ctr + (long long)team * team_counter_words(0), ctl, size, (int)blockIdx.x / nteams, 0u};
    if (!team_setup(tm)) return;
    double *base = scr + (long long)team * 6 * stride;
    double *tred = red + (long long)team * 6 * size;
    const CGWork wk{base + 2 * stride, base + 3 * stride, base + 4 * stride, tred};
    const CGWork2 wk2{{base + 2 * stride, base + 5 * stride}, {base + 3 * stride, base + 4 * stride}, tred};
    unsigned long long its = 0;
    for (int c = team; c < count; c += nteams) {
        const long long it = team_fine_theta<DIM, DIM == 3 ? 4 : 2>(tm, g, kind, r, steps, tol, maxit,
                                                                   src + c * sstride, dst + c * dstride, base,
                                                                   base + stride, wk, wk2);
        if (it < 0) return;
        its += (unsigned long long)it;
    }
    if (threadIdx.x == 0 && tm.rank == 0)
        __hip_atomic_fetch_add(cg_iters, its, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace pr
