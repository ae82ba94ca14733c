// Synchronous Parareal sweeps (equation (pr); Algorithm 1's guards).
//
// One iteration k of the synchronous driver is
//   (1) v_i = F(lambda_{i-1}^{k-1}) for every slice i >= k, all independent
//       (fine kernels, one launch over the batch of slices), then
//   (2) the sequential coarse sweep i = k..N:
//         w_new = G(lambda_{i-1}^k)          (skipped for i = k: its input is
//                                             exact and unchanged, so w_new = w_old)
//         lambda_i^k = v_i + (w_new - w_old)  (this evaluation order leaves
//                                             exactly v_i when w_new == w_old)
//         delta = max(delta, |lambda_i^k - lambda_i^{k-1}|)
// The sweep of (2) runs in one launch: a single wave in 1D, the whole GPU as
// one team in 2D/3D (the team barrier separates consecutive slices).  The
// initial coarse sweep lambda_i^0 = G(lambda_{i-1}^0), w_i = lambda_i^0 uses
// the same kernels in "init" mode.
#pragma once
#include "coarse.hpp"
#include "pcg.hpp"

namespace pr {

struct SweepArgs {
    double *lam;        // [(N+1) * npts], updated in place
    const double *v;    // [(N+1) * npts], v[i] = F(lambda_{i-1})
    double *w;          // [(N+1) * npts], w[i] = G of slice i's last coarse input
    double *wn;         // [npts] scratch for the new coarse value
    const double *wo;   // marching solvers (2D preconditioned, 3D), not incremental: [(N+1) * npts], the
                        // previous iteration's coarse values (then w receives the
                        // new ones directly); NULL: w is updated in place
    long long npts;
    int i0, i1;         // slices to sweep, inclusive
    int kguard;         // slice whose coarse input is known unchanged (-1: none)
    int init;           // 1: initial coarse sweep
    int incr;           // 1: coarse solves act on the change of their input
    double *d0, *d1;    // [npts] each: changes of consecutive slices (increment mode)
    double *delta;      // max-norm change (bit pattern max, zeroed by the host)
    unsigned long long *cg_iters;   // accumulated CG iterations (2D/3D)
    // 1D
    int n;
    double s;
    const double *inv_tab;
    // 2D/3D
    Geom g;
    double cg_tol;
    int cg_maxit;
    CGWork wk;
    CGWork2 wk2;        // 2D: one-synchronisation CG, products recomputed
    CGWorkP wkp;        // 2D: preconditioned CG
    unsigned *ctr;
    Control *ctl;
};

template <int R>
__global__ __launch_bounds__(64) void k_sweep_1d(SweepArgs a) {
    const int lane = threadIdx.x;
    const int n = a.n;
    double inv[R];
    load_inv<R>(a.inv_tab, inv);
    double x[R];   // input of the next coarse solve: lambda_{i-1} (new)
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int p = lane * R + e;
        x[e] = p < n ? a.lam[(a.i0 - 1) * a.npts + p] : 0.0;
    }
    double dmax = 0.0;
    const bool incr = a.incr && !a.init;
    if (incr) {
#pragma unroll
        for (int e = 0; e < R; ++e) x[e] = 0.0;   // the first slice's input is unchanged
    }
    for (int i = a.i0; i <= a.i1; ++i) {
        double *li = a.lam + i * a.npts;
        double *wi = a.w + i * a.npts;
        const double *vi = a.v + i * a.npts;
        double wnew[R];
        const bool skip = (i == a.kguard);
#pragma unroll
        for (int e = 0; e < R; ++e) wnew[e] = x[e];
        if (!skip) thomas_wave<R>(wnew, inv, n, a.s);   // G(input) or G(change of input)
#pragma unroll
        for (int e = 0; e < R; ++e) {
            const int p = lane * R + e;
            double nx = 0.0;
            if (p < n) {
                if (a.init) {
                    nx = wnew[e];
                    wi[p] = nx;
                    li[p] = nx;
                } else if (incr) {
                    const double ln = vi[p] + (skip ? 0.0 : wnew[e]);
                    nx = ln - li[p];                 // change of this slice = next input change
                    dmax = fmax(dmax, fabs(nx));
                    li[p] = ln;
                } else {
                    const double wold = wi[p];
                    const double wv = skip ? wold : wnew[e];
                    const double lnew = vi[p] + (wv - wold);
                    dmax = fmax(dmax, fabs(lnew - li[p]));
                    wi[p] = wv;
                    li[p] = lnew;
                    nx = lnew;
                }
            }
            x[e] = nx;
        }
    }
    dmax = wave_max(dmax);
    if (lane == 0 && !a.init) atomic_max_nonneg(a.delta, dmax);
}

// Sequential coarse sweep of slices i0..i1 of one problem by a team, with the
// fused correction and change norm (shared by the synchronous and the batched
// drivers).  kguard: slice whose coarse input is unchanged (skipped); init:
// initial sweep lambda_i = w_i = G(lambda_{i-1}).  Increment mode: the solve
// for slice i acts on the change d_{i-1} of its input (the previous slice's
// change, produced by its correction), to an absolute residual tol*||input||.
struct SweepBufs {
    double *lam;
    const double *v;
    double *w, *wn, *d0, *d1;
    const double *wo = nullptr;   // previous coarse values, when the corrections ride on the set-ups
};

template <int DIM>
__device__ __forceinline__ int team_cg(Team &tm, const Geom &g, double s, double tol, int maxit,
                                       const double *b, double *x, const CGWork &wk, double abs_thresh2,
                                       const double *xg = nullptr, const SetupCorr sc = SetupCorr{},
                                       double *dm = nullptr) {
    // 3D whole-GPU sweep: marching phases (7.7 s for the 3D workload against
    // 8.7 s with two chunks per wave in flight and 9.0 s with one; the
    // one-synchronisation form with w and s stored moves 80 B per point and
    // took 10.9 s)
    return cg_team_dim<DIM, 2, DIM == 3>(tm, g, s, tol, maxit, b, x, wk, abs_thresh2, xg, sc, dm);
}

template <int DIM>
__device__ __forceinline__ int team_cg(Team &tm, const Geom &g, double s, double tol, int maxit,
                                       const double *b, double *x, const CGWork2 &wk, double abs_thresh2,
                                       const double * = nullptr, const SetupCorr = SetupCorr{},
                                       double * = nullptr) {   // starts from b
    static_assert(DIM == 2, "the recomputing CG is two-dimensional");
    // the whole GPU has more waves than a state has rows per column strip:
    // every wave takes a few chunks (the marching sweep measured 1.6x slower)
    return cg_team_2d_r<false>(tm, g, s, tol, maxit, b, x, wk, abs_thresh2);
}

template <int DIM>
__device__ __forceinline__ int team_cg(Team &tm, const Geom &g, double s, double tol, int maxit,
                                       const double *b, double *x, const CGWork2M &wk, double abs_thresh2,
                                       const double * = nullptr, const SetupCorr = SetupCorr{},
                                       double * = nullptr) {   // starts from b
    static_assert(DIM == 2, "the recomputing CG is two-dimensional");
    return cg_team_2d_r<true>(tm, g, s, tol, maxit, b, x, wk, abs_thresh2);
}

template <int DIM>
__device__ __forceinline__ int team_cg(Team &tm, const Geom &g, double s, double tol, int maxit,
                                       const double *b, double *x, const CGWorkP &wk, double abs_thresh2,
                                       const double *xg = nullptr, const SetupCorr sc = SetupCorr{},
                                       double *dm = nullptr) {
    static_assert(DIM == 2, "the preconditioned CG is two-dimensional");
    return cg_team_2d_p<PCG_DEGREE, PCG_MINSEG_GPU, 4, true, true>(tm, g, s, tol, maxit, b, x, wk, abs_thresh2, xg,
                                                                   sc, dm);
}

template <int DIM>
__device__ __forceinline__ int team_cg(Team &tm, const Geom &g, double s, double tol, int maxit,
                                       const double *b, double *x, const CGWorkPT &wk, double abs_thresh2,
                                       const double *xg = nullptr, const SetupCorr = SetupCorr{},
                                       double * = nullptr) {
    static_assert(DIM == 2, "the preconditioned CG is two-dimensional");
    return cg_team_2d_p<PCG_DEGREE, PCG_MINSEG_TEAM, 2>(tm, g, s, tol, maxit, b, x, wk, abs_thresh2, xg);
}

template <int DIM, typename WK>
__device__ bool team_coarse_sweep(Team &tm, const Geom &g, double s, double tol, int maxit, long long npts,
                                  int i0, int i1, int kguard, bool init, bool incr, const SweepBufs &B,
                                  const WK &wk, double &dmax, unsigned long long &its, double *lds) {
    const ChunkRange cr = team_chunks(g, tm.rank, tm.size);
    const int w = wave_id();
    const int nw = nwaves();
    incr = incr && !init;
    // Corrections carried by the set-ups (B.wo given; literal form): slice i's
    // solve reads x0 from B.wo and writes G(lambda_{i-1}) into B.w directly,
    // and its set-up march forms the previous slice's correction where it
    // reads its input, so no pass and no barrier separate the solves; the
    // last slice's correction is a pass after the loop.
    const bool carry = B.wo != nullptr && !init && !incr;
    int pend = -1;            // slice whose correction is still to be made
    bool pend_skip = false;   // ... with its coarse solve skipped
    double *dprev = B.d0, *dnext = B.d1;
    double nrm_prev = 0.0;
    for (int i = i0; i <= i1; ++i) {
        const bool skip = (!init && i == kguard);
        double *li = B.lam + (long long)i * npts;
        double *wi = B.w + (long long)i * npts;
        const double *vi = B.v + (long long)i * npts;
        if (!skip) {
            SetupCorr sc{};
            if (carry && pend == i - 1) {
                const double *wo_p = B.wo + (long long)(i - 1) * npts;
                sc = SetupCorr{B.v + (long long)(i - 1) * npts, pend_skip ? wo_p : B.w + (long long)(i - 1) * npts,
                               wo_p, B.lam + (long long)(i - 1) * npts};
            }
            // one call site: the kernel holds a single copy of the solver.  A
            // solve of the literal form starts from the slice's last coarse
            // value G(lambda_{i-1}^{k-1}): its residual is then the change of
            // the input, small once the iteration settles (same stop rule)
            const int it = team_cg<DIM>(tm, g, s, tol, maxit, incr ? dprev : B.lam + (long long)(i - 1) * npts,
                                        carry ? wi : B.wn, wk, incr ? tol * tol * nrm_prev : -1.0,
                                        (init || incr) ? nullptr : (carry ? B.wo + (long long)i * npts : wi), sc,
                                        &dmax);
            if (it < 0) return false;
            its += (unsigned long long)it;
        }
        if (carry) {
            pend = i;
            pend_skip = skip;
            continue;
        }
        double nrm = 0.0;
        // the loads of STREAM_U chunks are in flight before any is used; every
        // lane visits its chunks in the same order as one at a time
        const bool use_n = !skip;                    // w_new
        const bool use_v = !init;                    // v and lambda
        const bool use_w = !init && !incr;           // w_old
        for (long long c = cr.begin + w; c < cr.end; c += (long long)STREAM_U * nw) {
            Point p[STREAM_U];
            chunk_points<STREAM_U>(g, c, cr.end, nw, p);
            double tn[STREAM_U], tv[STREAM_U], tl[STREAM_U], tw[STREAM_U];
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                const long long j = p[u].idx;
                tn[u] = use_n ? B.wn[j] : 0.0;
                tv[u] = use_v ? vi[j] : 0.0;
                tl[u] = use_v ? li[j] : 0.0;
                tw[u] = use_w ? wi[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                if (!p[u].valid) continue;
                const long long j = p[u].idx;
                if (init) {
                    li[j] = tn[u];
                    wi[j] = tn[u];
                } else if (incr) {
                    const double ln = tv[u] + tn[u];
                    const double d = ln - tl[u];
                    dmax = fmax(dmax, fabs(d));
                    dnext[j] = d;
                    nrm = __builtin_fma(ln, ln, nrm);
                    li[j] = ln;
                } else {
                    const double wv = skip ? tw[u] : tn[u];
                    const double lnew = tv[u] + (wv - tw[u]);
                    dmax = fmax(dmax, fabs(lnew - tl[u]));
                    li[j] = lnew;
                    wi[j] = wv;
                }
            }
        }
        if (incr) {
            if (!team_reduce<false>(tm, nrm, wk.red, nrm_prev, lds)) return false;
            double *t = dprev;
            dprev = dnext;
            dnext = t;
        } else if (!team_sync(tm)) {
            return false;
        }
    }
    if (carry && pend >= 0) {   // the last slice's correction (the launch ends after it)
        double *li = B.lam + (long long)pend * npts;
        const double *vi = B.v + (long long)pend * npts;
        const double *wo_p = B.wo + (long long)pend * npts;
        const double *wn_p = pend_skip ? wo_p : B.w + (long long)pend * npts;
        for (long long c = cr.begin + w; c < cr.end; c += (long long)STREAM_U * nw) {
            Point p[STREAM_U];
            chunk_points<STREAM_U>(g, c, cr.end, nw, p);
            double tv[STREAM_U], tn[STREAM_U], to[STREAM_U], tl[STREAM_U];
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                const long long j = p[u].idx;
                tv[u] = vi[j];
                tn[u] = wn_p[j];
                to[u] = wo_p[j];
                tl[u] = li[j];
            }
#pragma unroll
            for (int u = 0; u < STREAM_U; ++u) {
                if (!p[u].valid) continue;
                const double lnew = tv[u] + (tn[u] - to[u]);
                dmax = fmax(dmax, fabs(lnew - tl[u]));
                li[p[u].idx] = lnew;
            }
        }
    }
    return true;
}

// Cooperative launch: the whole grid is one team.
// one instantiation per dimension (2, 3): each kernel holds one solver copy
// 768 threads: 168 registers per lane hold the 2D solver with its preloaded
// chunk (1.16 s for the 1024^2, 64-slice sync solve; 1024 threads spill at
// 128 registers, 1.53 s, and 512 threads take 1.26 s)
constexpr int SWEEP_THREADS = 768;
// the preconditioned 2D CG holds its Chebyshev levels, row delay lines and
// four rows of loads in flight in registers: 512 threads (256 registers per lane)
constexpr int PCG_THREADS = 512;
__host__ __device__ constexpr int sweep_threads(bool pcg) { return pcg ? PCG_THREADS : SWEEP_THREADS; }
// PCG: 2D coarse solves by the preconditioned CG (pcg.hpp); otherwise the
// unpreconditioned one-synchronisation CG.
template <int DIM, bool PCG = false>
__global__ __launch_bounds__(sweep_threads(PCG)) void k_sweep_cg(SweepArgs a) {
    Team tm{a.ctr, a.ctl, (int)gridDim.x, (int)blockIdx.x, 0u};
    if (!team_setup(tm, true)) return;
    __shared__ double lds[MAX_WAVES];
    double dmax = 0.0;
    unsigned long long its = 0;
    const SweepBufs B{a.lam, a.v, a.w, a.wn, a.d0, a.d1, (DIM == 3 || PCG) ? a.wo : nullptr};
    bool ok;
    if constexpr (DIM == 2 && PCG)
        ok = team_coarse_sweep<2>(tm, a.g, a.s, a.cg_tol, a.cg_maxit, a.npts, a.i0, a.i1, a.kguard, a.init != 0,
                                  a.incr != 0, B, a.wkp, dmax, its, lds);
    else if constexpr (DIM == 2)
        ok = team_coarse_sweep<2>(tm, a.g, a.s, a.cg_tol, a.cg_maxit, a.npts, a.i0, a.i1, a.kguard, a.init != 0,
                                  a.incr != 0, B, a.wk2, dmax, its, lds);
    else
        ok = team_coarse_sweep<3>(tm, a.g, a.s, a.cg_tol, a.cg_maxit, a.npts, a.i0, a.i1, a.kguard, a.init != 0,
                                  a.incr != 0, B, a.wk, dmax, its, lds);
    if (!ok) return;
    dmax = block_reduce<true>(dmax, lds);
    if (threadIdx.x == 0) {
        if (!a.init) atomic_max_nonneg(a.delta, dmax);
        if (tm.rank == 0)
            __hip_atomic_fetch_add(a.cg_iters, its, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Batch of independent coarse solves (tests and the apply entry point):
// state c of the batch is solved by the whole grid, one after the other,
// with the solver of the synchronous sweep (2D: the one-synchronisation CG;
// 3D: the marching two-phase CG).
template <int DIM, bool PCG = false>
__global__ __launch_bounds__(sweep_threads(PCG)) void k_coarse_cg_batch(const double *src, double *dst, long long npts,
                                                           int count, Geom g, double s, double tol,
                                                           int maxit, CGWork wk, CGWork2 wk2, CGWorkP wkp,
                                                           unsigned *ctr, Control *ctl,
                                                           unsigned long long *cg_iters) {
    Team tm{ctr, ctl, (int)gridDim.x, (int)blockIdx.x, 0u};
    if (!team_setup(tm, true)) return;
    unsigned long long its = 0;
    for (int c = 0; c < count; ++c) {
        int it;
        if constexpr (DIM == 2 && PCG)
            it = team_cg<2>(tm, g, s, tol, maxit, src + c * npts, dst + c * npts, wkp, -1.0);
        else if constexpr (DIM == 2)
            it = team_cg<2>(tm, g, s, tol, maxit, src + c * npts, dst + c * npts, wk2, -1.0);
        else
            it = team_cg<3>(tm, g, s, tol, maxit, src + c * npts, dst + c * npts, wk, -1.0);
        if (it < 0) return;
        its += (unsigned long long)it;
        if (!team_sync(tm)) return;
    }
    if (threadIdx.x == 0 && tm.rank == 0)
        __hip_atomic_fetch_add(cg_iters, its, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_zero_words(unsigned *p, int nwords) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) p[i] = 0u;
}

__global__ void k_copy(const double *__restrict__ src, double *__restrict__ dst, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace pr
