// Many independent 2D heat problems (uneven grid size, slice count and
// diffusivity) solved by synchronous Parareal together.
//
// Every problem has its own descriptor (BProb) and device-resident state
// (BState: next iteration, active flag, last change), so one iteration of the
// whole batch is a fixed sequence of launches that reads its work from device
// memory -- the host captures it once as a hipGraph and replays it:
//   k_bfine   per size class and fine pass: every (problem, slice) unit of the
//             class still to be propagated this iteration advances one
//             temporally-blocked pass (inactive problems and exact slices
//             return at once);
//   k_bsweep  one persistent launch for the coarse sweeps of all problems:
//             fixed-size teams of workgroups take problems off an atomic
//             queue (largest work first) and run that problem's sequential
//             coarse sweep with the fused correction and change norm, then
//             update its state (iteration count, change, stop decision).
// A problem stops when its change drops below its eps or at k = N (finite
// termination); the host polls the active count between replays.  This is the
// per-slice / per-problem operator idea of the paper's remark on F_i, G_i
// applied across independent problems.
#pragma once
#include "fine.hpp"
#include "sync.hpp"

namespace pr {

struct BProb {
    int n, N, m, passes;   // grid side, slices, fine steps per slice, fine passes per slice
    int kmax, cg_maxit;
    int incr;              // coarse solves on the change of their input
    int pad;
    long long npts;
    long long off_lam;     // offset of lambda_0 in the concatenated iterate (and in v, w, tmp)
    double r, s, eps, cg_tol;
    Geom g;
};

struct BState {
    int k;                 // iteration to run next (0: initial coarse sweep pending)
    int active;
    int iters;             // iterations completed
    int pad;
    double delta;          // change of the last completed iteration
    unsigned long long cg_iters;
};

struct BatchArgs {
    int B;
    const BProb *prob;
    BState *st;
    double *lam, *v, *w;
    int nteams, tsz, ctr_stride;
    const int *team_of, *rank_of;
    unsigned *tctr;
    long long *tbc;
    double *tred;
    double *wn, *cgr, *cgr1, *cgp0, *cgp1, *d0, *d1;   // [nteams][maxnpts]
    double *cgw0, *cgw1;                               // [nteams][maxnpts], preconditioned CG only
    long long maxnpts;
    const int *order;
    unsigned *queue;
    Control *ctl;
};

template <int XP, int R, int D>
__global__ __launch_bounds__(BLOCK) void k_bfine(const BProb *__restrict__ prob, const BState *__restrict__ st,
                                                 const int *__restrict__ unit_b, const int *__restrict__ unit_i,
                                                 int nunits, int n, int nsx, int nsy, int pass, const double *lam,
                                                 double *v, double *tmp, int nblk) {
    const int L = xcd_remap(blockIdx.x, nblk);
    if (L >= nblk) return;
    const long long wv = (long long)L * WAVES_PER_BLOCK + wave_id();
    const long long per = (long long)nsx * nsy;
    const long long u = wv / per;
    if (u >= nunits) return;
    const int strip = (int)(wv - u * per);
    const int b = unit_b[u], i = unit_i[u];
    const BProb &P = prob[b];
    const BState &S = st[b];
    if (!S.active || S.k < 1 || i < S.k || pass >= P.passes) return;
    const int steps = min(D, P.m - pass * D);
    const long long here = P.off_lam + (long long)i * P.npts;
    auto target = [&](int p) { return ((P.passes - 1 - p) % 2 == 0) ? v + here : tmp + here; };
    const double *src = pass == 0 ? lam + P.off_lam + (long long)(i - 1) * P.npts : target(pass - 1);
    fine2d_strip<XP, R, D>(src, target(pass), n, P.r, steps, strip / nsy, strip % nsy);
}

template <int XP, int D>
__global__ __launch_bounds__(BLOCK) void k_bfine_sw(const BProb *__restrict__ prob, const BState *__restrict__ st,
                                                    const int *__restrict__ unit_b, const int *__restrict__ unit_i,
                                                    int nunits, int n, int nsx, int nsy, int ry, int pass,
                                                    const double *lam, double *v, double *tmp, int nblk) {
    const int L = xcd_remap(blockIdx.x, nblk);
    if (L >= nblk) return;
    const long long wv = (long long)L * WAVES_PER_BLOCK + wave_id();
    const long long per = (long long)nsx * nsy;
    const long long u = wv / per;
    if (u >= nunits) return;
    const int strip = (int)(wv - u * per);
    const int b = unit_b[u], i = unit_i[u];
    const BProb &P = prob[b];
    const BState &S = st[b];
    if (!S.active || S.k < 1 || i < S.k || pass >= P.passes) return;
    const int steps = min(D, P.m - pass * D);
    const long long here = P.off_lam + (long long)i * P.npts;
    auto target = [&](int p) { return ((P.passes - 1 - p) % 2 == 0) ? v + here : tmp + here; };
    const double *src = pass == 0 ? lam + P.off_lam + (long long)(i - 1) * P.npts : target(pass - 1);
    const int ya = (strip % nsy) * ry;
    fine2d_sw<XP, D>(src, target(pass), n, P.r, steps, strip / nsy, ya, min(n, ya + ry), (strip % nsy) & 1);
}

// Three workgroups per CU: 96 teams on the chip (11.0 s for the 512-problem
// batch against 11.9 s with two per CU and the registers the marching CG
// would take unbounded).  PCG: the preconditioned CG (its Chebyshev levels
// need the registers of two workgroups per CU).
template <bool PCG>
__global__ __launch_bounds__(BLOCK, PCG ? 2 : 3) void k_bsweep(BatchArgs a) {
    const int team = a.team_of[blockIdx.x];
    if (team < 0) return;
    Team tm{a.tctr + (long long)team * a.ctr_stride, a.ctl, a.tsz, a.rank_of[blockIdx.x], 0u};
    if (!team_setup(tm)) return;
    long long *bc = a.tbc + team * 16;
    double *wn = a.wn + team * a.maxnpts;
    // a team of 8 workgroups sweeps a whole problem: the marching CG
    const long long o = (long long)team * a.maxnpts;
    double *const red = a.tred + (long long)team * 8 * a.tsz;
    CGWork2M wk2;
    wk2.r[0] = a.cgr + o;
    wk2.r[1] = a.cgr1 + o;
    wk2.p[0] = a.cgp0 + o;
    wk2.p[1] = a.cgp1 + o;
    wk2.red = red;

    __shared__ double lds[MAX_WAVES];
    const bool leader = (tm.rank == 0 && threadIdx.x == 0);
    for (;;) {
        long long c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (leader) c[0] = __hip_atomic_fetch_add(a.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the queue word is read before the broadcast; the stop flag is never set here
        {
            __shared__ long long s_c;
            const int par = (tm.epoch + 1) & 1;
            if (leader) bc[par * 8] = c[0];
            if (!team_sync(tm)) return;
            if (threadIdx.x == 0) s_c = bc[par * 8];
            __syncthreads();
            c[0] = uniform(s_c);
            __syncthreads();
        }
        if (c[0] >= a.B) break;
        const int b = a.order[c[0]];
        const BProb &P = a.prob[b];
        BState &S = a.st[b];
        if (!S.active) continue;
        const int k = S.k;
        const bool init = (k == 0);
        double dmax = 0.0;
        unsigned long long its = 0;
        const SweepBufs SB{a.lam + P.off_lam, a.v + P.off_lam, a.w + P.off_lam, wn,
                           a.d0 + team * a.maxnpts, a.d1 + team * a.maxnpts};
        bool ok;
        if constexpr (PCG) {
            CGWorkPT wkp;
            wkp.r[0] = a.cgr + o;
            wkp.r[1] = a.cgr1 + o;
            wkp.u[0] = a.cgw0 + o;
            wkp.u[1] = a.cgw1 + o;
            wkp.p[0] = a.cgp0 + o;
            wkp.p[1] = a.cgp1 + o;
            wkp.red = red;
            ok = team_coarse_sweep<2>(tm, P.g, P.s, P.cg_tol, P.cg_maxit, P.npts, init ? 1 : k, P.N, init ? -1 : k,
                                      init, P.incr != 0, SB, wkp, dmax, its, lds);
        } else
            ok = team_coarse_sweep<2>(tm, P.g, P.s, P.cg_tol, P.cg_maxit, P.npts, init ? 1 : k, P.N, init ? -1 : k,
                                      init, P.incr != 0, SB, wk2, dmax, its, lds);
        if (!ok) return;
        double delta = 0.0;
        if (!team_reduce<true>(tm, dmax, red, delta, lds)) return;
        if (leader) {
            S.cg_iters += its;
            if (init) {
                S.k = 1;
            } else {
                S.delta = delta;
                S.iters = k;
                S.k = k + 1;
                if ((P.eps > 0 && delta < P.eps) || k >= P.N || k >= P.kmax) S.active = 0;
            }
        }
    }
}

// lambda_0 of every problem = its u0 (concatenated in problem order).
__global__ void k_bscatter(const double *u0, double *lam, const BProb *prob, const long long *u0_off) {
    const int b = blockIdx.y;
    const BProb &P = prob[b];
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < P.npts; p += (long long)gridDim.x * blockDim.x)
        lam[P.off_lam + p] = u0[u0_off[b] + p];
}

__global__ void k_binit(BState *st, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    BState s{};
    s.active = 1;
    st[b] = s;
}

struct BatchWork {
    BProb *prob = nullptr;
    BState *st = nullptr;
    double *v = nullptr, *w = nullptr, *tmp = nullptr;
    long long *u0_off = nullptr;
    int *order = nullptr, *team_of = nullptr, *rank_of = nullptr;
    unsigned *tctr = nullptr, *queue = nullptr;
    long long *tbc = nullptr;
    double *tred = nullptr, *wn = nullptr, *cgr = nullptr, *cgr1 = nullptr, *cgp0 = nullptr, *cgp1 = nullptr;
    double *cgw0 = nullptr, *cgw1 = nullptr;
    bool pcg = false;   // coarse solves by the preconditioned CG
    double *d0 = nullptr, *d1 = nullptr;
    long long maxnpts = 0, total = 0;
    int nteams = 0, tsz = 0, grid = 0;
    // per size class: side, units, fine shape
    int nclass = 0;
    int cls_n[8] = {}, cls_units[8] = {}, cls_shape[8] = {}, cls_passes[8] = {};
    int *cls_ub[8] = {}, *cls_ui[8] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const double *graph_lam = nullptr;   // iterate the captured graph writes
    int use_graph = 1;
};

}  // namespace pr
