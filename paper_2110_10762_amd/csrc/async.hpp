// Asynchronous Parareal (equation (apr) in the form of Algorithm 2), emulated
// on one GPU by one persistent cooperative launch.
//
// The grid is split into teams of workgroups (a team per slice, or per group
// of slices); teams never wait for each other.  Each local iteration of slice
// i does, exactly as Algorithm 2:
//     v      = F(x_old)                   x_old: the predecessor value its
//                                         previous coarse solve used
//     x_new  = newest published lambda_{i-1} (or the version a replay
//              schedule names)
//     w_new  = G(x_new)                   (= w_old when x_new is x_old: G is
//                                          deterministic, so nothing to solve)
//     lambda = v + (w_new - w_old)        (exactly v when the input is stale)
//     publish lambda as version ver+1;  x_old, w_old := x_new, w_new
// Publication: every slice owns a ring of R slots holding its newest
// versions; the slot data is written by the team, then the team leader
// stores the version number with agent-scope release semantics.  A reader
// acquires the version, copies the slot with the whole team, meets the team
// at a barrier and re-reads the version: the copy is valid if the writer
// cannot have started overwriting that slot before the last load returned
// (at most R-2 newer versions published).  Per-slice headers (change of the
// last update, accumulated change "drift", predecessor drift at the version
// read) are updated under a sequence lock so that a monitor can take a
// consistent snapshot by double collect.
//
// Stop rules (the paper delegates asynchronous termination to external
// protocols; these are this library's readings):
//   FREE   every slice has updated, its last update changed it by < eps, and
//          the predecessor version it read has since drifted by < eps (the
//          drift bounds the max-norm distance by the triangle inequality).
//          Value-preserving idling: a slice whose coarse input was stale in
//          its previous update and is still stale would recompute exactly the
//          value it already published, so it waits instead.
//   EXACT  finite termination (Section 3.2, nested-set proposition): a slice
//          is final once it updated with both inputs equal to its
//          predecessor's final value; stop when slice N is final.
//   REPLAY slice i's k-th coarse solve reads the predecessor version the host
//          schedule names (waiting for it if needed); all versions are kept.
#pragma once
#include "fine.hpp"
#include "coarse.hpp"
#include "pcg.hpp"
#include "implicit.hpp"

namespace pr {

constexpr int AMODE_FREE = 0, AMODE_EXACT = 1, AMODE_REPLAY = 2, AMODE_PIPELINED = 3;
// modes that keep every version and read scheduled ones
__host__ __device__ inline bool scheduled_reads(int mode) { return mode == AMODE_REPLAY || mode == AMODE_PIPELINED; }

struct alignas(64) SliceHdr {
    int seq;          // sequence lock (odd while the fields change)
    int ver;          // newest published version (release-stored)
    int k;            // local iterations performed (k_i)
    int g_ver;        // predecessor version read by the last coarse solve
    int final_from;   // EXACT: first version equal to the serial fine value, -1 before
    int done;         // the slice will not publish again (release-stored)
    int pad1, pad2;
    double delta;     // max-norm change made by the last update
    double drift;     // sum of the changes of versions 1..ver
    double stale_ref; // predecessor drift at version g_ver
    double pad3;
};

struct SliceLoc {     // team-private control state of a slice (leader only)
    int f_ver;        // predecessor version of x_old
    int xo, wo;       // which of the two x / w buffers hold x_old / w_old
    int f_final;      // x_old is the predecessor's final value (EXACT)
    int stale_streak; // consecutive updates with a stale coarse input
    int done;
    int unpub;        // its last computed value was not published (a lost message)
    int reset_done;   // the injected reset has happened
    int zero_noted;   // idling: the zero change of the skipped update is recorded
    double last_sref; // predecessor drift at the version the last computed value's G read
    int v_valid;      // v holds F(x_old) (2D explicit: F is batched per round)
};

struct AsyncWork {
    double *ring = nullptr, *X = nullptr, *W = nullptr, *V = nullptr, *S = nullptr;
    SliceHdr *hdr = nullptr;
    SliceLoc *loc = nullptr;
    double *slot_drift = nullptr;
    int *sched = nullptr, *delay = nullptr;
    int *team_of = nullptr, *rank_of = nullptr, *tsize = nullptr;
    unsigned *tctr = nullptr;
    long long *tbc = nullptr;
    double *tred = nullptr;
    double *cgr = nullptr, *cgr1 = nullptr, *cgp0 = nullptr, *cgp1 = nullptr, *cgb = nullptr;
    double *cgw0 = nullptr, *cgw1 = nullptr;   // 2D preconditioned CG: u (r and p shared)
    int *drop = nullptr, *reset = nullptr;   // failure injection, [N+1] each
    double *lam0 = nullptr;                  // [(N+1) npts] initial iterate (resets only)
    unsigned long long *counters = nullptr;
    unsigned long long *pub_t = nullptr;   // [(N+1) R] publication time of each slot's version
    int *pipe = nullptr;                   // PIPELINED: [N+2] publications per version, then K*
    unsigned long long *pipe_dmax = nullptr;   // PIPELINED: [N+2] max change per version (bits)
    void *args = nullptr;   // the launch's AsyncArgs, in device memory
    // the configuration these buffers were sized for
    int R = 0, L = 0, nteams = 0, grid = 0, withS = 0;   // nteams: CG sets held
};

struct AsyncArgs {
    int N, dim, n, m;
    long long npts;
    double r, s, eps, cg_tol;
    int cg_maxit;
    Geom g;
    int mode, R, L, idle_skip;
    int incr;                // coarse solves act on the change of their input
    double *ring;            // [R][(N+1) npts]
    double *X, *W;           // [2][(N+1) npts]
    double *V, *S;           // [(N+1) npts]; S only if a slice needs several fine passes
    SliceHdr *hdr;           // [N+1]
    SliceLoc *loc;           // [N+1]
    double *slot_drift;      // [(N+1) R]
    const int *sched;        // REPLAY: [N][L]
    const int *delay;        // [N+1] or NULL
    const int *drop;         // [N+1] or NULL: update j of slice i is not published if drop[i] | j
    const int *reset;        // [N+1] or NULL: slice i starts again from lambda^0 before update reset[i] + 1
    const double *lam0;      // [(N+1) npts] the initial iterate, when resets are injected
    unsigned long long *pub_t;    // [(N+1) R] wall-clock time each slot's version was published
    unsigned long long lat;       // ticks after publication before a version may be read
    int *pipe;                    // PIPELINED: [N+1] publication counts per version, [N+1] = K*
    unsigned long long *pipe_dmax;  // PIPELINED: [N+1] max change of each version (bits)
    int kcap;                     // PIPELINED: iteration cap (k = N is exact)
    int blocks;                   // slices per team: contiguous blocks (1) or every nteams-th (0)
    int fine_kind;                // FINE_EXPLICIT or an implicit theta-method
    const double *inv_tab_f;      // 1D implicit fine steps: Thomas factors of s = theta r
    double *cgb;                  // implicit trapezoidal fine steps: [nteams * cgs] right-hand sides
    int nteams, maxtsz;
    const int *team_of, *rank_of, *tsize;   // per workgroup / per team
    unsigned *tctr;          // [nteams * 16]
    long long *tbc;          // [nteams * 16] leader broadcasts
    double *tred;            // [nteams * 8 * maxtsz]
    double *cgr, *cgr1, *cgp0, *cgp1;   // [nteams * cgs]
    double *cgw0, *cgw1;                // [nteams * cgs], 2D preconditioned CG only
    long long cgs;               // per-team stride of the CG vectors
    Control *ctl;
    unsigned long long *counters;   // cg iterations, coarse solves, skipped solves, copy retries, idle rounds
    // fine-kernel geometry
    int nsx, nsy, nsz, zc;
    int rows;                // 2D: rows of a fine sliding-window segment
    const double *inv_tab;   // 1D Thomas factors
    unsigned long long t_limit;  // wall-clock ticks before the launch gives up
};

// Barrier that also broadcasts 8 words from the team leader and the global
// stop flag.  All workgroups of the team see the same words.  Returns false
// when the launch is aborted or stopped.
__device__ __forceinline__ bool team_bcast(Team &tm, long long *slots, long long (&v)[8]) {
    __shared__ long long s_v[8];
    const int par = (tm.epoch + 1) & 1;
    if (tm.rank == 0 && threadIdx.x == 0) {
        v[7] = __hip_atomic_load(&tm.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int j = 0; j < 8; ++j) slots[par * 8 + j] = v[j];
    }
    if (!team_sync(tm)) return false;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) s_v[j] = slots[par * 8 + j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = uniform(s_v[j]);
    __syncthreads();
    return v[7] == 0;
}

// ---- sequence-locked header access (leader threads only)
__device__ __forceinline__ void hdr_publish(SliceHdr *h, int ver, int k, int g_ver, int final_from,
                                            double delta, double drift, double stale_ref) {
    const int s = h->seq;
    __hip_atomic_store(&h->seq, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&h->k, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&h->g_ver, g_ver, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&h->final_from, final_from, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st_relaxed(&h->delta, delta);
    st_relaxed(&h->drift, drift);
    st_relaxed(&h->stale_ref, stale_ref);
    st_release(&h->ver, ver);
    __hip_atomic_store(&h->seq, s + 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

struct HdrView {
    int ver, k;
    double delta, drift, stale_ref;
};

__device__ __forceinline__ bool hdr_read(const SliceHdr *h, HdrView &o) {
    const int s1 = ld_acquire(&h->seq);
    if (s1 & 1) return false;
    o.ver = __hip_atomic_load(&h->ver, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    o.k = __hip_atomic_load(&h->k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    o.delta = ld_relaxed(&h->delta);
    o.drift = ld_relaxed(&h->drift);
    o.stale_ref = ld_relaxed(&h->stale_ref);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int s2 = __hip_atomic_load(&h->seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return s1 == s2;
}

__device__ __forceinline__ unsigned long long ld_relaxed_u64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed_u64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Double-collect snapshot of all headers; true if the FREE stop rule holds.
__device__ bool free_stop_rule(const AsyncArgs &a) {
    long long vsum[2] = {0, 0};
    bool ok = true;
    for (int pass = 0; pass < 2; ++pass) {
        double prev_drift = 0.0;
        for (int i = 1; i <= a.N; ++i) {
            HdrView v;
            if (!hdr_read(&a.hdr[i], v)) return false;
            vsum[pass] += v.ver;
            if (pass == 0) {
                if (v.k < 1 || !(v.delta < a.eps)) ok = false;
                if (i > 1 && !(prev_drift - v.stale_ref < a.eps)) ok = false;
            }
            prev_drift = v.drift;
        }
        if (!ok) return false;
    }
    return vsum[0] == vsum[1];
}

// Newest version of slice j a reader may use: with a message latency, a
// version becomes readable `lat` ticks after its publication (the emulated
// transfer); the reader then takes the newest one that has arrived, going
// back at most to the oldest version the slot ring still protects (waiting
// for that one if it is still in flight).
__device__ int visible_version(const AsyncArgs &a, int j) {
    const int newest = ld_acquire(&a.hdr[j].ver);
    if (a.lat == 0) return newest;
    const int oldest = max(0, newest - (a.R - 2));
    for (int v = newest; v > oldest; --v)
        if (wall_clock64() >= ld_relaxed_u64(&a.pub_t[j * a.R + v % a.R]) + a.lat) return v;
    const unsigned long long due = ld_relaxed_u64(&a.pub_t[j * a.R + oldest % a.R]) + a.lat;
    while (wall_clock64() < due) {
        if (__hip_atomic_load(&a.ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        __builtin_amdgcn_s_sleep(2);
    }
    return oldest;
}

// ---- team-parallel elementwise helpers (chunks of 64 x-values)
__device__ __forceinline__ void team_copy(const Team &tm, const Geom &g, const double *__restrict__ src,
                                          double *__restrict__ dst) {
    const ChunkRange cr = team_chunks(g, tm.rank, tm.size);
    const int nw = nwaves();
    for (long long c = cr.begin + wave_id(); c < cr.end; c += (long long)STREAM_U * nw) {
        Point p[STREAM_U];
        chunk_points<STREAM_U>(g, c, cr.end, nw, p);
        double t[STREAM_U];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) t[u] = src[p[u].idx];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u)
            if (p[u].valid) dst[p[u].idx] = t[u];
    }
}

// ---- fine propagation of one state by a team: passes of <= D steps
// IMPL: the implicit fine propagators (a separate instantiation, so that the
// explicit kernel carries none of their registers).
template <int DIM, int XP, int RR, int D, bool IMPL>
__device__ __forceinline__ bool team_fine(Team &tm, const AsyncArgs &a, const double *src, double *dst, double *scr,
                          const CGWork &wk, const CGWork2 &wk2, double *rhs, unsigned long long &fine_its) {
    if constexpr (IMPL) {   // implicit theta-steps: Thomas per wave (1D), team CG
        if constexpr (DIM == 1) {
            if (wave_id() == 0) {
                const double th = theta_of(a.fine_kind);
                double c[RR], rl[RR], inv[RR];
                load1d<RR>(src, a.n, (1.0 - th) * a.r, c, rl);
                load_inv<RR>(a.inv_tab_f, inv);
                fine1d_theta_regs<RR>(c, rl, inv, a.n, th * a.r, a.m, a.fine_kind == FINE_TRAPEZOIDAL);
                store1d<RR>(dst, a.n, c);
            }
            return team_sync(tm);
        } else {
            const long long it = team_fine_theta<DIM, 2, true>(tm, a.g, a.fine_kind, a.r, a.m, a.cg_tol, a.cg_maxit,
                                                          src, dst, scr, rhs, wk, wk2);
            if (it < 0) return false;
            fine_its += (unsigned long long)it;
            return true;
        }
    } else if constexpr (DIM == 1) {
        if (wave_id() == 0) {
            double c[RR], rl[RR];
            load1d<RR>(src, a.n, a.r, c, rl);
            fine1d_regs<RR>(c, rl, a.m);
            store1d<RR>(dst, a.n, c);
        }
        return team_sync(tm);
    } else {
        // 3D (2D explicit F runs batched per round: team_fine_2d_batch)
        static_assert(DIM == 3, "2D explicit F is batched");
        const int passes = a.m;   // one step per pass
        const double *cur = src;
        const int waves = tm.size * nwaves();
        const int wid = tm.rank * nwaves() + wave_id();
        for (int p = 0; p < passes; ++p) {
            double *tgt = ((passes - 1 - p) % 2 == 0) ? dst : scr;
            const int total = a.nsx * a.nsy * a.nsz;
            for (int sidx = wid; sidx < total; sidx += waves) {
                int rem = sidx;
                const int sy = rem % a.nsy;
                rem /= a.nsy;
                const int sz = rem % a.nsz;
                const int sx = rem / a.nsz;
                const int z0 = sz * a.zc;
                fine3d_strip<XP, RR>(cur, tgt, a.n, a.r, sx, sy, z0, min(a.n, z0 + a.zc));
            }
            if (!team_sync(tm)) return false;
            cur = tgt;
        }
        return true;
    }
}

// ---- 2D explicit F of several slices of the team's block at once: bit j of
// `mask` is slice i0 + j * istep, bit j of `xo_mask` the x buffer holding its
// x_old.  Each pass runs over every (slice, strip, segment) unit of the
// team, so a pass costs one team barrier for all the slices, and the
// segments are long (a single 1024^2 state on a quarter of the chip gets
// 24-row segments that recompute as many halo rows).  Passes ping-pong
// between v and the slice's scratch so that the last lands in v.
template <int XP, int D>
__device__ __forceinline__ bool team_fine_2d_batch(Team &tm, const AsyncArgs &a, int i0, int istep,
                                                   unsigned long long mask, unsigned long long xo_mask) {
    const int cnt = __popcll(mask);
    if (cnt == 0) return true;
    const int passes = (a.m + D - 1) / D;
    const int waves = tm.size * nwaves();
    const int wid = tm.rank * nwaves() + wave_id();
    const long long np = a.npts, all = (long long)(a.N + 1) * np;
    const int seg = march_seg(a.n, (long long)a.nsx * cnt, waves, 24);
    const int nseg = (a.n + seg - 1) / seg;
    const long long per = (long long)a.nsx * nseg;
    const long long units = per * cnt;
    for (int p = 0; p < passes; ++p) {
        const int st = min(D, a.m - p * D);
        const bool to_v = ((passes - 1 - p) % 2 == 0);
        for (long long u = wid; u < units; u += waves) {
            const int jj = (int)(u / per);   // the jj-th slice of the mask
            const int rem = (int)(u - (long long)jj * per);
            const int sx = rem % a.nsx;      // strips of the same rows side by side
            const int sy = rem / a.nsx;
            unsigned long long mm = mask;
            for (int q = 0; q < jj; ++q) mm &= mm - 1;
            const int j = __ffsll((long long)mm) - 1;
            const int i = i0 + j * istep;
            const double *src = p == 0 ? a.X + (long long)((xo_mask >> j) & 1) * all + i * np
                                       : (to_v ? a.S : a.V) + i * np;
            double *tgt = (to_v ? a.V : a.S) + i * np;
            const int ya = sy * seg;
            fine2d_sw<XP, D, 2, false>(src, tgt, a.n, a.r, st, sx, ya, min(a.n, ya + seg), sy & 1);
        }
        if (!team_sync(tm)) return false;
    }
    return true;
}

// ---- coarse solve of one state by a team; returns iterations or -1
template <int DIM, int RR, bool PCG>
__device__ int team_coarse(Team &tm, const AsyncArgs &a, const double *b, double *x, const CGWork &wk,
                           const CGWork2 &wk2, double abs_thresh2 = -1.0, const double *xg = nullptr) {
    if constexpr (DIM == 1) {
        if (wave_id() == 0) {
            double v[RR], inv[RR];
            load_inv<RR>(a.inv_tab, inv);
            const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
            for (int e = 0; e < RR; ++e) {
                const int p = lane * RR + e;
                v[e] = p < a.n ? b[p] : 0.0;
            }
            thomas_wave<RR>(v, inv, a.n, a.s);
#pragma unroll
            for (int e = 0; e < RR; ++e) {
                const int p = lane * RR + e;
                if (p < a.n) x[p] = v[e];
            }
        }
        return team_sync(tm) ? 0 : -1;
    } else {
        // 2D: one synchronisation per iteration, 48 B per point, and the
        // marching sweep: a team sweeps a whole state with an eighth of the
        // chip or less, so each wave owns a long run of rows and streams it
        // with its loads four rows ahead (1.33x faster than chunks visited
        // one or two at a time, whose load latency set the pace).  3D: the
        // two-phase CG with marching phases (26.6 s for the 3D workload with
        // one chunk per wave in flight, 11.7 s with four, 10.7 s marching).
        int it;
        if constexpr (DIM == 2 && PCG) {
            // the preconditioned CG (marching sweeps of a whole iteration)
            const long long o = (long long)a.team_of[blockIdx.x] * a.cgs;
            const CGWorkP wkp{{wk2.r[0], wk2.r[1]}, {a.cgw0 + o, a.cgw1 + o}, {wk2.p[0], wk2.p[1]}, wk2.red};
            it = cg_team_2d_p<PCG_DEGREE, PCG_MINSEG_TEAM, 1>(tm, a.g, a.s, a.cg_tol, a.cg_maxit, b, x, wkp,
                                                           abs_thresh2, xg);
        } else if constexpr (DIM == 2)
            it = cg_team_2d_r<true>(tm, a.g, a.s, a.cg_tol, a.cg_maxit, b, x, wk2, abs_thresh2);
        else
            it = cg_team_dim<DIM, 4, DIM == 3>(tm, a.g, a.s, a.cg_tol, a.cg_maxit, b, x, wk, abs_thresh2, xg);
        if (it < 0) return -1;
        return team_sync(tm) ? it : -1;
    }
}

enum { ACT_IDLE = 0, ACT_UPDATE = 1, ACT_DONE = 2 };

// The arguments live in device memory: read through a uniform pointer they
// stay in scalar registers, where a by-value struct passed on by reference
// would be copied to scratch.  XP: x points per lane of F; RR: points per
// lane in 1D, rows per strip in 3D (2D takes its fine segment length at run
// time, RR = 0); D: fine steps per pass.
template <int DIM, int XP, int RR, int D, bool IMPL = false, bool PCG = false>
// Two workgroups per CU in 2D and 3D: 256 registers per lane, room for the
// two chunks in flight of the 2D coarse solver without spills.
__global__ __launch_bounds__(BLOCK, DIM == 1 ? 1 : 2) void k_async(const AsyncArgs *__restrict__ ap) {
    const AsyncArgs &a = *ap;
    const int team = a.team_of[blockIdx.x];
    if (team < 0) return;
    const int rank = a.rank_of[blockIdx.x];
    Team tm{a.tctr + (long long)team * team_counter_words(a.maxtsz), a.ctl, a.tsize[team], rank, 0u};
    if (!team_setup(tm)) return;
    long long *bc = a.tbc + team * 16;
    double *const tred = a.tred + (long long)team * 8 * a.maxtsz;
    CGWork wk{a.cgr + (long long)team * a.cgs, a.cgp0 + (long long)team * a.cgs,
              a.cgp1 + (long long)team * a.cgs, tred};
    const CGWork2 wk2{{wk.r, a.cgr1 + (long long)team * a.cgs}, {wk.p0, wk.p1}, tred};
    __shared__ double lds[MAX_WAVES];
    const bool leader = (rank == 0 && threadIdx.x == 0);
    const long long np = a.npts;
    const long long all = (long long)(a.N + 1) * np;
    const unsigned long long t0 = wall_clock64();
    unsigned long long cg_its = 0, g_solves = 0, g_skips = 0, retries = 0, idles = 0, fine_its = 0;
    // wall-clock ticks the team spends per phase (leader's view)
    unsigned long long t_fine = 0, t_copy = 0, t_coarse = 0, t_corr = 0, tp = 0;

    for (;;) {
        bool any_active = false, any_work = false;
        // the team's slices: every nteams-th, or a contiguous block; visited in
        // increasing order, one update each per round
        const int i_first = a.blocks ? 1 + (int)((long long)team * a.N / a.nteams) : team + 1;
        const int i_last = a.blocks ? (int)((long long)(team + 1) * a.N / a.nteams) : a.N;
        const int i_step = a.blocks ? 1 : a.nteams;
        // 2D explicit: F of every live slice of the block whose v is not
        // F(x_old) yet, batched at the start of the round (x_old of a slice
        // changes only in its own update, so v stays valid through idle and
        // stale updates)
        constexpr bool FBATCH = DIM == 2 && !IMPL;
        if constexpr (FBATCH) {
            long long fb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (leader) {
                unsigned long long m = 0, xm = 0;
                for (int i = i_first, j = 0; i <= i_last && j < 64; i += i_step, ++j) {
                    SliceLoc &L = a.loc[i];
                    const bool live = !L.done && a.hdr[i].k < a.L &&
                                      !(a.mode == AMODE_EXACT && a.hdr[i].final_from >= 0);
                    if (live && !L.v_valid) {
                        m |= 1ull << j;
                        xm |= (unsigned long long)(L.xo & 1) << j;
                        L.v_valid = 1;
                    }
                }
                fb[0] = (long long)m;
                fb[1] = (long long)xm;
            }
            if (!team_bcast(tm, bc, fb)) goto out;
            tp = wall_clock64();
            if (!team_fine_2d_batch<XP, D>(tm, a, i_first, i_step, (unsigned long long)fb[0],
                                           (unsigned long long)fb[1]))
                goto out;
            t_fine += wall_clock64() - tp;
        }
        for (int i = i_first; i <= i_last; i += i_step) {
            // ---------------- leader decides, team follows
            long long b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (leader) {
                SliceLoc &L = a.loc[i];
                const int myver = a.hdr[i].ver;
                int action = ACT_UPDATE, pv = 0;
                // a final slice (EXACT) or one at its iteration cap publishes no more
                if (L.done || a.hdr[i].k >= a.L || (a.mode == AMODE_EXACT && a.hdr[i].final_from >= 0)) {
                    action = ACT_DONE;
                } else if (scheduled_reads(a.mode)) {
                    // REPLAY: the host schedule.  PIPELINED (Algorithm 1): update k
                    // reads version k+1 of the predecessor, or its last one, i-1,
                    // once it is exact; slice i is exact after i updates, and
                    // nothing past the stopping iteration K* is needed.  A team
                    // holding several slices visits them in increasing order, one
                    // update each per round, so the update it waits on only needs
                    // updates of lower slices from this round or earlier ones:
                    // every wait ends.
                    const int k = a.hdr[i].k;
                    int tgt;
                    if (a.mode == AMODE_REPLAY) {
                        tgt = a.sched[(long long)(i - 1) * a.L + k];
                    } else {
                        const int ks = ld_acquire(&a.pipe[a.N + 1]);
                        tgt = (k >= i || k >= ks) ? -1 : min(k + 1, i - 1);
                    }
                    if (tgt < 0) {
                        action = ACT_DONE;
                    } else {
                        pv = tgt;
                        if (i > 1) {
                            long long spins = 0;
                            for (;;) {
                                const int have = ld_acquire(&a.hdr[i - 1].ver);
                                if (have >= tgt && wall_clock64() >= ld_relaxed_u64(&a.pub_t[(i - 1) * a.R + tgt % a.R]) + a.lat)
                                    break;
                                if (a.mode == AMODE_PIPELINED && k >= ld_acquire(&a.pipe[a.N + 1])) {
                                    action = ACT_DONE;   // K* became known: this update is not needed
                                    break;
                                }
                                if (__hip_atomic_load(&a.ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                                if (++spins > SPIN_LIMIT) {
                                    __hip_atomic_store(&a.ctl->error, -7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                    __hip_atomic_store(&a.ctl->abort, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(2);
                            }
                        }
                    }
                } else {
                    if (a.reset && !L.reset_done && a.reset[i] >= 0 && a.hdr[i].k == a.reset[i]) {
                        // the slice loses its state: x_old, w_old go back to the
                        // initial guess (copied by the team below)
                        L.reset_done = 1;
                        L.f_ver = 0;
                        L.f_final = (i == 1) ? 1 : 0;
                        L.stale_streak = 0;
                        L.last_sref = 0.0;   // version 0 of the predecessor
                        L.v_valid = 0;
                        b[6] = 1;
                    }
                    pv = (i == 1) ? 0 : visible_version(a, i - 1);
                    const bool stale = (pv == L.f_ver);
                    if (a.idle_skip && stale && L.stale_streak >= 1 && !L.unpub) {
                        // Its last update already read this predecessor version, so
                        // another update would republish F(x_old) unchanged: record
                        // that (zero) change once, then wait.  Retire if nothing new
                        // can arrive.
                        if (!L.zero_noted) {
                            SliceHdr *h = &a.hdr[i];
                            hdr_publish(h, h->ver, h->k, h->g_ver, h->final_from, 0.0, h->drift, h->stale_ref);
                            L.zero_noted = 1;
                        }
                        const bool pred_done = (i == 1) || ld_acquire(&a.hdr[i - 1].done) != 0;
                        action = (pred_done && pv == ld_acquire(&a.hdr[i - 1].ver)) ? ACT_DONE : ACT_IDLE;
                    }
                }
                if (action == ACT_DONE && !L.done) {
                    L.done = 1;
                    st_release(&a.hdr[i].done, 1);
                }
                if (a.delay && action == ACT_UPDATE)
                    for (int j = 0; j < a.delay[i]; ++j) __builtin_amdgcn_s_sleep(127);
                if (wall_clock64() - t0 > a.t_limit) {
                    __hip_atomic_store(&a.ctl->error, -7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&a.ctl->abort, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
                b[0] = action;
                b[1] = pv;
                b[2] = L.xo;
                b[3] = L.wo;
                b[4] = myver;
                b[5] = (pv == L.f_ver) ? 1 : 0;
                b[7] = L.v_valid ? 0 : 1;   // F still to be computed for this update
                if (action == ACT_UPDATE) L.v_valid = 1;
            }
            if (!team_bcast(tm, bc, b)) goto out;
            const int action = (int)b[0];
            if (action == ACT_DONE) continue;
            any_active = true;
            if (action == ACT_IDLE) continue;
            any_work = true;
            int pv = (int)b[1];
            const int xo = (int)b[2], wo = (int)b[3], myver = (int)b[4];
            bool stale = b[5] != 0;
            double *x_old = a.X + xo * all + i * np;
            double *x_new = a.X + (xo ^ 1) * all + i * np;
            double *w_old = a.W + wo * all + i * np;
            double *w_new = a.W + (wo ^ 1) * all + i * np;
            double *v = a.V + i * np;
            if (b[6]) {   // injected reset: start again from the initial guess
                team_copy(tm, a.g, a.lam0 + (i - 1) * np, x_old);
                if (!a.incr) team_copy(tm, a.g, a.lam0 + i * np, w_old);
                if (!team_sync(tm)) goto out;
            }
            // ---------------- v = F(x_old), unless the round's batch made it
            tp = wall_clock64();
            if constexpr (FBATCH) {
                if (b[7] && !team_fine_2d_batch<XP, D>(tm, a, i, 1, 1ull, (unsigned long long)(xo & 1)))
                    goto out;
            } else {
                if (!team_fine<DIM, XP, RR, D, IMPL>(tm, a, x_old, v, a.S ? a.S + i * np : nullptr, wk, wk2,
                                               a.cgb ? a.cgb + (long long)team * a.cgs : nullptr, fine_its))
                    goto out;
            }
            {   // uniform code: the phase clocks stay in scalar registers
                const unsigned long long t = wall_clock64();
                t_fine += t - tp;
                tp = t;
            }
            // ---------------- newest predecessor (FREE/EXACT read it after F)
            double drift_read = 0.0;
            int g_final = 0;
            double nrm_part = 0.0;
            double *dbuf = a.W + i * np;          // increment mode: change of the input
            double *ybuf = a.W + all + i * np;    // increment mode: G(change)
            for (;;) {
                if (!scheduled_reads(a.mode)) {
                    long long c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    if (leader) {
                        c[0] = (i == 1) ? 0 : visible_version(a, i - 1);
                        c[1] = (c[0] == a.loc[i].f_ver) ? 1 : 0;
                    }
                    if (!team_bcast(tm, bc, c)) goto out;
                    pv = (int)c[0];
                    stale = c[1] != 0;
                }
                if (stale) break;
                const double *src = a.ring + (long long)(pv % a.R) * all + (i - 1) * np;
                if (a.incr) {
                    // x_new = copy, d = x_new - x_old, ||x_new||^2 (reduced once the copy is valid)
                    nrm_part = 0.0;
                    const ChunkRange cr = team_chunks(a.g, tm.rank, tm.size);
                    const int nw = nwaves();
                    for (long long cc = cr.begin + wave_id(); cc < cr.end; cc += (long long)STREAM_U * nw) {
                        Point p[STREAM_U];
                        chunk_points<STREAM_U>(a.g, cc, cr.end, nw, p);
                        double xs[STREAM_U], xp[STREAM_U];
#pragma unroll
                        for (int u = 0; u < STREAM_U; ++u) {
                            xs[u] = src[p[u].idx];
                            xp[u] = x_old[p[u].idx];
                        }
#pragma unroll
                        for (int u = 0; u < STREAM_U; ++u) {
                            if (!p[u].valid) continue;
                            x_new[p[u].idx] = xs[u];
                            dbuf[p[u].idx] = xs[u] - xp[u];
                            nrm_part = __builtin_fma(xs[u], xs[u], nrm_part);
                        }
                    }
                } else {
                    team_copy(tm, a.g, src, x_new);
                }
                // Ring slots are reused: the copy is valid only if the writer had
                // not started on this slot again when the LAST load of every
                // workgroup of the team had returned, so the version is re-read
                // after a team barrier (scheduled reads keep every version).
                if (!scheduled_reads(a.mode) && i > 1 && !team_sync(tm)) goto out;
                long long c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (leader) {
                    const double dr = a.slot_drift[(i - 1) * a.R + pv % a.R];
                    const int ff = __hip_atomic_load(&a.hdr[i - 1].final_from, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    const int after = (i == 1) ? pv : ld_acquire(&a.hdr[i - 1].ver);
                    c[0] = (scheduled_reads(a.mode) || after - pv <= a.R - 2) ? 1 : 0;
                    c[1] = __double_as_longlong(dr);
                    c[2] = (i == 1) ? 1 : ((ff >= 0 && pv >= ff) ? 1 : 0);
                }
                if (!team_bcast(tm, bc, c)) goto out;
                if (c[0]) {
                    drift_read = __longlong_as_double(c[1]);
                    g_final = (int)c[2];
                    break;
                }
                if (++retries > 100000) {
                    if (leader) {
                        __hip_atomic_store(&a.ctl->error, -7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&a.ctl->abort, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    goto out;
                }
            }
            // ---------------- w_new = G(x_new) (or G(x_new - x_old)), or nothing if stale
            {   // uniform code: the phase clocks stay in scalar registers
                const unsigned long long t = wall_clock64();
                t_copy += t - tp;
                tp = t;
            }
            const double *wv = w_old;
            if (!stale) {
                // one call site: the kernel holds a single copy of the solver
                double thr = -1.0;
                if (a.incr) {
                    double nrm = 0.0;
                    if (!team_reduce<false>(tm, nrm_part, wk.red, nrm, lds)) goto out;
                    thr = a.cg_tol * a.cg_tol * nrm;
                }
                // the literal form starts from the last coarse value G(x_old)
                const int it = team_coarse<DIM, RR, PCG>(tm, a, a.incr ? dbuf : x_new, a.incr ? ybuf : w_new, wk, wk2,
                                                         thr, a.incr ? nullptr : w_old);
                if (it < 0) goto out;
                cg_its += (unsigned long long)it;
                ++g_solves;
                wv = w_new;
            } else {
                ++g_skips;
            }
            // ---------------- lambda = v + (w_new - w_old), change norm, write the next slot
            {   // uniform code: the phase clocks stay in scalar registers
                const unsigned long long t = wall_clock64();
                t_coarse += t - tp;
                tp = t;
            }
            const int nslot = (myver + 1) % a.R;
            const double *cur = a.ring + (long long)(myver % a.R) * all + i * np;
            double *nxt = a.ring + (long long)nslot * all + i * np;
            double dmax = 0.0;
            {
                const ChunkRange cr = team_chunks(a.g, tm.rank, tm.size);
                const int nw = nwaves();
                // increment form: y = G(change), or 0 when stale; literal form:
                // w_new and w_old
                const double *pa = a.incr ? ybuf : wv;
                const bool use_b = !a.incr;
                const bool use_a = !(a.incr && stale);
                for (long long c = cr.begin + wave_id(); c < cr.end; c += (long long)STREAM_U * nw) {
                    Point p[STREAM_U];
                    chunk_points<STREAM_U>(a.g, c, cr.end, nw, p);
                    double tv[STREAM_U], ta[STREAM_U], tb[STREAM_U], tc[STREAM_U];
#pragma unroll
                    for (int u = 0; u < STREAM_U; ++u) {
                        const long long j = p[u].idx;
                        tv[u] = v[j];
                        ta[u] = use_a ? pa[j] : 0.0;
                        tb[u] = use_b ? w_old[j] : 0.0;
                        tc[u] = cur[j];
                    }
#pragma unroll
                    for (int u = 0; u < STREAM_U; ++u) {
                        if (!p[u].valid) continue;
                        const double ln = use_b ? tv[u] + (ta[u] - tb[u]) : tv[u] + ta[u];
                        dmax = fmax(dmax, fabs(ln - tc[u]));
                        nxt[p[u].idx] = ln;
                    }
                }
            }
            double delta;
            if (!team_reduce<true>(tm, dmax, wk.red, delta, lds)) goto out;
            // ---------------- publish (leader), update the slice's control state
            if (leader) {
                SliceLoc &L = a.loc[i];
                SliceHdr *h = &a.hdr[i];
                const double drift = h->drift + delta;
                // a stale update's G input is that of the last computed value
                // (published or lost), whose predecessor drift is kept locally
                const double sref = stale ? L.last_sref : drift_read;
                L.last_sref = sref;
                const int gf = stale ? L.f_final : g_final;
                int ff = h->final_from;
                if (ff < 0 && L.f_final && gf) ff = myver + 1;
                // injected message loss: the update counts, its value is not published
                const bool lost = a.drop && a.drop[i] > 0 && (h->k + 1) % a.drop[i] == 0;
                if (lost) {
                    hdr_publish(h, myver, h->k + 1, h->g_ver, h->final_from, h->delta, h->drift, h->stale_ref);
                    ff = -1;
                } else {
                    a.slot_drift[i * a.R + nslot] = drift;
                    st_relaxed_u64(&a.pub_t[i * a.R + nslot], wall_clock64());   // ordered by the publication
                    hdr_publish(h, myver + 1, h->k + 1, pv, ff, delta, drift, sref);
                }
                L.unpub = lost ? 1 : 0;
                L.zero_noted = 0;
                if (a.mode == AMODE_PIPELINED) {
                    // version v is complete once slices v..N have published it; the
                    // first complete version with a change below eps (or v = N, or
                    // the cap) is the stopping iteration K* of the synchronous test
                    const int v = myver + 1;
                    __hip_atomic_fetch_max(&a.pipe_dmax[v], (unsigned long long)__double_as_longlong(delta),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int seen = __hip_atomic_fetch_add(&a.pipe[v], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
                    if (seen == a.N - v + 1) {
                        const double dv = __longlong_as_double((long long)__hip_atomic_load(
                            &a.pipe_dmax[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        if (dv < a.eps || v >= a.kcap) {
                            __hip_atomic_fetch_min(&a.pipe[a.N + 1], v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                            __hip_atomic_store(&a.ctl->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
                if (!stale) {
                    L.xo ^= 1;
                    if (!a.incr) L.wo ^= 1;
                    L.v_valid = 0;   // x_old moved on
                }
                L.f_ver = pv;
                L.f_final = gf;
                L.stale_streak = stale ? L.stale_streak + 1 : 0;
                if (a.mode == AMODE_EXACT && i == a.N && ff >= 0)
                    __hip_atomic_store(&a.ctl->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                if (a.mode == AMODE_FREE && delta < a.eps && free_stop_rule(a))
                    __hip_atomic_store(&a.ctl->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            t_corr += wall_clock64() - tp;
        }
        if (!any_active) {
            // every slice of this team has retired: the state may now satisfy
            // the stop rule with nobody left to notice, so look once more
            if (leader && a.mode == AMODE_FREE && free_stop_rule(a))
                __hip_atomic_store(&a.ctl->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        if (!any_work) {
            ++idles;
            if (leader) {
                if (a.mode == AMODE_FREE && free_stop_rule(a))
                    __hip_atomic_store(&a.ctl->stop, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_s_sleep(32);
            }
        }
    }
out:
    if (leader) {
        __hip_atomic_fetch_add(&a.counters[0], cg_its, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[1], g_solves, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[2], g_skips, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[3], retries, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[4], idles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[5], t_fine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[6], t_copy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[7], t_coarse, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[8], t_corr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[9], wall_clock64() - t0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&a.counters[10], fine_its, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Pipelined driver: no version complete yet, stopping iteration unknown (N+1).
__global__ void k_pipe_init(int *pipe, int N) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v <= N + 1) pipe[v] = (v == N + 1) ? N + 1 : 0;
}

// Initial per-slice control state: x_old = lambda_{i-1}^0 in X[0], w_old =
// lambda_i^0 in W[0], version 0 in ring slot 0.
__global__ void k_async_init(SliceHdr *hdr, SliceLoc *loc, double *slot_drift, int N, int R) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    SliceHdr h{};
    h.final_from = (i == 0) ? 0 : -1;
    h.done = (i == 0) ? 1 : 0;
    hdr[i] = h;
    SliceLoc l{};
    l.f_final = (i == 1) ? 1 : 0;
    loc[i] = l;
    for (int j = 0; j < R; ++j) slot_drift[i * R + j] = 0.0;
}

// lambda_out[i] = newest published version of slice i, capped at vcap (the
// stopping iteration of the pipelined driver; slices ran ahead of it).
__global__ void k_async_gather(const double *ring, const SliceHdr *hdr, double *out, long long npts, int N,
                               int R, const int *vcap) {
    const long long all = (long long)(N + 1) * npts;
    const int i = blockIdx.y;
    const int slot = (vcap ? min(hdr[i].ver, *vcap) : hdr[i].ver) % R;
    const double *src = ring + slot * all + i * npts;
    double *dst = out + i * npts;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x)
        dst[p] = src[p];
}

}  // namespace pr
