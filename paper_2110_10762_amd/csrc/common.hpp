// Device-side building blocks shared by every kernel of the library:
// wave64 DPP lane shifts, odd-reflection indexing of the zero-Dirichlet
// extension, deterministic wave/block/team reductions, and a bounded
// team barrier built on agent-scope atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pr {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;            // threads per workgroup for all kernels
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;
constexpr int MAX_WAVES = 16;         // largest workgroup: 1024 threads

// Waves in this workgroup (uniform).
__device__ __forceinline__ int nwaves() { return (int)(blockDim.x / WAVE); }

// Index of this wave in its workgroup, as a wave-uniform (scalar) value so
// that everything derived from it stays in scalar registers.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
}

// ---------------------------------------------------------------- lane shifts
// Whole-wave DPP row moves: wave_shr:1 moves data to the next higher lane
// (lane l receives lane l-1), wave_shl:1 to the next lower lane.  Lanes
// whose source is outside the wave receive 0.
// (bound_ctrl set: the lane without a source, 0 resp. 63, reads 0)
__device__ __forceinline__ double from_lower_lane(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_upper_lane(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// A value every lane of the wave holds alike, moved to scalar registers (so
// that what is derived from it, addresses above all, stays scalar too).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform(long long v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double uniform(double v) {
    return __longlong_as_double(uniform((long long)__double_as_longlong(v)));
}

// ---------------------------------------------------------------- boundaries
// Zero Dirichlet ghosts at index -1 and n are kept exactly zero by extending
// the grid function oddly about them (period 2(n+1)): the explicit stencil
// commutes with that reflection, so a strip that loads the extension instead
// of masking computes the interior values bit for bit.  Returns the interior
// index to load and the sign (+1, -1, or 0 for a ghost).
__device__ __forceinline__ int reflect(int y, int n, double &sgn) {
    const int P = 2 * (n + 1);
    int t = (y + 1) % P;
    if (t < 0) t += P;
    if (t == 0 || t == n + 1) { sgn = 0.0; return 0; }
    if (t <= n) { sgn = 1.0; return t - 1; }
    sgn = -1.0;
    return P - t - 1;
}

// One explicit-Euler update with a fixed evaluation order (explicit fma so
// every kernel shape rounds identically).  s2 = (up+down), s1 = (left+right).
__device__ __forceinline__ double euler_update(double cur, double s1, double s2,
                                               double twod, double r) {
    double s = s2 + s1;
    double t = __builtin_fma(-twod, cur, s);
    return __builtin_fma(r, t, cur);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Block reduction in a fixed order; every thread gets the result.
template <bool MAX>
__device__ __forceinline__ double block_reduce(double v, double *lds /*[MAX_WAVES]*/) {
    v = MAX ? wave_max(v) : wave_sum(v);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[w] = v;
    __syncthreads();
    double t = lds[0];
    const int nw = nwaves();
    for (int i = 1; i < nw; ++i) t = MAX ? fmax(t, lds[i]) : t + lds[i];
    return t;
}

// ---------------------------------------------------------------- atomics
__device__ __forceinline__ unsigned ld_acquire(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_acquire(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(unsigned *p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_acquire(const double *p) {
    unsigned long long u = __hip_atomic_load((const unsigned long long *)p, __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)u);
}
__device__ __forceinline__ double ld_relaxed(const double *p) {
    unsigned long long u = __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)u);
}
__device__ __forceinline__ void st_relaxed(double *p, double v) {
    __hip_atomic_store((unsigned long long *)p, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// max of non-negative doubles through their (order-preserving) bit patterns
__device__ __forceinline__ void atomic_max_nonneg(double *p, double v) {
    __hip_atomic_fetch_max((unsigned long long *)p, (unsigned long long)__double_as_longlong(v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- control block
// Shared by all workgroups of a launch: an abort flag that every bounded wait
// checks, and the error code of the first wait that ran out.
struct Control {
    int abort;
    int error;        // 0 or PR_ETIMEOUT
    int stop;         // asynchronous driver: set once the stop rule holds
    int pad;
};

constexpr long long SPIN_LIMIT = 1ll << 27;   // ~ seconds of s_sleep(1) polling

// Waits (single thread) until (int)(*ctr - target) >= 0.  Returns false if the
// launch was aborted or the wait ran out (then the launch is aborted).
__device__ __forceinline__ unsigned ld_relaxed(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls (single thread) with relaxed atomic loads until (int)(*ctr - target)
// >= 0, then issues one agent-scope acquire fence.  Returns false if the
// launch was aborted or the wait ran out (then the launch is aborted).
// The abort flag is read every 16th poll only: a poll is a round trip to the
// memory side, and the barrier latency is a chain of them.
__device__ __forceinline__ bool wait_counter(const unsigned *ctr, unsigned target, Control *ctl) {
    long long spins = 0;
    while ((int)(ld_relaxed(ctr) - target) < 0) {
        if ((++spins & 15) == 0) {
            if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
            if (spins > SPIN_LIMIT) {
                __hip_atomic_store(&ctl->error, -7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// A team is a fixed set of co-resident workgroups that cooperate on one
// state.  Its barrier is two-level and follows the chip's cache hierarchy:
// the workgroups of the team that sit on the same XCD (read from the
// hardware XCC_ID register when the launch starts) count their arrivals on
// that XCD's counter; the last arrival of each XCD writes the XCD's L2 back
// (agent-scope release) and, if the team spans several XCDs, meets the other
// XCDs' last arrivals on the top counter; it then raises the XCD's
// generation word, which the other workgroups of the XCD poll.  Every
// workgroup ends with an agent-scope acquire.  Counters are monotone (the
// e-th barrier waits for e * count), polled with relaxed agent-scope loads,
// and every wait is bounded.  Counter block (words, one cache line each):
// top at 0, arrivals of XCD x at 32*(1+x), generation of XCD x at 32*(9+x),
// registrations of XCD x at 32*(17+x), set-up arrivals at 32*25.
constexpr int TEAM_CTR_WORDS = 32 * 26;

__host__ __device__ inline int team_counter_words(int) { return TEAM_CTR_WORDS; }

__device__ __forceinline__ int xcc_id() {
    // s_getreg_b32 hwreg(HW_REG_XCC_ID, 0, 16)
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((16 - 1) << 11)) & 7;
}

struct Team {
    unsigned *ctr;    // counter block (zeroed before the launch)
    Control *ctl;
    int size;         // workgroups in the team
    int rank;         // this workgroup's index in the team
    unsigned epoch;   // barriers passed so far (identical in all threads)
    int xcc;          // this workgroup's XCD
    int gx;           // workgroups of this team on that XCD
    int nx;           // XCDs the team spans
    int rpar;         // reduction slot set used by the next team_reduce (alternates)
};

// Must be called once by every workgroup of the team before any team_sync.
// xcd_ranks: renumber the workgroups so that those on one XCD hold
// consecutive ranks (XCD 0 first, arrival order within an XCD); the chunks a
// rank owns are then neighbours in memory, so the halo rows a workgroup
// reads mostly sit in its own XCD's L2.  Any numbering gives the same
// results: a rank's chunk range and reduction slot do not depend on which
// workgroup holds it.
__device__ __forceinline__ bool team_setup(Team &tm, bool xcd_ranks = false) {
    __shared__ int s_gx, s_nx, s_ok, s_rank;
    tm.xcc = xcc_id();
    if (threadIdx.x == 0) {
        bool ok = true;
        int gx = 1, nx = 1, rank = tm.rank;
        if (tm.size > 1) {
            const unsigned ticket = __hip_atomic_fetch_add(tm.ctr + 32 * (17 + tm.xcc), 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(tm.ctr + 32 * 25, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            ok = wait_counter(tm.ctr + 32 * 25, (unsigned)tm.size, tm.ctl);
            nx = 0;
            int before = 0;
            for (int x = 0; x < 8; ++x) {
                const unsigned cx = ld_relaxed(tm.ctr + 32 * (17 + x));
                nx += cx > 0u;
                if (x < tm.xcc) before += (int)cx;
            }
            gx = (int)ld_relaxed(tm.ctr + 32 * (17 + tm.xcc));
            if (xcd_ranks) rank = before + (int)ticket;
        }
        s_gx = gx;
        s_nx = nx;
        s_ok = ok;
        s_rank = rank;
    }
    __syncthreads();
    tm.gx = s_gx;
    tm.nx = s_nx;
    tm.rank = uniform(s_rank);
    tm.epoch = 0;
    tm.rpar = 0;
    const bool ok = s_ok != 0;
    __syncthreads();
    return ok;
}

// Team barrier with agent-scope release/acquire ordering.  Returns false if
// the launch was aborted (every caller then unwinds).  All threads of all
// team workgroups must call it.
__device__ __forceinline__ bool team_sync(Team &tm) {
    __shared__ int s_ok;
    tm.epoch += 1;
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached L2
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        if (tm.size > 1) {
            const unsigned old = __hip_atomic_fetch_add(tm.ctr + 32 * (1 + tm.xcc), 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            if (old + 1u == tm.epoch * (unsigned)tm.gx) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // write this XCD's L2 back
                if (tm.nx > 1) {
                    __hip_atomic_fetch_add(tm.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = wait_counter(tm.ctr, tm.epoch * (unsigned)tm.nx, tm.ctl);   // ends with the acquire
                } else {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                __hip_atomic_store(tm.ctr + 32 * (9 + tm.xcc), tm.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = wait_counter(tm.ctr + 32 * (9 + tm.xcc), tm.epoch, tm.ctl);   // ends with the acquire
            }
        }
        // an abort raised elsewhere while this barrier completed is seen at
        // the next wait
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Slots a lane loads at once when it sums the team's partials (one round
// trip for teams of up to 256 workgroups).  Lanes sum their slots j, j + 64,
// ... in increasing order, padding with zeros, whatever the batch.
constexpr int SLOT_BATCH = 4;

// Deterministic team all-reduce: every workgroup writes its partial to its
// slot; after the barrier every workgroup sums (or maxes) the slots in the
// same fixed order, so all of them hold bit-identical results.  `base` holds
// two sets of `size` slots; consecutive reductions alternate between them so
// that a fast workgroup never overwrites a slot a slow one is still reading.
template <bool MAX>
__device__ __forceinline__ bool team_reduce(Team &tm, double part, double *base, double &out, double *lds) {
    double *buf = base + tm.rpar * tm.size;
    tm.rpar ^= 1;
    part = block_reduce<MAX>(part, lds);
    if (threadIdx.x == 0) buf[tm.rank] = part;
    if (!team_sync(tm)) return false;
    if (threadIdx.x < WAVE) {
        double acc = 0.0;
        for (int j0 = 0; j0 < tm.size; j0 += SLOT_BATCH * WAVE) {
            double b[SLOT_BATCH];
#pragma unroll
            for (int t = 0; t < SLOT_BATCH; ++t) {
                const int j = j0 + t * WAVE + (int)threadIdx.x;
                b[t] = j < tm.size ? buf[j] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < SLOT_BATCH; ++t) acc = MAX ? fmax(acc, b[t]) : acc + b[t];
        }
        const double v = MAX ? wave_max(acc) : wave_sum(acc);
        if (threadIdx.x == 0) lds[0] = v;
    }
    __syncthreads();
    out = uniform(lds[0]);
    __syncthreads();
    return true;
}

// K sums at once, one barrier.  `base` holds 2 K * size slots; value k of
// slot set q (q = 0, 1 alternating) sits at [(2k + q) size, (2k + q + 1)
// size), so set q of one call never meets set 1 - q of the next, whichever
// of team_reduce and team_reduce_n makes it.  Per value, the order of the
// additions is that of team_reduce.
//
// Split form, for callers that issue loads while the partials travel:
// team_reduce_begin writes this workgroup's partials and passes the barrier
// (returns the slot set, or -1 if the launch was aborted); team_reduce_end
// sums the slots.  No slot write of the team may come in between.
template <int K>
__device__ __forceinline__ int team_reduce_begin(Team &tm, const double (&part)[K], double *base) {
    __shared__ double sl[MAX_WAVES * K];
    const int q = tm.rpar;
    tm.rpar ^= 1;
    const int w = threadIdx.x / WAVE;
    const int nw = nwaves();
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(part[k]);
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sl[w * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = sl[k];
            for (int i = 1; i < nw; ++i) t = t + sl[i * K + k];
            base[(long long)(2 * k + q) * tm.size + tm.rank] = t;
        }
    }
    return team_sync(tm) ? q : -1;
}

template <int K>
__device__ __forceinline__ void team_reduce_end(const Team &tm, const double *base, int q, double (&out)[K]) {
    __shared__ double so[K];
    if (threadIdx.x < WAVE) {
        double acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = 0.0;
        for (int j0 = 0; j0 < tm.size; j0 += SLOT_BATCH * WAVE) {
            double b[K][SLOT_BATCH];
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int t = 0; t < SLOT_BATCH; ++t) {
                    const int j = j0 + t * WAVE + (int)threadIdx.x;
                    b[k][t] = j < tm.size ? base[(long long)(2 * k + q) * tm.size + j] : 0.0;
                }
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int t = 0; t < SLOT_BATCH; ++t) acc[k] += b[k][t];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double r = wave_sum(acc[k]);
            if (threadIdx.x == 0) so[k] = r;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = uniform(so[k]);
    __syncthreads();
}

template <int K>
__device__ __forceinline__ bool team_reduce_n(Team &tm, const double (&part)[K], double *base, double (&out)[K]) {
    const int q = team_reduce_begin<K>(tm, part, base);
    if (q < 0) return false;
    team_reduce_end<K>(tm, base, q, out);
    return true;
}

}  // namespace pr
