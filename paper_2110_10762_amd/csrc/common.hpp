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
__device__ __forceinline__ double from_lower_lane(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_upper_lane(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
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
__device__ __forceinline__ bool wait_counter(const unsigned *ctr, unsigned target, Control *ctl) {
    long long spins = 0;
    while ((int)(ld_relaxed(ctr) - target) < 0) {
        if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (++spins > SPIN_LIMIT) {
            __hip_atomic_store(&ctl->error, -7, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// A team is a fixed set of co-resident workgroups that cooperate on one
// state.  Its barrier counts arrivals on monotonically increasing counters:
// workgroups are split into groups of at most TEAM_GROUP, each group has its
// own counter on its own cache line, and the last arrival of a group bumps
// the top counter; the e-th barrier completes when the top counter reaches
// e * (number of groups).  Counter block layout (words): top at 0, group g at
// 32 * (1 + g); team_counter_words() gives its size.
constexpr int TEAM_GROUP = 32;

__host__ __device__ inline int team_groups(int size) { return (size + TEAM_GROUP - 1) / TEAM_GROUP; }
__host__ __device__ inline int team_counter_words(int size) { return 32 * (1 + team_groups(size)); }

struct Team {
    unsigned *ctr;    // counter block (zeroed before the launch)
    Control *ctl;
    int size;         // workgroups in the team
    int rank;         // this workgroup's index in the team
    unsigned epoch;   // barriers passed so far (identical in all threads)
};

// Team barrier with agent-scope release/acquire ordering.  Returns false if
// the launch was aborted (every caller then unwinds).  All threads of all
// team workgroups must call it.
__device__ __forceinline__ bool team_sync(Team &tm) {
    __shared__ int s_ok;
    tm.epoch += 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        if (tm.size > 1) {
            const int ng = team_groups(tm.size);
            unsigned target;
            if (ng == 1) {
                __hip_atomic_fetch_add(tm.ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                target = tm.epoch * (unsigned)tm.size;
            } else {
                const int g = tm.rank / TEAM_GROUP;
                const unsigned gsize = (unsigned)min(TEAM_GROUP, tm.size - g * TEAM_GROUP);
                const unsigned old = __hip_atomic_fetch_add(tm.ctr + 32 * (1 + g), 1u, __ATOMIC_ACQ_REL,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                if (old + 1u == tm.epoch * gsize)
                    __hip_atomic_fetch_add(tm.ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                target = tm.epoch * (unsigned)ng;
            }
            ok = wait_counter(tm.ctr, target, tm.ctl);
        }
        s_ok = ok && !__hip_atomic_load(&tm.ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return s_ok != 0;
}

// Deterministic team all-reduce: every workgroup writes its partial to
// buf[rank]; after the barrier every workgroup sums (or maxes) buf[0..size)
// in the same fixed order, so all of them hold bit-identical results.
template <bool MAX>
__device__ __forceinline__ bool team_reduce(Team &tm, double part, double *buf, double &out,
                                            double *lds) {
    part = block_reduce<MAX>(part, lds);
    if (threadIdx.x == 0) buf[tm.rank] = part;
    if (!team_sync(tm)) return false;
    double v = MAX ? 0.0 : 0.0;
    if (threadIdx.x < WAVE) {
        double acc = MAX ? 0.0 : 0.0;
        for (int j = threadIdx.x; j < tm.size; j += WAVE) {
            double b = buf[j];
            acc = MAX ? fmax(acc, b) : acc + b;
        }
        v = MAX ? wave_max(acc) : wave_sum(acc);
        if (threadIdx.x == 0) lds[0] = v;
    }
    __syncthreads();
    out = lds[0];
    __syncthreads();
    return true;
}

}  // namespace pr
