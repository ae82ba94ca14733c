// Adjoint of the fine integration (gradient of L = 1/2 ||u(T) - u_target||^2
// with respect to u0 and nu).
//
// The fine solution is u_{n+1} = A u_n with A = I + nu dt L_h (M = N*m steps,
// dt fixed by the slicing).  With mu_M = dL/du(T) and mu_n = A^T mu_{n+1}:
//     dL/du0 = mu_0,      dL/dnu = sum_n mu_{n+1}^T (dt L_h u_n).
// A is symmetric (same stencil weights both ways, zero ghosts), so A^T mu is
// the explicit-Euler step applied to mu.  The slice-boundary adjoints
// mu_{i-1} = (A^T)^m mu_i are computed first, sequentially; then every slice
// works in parallel: its forward states are recomputed from the checkpoint
// lambda_{i-1} (sub-checkpoints every c ~ sqrt(m) steps, one segment at a
// time), and k_adjoint_step walks the segment backwards, producing mu_n and
// the per-block partial sums of mu_{n+1}^T (h^2 L_h u_n).
#pragma once
#include "coarse.hpp"

namespace pr {

struct AdjWork {
    double *mu = nullptr;      // [(N+1) npts] slice-boundary adjoints
    double *subck = nullptr;   // [nseg][N][npts] forward sub-checkpoints
    double *seg = nullptr;     // [c][N][npts] recomputed forward states of a segment
    double *mw = nullptr;      // [2][N][npts] running adjoint of every slice
    double *tmp = nullptr;     // [N][npts] fine-pass scratch
    double *acc = nullptr;     // [N][nblk] partial sums
    int c = 0, nseg = 0, nblk = 0;
};

// mu_out = A mu_in for `count` states (blockIdx.y), and
// acc[state][block] += <mu_in, h^2 L_h u> over the block's chunks.  The block
// -> chunk assignment is the same in every launch, so each slot accumulates
// in a fixed order.
__global__ __launch_bounds__(BLOCK) void k_adjoint_step(const double *__restrict__ mu_in, double *__restrict__ mu_out,
                                                        const double *__restrict__ u, long long stride, Geom g,
                                                        double r, double *acc) {
    __shared__ double lds[MAX_WAVES];
    const int st = blockIdx.y;
    const double *mi = mu_in + st * stride;
    double *mo = mu_out + st * stride;
    const double *us = u + st * stride;
    const double twod = 2.0 * g.dim;
    const ChunkRange cr = team_chunks(g, blockIdx.x, gridDim.x);
    double part = 0.0;
    for (long long c = cr.begin + wave_id(); c < cr.end; c += nwaves()) {
        const Point p = chunk_point(g, c);
        const double mc = p.valid ? mi[p.idx] : 0.0;
        const double uc = p.valid ? us[p.idx] : 0.0;
        const double nm = neighbour_sum(g, p, mc, [&](long long j) { return mi[j]; });
        const double nu = neighbour_sum(g, p, uc, [&](long long j) { return us[j]; });
        const double lap_mu = __builtin_fma(-twod, mc, nm);
        const double lap_u = __builtin_fma(-twod, uc, nu);
        if (p.valid) {
            mo[p.idx] = __builtin_fma(r, lap_mu, mc);
            part = __builtin_fma(mc, lap_u, part);
        }
    }
    part = block_reduce<false>(part, lds);
    if (threadIdx.x == 0) acc[(long long)st * gridDim.x + blockIdx.x] += part;
}

}  // namespace pr
