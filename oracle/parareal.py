"""Synchronous and asynchronous Parareal (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Synchronous Parareal follows equation (pr) of Section 3.1 literally: every
slice is recomputed at every iteration, including the ones that are already
exact (the distributed algorithm of Section 4.1 skips them; the values are the
same bit for bit).  Asynchronous Parareal follows equation (apr) in the form of
Algorithm 2 (Section 4.1): each slice keeps the predecessor iterate its last
coarse solve used; its next fine solve starts from that iterate, its next
coarse solve uses whichever predecessor version the schedule delivers.  The
schedule stands for the update sets P^(k) and the delays of equation (ai)
(Section 2.1); the replay is deterministic so that tests can pin it.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Iterable, List, Optional, Tuple

import numpy as np


def coarse_sweep(u0: np.ndarray, G: Callable, nslices: int) -> np.ndarray:
    """Initial guess of Section 3.1: lambda_0 = u0, lambda_i = G(lambda_{i-1})."""
    lam = np.empty((nslices + 1,) + u0.shape)
    lam[0] = u0
    for i in range(1, nslices + 1):
        lam[i] = G(lam[i - 1])
    return lam


def correction(v: np.ndarray, w_new: np.ndarray, w_old: np.ndarray) -> np.ndarray:
    """lambda_i^{k+1} = G(new input) + F(old input) - G(old input), evaluated
    as v + (w_new - w_old): equal inputs then give exactly v."""
    return v + (w_new - w_old)


@dataclasses.dataclass
class SyncResult:
    lam: np.ndarray                 # final iterate, shape (N+1,) + u0.shape
    iters: int                      # k at which the loop stopped
    deltas: List[float]             # ||lambda^k - lambda^{k-1}||_inf for k = 1..iters
    history: Optional[List[np.ndarray]] = None   # lambda^0 .. lambda^iters if kept


def parareal_sync(u0: np.ndarray, F: Callable, G: Callable, nslices: int,
                  eps: float = 1e-10, kmax: Optional[int] = None,
                  keep_history: bool = False) -> SyncResult:
    """Equation (pr): lambda_0^{k+1} = lambda_0^k and, for every slice,
    lambda_i^{k+1} = G(lambda_{i-1}^{k+1}) + F(lambda_{i-1}^k) - G(lambda_{i-1}^k).

    G(lambda_{i-1}^k) is the value computed for slice i at the previous
    iteration (Algorithm 1 keeps it as w_i^k).  Stops at the first k with
    ||lambda^k - lambda^{k-1}||_inf < eps (eq. (thresh)), at k = N (finite
    termination) or at kmax.  eps <= 0 runs exactly kmax (or N) iterations.
    """
    N = nslices
    if kmax is None or kmax > N:
        kmax = N
    lam = coarse_sweep(u0, G, N)
    w = lam.copy()                       # w_i^0 = G(lambda_{i-1}^0) = lambda_i^0
    hist = [lam.copy()] if keep_history else None
    deltas: List[float] = []
    k = 0
    while k < kmax:
        v = np.empty_like(lam)
        for i in range(1, N + 1):
            v[i] = F(lam[i - 1])        # F(lambda_{i-1}^k), all slices independent
        new = lam.copy()
        for i in range(1, N + 1):       # sequential coarse sweep
            w_new = G(new[i - 1])        # G(lambda_{i-1}^{k+1})
            new[i] = correction(v[i], w_new, w[i])
            w[i] = w_new
        delta = float(np.max(np.abs(new - lam)))
        lam = new
        k += 1
        deltas.append(delta)
        if hist is not None:
            hist.append(lam.copy())
        if eps > 0 and delta < eps:
            break
    return SyncResult(lam, k, deltas, hist)


class AsyncReplay:
    """Deterministic replay of asynchronous Parareal (Algorithm 2).

    Per slice i = 1..N the state is
      versions[i] -- every iterate slice i has published; version 0 is the
                     coarse guess lambda_i^0, version j its j-th local update
      f_ver[i]    -- predecessor version its next F starts from (the version
                     its last G used; initially 0, the coarse guess)
      w_old[i]    -- G(versions[i-1][f_ver[i]])
      k[i]        -- local iteration count k_i
    ``step(i, j)`` performs one local iteration of slice i whose coarse solve
    reads predecessor version j (j >= f_ver[i], j <= newest): this is one
    element of P^(k) with delay tau = j.  Slice 0 is u0, whose only version is 0.
    """

    def __init__(self, u0: np.ndarray, F: Callable, G: Callable, nslices: int):
        self.F, self.G, self.N = F, G, nslices
        lam0 = coarse_sweep(u0, G, nslices)
        self.versions: List[List[np.ndarray]] = [[lam0[i]] for i in range(nslices + 1)]
        self.f_ver = [0] * (nslices + 1)
        self.w_old = [lam0[i].copy() for i in range(nslices + 1)]
        self.k = [0] * (nslices + 1)
        self.delta = [np.inf] * (nslices + 1)     # change made by the last update
        self.g_ver = [-1] * (nslices + 1)         # predecessor version the last G read
        self.last_f_ver = [-1] * (nslices + 1)    # predecessor version the last F read
        self.final_from = [0] + [-1] * nslices    # first version known to equal lambda*
        # drift[i][v] = sum of the changes of versions 1..v of slice i: by the
        # triangle inequality it bounds ||versions[i][v'] - versions[i][v]||_inf
        # by drift[i][v'] - drift[i][v]
        self.drift: List[List[float]] = [[0.0] for _ in range(nslices + 1)]
        self.events: List[Tuple[int, int]] = []

    def newest(self, i: int) -> int:
        return len(self.versions[i]) - 1

    def step(self, i: int, j: int) -> None:
        if not 1 <= i <= self.N:
            raise ValueError("slice index out of range")
        if not self.f_ver[i] <= j <= self.newest(i - 1):
            raise ValueError(f"slice {i}: version {j} not in [{self.f_ver[i]}, {self.newest(i - 1)}]")
        x_old = self.versions[i - 1][self.f_ver[i]]
        x_new = self.versions[i - 1][j]
        v = self.F(x_old)                          # v_i^{k_i} = F(lambda_{i-1}^{k_i})
        w_new = self.G(x_new)                      # w_i^{k_i+1} = G(lambda_{i-1}^{k_i+1})
        lam_new = correction(v, w_new, self.w_old[i])
        self.delta[i] = float(np.max(np.abs(lam_new - self.versions[i][-1])))
        self.drift[i].append(self.drift[i][-1] + self.delta[i])
        self.last_f_ver[i] = self.f_ver[i]
        self.g_ver[i] = j
        self.versions[i].append(lam_new)           # "send lambda_i^{k_i+1} to i+1"
        self.f_ver[i] = j
        self.w_old[i] = w_new
        self.k[i] += 1
        # finite-termination bookkeeping (Proposition on nested sets, Section 3.2):
        # both inputs equal to the predecessor's final value make this slice final.
        ff = self.final_from[i - 1]
        if self.final_from[i] < 0 and ff >= 0 and self.last_f_ver[i] >= ff and j >= ff:
            self.final_from[i] = self.newest(i)
        self.events.append((i, j))

    def reset(self, i: int) -> None:
        """Slice i loses its local state (a restarted processor): its next
        update starts again from the initial guess, F from the predecessor's
        coarse guess lambda_{i-1}^0 and w_old = G(lambda_{i-1}^0) = lambda_i^0,
        as at the start of Algorithm 2.  Its published versions and k_i stay.
        The finite-termination bookkeeping of this slice restarts: it is final
        again only after an update whose both inputs are final (Section 3.2)."""
        if not 1 <= i <= self.N:
            raise ValueError("slice index out of range")
        self.f_ver[i] = 0
        self.w_old[i] = self.versions[i][0].copy()
        self.last_f_ver[i] = -1
        # its next versions are not final, nor those of any successor that
        # reads them: the final marks downstream are re-established later
        for j in range(i, self.N + 1):
            self.final_from[j] = -1

    def current(self) -> np.ndarray:
        return np.stack([self.versions[i][-1] for i in range(self.N + 1)])

    def staleness(self, i: int) -> float:
        """Upper bound on ||newest predecessor - predecessor read by slice i's
        last coarse solve||_inf (0 for slice 1, whose predecessor is u0)."""
        d = self.drift[i - 1]
        return d[-1] - d[self.g_ver[i]] if self.g_ver[i] >= 0 else np.inf

    def converged_tol(self, eps: float) -> bool:
        """Tolerance stop, the asynchronous reading of eq. (thresh): every slice
        has updated at least once, its last update changed it by less than eps
        in the max norm, and the predecessor it last read has since moved by
        less than eps (bounded through the recorded changes)."""
        for i in range(1, self.N + 1):
            if self.k[i] == 0 or self.delta[i] >= eps or self.staleness(i) >= eps:
                return False
        return True

    def converged_exact(self) -> bool:
        """Exact stop: the finite-termination cascade has reached slice N."""
        return self.final_from[self.N] >= 0

    @property
    def kappa(self) -> int:
        """kappa = max_i k_i (Section 4.1)."""
        return max(self.k[1:])


def sync_schedule(nslices: int, iters: int) -> List[Tuple[int, int]]:
    """The synchronous iteration written as an asynchronous schedule: at sweep
    k every slice updates once, in order, reading predecessor version k
    (Section 2.1: synchronous iterations are the special case of full update
    sets and no delay)."""
    ev = []
    for k in range(1, iters + 1):
        for i in range(1, nslices + 1):
            ev.append((i, k if i > 1 else 0))
    return ev


def replay(u0, F, G, nslices, schedule: Iterable[Tuple[int, int]]) -> AsyncReplay:
    st = AsyncReplay(u0, F, G, nslices)
    for i, j in schedule:
        st.step(i, j)
    return st


def run_random(u0, F, G, nslices: int, seed: int, max_delay: int = 3,
               eps: float = 0.0, max_rounds: int = 10_000,
               exact: bool = False, resets=None) -> AsyncReplay:
    """Fair, bounded-delay random schedule (the two assumptions of Section 2.1).

    Rounds: each round updates every slice once in a random order (fairness),
    and each coarse solve reads a uniformly random version among the newest
    ``max_delay + 1`` that are allowed (bounded delay).  Stops by the tolerance
    rule (eps > 0) or the exact rule (exact=True), else after max_rounds.
    resets: {slice: k} resets that slice (AsyncReplay.reset) once, just
    before its update number k + 1."""
    rng = np.random.default_rng(seed)
    st = AsyncReplay(u0, F, G, nslices)
    pending = dict(resets or {})
    for _ in range(max_rounds):
        for i in rng.permutation(np.arange(1, nslices + 1)):
            i = int(i)
            if pending.get(i) == st.k[i]:
                st.reset(i)
                del pending[i]
            hi = st.newest(i - 1)
            lo = max(st.f_ver[i], hi - max_delay)
            j = int(rng.integers(lo, hi + 1))
            st.step(i, j)
        if exact and st.converged_exact():
            break
        if eps > 0 and st.converged_tol(eps):
            break
    return st
