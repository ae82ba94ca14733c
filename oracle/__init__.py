"""FP64 CPU oracle for Parareal / asynchronous Parareal on the heat equation.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct NumPy code that the
tests, the smoke check and the benchmark's CPU-baseline leg compare the HIP
library against.  The library never imports, links or calls anything here, and
nothing here imports the library.

Modules
  heat      -- grid derivation, explicit-Euler fine propagator F, backward-Euler
               coarse propagator G (Thomas, textbook CG, dense), serial fine run
  parareal  -- synchronous Parareal (eq. (pr)), asynchronous Parareal replay
               (eq. (apr), Algorithm 2) and its termination tests
  spectral  -- exact sine-mode closed forms used to pin the above and to check
               full-size GPU results at sampled outputs
  adjoint   -- gradients of L = 1/2 ||u(T) - u_target||^2 (closed form and a
               plain reverse sweep)

Every function states the passage of the paper (or the reading of it) that it
follows.  Points where the paper is silent use these readings:
  * grid: h = 1/(n+1), interior nodes only, zero ghost values;
  * fine step count m = max(1, ceil(dT/dt_nominal - 1e-9)), dt = dT/m, so the
    step never exceeds the requested one;
  * the correction is evaluated as F(x_old) + (G(x_new) - G(x_old)), so an
    unchanged coarse input leaves exactly F(x_old) (Section 4.2's remark on
    stale inputs) and Parareal after N iterations equals the serial fine run
    bit for bit;
  * stopping test (eq. (thresh)): absolute, strict '<', max over all slices and
    nodes; iteration k = N always stops (finite termination, Section 3.2).
"""
from . import heat, parareal, spectral, adjoint  # noqa: F401
