"""Plain FP64 CPU oracle for the flux reconstruction stochastic Galerkin (FR-SG) method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or run anything in this
package.  The product path (the HIP library and its Python binding) never
routes through it, and the oracle shares no code, tables or helpers with it.

It follows Xiao, Kusch, Koellermeier & Frank, "A flux reconstruction
stochastic Galerkin scheme for hyperbolic conservation laws" (arXiv
2112.05946):

* Sec. 2.1, Eq. (polynomial chaos) .. Eq. (sg conservation laws): gPC
  expansion, orthonormal basis, quadrature inner product, Galerkin projection;
* Sec. 3.1-3.5: flux reconstruction (Lagrange solution polynomial, discontinuous
  flux, Radau correction functions h_L/h_R, interactive flux, total-flux
  derivative, tensor-product multi-dimensional extension);
* Sec. 4 (Eq. modal solution, Eq. vandermonde matrix): nodal/modal transform;
* Sec. 4.1.1-4.1.2: exponential and L2 filters;
* Sec. 4.2 (Eq. detector): modal-decay discontinuity sensor;
* Sec. 4.1.3: Lasso filter with automatic strengths;
* Sec. 4.3 (Eq. schemefullDiscr): positivity-preserving slope limiter;
* Sec. 3.3 and Tables 5-6: Lax-Friedrichs and HLL interactive fluxes;
* Sec. 3.1 and 3.5 on triangles (``tri.py``): reference triangle, vector
  correction fields, unstructured meshes.

Time integration: the three-stage strong-stability-preserving Runge-Kutta
scheme of Shu and Osher, with the limiter after each stage and the
sensor-gated filter at the end of the step (the paper's forward-Euler ordering
"limit, update, filter", Eq. schemefullDiscr, applied stage-wise), or the
paper's RK4, Tsitouras 5(4) and Bogacki-Shampine 3(2) tableaux at the same
CFL step.

Everything is float64 NumPy.  Every function is pinned by tests that do not
restate it (closed forms, library routines, an independent discontinuous
Galerkin weak form, published stability limits, the paper's printed tables);
a function without such a pin would say "parity unpinned" in its docstring,
and none does.
"""

from .tables import Tables1D, RandomTables, build_tables  # noqa: F401
from .problem import Problem  # noqa: F401
from .fr import rhs  # noqa: F401
from .stabilize import limit, sensor_filter, sensor_flags  # noqa: F401
from .stepper import step, cfl_dt, solve  # noqa: F401
