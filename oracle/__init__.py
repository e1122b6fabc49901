"""FP64 CPU oracle for the fast spectral Boltzmann collision operator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or link
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it. It shares no code, tables or constants with the HIP library.

Contents (each function cites the passage of the paper it follows):
  spectral  -- O1: the fast spectral operator Q_h of section 3.3 (FFT based)
  direct    -- O2: the same Q_h as the direct mode sum of eq. (ode)
  brute     -- O3: the same Q_h by real-space quadrature of the trigonometric
               interpolant (Carleman form, eq. (defQBCarleman))
  sigma     -- O4: modelling check, the sigma/omega form of eq. (Boltzmann)
  bkw       -- the BKW closed form of section 4.1 and its time derivative
  stepping  -- explicit Euler and penalised IMEX steps (section 3.4)
  galerkin  -- the dealiased (non-wrapping) variant of Q_h, 3/2 rule and
               literal mode sum (section 3.3)
  transport -- CWENO reconstruction and Rusanov fluxes on polygonal meshes
               (section 2.2)
  classical -- the classical O(N^4) method: direct double sum with exact
               kernel modes (section 3.3)

Pin status of every function is listed in the module docstrings; a function
with no independent pin says "parity unpinned" there.
"""

from .spectral import (  # noqa: F401
    Setup,
    default_radius,
    default_coupling,
    mode_indices,
    active_mask,
    forward_dft,
    inverse_dft,
    phi_segment,
    phi_weighted_segment,
    psi_disc,
    hs2d_radial_expansion,
    directions,
    filter_bank,
    loss_multiplier,
    q_fast,
    moment_matrix,
    moments,
    project_conservative,
)
