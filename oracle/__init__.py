"""Plain FP64 CPU oracle of the THOR dynamical-core step (Mendonca et al. 2016).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under ``oracle/``; only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark do.  The oracle shares no code with the
HIP library: it is a slow, readable NumPy restatement of the paper's method
(section 2 grid and operators, section 3 time integration, section 4
dissipation, section 5 forcing), written so a reader can check each step
against the paper by eye.

Modules
  grid       icosahedral grid, spring dynamics, centroids, control-volume
             geometry (Sec. 2.1-2.2, Eqs. grid_qts, int_grid, spring_force,
             dbar, centroid equation)
  operators  finite-volume divergence, gradient and triangle-gradient
             Laplacian (Eqs. flx_div, div_gauss, grad; Sec. 4 Laplacian)
  dynamics   HEVI split-explicit large step, hyperdiffusion, divergence
             damping, Newtonian relaxation, diagnostics (Sec. 3-5)
  rng        SplitMix64 counter-based noise, from its published definition
  mlp        FP64 reference of the per-column corrector network
"""
