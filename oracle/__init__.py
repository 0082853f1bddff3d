"""Plain, slow FP64 CPU oracle of the windowed regularized LBM-LES step and
its discrete adjoint.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) may import, call or execute this package; only the tests, the
smoke entry point and the CPU-baseline leg of the benchmark use it. It shares
no code with the GPU path: no kernels, headers, helpers or constant tables.

Every function follows the paper ("Adaptive Time Windows for Discrete Adjoint
Topology Optimization of Unsteady Flows") equation by equation, vectorised
over lattice nodes with numpy and generic in the scalar type, so the same code
runs with complex128 inputs for complex-step differentiation.

Modules
-------
lattice   D2Q9 (Sec. 2.1.1) and D3Q19 velocity sets.
forward   equilibrium, moments, LES closure, regularized collision, partial
          bounce-back, streaming, wall / Zou-He boundaries, objective samples,
          consecutive-window driver (Sec. 2, Sec. 3.1, Algorithm "LES solver").
adjoint   adjoint boundary rules, adjoint streaming, explicit per-node
          collision Jacobian, sensitivity and the reverse sweep over the
          representative window (Sec. 3.2).
design    density filter, Heaviside projection, volume fraction, their
          chain-rule transposes and a projected-gradient design update
          (Sec. "Topology optimization procedure", Algorithm "Optimization
          iteration"; the update stands in for MMA).

Parity status: every function is pinned by the CPU tests under tests/
(lattice identities, conservation, closed-form Poiseuille and Taylor-Green
flows, transposes of the boundary rules, complex-step derivatives). The
paper's printed optimisation results need the outer design loop and are not
used ("parity unpinned" for those, which this package does not compute).
"""

from . import lattice, forward, adjoint, design  # noqa: F401
