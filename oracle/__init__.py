"""Plain fp64 CPU oracle of the biorthonormal CCSD derivative-coupling path.

TEST INFRASTRUCTURE ONLY: this package exists to check the GPU library.  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product path never calls it and shares no
code with it.

Modules:
* ``detspace`` - determinant-space second quantization (CC by definition, FCI);
* ``ccsd``     - closed-shell T1-transformed CCSD residual, energy, solver;
* ``response`` - Jacobians by automatic differentiation, EOM, multipliers,
                 densities, coupling (direct and density routes);
* ``fd``       - finite-difference couplings (unrelaxed and orbital-relaxed).
"""
