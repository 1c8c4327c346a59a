"""Plain FP64 CPU oracle for the SIPG hp-DG elliptic operator and its multigrid solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its Python
binding) imports, links or calls this package; only the tests, the smoke check and
the CPU-baseline leg of the benchmark do.  It shares no code with the GPU path;
both read the same neutral problem descriptions from ``meshgen``.

The oracle writes the method out from its definitions in the paper
(arXiv:1907.01572), in FP64 numpy, without blocking or fusion:

* ``rules``     LGL / GL nodes and weights, Lagrange matrices (Sec. II.A.3, II.A.5)
* ``geometry``  macro maps and element maps, Jacobians (Sec. II.A.1, II.A.5, Sec. III.C)
* ``mesh``      mortar decomposition of the fine mesh and multigrid mesh hierarchy
                (Sec. II.A.1, II.D.3)
* ``operator``  SIPG bilinear form applied matrix-free by quadrature, a brute-force
                assembled form, the right-hand side, penalty, norms
                (Eqs. lh2, Fh2, stiffness/harald-stiff, temp-E, penaltyparameter, norms)
* ``solvers``   prolongation/restriction, Chebyshev smoother, CG spectral bound,
                V-cycle, flexible CG, PCG (Algs. 2-5, Eqs. psi-interpolation, temp-G)
* ``problems``  manufactured solutions and coefficients named by ``meshgen`` descriptors

Functions without an independent pin say "parity unpinned" in their docstring.
"""
