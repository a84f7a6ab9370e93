"""Plain FP64 CPU oracle for the high-order Riesz-map solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the library: it is an independent, deliberately
slow and literal restatement of the paper's construction (Brubeck, Farrell,
Kirby, Parker, "Fast solvers for the high-order FEM simplicial de Rham
complex", arXiv:2506.17406):

* ``simplex``  -- reference simplices, quadrature, orthonormal polynomials;
* ``element``  -- the orthogonality-promoting dual bases (Sec. 3-4);
* ``mesh``     -- Freudenthal/Kuhn topology and entity-major dof numbering;
* ``operator`` -- cell matrices of the weak form (Sec. 2) and assembly;
* ``precond``  -- the interior-interface split Schwarz preconditioners
                  (Sec. 6, eq:approx-sc-pafw, eq:hcurl-decomp, eq:hdiv-decomp);
* ``pcg``      -- preconditioned conjugate gradients with a Lanczos condition
                  estimate (Sec. 7).

Every function cites the passage it follows.  Where the paper leaves a
choice open, the reading taken is stated at the point of use.
"""
