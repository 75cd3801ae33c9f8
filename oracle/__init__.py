"""Plain FP64 CPU oracle of the MGM solve phase (test infrastructure only).

This package is the checker, not the product. Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the HIP
library never calls into it and shares no code with it (the two take the same
seeded inputs from the separate `synth` module and nothing else).

Every function follows the paper (Wright, Jones & Shankar, "MGM: A meshfree
geometric multilevel method for systems arising from elliptic equations on
point cloud surfaces", arXiv 2204.06154) in its order and notation, written
for readability rather than speed:

  knn          -- stencil selection (Sec. 2, nearest neighbours in R^3)
  discretize   -- tangent-plane projection, RBF-FD and GFD Laplace-Beltrami
                  weights, assembly of D_h and L_h (Sec. 2.1-2.3,
                  eqs. tp_pts, rbf_fd_lap, wls_fd_lap, discrete_system)
  coarsen      -- weighted sample elimination and the level count
                  (Sec. 4.1, Alg. 2)
  transfer     -- PHS interpolation I_H^h and restriction (Sec. 3,
                  eq. rbf_fd_interp)
  galerkin     -- Galerkin coarse operators, bordered variant (Sec. 4.2,
                  eq. galerkin; Sec. 4.4, eq. gco_saddle_point)
  colouring    -- multicolour ordering that replaces RCM for the smoother
  hierarchy    -- the preprocessing phase (Alg. 2) and the coarse LU
  smoother     -- Gauss-Seidel (Sec. 4.3, eq. smoother; Sec. 4.4 Uzawa form)
  vcycle       -- the V(nu1,nu2)-cycle (Alg. 3) incl. the bordered system
  krylov       -- right-preconditioned FGMRES and BiCGSTAB (Sec. 4.6)
  precision    -- FP32 / FP16-with-row-scale emulation of the V-cycle
"""
