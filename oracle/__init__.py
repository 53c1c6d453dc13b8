"""Plain FP64 CPU oracle for the Chebyshev-filtered subspace iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python
binding imports, calls or links this package; only the tests, the smoke
check and the CPU-baseline leg of the benchmark use it.  It is slow on
purpose: every function is the plain definition of what the method computes
(assembled sparse matrices, library direct solves, the dense generalized
eigendecomposition) or the method's steps in the paper's order and notation.

Modules
-------
operators  global H^E, M^E assembled from the element blocks; H X, M X,
           M^-1 X by a sparse direct solve, and the block-wise inverse of
           Sec. IV.D written out as stated.
filters    Chebyshev polynomials, the three-term recurrence filter and the
           exact filter through the generalized eigendecomposition (Sec. V).
subspace   Cholesky-QR, Rayleigh-Ritz, Lanczos spectrum bounds, one
           subspace-iteration step and the error metrics (Sec. V).
cellwise   the same H^E X, M^E X and block-wise (M^E)^-1 summed cell by cell
           from the element blocks (torch CPU, all host threads), for
           problems whose global matrices do not fit: the fixed point of the
           30-atom workload and the CPU baseline.
mlp        the learned-bounds network: FP64 forward, backpropagated
           mean-squared-error gradient, Adam.
assembly   the classical element block of a plain cell as the quadrature
           sum over its Gauss points (Eq. HBlocks).
enriched   the element blocks of a cell with the adaptive rule (Sec. IV.C):
           Lagrange basis, smooth cutoff, Slater-type radials and real
           harmonics evaluated point by point (Eq. HBlocks, MBlocks).
scf        the self-consistent field quantities (Sec. II, V): Fermi level,
           density, LDA, the Hartree Poisson problem, Anderson mixing.

Parity pins: see the `-m "not gpu"` tests under tests/ (closed forms,
textbook limits, library routines, brute force on tiny meshes).
"""
