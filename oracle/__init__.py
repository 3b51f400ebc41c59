"""CPU oracle for the matrix-free BCSR Hamiltonian (test infrastructure only).

This package is a plain, slow, obviously correct float64 implementation of
what the GPU library computes, written from the paper (Davydov & Kronbichler,
"Algorithms and data structures for matrix-free finite element operators with
MPI-parallel sparse multi-vectors", arXiv 1907.01005).  It is test
infrastructure: only the test-suite, the smoke entry point and the CPU
baseline leg of the benchmark may import it.  The GPU library never calls it
and shares no code with it.

Modules
-------
fe1d     1D Lagrange basis on Gauss-Lobatto nodes, Gauss quadrature (Sec. 3.1)
element  explicit element matrices H_K = K_K + M_K[V] (eq. fe_matrices)
mesh     box mesh numbering, quadrature points, Dirichlet nodes
hilbert  Hilbert space-filling-curve index (Alg. 1 step 2, Alg. 2 step 3)
pattern  batch order, row blocks, column order and blocks, BCSR pattern
         (Alg. 1, Alg. 2, Sec. 4 support construction)
apply    Y = mask(H X) cell by cell (eq. fe_matrices_cell_based, Alg. 6),
         S = X^T Y (Alg. 8), trace; dense assembly for pins
"""
