"""Independent float64 CPU oracle for the H-matrix MGWR path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package; the product library
(paper_1706_07632_amd) never does, and the two share no code.  The only shared
module is `workloads`, which generates the seeded inputs and holds none of the
method's arithmetic.

What it computes: the plain definition of the result of multigrid waveform
relaxation, namely the solution of the fully discrete system
(Rt (x) I + I (x) A_h) U = F + a_{.,1} g, obtained by marching in time with a
direct spatial solve (Rt lower triangular), where Rt is either the L1 matrix R
of Section 2 (k = None) or its H-matrix representation of Section 3.

oracle.mgwr (imported on its own) takes the steps of one cycle of Algorithm
2 (zebra-in-time line relaxation, defect, full weighting, coarse cycles,
linear interpolation), so that iterates after a fixed number of cycles can be
compared as well.

Pins (tests/test_oracle_*.py):
* R: invariants with closed forms (row sums, exactness on linear functions,
  the uniform-mesh L1 coefficients), the defining integral evaluated with
  mpmath quadrature at 30 digits;
* Rt: the entrywise bound in the proof of Theorem 3.1 and the 3^-k decay;
* time marching: dense Kronecker LU on tiny grids, single-sine-mode reduction
  (eigenvectors of the finite-difference Laplacian);
* the whole chain: the maximum errors printed in Table 1 and the graded-mesh
  convergence order for the manufactured solution;
* the cycle (oracle.mgwr): on two grids it reproduces the semi-algebraic mode
  analysis blocks of oracle.sama element by element (1D and 2D), the direct
  solution is its fixed point, cycles converge to it.
"""
from .l1 import steps, pow_diff, l1_weights, l1_matrix, initial_value_weights  # noqa: F401
from .hmatrix import (cluster_tree, admissible, block_partition, taylor_coeffs, rk_factors,  # noqa: F401
                      hmatrix_dense, theorem_bound)
from .direct import (laplacian_apply, laplacian_dense, laplacian_eigs, rhs, timestep_solve,  # noqa: F401
                     residual, residual_columns, residual_sampled, single_mode_profile, mode_eigenvalue, kron_solve,
                     solve_shifted_spatial)
from .special import mittag_leffler  # noqa: F401


def operator(t, alpha, k=None, leaf=16):
    """Rt: the dense L1 matrix (k None) or its rank-k H-matrix representation."""
    if k is None:
        return l1_matrix(t, alpha)
    return hmatrix_dense(t, alpha, k, leaf)


def solve(problem, k="problem", Rt=None):
    """Direct solution U [M][N] of the problem's discrete system."""
    kk = problem.k if k == "problem" else k
    if Rt is None:
        Rt = operator(problem.t, problem.alpha, kk, problem.leaf)
    B = rhs(problem.f, problem.t, problem.alpha, problem.g)
    return timestep_solve(Rt, B, problem.dim, problem.n, problem.length)
