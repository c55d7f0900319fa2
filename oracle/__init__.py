"""CPU FP64 oracle for the Krylov interior point method of Liu, Fredriksson and
Markidis, "Krylov Solvers for Interior Point Methods with Applications in
Radiation Therapy and Support Vector Machines" (arXiv 2308.00637).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or calls
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It is deliberately plain and slow: dense matrices, library Cholesky /
LU solves and unblocked NumPy expressions written in the paper's notation, so
that each function can be checked against the paper by eye.  It shares no code
with the HIP path (the seeded generators in `paper_2308_00637_amd.workloads`
are the only common inputs, and hold none of the method's arithmetic).
"""
from .ipm import (Problem, State, Residuals, from_spec, index_sets, initial_point,
                  residuals, stacked_norm, infeasibilities, reduced_system,
                  doubly_augmented, newton_rhs_doubly, jacobi_diagonal,
                  direction_from_solution, newton_direction, step_lengths,
                  take_step, solve, objective, kkt_matvec, IPMOptions, IPMResult,
                  NotSPDError)
from .pcg import pcg
from .fullsystem import full_newton_matrix, full_newton_direction
from .bruteforce import brute_force_qp
from .adjoint import adjoint_gradients, center
from .woodbury import woodbury_direction, schur_direction
from .mehrotra import solve_mpc, target_residuals, complementarity, pair_count
from .spectrum import (kkt_dense, jacobi_spectrum, condition_numbers, condest,
                       condest_path, onenorm_inverse_estimate)

__all__ = [n for n in dir() if not n.startswith("_")]
