"""FP64 CPU oracle for the boundary-integral water-wave solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
path: it is written directly from the paper's formulas in plain PyTorch CPU
operations in float64/complex128, builds every matrix block literally from
the kernel table of Sec. 3.2 (and the transposed "dagger" blocks of Sec.
4.1), applies spectral operators with the FFT, and solves by dense LU with
one step of iterative refinement (residual in extended precision) or, for
systems too large for that, by a plain restarted GMRES on the stored
matrix.  Gradients come from PyTorch autograd through these same plain
operations; directional derivatives from the tangent-linear model
(forward-mode derivatives of the assembly and of the U map around one
extra solve).
"""
from .bim import (OGeom, assemble_A, A_rows, rhs, solve_phi, solve_gamma, spectral, split,
                  K_block, G_block, A_block, wall_matrix, psi_on_surface,
                  psi_mv, u_mv, energy, surface_from_periodic, J_and_grad, dphi_dn_from_omega,
                  dphi_ds_from_omega, gamma_t_matrix, gamma_t_rhs, solve_gamma_t, F_operators,
                  surface_velocity_state, graph_surface, hls_reconstruct, hls_V, stage_rhs,
                  rk_step, boundary_dPhi, helsing_ojala, dphi_dn_all,
                  layer_potential_direct, boundary_Phi, pressure, spectral_tail,
                  assemble_A_blocked, gmres, dphi_dn_from_omega_chunked, A_times_blocked,
                  tangent_J, tangent_J_nodes, J_and_grad_nodes, dense_solve, residual_ext)

__all__ = ["OGeom", "assemble_A", "A_rows", "rhs", "solve_phi", "solve_gamma", "spectral", "split",
           "K_block", "G_block", "A_block", "wall_matrix", "psi_on_surface",
           "psi_mv", "u_mv", "energy", "surface_from_periodic", "J_and_grad",
           "dphi_dn_from_omega", "dphi_ds_from_omega",
           "gamma_t_matrix", "gamma_t_rhs", "solve_gamma_t", "F_operators", "surface_velocity_state",
           "graph_surface", "hls_reconstruct", "hls_V", "stage_rhs", "rk_step",
           "boundary_dPhi", "helsing_ojala", "dphi_dn_all",
           "layer_potential_direct", "boundary_Phi", "pressure", "spectral_tail",
           "assemble_A_blocked", "gmres", "dphi_dn_from_omega_chunked", "A_times_blocked",
           "tangent_J", "tangent_J_nodes", "J_and_grad_nodes", "dense_solve", "residual_ext"]
