"""Pins of the deformation-state oracle (oracle/bl_deform.py) against facts fixed by the paper's
definitions and by mathematics; the checks themselves live in deform_pin_checks.py so that the
mutation check can rerun them on planted-mistake copies.

Measured on the unmodified oracle: truncated convolution 1e-15 from its double sum; transposes
exact to 1e-15; the incremental state and the adjoint sweep are the exact derivative (2.5e-10
from central differences) and transpose (8e-16) of the discrete state map; in-band inverse map
within 8e-6 (2D) and 1.3e-5 (3D, non-cubic) of the exact inverse flow, relative to the largest
displacement; constant-velocity closed forms 1.5e-7 (g) and 1e-6 (H); zero-velocity closed forms 1e-15; Gauss-Newton symmetry 1e-16 (2D) and 1.5e-15
(3D) at realistic velocities; gradient 0.5% and Hessian 3% from finite differences (the image
level uses the interpolated central-difference gradient of I0 instead of the derivative of the
interpolant, reading R-D4)."""
import numpy as np
import pytest

import oracle as O
import oracle.bl_deform as D
import deform_pin_checks as P
from paper_1807_05117_amd import phantoms


def test_truncated_convolution_is_its_double_sum():
    assert P.check_star_bruteforce(D) < 1e-12


def test_transport_operators_are_mutual_transposes():
    assert P.check_transposes(D) < 1e-12


@pytest.mark.parametrize("dim,bound", [(2, 5e-5), (3, 1e-4)])
def test_in_band_map_is_the_exact_inverse_flow(dim, bound):
    assert P.check_inverse_flow(D, dim=dim) < bound


def test_in_band_map_converges_in_time():
    """fewer steps give a larger error, down to the band-truncation floor"""
    e5, e10 = P.check_inverse_flow(D, nt=5), P.check_inverse_flow(D, nt=10)
    assert e10 < e5


def test_state_map_linearisation_and_transpose_are_exact():
    """the incremental state is the derivative of the discrete state map (central differences,
    2.5e-10) and the adjoint sweep is exactly its negative transpose (8e-16)"""
    e_lin, e_fd, e_tr = P.check_state_map_derivatives(D)
    assert e_lin < 1e-7 and e_fd < 1e-7 and e_tr < 1e-12


def test_constant_velocity_closed_forms():
    exact, e_g, e_h = P.check_constant_velocity(D)
    assert exact < 1e-12
    assert e_g < 1e-5 and e_h < 1e-5


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_velocity_closed_forms(dim):
    e_g, e_h = P.check_zero_velocity(D, dim=dim)
    assert e_g < 1e-10 and e_h < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_gauss_newton_exactly_symmetric_and_above_regulariser(dim):
    defect, pos = P.check_symmetry(D, dim=dim)
    assert defect < 1e-12
    assert pos > 0.999


def test_gradient_matches_finite_differences():
    assert P.check_fd_gradient(D) < 0.02


def test_gauss_newton_matches_derivative_of_gradient_at_zero_residual():
    assert P.check_fd_hessian_zero_residual(D) < 0.06


def test_registration_recovers_known_warp():
    prob, I0, vs = P.blob_case()
    I1 = D.def_warp(I0, vs, prob)
    vh, m1, st = D.def_register(I0, I1, np.zeros_like(vs), prob, O.SolverOpts(max_gn=6))
    assert st["status"] in (O.CONVERGED, O.MAXITER)
    assert all(b <= a for a, b in zip(st["E"], st["E"][1:]))
    assert st["mse_rel"][-1] < 2.0


def test_incompressible_outputs_divergence_free_and_registration():
    prob = O.Problem(2, (32, 32), (12, 12), 6, alpha=5e-3, s=1, gamma=1)
    I0 = phantoms.blobs_2d(0, 32)
    vs = O.project(phantoms.raw_band_velocity(0, 2, prob.k), prob)
    vs *= 3.0 / O.max_displacement_voxels(vs, prob)
    assert np.abs(O.div_band(vs, prob)).max() < 1e-12
    I1 = D.def_warp(I0, vs, prob)
    st = D.def_evaluate(0.5 * vs, I0, I1, prob)
    g = D.def_gradient(st)
    H = D.def_hessvec(st, P.rand_adm(prob, 3))
    assert np.abs(O.div_band(g, prob)).max() < 1e-10 * np.abs(g).max() * prob.nref
    assert np.abs(O.div_band(H, prob)).max() < 1e-10 * np.abs(H).max() * prob.nref
    vh, m1, stats = D.def_register(I0, I1, np.zeros_like(vs), prob, O.SolverOpts(max_gn=6))
    assert stats["mse_rel"][-1] < 5.0
