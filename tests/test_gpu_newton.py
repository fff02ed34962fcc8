"""GPU parity of the full Newton Hessian-vector product (BL_NEWTON): the incremental adjoint
with its source div(lambda dv) and the product with pi(lambda grad dm), against the oracle's
hessvec_newton (relative 1e-5 plain, 1e-4 mixed); exact symmetry on permutation transports
(to FP32 rounding); equality with the Gauss-Newton product at zero residual; a Newton
registration with the oracle's solver decisions."""
import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B
from paper_1807_05117_amd import phantoms

from parity_cases import bl_problem, case, check_hessvec, check_mse_rel, oracle_hessvec_newton, rel2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [(B.BL_FP32, 1e-5), (B.BL_MIXED, 1e-4)],
                         ids=["fp32", "mixed"])
@pytest.mark.parametrize("name", ["c1_2d", "ragged_3d", "brainlike_small", "c2_full"])
def test_newton_hessvec_parity(gpu_lib, name, precision, tol):
    prob, I0, I1, vs, vh, dv = case(name)
    # a product without a gradient first (the adjoint is formed inside) ...
    ctx = B.Ctx(bl_problem(prob, precision=precision, newton=True), I0, I1)
    ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64), want_gradient=False)
    H1 = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
    # ... and after one (the gradient's adjoint is reused): the same product
    ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64))
    H2 = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
    ctx.close()
    check_hessvec(H1, oracle_hessvec_newton(name), tol, f"newton {name}")
    assert np.array_equal(H1, H2)


@pytest.mark.parametrize("dim", [2, 3])
def test_newton_symmetric_on_permutation_transports(gpu_lib, dim):
    nt = 8
    n = (32,) * dim if dim == 2 else (32, 16, 16)
    prob = O.Problem(dim, n, (8,) * dim, nt, sigma=0.8)
    vh = np.zeros((dim,) + prob.bshape, np.complex64)
    centre = tuple(K // 2 for K in prob.bshape)
    for j in range(dim):
        vh[(j,) + centre] = (1, -1, 1)[j] * nt / prob.nref
    I0 = (phantoms.blobs_2d(3, 32) if dim == 2 else phantoms.shells_3d(3, n)).astype(np.float32)
    I1 = (np.roll(I0, 2, axis=0) + 0.1).astype(np.float32)
    ctx = B.Ctx(bl_problem(prob, newton=True), I0, I1)
    ctx.bl_lddmm_ctx_set_velocity(vh, want_gradient=False)
    d1 = O.project(phantoms.random_band_direction(7, dim, prob.k), prob).astype(np.complex64)
    d2 = O.project(phantoms.random_band_direction(8, dim, prob.k), prob).astype(np.complex64)
    H1 = ctx.bl_lddmm_ctx_hessvec(d1).astype(np.complex128)
    H2 = ctx.bl_lddmm_ctx_hessvec(d2).astype(np.complex128)
    ctx.close()
    a, b = O.dot(H1, d2), O.dot(d1, H2)
    print(f"newton symmetry defect {abs(a - b) / (abs(a) + abs(b)):.1e}", flush=True)
    assert abs(a - b) <= 1e-5 * (abs(a) + abs(b))


def test_newton_equals_gauss_newton_at_zero_residual(gpu_lib):
    prob, I0, I1, vs, vh, dv = case("ragged_3d")
    I1z = O.warp(I0, vh, prob).astype(np.float32)
    HN = B.bl_lddmm_hessvec(bl_problem(prob, newton=True), I0, I1z, vh, dv)
    HG = B.bl_lddmm_hessvec(bl_problem(prob), I0, I1z, vh, dv)
    # lambda is the FP32 residual of the state, not exactly 0: agreement to FP32 level
    assert rel2(HN, HG) < 1e-4


def test_newton_register_c1_against_oracle(gpu_lib):
    prob, I0, I1, vs, vh, dv = case("c1_2d")
    v0 = np.zeros_like(vh)
    v_ref, m_ref, st_ref = O.register(I0, I1, v0, prob, O.SolverOpts(max_gn=5, newton=True))
    v_gpu, m_gpu, st = B.bl_lddmm_register(bl_problem(prob, newton=True), I0, I1,
                                           v0.astype(np.complex64), B.opts_struct(max_gn=5))
    print("newton gpu", st["pcg_iters"], st["ls_trials"], st["mse_rel"][-1], " oracle",
          st_ref["pcg_iters"], st_ref["ls_trials"], st_ref["mse_rel"][-1], flush=True)
    assert st["status"] == st_ref["status"]
    assert st["pcg_iters"] == st_ref["pcg_iters"]
    assert st["ls_trials"] == st_ref["ls_trials"]
    assert np.allclose(st["E"], st_ref["E"], rtol=1e-4, atol=0)
    check_mse_rel(st, st_ref, 1e-5, "newton c1_2d")
