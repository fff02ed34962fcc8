"""GPU parity of the incompressible flow model (gamma = 1, here with the H^1 regulariser
s = 1): velocities are projected divergence-free, and gradients and Hessian products are the
divergence-free parts of the gamma = 0 expressions.  Same tolerances as the plain path
(relative 1e-5, in the 2-norm and element by element); the outputs' spectral divergence and
the unit reaction factor are checked directly."""
import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B

from parity_cases import (bl_problem, case, check_gradient, check_hessvec, check_mse_rel,
                          oracle_gradient, oracle_hessvec, oracle_state, rel2)

pytestmark = pytest.mark.gpu

CASES = ["h1_incomp_3d", "h1_incomp_2d"]


def _div_rel(vh, prob):
    return float(np.abs(O.div_band(vh.astype(np.complex128), prob)).max()
                 / (np.abs(vh).max() * 2 * np.pi * max(prob.k)))


@pytest.mark.parametrize("precision,tol", [(B.BL_FP32, 1e-5), (B.BL_MIXED, 1e-4)],
                         ids=["fp32", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_incompressible_gradient_and_hessvec(gpu_lib, name, precision, tol):
    prob, I0, I1, vs, vh, dv = case(name)
    ctx = B.Ctx(bl_problem(prob, precision=precision), I0, I1)
    E, g = ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64))
    H = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
    a = ctx.bl_lddmm_ctx_get_field("a", 0)
    ctx.close()
    print(f"{name}: div g {_div_rel(g, prob):.1e}, div Hv {_div_rel(H, prob):.1e}, "
          f"max|a-1| {np.abs(a - 1).max():.1e}", flush=True)
    check_gradient(g, oracle_gradient(name), prob, vh, tol, name)
    check_hessvec(H, oracle_hessvec(name), tol, name)
    assert abs(E - oracle_state(name).E) <= tol * oracle_state(name).E
    assert _div_rel(g, prob) < 1e-6 and _div_rel(H, prob) < 1e-6
    assert np.abs(a - 1).max() < 1e-5


def test_incompressible_register_2d_against_oracle(gpu_lib):
    prob, I0, I1, vs, vh, dv = case("h1_incomp_2d")
    v0 = np.zeros_like(vh)
    opts = O.SolverOpts(max_gn=6)
    v_ref, m_ref, st_ref = O.register(I0, I1, v0, prob, opts)
    v_gpu, m_gpu, st = B.bl_lddmm_register(bl_problem(prob), I0, I1, v0.astype(np.complex64),
                                           B.opts_struct(max_gn=6))
    print("gpu", st["pcg_iters"], st["mse_rel"][-1], " oracle", st_ref["pcg_iters"],
          st_ref["mse_rel"][-1], flush=True)
    assert st["status"] == st_ref["status"]
    assert st["pcg_iters"] == st_ref["pcg_iters"]
    assert st["ls_trials"] == st_ref["ls_trials"]
    assert np.allclose(st["E"], st_ref["E"], rtol=1e-4, atol=0)
    check_mse_rel(st, st_ref, 1e-5, "h1_incomp_2d")
    assert rel2(v_gpu, v_ref) < 1e-3
    assert _div_rel(v_gpu, prob) < 1e-6


@pytest.mark.parametrize("name", CASES)
def test_incompressible_full_newton_product(gpu_lib, name):
    """gamma = 1 with the full Newton product (BL_NEWTON): the oracle's Newton product,
    divergence-free output"""
    prob, I0, I1, vs, vh, dv = case(name)
    ctx = B.Ctx(bl_problem(prob, newton=True), I0, I1)
    ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64))
    H = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
    ctx.close()
    check_hessvec(H, O.hessvec_newton(oracle_state(name), dv), 1e-5, f"newton {name}")
    assert _div_rel(H, prob) < 1e-6


@pytest.mark.parametrize("name", CASES)
def test_incompressible_nonstationary(gpu_lib, name):
    """gamma = 1 with a non-stationary velocity (BL_NONSTATIONARY): per-node gradient and
    product against the oracle's, every node's outputs divergence-free"""
    from paper_1807_05117_amd import phantoms

    prob, I0, I1, vs, vh, dv = case(name)
    nodes = prob.nt + 1
    V = np.stack([vh * (1.0 + 0.3 * np.sin(n)) for n in range(nodes)])
    V = V.astype(np.complex64).astype(np.complex128)
    D = np.stack([O.project(phantoms.random_band_direction(100 + n, prob.dim, prob.k), prob)
                  for n in range(nodes)])
    D = (D / np.abs(D).max()).astype(np.complex64).astype(np.complex128)
    st = O.ns_evaluate(V, I0, I1, prob)
    gref, href = O.ns_gradient(st), O.ns_hessvec(st, D)
    ctx = B.Ctx(bl_problem(prob, nonstationary=True), I0, I1)
    E, g = ctx.bl_lddmm_ctx_set_velocity(V.astype(np.complex64))
    H = ctx.bl_lddmm_ctx_hessvec(D.astype(np.complex64))
    ctx.close()
    assert abs(E - st.E) <= 1e-5 * st.E
    # gradient error per (node, component) relative to max |L v| + max |pi(b)|, the two parts
    # normalised separately as in the stationary gradient checks
    Lv = O.L_hat(prob)[None, None] * O.ns_project(V, prob)
    G, R, L = (np.asarray(a).reshape(a.shape[0] * a.shape[1], -1) for a in (g, gref, Lv))
    eg = max(np.abs(G[i] - R[i]).max() / (np.abs(L[i]).max() + np.abs(R[i] - L[i]).max())
             for i in range(R.shape[0]))
    print(f"non-stationary {name}: gradient element-wise {eg:.2e}", flush=True)
    assert eg < 1e-5
    check_hessvec(H, href, 1e-5, f"non-stationary {name}", lead=2)
    for n in range(nodes):
        assert _div_rel(g[n], prob) < 1e-6 and _div_rel(H[n], prob) < 1e-6, n
