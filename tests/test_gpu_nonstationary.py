"""GPU parity of the non-stationary velocity (BL_NONSTATIONARY): one band field per time node,
per-step offsets from both ends of a step, gradients and Gauss-Newton products per node,
against the oracle's ns_* functions (relative 1e-5 plain, 1e-4 mixed, in the 2-norm and per
node and component element by element), the stationary limit,
and a 2D registration with the oracle's solver decisions."""
import functools

import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B
from paper_1807_05117_amd import phantoms

from parity_cases import bl_problem, case, check_hessvec, check_mse_rel, rel2

pytestmark = pytest.mark.gpu

CASES = ["c1_2d", "ragged_3d", "brainlike_small"]


@functools.lru_cache(maxsize=None)
def ns_case(name):
    """the case's images; a velocity that varies over the nodes, a direction per node"""
    prob, I0, I1, vs, vh, dv = case(name)
    nodes = prob.nt + 1
    V = np.stack([vh * (1.0 + 0.3 * np.sin(n)) for n in range(nodes)])
    V = V.astype(np.complex64).astype(np.complex128)
    D = np.stack([O.project(phantoms.random_band_direction(100 + n, prob.dim, prob.k), prob)
                  for n in range(nodes)])
    D = (D / np.abs(D).max()).astype(np.complex64).astype(np.complex128)
    st = O.ns_evaluate(V, I0, I1, prob)
    return prob, I0, I1, V, D, st, O.ns_gradient(st), O.ns_hessvec(st, D)


def _grad_err(g, gref, prob, V):
    Lv = O.L_hat(prob)[None, None] * O.ns_project(V, prob)
    den = np.linalg.norm(Lv.ravel()) + np.linalg.norm((gref - Lv).ravel())
    return float(np.linalg.norm((np.asarray(g) - gref).ravel()) / den)


def _grad_elem_err(g, gref, prob, V):
    """worst (node, component) of max |dg| / (max |L v| + max |pi(b)|)"""
    Lv = O.L_hat(prob)[None, None] * O.ns_project(V, prob)
    G, R, L = (np.asarray(a).reshape(a.shape[0] * a.shape[1], -1) for a in (g, gref, Lv))
    return float(max(np.abs(G[i] - R[i]).max() / (np.abs(L[i]).max() + np.abs(R[i] - L[i]).max())
                     for i in range(R.shape[0])))


@pytest.mark.parametrize("precision,tol", [(B.BL_FP32, 1e-5), (B.BL_MIXED, 1e-4)],
                         ids=["fp32", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_ns_gradient_and_hessvec(gpu_lib, name, precision, tol):
    prob, I0, I1, V, D, st, gref, href = ns_case(name)
    ctx = B.Ctx(bl_problem(prob, precision=precision, nonstationary=True), I0, I1)
    E, g = ctx.bl_lddmm_ctx_set_velocity(V.astype(np.complex64))
    H = ctx.bl_lddmm_ctx_hessvec(D.astype(np.complex64))
    ctx.close()
    eg, ee = _grad_err(g, gref, prob, V), _grad_elem_err(g, gref, prob, V)
    print(f"non-stationary {name}: gradient rel err 2-norm {eg:.2e}, element-wise {ee:.2e}",
          flush=True)
    assert eg < tol and ee < tol
    check_hessvec(H, href, tol, f"non-stationary {name}", lead=2)
    assert abs(E - st.E) <= tol * st.E


def test_ns_stationary_limit(gpu_lib):
    """equal nodes: the trapezoid-weighted sums of the per-node gradient and product are the
    stationary ones (same kernels up to the per-node body force and transforms)"""
    prob, I0, I1, vs, vh, dv = case("ragged_3d")
    nodes = prob.nt + 1
    w = O.trapezoid_weights(prob.nt)
    ctx = B.Ctx(bl_problem(prob, nonstationary=True), I0, I1)
    En, gn = ctx.bl_lddmm_ctx_set_velocity(np.stack([vh] * nodes).astype(np.complex64))
    Hn = ctx.bl_lddmm_ctx_hessvec(np.stack([dv] * nodes).astype(np.complex64))
    ctx.close()
    ctx = B.Ctx(bl_problem(prob), I0, I1)
    Es, gs = ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64))
    Hs = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
    ctx.close()
    assert abs(En - Es) <= 1e-6 * Es
    assert rel2(sum(w[n] * gn[n].astype(np.complex128) for n in range(nodes)), gs) < 1e-5
    assert rel2(sum(w[n] * Hn[n].astype(np.complex128) for n in range(nodes)), Hs) < 1e-5


def test_ns_register_2d_against_oracle(gpu_lib):
    prob, I0, I1, vs, vh, dv = case("c1_2d")
    V0 = np.zeros((prob.nt + 1,) + vh.shape, np.complex64)
    v_ref, m_ref, st_ref = O.ns_register(I0, I1, V0, prob, O.SolverOpts(max_gn=4))
    v_gpu, m_gpu, st = B.bl_lddmm_register(bl_problem(prob, nonstationary=True), I0, I1, V0,
                                           B.opts_struct(max_gn=4))
    print("non-stationary gpu", st["pcg_iters"], st["mse_rel"][-1], " oracle",
          st_ref["pcg_iters"], st_ref["mse_rel"][-1], flush=True)
    assert st["status"] == st_ref["status"]
    assert st["pcg_iters"] == st_ref["pcg_iters"]
    assert st["ls_trials"] == st_ref["ls_trials"]
    assert np.allclose(st["E"], st_ref["E"], rtol=1e-4, atol=0)
    check_mse_rel(st, st_ref, 1e-5, "non-stationary c1_2d")
    assert rel2(v_gpu, v_ref) < 1e-3
