"""GPU tests of the cohort server (bl_server_create_batched): pairs of equal problems advanced
together by one launch per kernel and one graph replay per Newton step.  Every served result
must be bitwise the one bl_lddmm_register gives alone (velocity, warped image and every
statistic), whatever the companions, the slot, the admission order or the budget; the cohort
budget must hold; unsupported models are refused; a served 3D pair meets the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B
from paper_1807_05117_amd import phantoms

pytestmark = pytest.mark.gpu

# (dim, grid, band, nt, precision, seed, opts): several pairs per problem, so cohorts hold
# more than one pair; one request with a strict Armijo constant and few halvings, so trials
# are rejected (retries across steps) and the line search may stall
MIX = [(3, (32, 32, 32), (8, 8, 8), 5, B.BL_FP32, 1, dict(max_gn=4, max_pcg=5)),
       (3, (32, 32, 32), (8, 8, 8), 5, B.BL_FP32, 2, dict(max_gn=4, max_pcg=5)),
       (3, (40, 48, 40), (10, 12, 10), 4, B.BL_MIXED, 3, dict(max_gn=3, max_pcg=6)),
       (3, (32, 32, 32), (8, 8, 8), 5, B.BL_FP32, 4, dict(max_gn=5, max_pcg=3)),
       (3, (40, 48, 40), (10, 12, 10), 4, B.BL_MIXED, 5, dict(max_gn=3, max_pcg=6)),
       (2, (64, 64, 1), (16, 16, 1), 10, B.BL_FP32, 6, dict(max_gn=6, max_pcg=10)),
       (3, (32, 32, 32), (8, 8, 8), 5, B.BL_FP32, 7, dict(max_gn=4, max_pcg=5, c1=0.9,
                                                          max_halvings=1)),
       (2, (64, 64, 1), (16, 16, 1), 10, B.BL_FP32, 8, dict(max_gn=6, max_pcg=10)),
       (3, (24, 24, 24), (8, 8, 8), 6, B.BL_FP32, 9, dict(max_gn=3, max_pcg=4))]


def make_pair(dim, grid, band, nt, seed, disp=2.0):
    if dim == 2:
        prob = O.Problem(2, grid[:2], band[:2], nt)
        I0 = phantoms.blobs_2d(seed, grid[0]).astype(np.float32)
        vs = O.project(phantoms.raw_band_velocity(seed, 2, band[:2]), prob)
    else:
        prob = O.Problem(3, grid, band, nt)
        I0 = phantoms.shells_3d(seed, grid).astype(np.float32)
        vs = O.project(phantoms.raw_band_velocity(seed, 3, band), prob)
    vs *= disp / O.max_displacement_voxels(vs, prob)
    I1 = O.warp(I0.astype(np.float64), vs, prob).astype(np.float32)
    return I0, I1


def problem(i):
    dim, g, k, nt, prec, _, _ = MIX[i]
    if dim == 2:
        return B.make_problem(2, g[:2], k[:2], nt, precision=prec)
    return B.make_problem(3, g, k, nt, precision=prec)


def opts(i):
    return B.opts_struct(**MIX[i][6])


@pytest.fixture(scope="module")
def pairs():
    return [make_pair(d, g, k, nt, sd) for d, g, k, nt, _, sd, _ in MIX]


@pytest.fixture(scope="module")
def alone(gpu_lib, pairs):
    out = []
    for i, (I0, I1) in enumerate(pairs):
        p = problem(i)
        out.append(B.bl_lddmm_register(p, I0, I1, np.zeros(B.band_shape(p), np.complex64),
                                       opts(i)))
    return out


STAT_KEYS = ("status", "gn_iters", "hessvecs", "gradients", "evaluations", "pcg_total", "E",
             "mse_rel", "ginf_rel", "pcg_iters", "ls_trials", "eps")


def assert_same(i, got, ref):
    rc, v, w, st, times = got
    va, wa, sa = ref
    assert rc == B.BL_OK, (i, rc)
    assert np.array_equal(v, va), i
    assert np.array_equal(w, wa), i
    for k in STAT_KEYS:
        assert st[k] == sa[k], (i, k, st[k], sa[k])


def serve(order, pairs, **kw):
    srv = B.Server(batched=True, **kw)
    tickets = {i: srv.submit(problem(i), *pairs[i], opts=opts(i)) for i in order}
    res = {i: srv.wait(t) for i, t in tickets.items()}
    info = srv.info()
    srv.close()
    return res, info


def test_batched_results_identical_alone_and_in_mix(pairs, alone):
    res, info = serve(range(len(MIX)), pairs, max_slots=4)
    print("cohort server info", info, flush=True)
    for i in range(len(MIX)):
        assert_same(i, res[i], alone[i])
    assert info["completed"] == len(MIX)
    assert info["peak_resident"] >= 4   # several pairs resident at once
    # a stalled line search is among the cases only if the strict request stalls alone too
    print("strict-Armijo request:", alone[6][2]["status"], alone[6][2]["ls_trials"], flush=True)


def test_batched_independent_of_order_and_slots(pairs, alone):
    """reversed submission order, two pairs per cohort: other companions, other slots"""
    res, _ = serve(list(reversed(range(len(MIX)))), pairs, max_slots=2)
    for i in range(len(MIX)):
        assert_same(i, res[i], alone[i])


def test_batched_budget_with_mixed_sizes(pairs, alone):
    """a budget below the mix's total: cohorts are sized to it, freed when empty and another
    problem needs the memory, and the memory held never exceeds the budget"""
    fps = sorted({B.bl_lddmm_footprint(problem(i)) for i in range(len(MIX))})
    budget = int(2.2 * fps[-1])
    res, info = serve(range(len(MIX)), pairs, max_slots=4, budget_bytes=budget)
    print("budget", budget, "info", info, flush=True)
    assert info["peak_bytes"] <= budget
    assert info["completed"] == len(MIX)
    for i in range(len(MIX)):
        assert_same(i, res[i], alone[i])


def test_threads_budget_with_mixed_sizes(pairs, alone):
    """the slot-thread server charges every slot's arena while the slot holds it: with mixed
    sizes the memory held stays within the budget"""
    fps = [B.bl_lddmm_footprint(problem(i)) for i in range(len(MIX))]
    budget = int(1.6 * max(fps))
    srv = B.Server(max_slots=4, budget_bytes=budget)
    tickets = [srv.submit(problem(i), *pairs[i], opts=opts(i)) for i in range(len(MIX))]
    got = [srv.wait(t) for t in tickets]
    info = srv.info()
    srv.close()
    print("budget", budget, "info", info, flush=True)
    assert info["peak_bytes"] <= budget
    for i in range(len(MIX)):
        assert_same(i, got[i], alone[i])


def test_batched_refuses_other_models(pairs):
    srv = B.Server(batched=True, max_slots=2)
    p = B.make_problem(3, (32, 32, 32), (8, 8, 8), 5, newton=True)
    t = srv.submit(p, *pairs[0], opts=opts(0))
    assert srv.wait(t)[0] == B.BL_E_UNSUPPORTED
    t = srv.submit(problem(0), *pairs[0], opts=opts(0))
    assert srv.wait(t)[0] == B.BL_OK
    srv.close()


def test_batched_served_pair_matches_oracle(pairs, alone):
    """the first 3D pair, served in a cohort with two companions, against the FP64 oracle's
    registration: solver decisions, energies, MSE_rel, final v~ and m(1)"""
    dim, g, k, nt, _, _, o = MIX[0]
    res, _ = serve([0, 1, 3], pairs, max_slots=3)
    rc, v, w, st, _ = res[0]
    assert rc == B.BL_OK
    prob = O.Problem(3, g, k, nt)
    I0, I1 = pairs[0]
    v_ref, m_ref, st_ref = O.register(I0.astype(np.float64), I1.astype(np.float64),
                                      np.zeros((3,) + prob.bshape, complex), prob,
                                      O.SolverOpts(max_gn=o["max_gn"], max_pcg=o["max_pcg"]))
    print("served", st["pcg_iters"], st["ls_trials"], " oracle", st_ref["pcg_iters"],
          st_ref["ls_trials"], flush=True)
    assert st["status"] == st_ref["status"]
    assert st["pcg_iters"] == st_ref["pcg_iters"]
    assert st["ls_trials"] == st_ref["ls_trials"]
    assert np.allclose(st["E"], st_ref["E"], rtol=1e-5, atol=0)
    assert np.allclose(st["mse_rel"], st_ref["mse_rel"], rtol=1e-5, atol=0)
    assert np.linalg.norm((v - v_ref).ravel()) < 1e-3 * np.linalg.norm(v_ref.ravel())
    assert np.abs(w - m_ref).max() < 1e-4 * np.abs(m_ref).max()
