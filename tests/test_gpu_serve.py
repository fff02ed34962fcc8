"""GPU tests of the serving loop: results are the same alone and in the mix, admission
respects the device-memory budget, cancellation and oversize rejection."""
import time

import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B
from paper_1807_05117_amd import phantoms

pytestmark = pytest.mark.gpu

# (grid, band, nt, precision, seed): a mix of grid sizes, band sizes, time steps, precisions
MIX = [((32, 32, 32), (8, 8, 8), 5, B.BL_FP32, 1),
       ((40, 48, 40), (10, 12, 10), 4, B.BL_MIXED, 2),
       ((24, 24, 24), (8, 8, 8), 6, B.BL_FP32, 3),
       ((48, 32, 40), (12, 8, 10), 5, B.BL_MIXED, 4),
       ((32, 32, 32), (8, 8, 8), 5, B.BL_MIXED, 5),
       ((40, 48, 40), (10, 12, 10), 4, B.BL_FP32, 6)]


def make_pair(grid, band, nt, seed, disp=2.0):
    prob = O.Problem(3, grid, band, nt)
    I0 = phantoms.shells_3d(seed, grid).astype(np.float32)
    vs = O.project(phantoms.raw_band_velocity(seed, 3, band), prob)
    vs *= disp / O.max_displacement_voxels(vs, prob)
    I1 = O.warp(I0.astype(np.float64), vs, prob).astype(np.float32)
    return I0, I1


@pytest.fixture(scope="module")
def pairs():
    return [make_pair(g, k, nt, sd) for g, k, nt, _, sd in MIX]


def _problem(i):
    g, k, nt, prec, _ = MIX[i]
    return B.make_problem(3, g, k, nt, precision=prec)


def test_results_identical_alone_and_in_mix(gpu_lib, pairs):
    opts = B.opts_struct(max_gn=4, max_pcg=5)
    alone = []
    for i, (I0, I1) in enumerate(pairs):
        p = _problem(i)
        v0 = np.zeros(B.band_shape(p), np.complex64)
        alone.append(B.bl_lddmm_register(p, I0, I1, v0, opts))
    srv = B.Server(max_slots=4)
    tickets = [srv.submit(_problem(i), I0, I1, opts=opts) for i, (I0, I1) in enumerate(pairs)]
    for i, t in enumerate(tickets):
        rc, v, w, st, times = srv.wait(t)
        assert rc == B.BL_OK
        va, wa, sa = alone[i]
        # same kernels, launch shapes and reduction orders: identical up to nothing
        assert np.array_equal(v, va), i
        assert np.array_equal(w, wa), i
        assert st["pcg_iters"] == sa["pcg_iters"] and st["E"] == sa["E"]
        assert times["submitted"] <= times["admitted"] <= times["finished"]
    info = srv.info()
    print("server info", info, flush=True)
    assert info["completed"] == len(pairs) and info["peak_resident"] >= 2
    srv.close()


# every model variant of the library in one serving mix: (grid, band, nt, make_problem options)
VARIANTS = [((32, 32, 32), (8, 8, 8), 5, dict(deformation=True)),
            ((40, 48, 40), (10, 12, 10), 4, dict(nonstationary=True)),
            ((32, 32, 32), (8, 8, 8), 5, dict(newton=True)),
            ((40, 48, 40), (10, 12, 10), 4, dict(gamma=1, s=1, alpha=5e-3)),
            ((32, 32, 32), (8, 8, 8), 5, dict(deformation=True, precision=B.BL_MIXED)),
            ((24, 24, 24), (8, 8, 8), 6, dict())]


def test_model_variants_identical_alone_and_in_mix(gpu_lib):
    """deformation, non-stationary, Newton, incompressible and plain problems served together:
    each result is bitwise the one bl_lddmm_register gives alone"""
    opts = B.opts_struct(max_gn=3, max_pcg=4)
    probs, data, alone = [], [], []
    for i, (g, k, nt, kw) in enumerate(VARIANTS):
        p = B.make_problem(3, g, k, nt, **kw)
        I0, I1 = make_pair(g, k, nt, 10 + i)
        v0 = np.zeros(B.band_shape(p), np.complex64)
        probs.append(p)
        data.append((I0, I1))
        alone.append(B.bl_lddmm_register(p, I0, I1, v0, opts))
    srv = B.Server(max_slots=3)
    tickets = [srv.submit(p, I0, I1, opts=opts) for p, (I0, I1) in zip(probs, data)]
    for i, t in enumerate(tickets):
        rc, v, w, st, times = srv.wait(t)
        assert rc == B.BL_OK, i
        va, wa, sa = alone[i]
        assert np.array_equal(v, va), VARIANTS[i]
        assert np.array_equal(w, wa), VARIANTS[i]
        assert st["pcg_iters"] == sa["pcg_iters"] and st["E"] == sa["E"], VARIANTS[i]
    assert srv.info()["completed"] == len(VARIANTS)
    srv.close()


def test_served_pair_matches_oracle(gpu_lib, pairs):
    """a 3D pair registered by the serving loop (in a mix with the other pairs) against the
    FP64 oracle's registration: solver decisions, energies, MSE_rel, final v~ and m(1)"""
    g, k, nt, prec, _ = MIX[0]
    prob = O.Problem(3, g, k, nt)
    I0, I1 = pairs[0]
    opts = B.opts_struct(max_gn=4, max_pcg=5)
    srv = B.Server(max_slots=3)
    tickets = [srv.submit(_problem(i), *pairs[i], opts=opts) for i in range(3)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    rc, v, w, st, _ = res[0]
    assert rc == B.BL_OK
    v_ref, m_ref, st_ref = O.register(I0.astype(np.float64), I1.astype(np.float64),
                                      np.zeros((3,) + prob.bshape, complex), prob,
                                      O.SolverOpts(max_gn=4, max_pcg=5))
    print("served", st["pcg_iters"], st["ls_trials"], " oracle", st_ref["pcg_iters"],
          st_ref["ls_trials"], flush=True)
    assert st["status"] == st_ref["status"]
    assert st["pcg_iters"] == st_ref["pcg_iters"]
    assert st["ls_trials"] == st_ref["ls_trials"]
    assert np.allclose(st["E"], st_ref["E"], rtol=1e-5, atol=0)
    assert np.allclose(st["mse_rel"], st_ref["mse_rel"], rtol=1e-5, atol=0)
    assert np.linalg.norm((v - v_ref).ravel()) < 1e-3 * np.linalg.norm(v_ref.ravel())
    assert np.abs(w - m_ref).max() < 1e-4 * np.abs(m_ref).max()


def test_budget_limits_resident_pairs(gpu_lib, pairs):
    p0 = _problem(0)
    fp = B.bl_lddmm_footprint(p0)
    srv = B.Server(budget_bytes=int(2.5 * fp), max_slots=6)
    tickets = [srv.submit(p0, *pairs[0], opts=B.opts_struct(max_gn=2, max_pcg=3)) for _ in range(6)]
    for t in tickets:
        assert srv.wait(t)[0] == B.BL_OK
    info = srv.info()
    assert info["peak_resident"] <= 2 and info["peak_bytes"] <= int(2.5 * fp)
    srv.close()


def test_oversize_rejected_and_cancel(gpu_lib, pairs):
    p1 = _problem(1)
    srv = B.Server(budget_bytes=B.bl_lddmm_footprint(p1) - 1, max_slots=1)
    with pytest.raises(B.BLError) as e:
        srv.submit(p1, *pairs[1])
    assert e.value.code == B.BL_E_NOMEM
    srv.close()
    srv = B.Server(max_slots=1)
    p0 = _problem(0)
    ts = [srv.submit(p0, *pairs[0], opts=B.opts_struct(max_gn=3, max_pcg=5)) for _ in range(4)]
    assert srv.cancel(ts[-1]) == B.BL_OK
    assert srv.wait(ts[-1])[0] == B.BL_E_CANCELLED
    for t in ts[:-1]:
        assert srv.wait(t)[0] == B.BL_OK
    assert srv.info()["cancelled"] == 1
    srv.close()


def test_wait_timeout_returns_pending(gpu_lib, pairs):
    srv = B.Server(max_slots=1)
    p0 = _problem(0)
    ts = [srv.submit(p0, *pairs[0]) for _ in range(3)]
    rc = srv.wait(ts[-1], timeout=0.0)[0]
    assert rc in (B.BL_PENDING, B.BL_OK)
    for t in ts:
        if rc == B.BL_OK and t == ts[-1]:
            continue
        assert srv.wait(t)[0] == B.BL_OK
    srv.close()
