"""GPU parity on the degenerate cases of the method, against the FP64 oracle on the same seeded
float32 inputs: one time step, the full band k = n, the smallest band k = 2, and the smallest
grids the library accepts (see parity_cases.CASES).  Same bar as the other parity tests: the
transforms within 2e-6, gradient and H v within relative 1e-5 in the 2-norm and element by
element, the energy within 1e-5, and a full registration with the oracle's solver decisions
reproduced exactly."""
import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import binding as B

from parity_cases import (bl_problem, case, check_gradient, check_hessvec, check_mse_rel,
                          oracle_gradient, oracle_hessvec, oracle_state, rel2)

pytestmark = pytest.mark.gpu

EDGE = ["nt1_3d", "fullband_2d", "fullband_3d", "minband_3d", "tiny_3d", "min_grid_2d"]


def _log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("name", EDGE)
def test_edge_band_to_grid_and_back(gpu_lib, name):
    """iota and pi at the degenerate band sizes, element by element against the oracle (same
    bound as the other transform tests), and pi's output exactly Hermitian with zero unpaired
    planes"""
    prob, I0, I1, vs, vh, dv = case(name)
    p = bl_problem(prob)
    _log("case", name, "band_to_grid / grid_to_band")
    grid = B.bl_band_to_grid(p, vh)
    for c in range(prob.dim):
        ref = O.iota(O.project(vh[c], prob), prob)
        assert np.abs(grid[c] - ref).max() <= 2e-6 * np.abs(ref).max(), c
    f = np.stack([I0, I1]).astype(np.float32)
    band = B.bl_grid_to_band(p, f)
    for c in range(2):
        ref = O.pi_(f[c].astype(np.float64), prob)
        assert rel2(band[c], ref) < 2e-6
        assert np.array_equal(O.project(band[c].astype(np.complex128), prob),
                              band[c].astype(np.complex128))


@pytest.mark.parametrize("name", EDGE)
def test_edge_gradient_and_energy(gpu_lib, name):
    prob, I0, I1, vs, vh, dv = case(name)
    _log("case", name, "gradient")
    g, E = B.bl_lddmm_gradient(bl_problem(prob), I0, I1, vh)
    check_gradient(g, oracle_gradient(name), prob, vh, 1e-5, name)
    assert abs(E - oracle_state(name).E) <= 1e-5 * oracle_state(name).E


@pytest.mark.parametrize("name", EDGE)
def test_edge_hessvec(gpu_lib, name):
    prob, I0, I1, vs, vh, dv = case(name)
    _log("case", name, "hessvec")
    H = B.bl_lddmm_hessvec(bl_problem(prob), I0, I1, vh, dv)
    check_hessvec(H, oracle_hessvec(name), 1e-5, name)


@pytest.mark.parametrize("name", EDGE)
def test_edge_register(gpu_lib, name):
    prob, I0, I1, vs, vh, dv = case(name)
    v0 = np.zeros_like(vh)
    _log("case", name, "register")
    v_ref, m_ref, st_ref = O.register(I0, I1, v0, prob, O.SolverOpts())
    v_gpu, m_gpu, st = B.bl_lddmm_register(bl_problem(prob), I0, I1, v0.astype(np.complex64))
    _log("  gpu", st["status"], st["pcg_iters"], st["ls_trials"], " oracle", st_ref["status"],
         st_ref["pcg_iters"], st_ref["ls_trials"])
    assert st["status"] == st_ref["status"]
    assert st["pcg_iters"] == st_ref["pcg_iters"]
    assert st["ls_trials"] == st_ref["ls_trials"]
    assert np.allclose(st["E"], st_ref["E"], rtol=1e-4, atol=0)
    check_mse_rel(st, st_ref, 1e-5, name)
    assert rel2(v_gpu, v_ref) < 1e-3
    assert np.abs(m_gpu - m_ref).max() < 1e-3 * np.abs(m_ref).max()


def test_edge_largest_grid_over_device_memory(gpu_lib):
    """the largest grid the library accepts (2048 x 2048 x 255 voxels, just under 2^30) with
    Nt = 256 needs far more device memory than one GPU has: the call fails with BL_E_NOMEM
    before any device work (the inputs are never read), and the next call works as before"""
    prob = O.Problem(3, (2048, 2048, 255), (8, 8, 8), 256)
    p = bl_problem(prob)
    assert B.bl_lddmm_footprint(p) > 300 * 2 ** 30
    I0 = np.zeros(prob.shape, np.float32)   # untouched pages: no host memory is used
    vh = np.zeros((3,) + prob.bshape, np.complex64)
    with pytest.raises(B.BLError) as e:
        B.bl_lddmm_gradient(p, I0, I0, vh)
    assert e.value.code == B.BL_E_NOMEM, e.value
    del I0
    name = "tiny_3d"
    prob, I0, I1, vs, vh, dv = case(name)
    g, E = B.bl_lddmm_gradient(bl_problem(prob), I0, I1, vh)
    check_gradient(g, oracle_gradient(name), prob, vh, 1e-5, name)
