"""GPU: the transport launch shapes (64 x 4 x zv voxel tiles, zv chosen per grid shape by
timing) change only speed: gradient, H v and the registration are bitwise the same for every
shape, so the tuned choice cannot make a result depend on the run."""
import os

import numpy as np
import pytest

from paper_1807_05117_amd import binding as B

from parity_cases import bl_problem, case

pytestmark = pytest.mark.gpu


def _run(name, zv):
    prob, I0, I1, vs, vh, dv = case(name)
    old = os.environ.get("BL_TRANSPORT_ZV")
    if zv is None:
        os.environ.pop("BL_TRANSPORT_ZV", None)
    else:
        os.environ["BL_TRANSPORT_ZV"] = str(zv)
    try:
        ctx = B.Ctx(bl_problem(prob), I0, I1)
        E, g = ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64))
        H = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
        shapes = ctx.bl_lddmm_ctx_launch_shapes()
        ctx.close()
    finally:
        if old is None:
            os.environ.pop("BL_TRANSPORT_ZV", None)
        else:
            os.environ["BL_TRANSPORT_ZV"] = old
    return E, g, H, shapes


@pytest.mark.parametrize("name", ["ragged_3d", "c2_full"])
def test_every_launch_shape_gives_identical_results(gpu_lib, name):
    ref = _run(name, None)
    print(name, "tuned launch shapes", ref[3], flush=True)
    assert all(z in (1, 2, 4, 8) for z in ref[3])
    for zv in (1, 2, 4, 8):
        E, g, H, shapes = _run(name, zv)
        assert shapes == (zv,) * 4
        assert E == ref[0], zv
        assert np.array_equal(g, ref[1]), zv
        assert np.array_equal(H, ref[2]), zv
