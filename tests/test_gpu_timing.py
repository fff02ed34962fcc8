"""GPU: per-kernel timing (bl_kernel_timing_*).  Every timed launch records an event pair at its
own dispatch's start and end; the counts per class follow the operation sequence, the times
are positive and the results do not depend on whether timing is on."""
import numpy as np
import pytest

from paper_1807_05117_amd import binding as B

from parity_cases import bl_problem, case

pytestmark = pytest.mark.gpu

# classes: 0 state step, 1 incremental step, 2 adjoint step, 3 iota z stage of a product,
# 4 pi z stage of a product, 5 body force, 6 setup


@pytest.mark.parametrize("name", ["ragged_3d", "c1_2d"])
def test_timed_counts_and_results(gpu_lib, name):
    prob, I0, I1, vs, vh, dv = case(name)
    nt = prob.nt
    vh = vh.astype(np.complex64)
    dv = dv.astype(np.complex64)

    ctx = B.Ctx(bl_problem(prob), I0, I1)
    E_ref, g_ref = ctx.bl_lddmm_ctx_set_velocity(vh)
    H_ref = ctx.bl_lddmm_ctx_hessvec(dv)

    ctx.bl_kernel_timing_enable(True)
    E, g = ctx.bl_lddmm_ctx_set_velocity(vh)   # one evaluation and one gradient
    H = [ctx.bl_lddmm_ctx_hessvec(dv) for _ in range(3)]
    got = {k: ctx.bl_kernel_timing_read(k) for k in range(7)}
    ctx.bl_kernel_timing_enable(False)
    again = {k: ctx.bl_kernel_timing_read(k) for k in range(7)}   # read resets
    ctx.close()
    print(name, got, flush=True)

    assert E == E_ref and np.array_equal(g, g_ref)
    for h in H:
        assert np.array_equal(h, H_ref)
    # the adjoint sweeps stop at lambda^1 (the body force forms lambda^0): nt - 1 steps each
    want = {0: nt, 1: 3 * (nt - 1), 2: 4 * (nt - 1), 3: 3, 4: 3, 5: 1 + 3, 6: 1}
    for k, n in want.items():
        launches, ms = got[k]
        assert launches == n, (k, launches, n)
        assert ms > 0.0, k
        assert again[k] == (0, 0.0), k


def test_timing_class_out_of_range(gpu_lib):
    prob, I0, I1, vs, vh, dv = case("c1_2d")
    ctx = B.Ctx(bl_problem(prob), I0, I1)
    with pytest.raises(Exception):
        ctx.bl_kernel_timing_read(7)
    ctx.close()
