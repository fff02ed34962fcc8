"""GPU test of the allocation-free product bl_lddmm_hessvec_noalloc: through the C interface,
two calls in a row (the second on a smaller problem, so the shared scratch array holds the
first call's contents), each bitwise equal to bl_lddmm_hessvec on the same inputs and within
the plain path's tolerance of the FP64 oracle; host pointers, mixed precision, and device
pointers on a caller's stream."""
import numpy as np
import pytest

from paper_1807_05117_amd import binding as B
from parity_cases import bl_problem, case, oracle_hessvec, rel2

pytestmark = pytest.mark.gpu

# larger first, then smaller: brain-shaped 40x48x40 (Nt = 6), then ragged 72x21x13 (Nt = 5)
ORDER = ["brainlike_small", "ragged_3d"]


@pytest.mark.parametrize("precision", [B.BL_FP32, B.BL_MIXED])
def test_noalloc_matches_hessvec_two_calls(gpu_lib, precision):
    for name in ORDER:
        prob, I0, I1, vs, vh, dv = case(name)
        p = bl_problem(prob, precision=precision)
        ref = B.bl_lddmm_hessvec(p, I0, I1, vh, dv)
        got = B.bl_lddmm_hessvec_noalloc(p, I0, I1, vh, dv)
        err = rel2(got, oracle_hessvec(name))
        print(f"{name} precision {precision}: noalloc vs oracle {err:.2e}", flush=True)
        assert np.array_equal(got, ref), name
        assert err < (1e-5 if precision == B.BL_FP32 else 1e-4), name


def test_noalloc_device_pointers_on_a_stream(gpu_lib):
    import torch

    for name in ORDER:
        prob, I0, I1, vs, vh, dv = case(name)
        ref = B.bl_lddmm_hessvec(bl_problem(prob), I0, I1, vh, dv)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            p = bl_problem(prob, device=True, stream=stream.cuda_stream)
            dI0 = torch.from_numpy(I0.astype(np.float32)).cuda()
            dI1 = torch.from_numpy(I1.astype(np.float32)).cuda()
            dvh = torch.from_numpy(vh.astype(np.complex64)).cuda()
            ddv = torch.from_numpy(dv.astype(np.complex64)).cuda()
            out = torch.empty_like(ddv)
            stream.synchronize()
            rc = B.load().bl_lddmm_hessvec_noalloc(
                B.C.byref(p), B._tptr(dI0), B._tptr(dI1), B._tptr(dvh), B._tptr(ddv),
                B._tptr(out))
            assert rc == B.BL_OK, B.load().bl_lddmm_last_error()
            got = out.cpu().numpy()
        assert np.array_equal(got, ref), name


def test_noalloc_limit_reported(gpu_lib):
    assert B.bl_lddmm_noalloc_limit() == 512 << 20
    prob, I0, I1, vs, vh, dv = case("ragged_3d")
    big = B.make_problem(3, (256, 256, 256), (64, 64, 64), 20)
    with pytest.raises(B.BLError) as e:
        B.bl_lddmm_hessvec_noalloc(big, np.zeros((256,) * 3, np.float32),
                                   np.zeros((256,) * 3, np.float32),
                                   np.zeros(B.band_shape(big), np.complex64),
                                   np.zeros(B.band_shape(big), np.complex64))
    assert e.value.code == B.BL_E_NOMEM
    # the scratch array still serves a problem that fits, after the refusal
    ref = B.bl_lddmm_hessvec(bl_problem(prob), I0, I1, vh, dv)
    assert np.array_equal(B.bl_lddmm_hessvec_noalloc(bl_problem(prob), I0, I1, vh, dv), ref)
