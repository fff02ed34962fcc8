"""GPU: the one-shot calls reuse an idle cached context of the same problem; results are
bitwise those of a fresh context, device-pointer registrations equal host-pointer ones, and
releasing the cache leaves later calls working."""
import numpy as np
import pytest

from paper_1807_05117_amd import binding as B

from parity_cases import bl_problem, case

pytestmark = pytest.mark.gpu


def test_repeated_and_interleaved_calls_are_identical(gpu_lib):
    B.bl_lddmm_release_cached()
    pa, I0a, I1a, _, vha, dva = case("ragged_3d")
    pb, I0b, I1b, _, vhb, dvb = case("brainlike_small")
    first_a = B.bl_lddmm_hessvec(bl_problem(pa), I0a, I1a, vha, dva)   # fresh context
    first_b = B.bl_lddmm_gradient(bl_problem(pb), I0b, I1b, vhb)
    for _ in range(2):                                                # cached contexts
        assert np.array_equal(B.bl_lddmm_hessvec(bl_problem(pa), I0a, I1a, vha, dva), first_a)
        g, E = B.bl_lddmm_gradient(bl_problem(pb), I0b, I1b, vhb)
        assert np.array_equal(g, first_b[0]) and E == first_b[1]
    B.bl_lddmm_release_cached()
    assert np.array_equal(B.bl_lddmm_hessvec(bl_problem(pa), I0a, I1a, vha, dva), first_a)


def test_device_pointer_registration_matches_host(gpu_lib):
    import torch

    prob, I0, I1, vs, vh, dv = case("brainlike_small")
    opts = B.opts_struct(max_gn=3, max_pcg=5)
    v0 = np.zeros_like(vh, dtype=np.complex64)
    vh_host, w_host, st_host = B.bl_lddmm_register(bl_problem(prob), I0, I1, v0, opts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p = bl_problem(prob, device=True, stream=stream.cuda_stream)
        dI0 = torch.from_numpy(I0.astype(np.float32)).cuda()
        dI1 = torch.from_numpy(I1.astype(np.float32)).cuda()
        for _ in range(2):   # second call runs on the cached context
            v = torch.zeros(v0.shape, dtype=torch.complex64, device="cuda")
            w = torch.empty_like(dI0)
            st = B.bl_lddmm_register_device(p, dI0, dI1, v, w, opts)
            stream.synchronize()
            assert np.array_equal(v.cpu().numpy(), vh_host)
            assert np.array_equal(w.cpu().numpy(), w_host)
            assert st["pcg_iters"] == st_host["pcg_iters"] and st["E"] == st_host["E"]
