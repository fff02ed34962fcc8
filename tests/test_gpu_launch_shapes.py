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


def _run_shapes(name, shapes, precision=B.BL_FP32):
    """gradient and H v with every launch-shape class fixed (BL_LAUNCH_SHAPES)"""
    prob, I0, I1, vs, vh, dv = case(name)
    os.environ["BL_LAUNCH_SHAPES"] = ",".join(str(v) for v in shapes)
    try:
        ctx = B.Ctx(bl_problem(prob, precision=precision), I0, I1)
        E, g = ctx.bl_lddmm_ctx_set_velocity(vh.astype(np.complex64))
        H = ctx.bl_lddmm_ctx_hessvec(dv.astype(np.complex64))
        ctx.close()
    finally:
        os.environ.pop("BL_LAUNCH_SHAPES", None)
    return E, g, H


# transports and setup (voxels per thread), iota z-chunk multiplier, fused iota x/y rows
SHAPES = [(2, 2, 2, 1, 1, 1, 0), (1, 4, 8, 2, 2, 2, 16), (8, 1, 4, 8, 4, 4, 16),
          (4, 8, 1, 4, 8, 1, 32)]


@pytest.mark.parametrize("name", ["ragged_3d", "brainlike_small"])
@pytest.mark.parametrize("precision", [B.BL_FP32, B.BL_MIXED])
def test_every_tuned_class_gives_identical_results(gpu_lib, name, precision):
    """every class of the autotuner (setup voxels per thread, the iota z stage's chunking, the
    fused iota x/y stage's rows per block, the transports) changes only speed"""
    ref = _run_shapes(name, SHAPES[0], precision)
    for shp in SHAPES[1:]:
        E, g, H = _run_shapes(name, shp, precision)
        assert E == ref[0], shp
        assert np.array_equal(g, ref[1]), shp
        assert np.array_equal(H, ref[2]), shp


def test_tuned_shapes_persist_in_the_cache_file(gpu_lib, tmp_path):
    """the autotuner appends its choice for a new problem shape to the cache file; after the
    process forgets its choices (bl_lddmm_tune_reload) a new context takes them from the file
    without timing (no second line) and uses the same shapes"""
    import oracle as O
    from paper_1807_05117_amd import phantoms

    cache = tmp_path / "shapes.txt"
    old = os.environ.get("BL_TUNE_CACHE")
    os.environ["BL_TUNE_CACHE"] = str(cache)
    for k in ("BL_TRANSPORT_ZV", "BL_LAUNCH_SHAPES"):
        os.environ.pop(k, None)
    try:
        prob = O.Problem(3, (36, 20, 12), (8, 8, 6), 4)   # a shape no other test uses
        I0 = phantoms.shells_3d(5, prob.n).astype(np.float32)
        vh = (0.1 * O.project(phantoms.raw_band_velocity(5, 3, prob.k), prob)).astype(np.complex64)

        def shapes():
            ctx = B.Ctx(bl_problem(prob), I0, I0)
            ctx.bl_lddmm_ctx_set_velocity(vh)
            out = ctx.bl_lddmm_ctx_launch_shapes()
            ctx.close()
            return out

        first = shapes()
        lines = cache.read_text().splitlines()
        assert len(lines) == 1, lines
        key, vals = lines[0].split(":")
        assert key.split()[1:8] == ["3", "36", "20", "12", "8", "8", "6"]
        assert [int(v) for v in vals.split()][:4] == list(first)
        B.load().bl_lddmm_tune_reload()
        assert shapes() == first
        assert len(cache.read_text().splitlines()) == 1
    finally:
        if old is None:
            os.environ.pop("BL_TUNE_CACHE", None)
        else:
            os.environ["BL_TUNE_CACHE"] = old
        B.load().bl_lddmm_tune_reload()


def test_cache_file_lines_are_validated(gpu_lib, tmp_path):
    """a cache line with a value no class accepts is skipped (the shape is tuned again and a
    valid line appended); a valid line is used as written, without timing"""
    import oracle as O
    from paper_1807_05117_amd import phantoms

    cache = tmp_path / "shapes.txt"
    old = os.environ.get("BL_TUNE_CACHE")
    os.environ["BL_TUNE_CACHE"] = str(cache)
    for k in ("BL_TRANSPORT_ZV", "BL_LAUNCH_SHAPES"):
        os.environ.pop(k, None)
    try:
        bad = O.Problem(3, (36, 20, 14), (8, 8, 6), 4)    # shapes no other test uses
        good = O.Problem(3, (36, 20, 16), (8, 8, 6), 4)
        arch = None

        def run(prob):
            I0 = phantoms.shells_3d(5, prob.n).astype(np.float32)
            vh = (0.1 * O.project(phantoms.raw_band_velocity(5, 3, prob.k), prob)).astype(np.complex64)
            ctx = B.Ctx(bl_problem(prob), I0, I0)
            ctx.bl_lddmm_ctx_set_velocity(vh)
            out = ctx.bl_lddmm_ctx_launch_shapes()
            ctx.close()
            return out

        # learn the key format (architecture name) from a first tuning of the bad shape
        run(bad)
        arch = cache.read_text().split()[0]
        cache.write_text(f"{arch} 3 36 20 14 8 8 6 0 : 3 2 2 2 1 1 0\n"
                         f"{arch} 3 36 20 16 8 8 6 0 : 1 4 1 8 2 1 0\n")
        B.load().bl_lddmm_tune_reload()
        got_bad = run(bad)
        assert all(v in (1, 2, 4, 8) for v in got_bad), got_bad
        lines = cache.read_text().splitlines()
        assert len(lines) == 3, lines                      # re-tuned: one valid line appended
        assert lines[2].startswith(f"{arch} 3 36 20 14 ")
        assert run(good) == (1, 4, 1, 8)                   # taken from the file as written
        assert len(cache.read_text().splitlines()) == 3    # no timing, nothing appended
    finally:
        if old is None:
            os.environ.pop("BL_TUNE_CACHE", None)
        else:
            os.environ["BL_TUNE_CACHE"] = old
        B.load().bl_lddmm_tune_reload()
