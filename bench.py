"""Benchmark of band-limited PDE-LDDMM (state equation, Gauss-Newton-Krylov) on one MI355X.

Workload: a synthetic 128^3 brain-like phantom (3 nested ellipsoidal tissue shells,
intensities 0.2/0.5/0.8, Gaussian smoothing sigma = 1 voxel, N(0, 0.01^2) noise), target =
the phantom warped by a random band-limited velocity (band 32^3, coefficients
N(0,1)/(1 + |k|^2), 6 voxels maximal displacement), band 32^3, Nt = 10, alpha = 1e-3,
s = 2, sigma = 1.  One step = one full registration (10 Gauss-Newton iterations with at
most 10 PCG steps each), which runs every stage of the path: band<->grid transforms,
departure-point setup, forward state, energy, adjoint and body force, incremental state,
incremental adjoint, regulariser, PCG and line search.

Printed: one JSON line with registrations/min as the value, plus Gauss-Newton
Hessian-vector products per second (200 products at a cached mid-optimisation state),
per-registration and per-product p50/p99 latency, the roofline of the dominant kernel
(timed with HIP events on the library's stream) and the FP64 oracle's rate on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1807_05117_amd import binding as B  # noqa: E402
from paper_1807_05117_amd import phantoms  # noqa: E402

GRID = (128, 128, 128)
BAND = (32, 32, 32)
NT = 10
DISP = 6.0
HBM_PEAK_GBS = 8000.0
# algorithmic FP32 bytes per voxel of one launch of each timed kernel class:
#   state step      X (12) + m^n (4) read, m^{n+1} (4) written                 = 20
#   incremental     X (12) + t^n (4) + m^{n+1} (4) + dv (12) read, t^{n+1} (4)  = 36
#   adjoint step    (Y, a) packed (16) + lambda^{n+1} (4) read, lambda^n (4)    = 24
#                   written (the body force is a separate pass over the stored lambda^n)
#   iota z stage    3 grid planes written (12) + the kz >= 0 half-spectrum columns read
#                   (3 kzh complex per column = 24 kzh / nz per voxel)
#   pi z stage      the same bytes in the other direction
#   body force      lambda^n, m^n read for n = 0..Nt (8 (Nt + 1)), b written (12)
#   setup           v, r read (16), X (12) and (Y, a) (16) written              = 44
KCLASS = {0: ("state_step", 20), 1: ("inc_step", 36), 2: ("adj_step", 24)}
KNAMES = {3: "iota_z", 4: "pi_z", 5: "body_force", 6: "setup"}


def class_bytes(k, grid, band, nt):
    """algorithmic bytes per voxel of kernel class k"""
    if k in KCLASS:
        return KCLASS[k][1]
    if k in (3, 4):
        return 12.0 + 24.0 * (band[2] // 2) / grid[2]
    if k == 5:
        # m^0..m^nt and lambda^1..lambda^nt read, (Y, a) read to form lambda^0, b written
        return 4.0 * (nt + 1) + 4.0 * nt + 16.0 + 12.0
    return 44.0


def class_name(k):
    return KCLASS[k][0] if k in KCLASS else KNAMES[k]


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


# the large single instance: 256^3, six tissue classes, 8 voxels, band 64^3, Nt = 20
LARGE = dict(grid=(256, 256, 256), band=(64, 64, 64), nt=20, disp=8.0, ncls=6)


def make_inputs(seed=0, grid=None, band=None, nt=None, disp=None, ncls=3, **model):
    grid, band = grid or GRID, band or BAND
    nt, disp = nt or NT, disp or DISP
    I0 = phantoms.shells_3d(seed, grid, n_classes=ncls).astype(np.float32)
    raw = phantoms.raw_band_velocity(seed, 3, band).astype(np.complex64)
    p = B.make_problem(3, grid, band, nt, **model)
    v = B.bl_band_to_grid(p, raw)                       # projected inside the library
    vmax = float(np.sqrt((v.astype(np.float64) ** 2).sum(axis=0)).max()) * max(grid)
    vs = (raw * (disp / vmax)).astype(np.complex64)
    I1 = B.bl_lddmm_warp(p, I0, vs)
    return I0, I1, vs


def kernel_table(kern, grid, band, nt):
    """average launch time and algorithmic GB/s (fraction of the 8 TB/s peak) per class"""
    M = int(np.prod(grid))
    out = {}
    for k, (n, ms) in kern.items():
        if not n:
            continue
        avg = ms / 1000.0 / n
        gbs = class_bytes(k, grid, band, nt) * M / avg / 1e9
        out[class_name(k)] = {"launches": n, "avg_us": avg * 1e6, "gbs_algorithmic": gbs,
                              "frac_of_peak": gbs / HBM_PEAK_GBS}
    return out


def gpu_leg(steps, warmup, n_hv=200, n_lat=50, n_grad=20, precision=B.BL_FP32, inputs=None,
            model=None, size=None):
    import torch

    model = model or {}
    size = size or {}
    grid, band, nt = size.get("grid", GRID), size.get("band", BAND), size.get("nt", NT)
    p = B.make_problem(3, grid, band, nt, precision=precision, **model)
    I0, I1, vs = inputs if inputs is not None else make_inputs(0, **size, **model)
    v0 = np.zeros_like(vs)
    # registrations on resident device inputs, the library's calls ordered on torch's stream;
    # every registration starts from its own zero initial guess allocated beforehand
    stream = torch.cuda.current_stream()
    pr = B.make_problem(3, grid, band, nt, device=True, stream=stream.cuda_stream,
                        precision=precision, **model)
    rI0 = torch.from_numpy(I0).cuda()
    rI1 = torch.from_numpy(I1).cuda()
    rw = torch.empty_like(rI0)
    guesses = [torch.zeros(vs.shape, dtype=torch.complex64, device="cuda")
               for _ in range(warmup + steps)]
    progress("inputs ready; warmup")
    for i in range(warmup):
        B.bl_lddmm_register_device(pr, rI0, rI1, guesses[i], rw)
    torch.cuda.synchronize()
    lat = []
    stats = None
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        stats = B.bl_lddmm_register_device(pr, rI0, rI1, guesses[warmup + i], rw)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    warped = rw.cpu().numpy()
    progress(f"{steps} registrations in {elapsed:.3f} s; host-pointer calls")
    # the same through host buffers (PCIe transfers of I0, I1, v and m(1) included)
    t_host = []
    for _ in range(3):
        ts = time.perf_counter()
        B.bl_lddmm_register(p, I0, I1, v0)
        t_host.append(time.perf_counter() - ts)
    progress("Hessian-vector products")

    # Hessian-vector products at a cached mid-optimisation state, device pointers on the
    # library's own context stream = torch's current stream
    stream = torch.cuda.current_stream()
    pd = B.make_problem(3, grid, band, nt, device=True, stream=stream.cuda_stream,
                        precision=precision, **model)
    dI0 = torch.from_numpy(I0).cuda()
    dI1 = torch.from_numpy(I1).cuda()
    ctx = B.Ctx(pd, dI0, dI1)
    vh = torch.from_numpy(np.ascontiguousarray(0.5 * vs)).cuda()
    gen = np.random.default_rng(1)
    dvn = (gen.standard_normal(vs.shape) + 1j * gen.standard_normal(vs.shape)).astype(np.complex64)
    dv = torch.from_numpy(dvn).cuda()
    out = torch.empty_like(dv)
    E, g = ctx.bl_lddmm_ctx_set_velocity(vh)
    for _ in range(20):
        ctx.bl_lddmm_ctx_hessvec(dv, out)
    torch.cuda.synchronize()
    # throughput: back-to-back products
    t1 = time.perf_counter()
    for _ in range(n_hv):
        ctx.bl_lddmm_ctx_hessvec(dv, out)
    torch.cuda.synchronize()
    hv_s = n_hv / (time.perf_counter() - t1)
    # latency: one product at a time, HIP events on the same stream
    hv_lat = []
    for _ in range(n_lat):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.bl_lddmm_ctx_hessvec(dv, out)
        e1.record(stream)
        e1.synchronize()
        hv_lat.append(e0.elapsed_time(e1))
    # gradients per second (set_velocity + gradient)
    t2 = time.perf_counter()
    for _ in range(n_grad):
        ctx.bl_lddmm_ctx_set_velocity(vh)
    torch.cuda.synchronize()
    grad_s = n_grad / (time.perf_counter() - t2)
    # per-kernel durations with HIP events on the context's stream
    ctx.bl_kernel_timing_enable(True)
    ctx.bl_lddmm_ctx_set_velocity(vh)
    for _ in range(20):
        ctx.bl_lddmm_ctx_hessvec(dv, out)
    torch.cuda.synchronize()
    kern = {}
    for k in range(7):
        n, ms = ctx.bl_kernel_timing_read(k)
        kern[k] = (n, ms)
    ctx.bl_kernel_timing_enable(False)
    shapes = dict(zip(("state", "incremental", "adjoint", "body_force"),
                      ctx.bl_lddmm_ctx_launch_shapes()))
    ctx.close()
    if precision != B.BL_FP32 or model or size:
        return dict(elapsed=elapsed, lat=lat, stats=stats, hv_s=hv_s, hv_lat=hv_lat,
                    grad_s=grad_s, kern=kern, shapes=shapes, E=E, inputs=(I0, I1, vs),
                    warped=warped, t_host=t_host)
    # achievable HBM bandwidth: a plain 1 GiB device-to-device copy (also the reference
    # kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) / 1000.0) / 1e9
    # an in-place read-modify-write of the same 1 GiB reaches more than a copy on this chip
    for _ in range(3):
        dst.add_(1.0)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        dst.add_(1.0)
    e1.record()
    e1.synchronize()
    rmw_gbs = 10 * 2 * dst.numel() * 4 / (e0.elapsed_time(e1) / 1000.0) / 1e9
    del src, dst
    return dict(copy_gbs=copy_gbs, rmw_gbs=rmw_gbs, inputs=(I0, I1, vs), warped=warped, elapsed=elapsed, lat=lat,
                stats=stats, hv_s=hv_s, hv_lat=hv_lat, grad_s=grad_s, kern=kern, shapes=shapes, E=E,
                t_host=t_host)


def cpu_leg(stats, repeats=3):
    """The FP64 oracle on the host: an energy evaluation, a gradient and a Hessian-vector
    product at 128^3 (median of `repeats` runs each), scaled by the registration's operation
    counts."""
    from threadpoolctl import threadpool_limits

    import oracle as O

    with threadpool_limits(limits=1):
        prob = O.Problem(3, GRID, BAND, NT)
        I0 = phantoms.shells_3d(0, GRID, n_classes=3).astype(np.float32).astype(np.float64)
        vs = O.project(phantoms.raw_band_velocity(0, 3, BAND), prob)
        vs *= DISP / O.max_displacement_voxels(vs, prob)
        I1 = O.warp(I0, vs, prob).astype(np.float32).astype(np.float64)
        d = O.project(phantoms.random_band_direction(1, 3, BAND), prob)
        te, tg, th = [], [], []
        for _ in range(repeats):
            t = time.perf_counter()
            st = O.evaluate(0.5 * vs, I0, I1, prob)
            te.append(time.perf_counter() - t)
            t = time.perf_counter()
            O.gradient(st)
            tg.append(time.perf_counter() - t)
            t = time.perf_counter()
            O.hessvec(st, d)
            th.append(time.perf_counter() - t)
    t_eval, t_grad, t_hv = (float(np.median(x)) for x in (te, tg, th))
    progress(f"oracle: evaluation {t_eval:.1f} s, gradient {t_grad:.1f} s, product {t_hv:.1f} s "
             f"(medians of {repeats})")
    t_reg = (stats["evaluations"] * t_eval + stats["gradients"] * t_grad
             + stats["hessvecs"] * t_hv)
    return {"value": 60.0 / t_reg, "unit": "registrations/min", "cores": 1, "kind": "oracle",
            "sample": (f"medians of {repeats} runs each of an energy evaluation ({t_eval:.1f} s), "
                       f"a gradient ({t_grad:.1f} s) and a Hessian-vector product ({t_hv:.1f} s) "
                       f"at 128^3/32^3/Nt=10, FP64 NumPy on 1 thread, scaled by the "
                       f"registration's counts ({stats['evaluations']} evaluations, "
                       f"{stats['gradients']} gradients, {stats['hessvecs']} products)"),
            "runs_s": {"evaluation": te, "gradient": tg, "hessvec": th},
            "hv_per_s": 1.0 / t_hv, "gradients_per_s": 1.0 / (t_eval + t_grad)}


def oracle_register_leg():
    """One full FP64 oracle registration of the headline pair (10 GN x <= 10 PCG), timed."""
    from threadpoolctl import threadpool_limits

    import oracle as O

    progress("oracle: one full registration at 128^3 (minutes)")
    with threadpool_limits(limits=1):
        prob = O.Problem(3, GRID, BAND, NT)
        I0 = phantoms.shells_3d(0, GRID, n_classes=3).astype(np.float32).astype(np.float64)
        vs = O.project(phantoms.raw_band_velocity(0, 3, BAND), prob)
        vs *= DISP / O.max_displacement_voxels(vs, prob)
        I1 = O.warp(I0, vs, prob).astype(np.float32).astype(np.float64)
        t = time.perf_counter()
        _, _, st = O.register(
            I0, I1, np.zeros_like(vs), prob, O.SolverOpts(),
            on_iteration=lambda s: progress(f"oracle registration: iteration {s['gn_iters']} "
                                            f"({s['pcg_iters'][-1]} PCG steps) at "
                                            f"{time.perf_counter() - t:.0f} s"))
        dt = time.perf_counter() - t
    return {"seconds": dt, "registrations_per_min": 60.0 / dt, "gn_iters": st["gn_iters"],
            "pcg_iters": st["pcg_iters"], "final_mse_rel": st["mse_rel"][-1], "cores": 1}


SERVE_SIZES = [(96, 96, 96), (128, 128, 128), (160, 192, 160)]


def _serve_phantom(args):
    seed, shp = args
    return phantoms.shells_3d(seed, shp, n_classes=3 if shp[0] < 160 else 5).astype(np.float32)


def serve_deformation_leg(n_pairs=8, slots=4):
    """Saturated serving of 128^3 deformation-state pairs (the model whose single-pair kernels
    are latency bound) by the slot-thread server against one registration after the other;
    the served results must be bitwise those of the sequential ones."""
    progress(f"serving: {n_pairs} deformation-state pairs, slot threads")
    pairs = [make_inputs(seed) for seed in range(n_pairs)]

    def prob():
        return B.make_problem(3, GRID, BAND, NT, deformation=True)

    v0 = np.zeros(B.band_shape(prob()), np.complex64)
    B.bl_lddmm_register(prob(), pairs[0][0], pairs[0][1], v0)   # first-use work, untimed
    t0 = time.perf_counter()
    seq = [B.bl_lddmm_register(prob(), I0, I1, v0)[0] for I0, I1, _ in pairs]
    t_seq = time.perf_counter() - t0
    B.bl_lddmm_release_cached()
    srv = B.Server(max_slots=slots, batched=False)
    t0 = time.perf_counter()
    tickets = [srv.submit(prob(), I0, I1) for I0, I1, _ in pairs]
    res = [srv.wait(t) for t in tickets]
    wall = time.perf_counter() - t0
    srv.close()
    if any(r[0] != B.BL_OK for r in res):
        raise RuntimeError("deformation serving request failed")
    return {"pairs": n_pairs, "slots": slots,
            "workload": "128^3 deformation state equation, band 32^3, Nt = 10, per-pair seeds",
            "sequential_registrations_per_min": 60.0 * n_pairs / t_seq,
            "saturated_registrations_per_min": 60.0 * n_pairs / wall,
            "speedup_saturated_vs_sequential": t_seq / wall,
            "results_bitwise_equal_to_sequential": all(
                np.array_equal(r[1], v) for r, v in zip(res, seq))}


def serve_leg(n_pairs=64, rate=4.0, slots=8, thread_slots=4, seed=1000):
    """Continuous-batching request loop on a stream of registration pairs of mixed sizes:
    grids uniform over 96^3, 128^3 and 160x192x160, band = grid/4 per axis, Nt in {5, 10},
    per-pair phantom and velocity seeds (6 voxels).  Runs over the same pairs: sequential plain
    FP32 (one bl_lddmm_register after the other), saturated serving (all pairs queued at
    t = 0) by the slot-thread server and by the cohort server, and open-loop serving with
    Poisson arrivals by the cohort server.  The slot-thread server runs as many slots as a
    process has hardware queues (4): more slots contend and serve fewer pairs per second."""
    from concurrent.futures import ThreadPoolExecutor

    rng = np.random.default_rng(seed)
    shapes = [SERVE_SIZES[int(rng.integers(len(SERVE_SIZES)))] for _ in range(n_pairs)]
    nts = [int(rng.choice([5, 10])) for _ in range(n_pairs)]
    with ThreadPoolExecutor(max_workers=8) as ex:   # NumPy releases the GIL in the bulk work
        sources = list(ex.map(_serve_phantom, [(seed + 100 + i, shapes[i]) for i in range(n_pairs)]))
    pairs = []
    for i in range(n_pairs):
        shp, nt = shapes[i], nts[i]
        band = tuple(n // 4 for n in shp)
        raw = phantoms.raw_band_velocity(seed + 10 + i, 3, band).astype(np.complex64)
        p = B.make_problem(3, shp, band, nt)
        v = B.bl_band_to_grid(p, raw)
        vmax = float(np.sqrt((v.astype(np.float64) ** 2).sum(axis=0)).max()) * max(shp)
        I1 = B.bl_lddmm_warp(p, sources[i], (raw * (DISP / vmax)).astype(np.complex64))
        pairs.append((shp, band, nt, sources[i], I1))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_pairs))
    progress(f"serving: {n_pairs} pairs ready; sequential FP32")

    def prob(i, precision):
        shp, band, nt, _, _ = pairs[i]
        return B.make_problem(3, shp, band, nt, precision=precision)

    def sequential(precision):
        mse, vs = [], []
        t0 = time.perf_counter()
        for i, (shp, band, nt, I0, I1) in enumerate(pairs):
            v0 = np.zeros(B.band_shape(prob(i, precision)), np.complex64)
            v, _, st = B.bl_lddmm_register(prob(i, precision), I0, I1, v0)
            mse.append(st["mse_rel"][-1])
            vs.append(v)
        return time.perf_counter() - t0, mse, vs

    t_seq, seq_mse, _ = sequential(B.BL_FP32)
    B.bl_lddmm_release_cached()

    def serve(arrive, batched, precision):
        srv = B.Server(max_slots=slots if batched else thread_slots, batched=batched)
        t_start = time.perf_counter()
        tickets = []
        for i, (shp, band, nt, I0, I1) in enumerate(pairs):
            if arrive is not None:
                delay = arrive[i] - (time.perf_counter() - t_start)
                if delay > 0:
                    time.sleep(delay)
            tickets.append(srv.submit(prob(i, precision), I0, I1))
        lat, mse, vs = [], [], []
        for t in tickets:
            rc, v, _, st, tm = srv.wait(t)
            if rc != B.BL_OK:
                raise RuntimeError(f"serving request failed: {rc}")
            lat.append(tm["finished"] - tm["submitted"])
            mse.append(st["mse_rel"][-1])
            vs.append(v)
        wall = time.perf_counter() - t_start
        info = srv.info()
        srv.close()
        return dict(wall=wall, lat=lat, mse=mse, info=info, v=vs)

    def record(r):
        return {"registrations_per_min": 60.0 * n_pairs / r["wall"], "seconds": r["wall"],
                "p50_ms": 1000 * percentile(r["lat"], 50), "p99_ms": 1000 * percentile(r["lat"], 99),
                "peak_resident": r["info"]["peak_resident"],
                "peak_gb": r["info"]["peak_bytes"] / 1e9,
                "final_mse_rel_max_rel_diff_vs_fp32": max(
                    abs(a - b) / max(abs(b), 1e-12) for a, b in zip(r["mse"], seq_mse))}

    progress("serving: saturated, slot threads (mixed)")
    thr = serve(None, False, B.BL_MIXED)
    progress("serving: saturated, cohorts (mixed)")
    coh = serve(None, True, B.BL_MIXED)
    progress("serving: saturated, cohorts (fp32)")
    coh32 = serve(None, True, B.BL_FP32)
    progress("serving: Poisson arrivals, cohorts (mixed)")
    poi = serve(arrivals, True, B.BL_MIXED)
    # the cohort server's results are bitwise those of one-pair registrations
    t_seqm, _, seqm_v = sequential(B.BL_MIXED)
    identical = all(np.array_equal(a, b) for a, b in zip(coh["v"], seqm_v))
    return {
        "pairs": n_pairs, "slots": slots, "slot_threads": thread_slots,
        "grids": [list(g) for g in SERVE_SIZES], "band": "grid/4", "nt": [5, 10],
        "phantoms": "per-pair seeds",
        "sequential_fp32": {"registrations_per_min": 60.0 * n_pairs / t_seq, "seconds": t_seq},
        "sequential_mixed": {"registrations_per_min": 60.0 * n_pairs / t_seqm, "seconds": t_seqm},
        "saturated_mixed_slot_threads": record(thr),
        "saturated_mixed_cohorts": record(coh),
        "saturated_fp32_cohorts": record(coh32),
        "poisson_mixed_cohorts": dict(record(poi), rate_per_s=rate),
        "speedup_saturated_vs_sequential_fp32": t_seq / coh["wall"],
        "speedup_slot_threads_vs_sequential_fp32": t_seq / thr["wall"],
        "cohort_results_bitwise_equal_to_one_pair_mixed": identical,
        "deformation_state_slot_threads": serve_deformation_leg(),
    }


def traffic_record(kernel):
    """Per-launch HBM bytes of `kernel` from the committed counter summary, if it was taken on
    the kernel source that is built now (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_c2_128cube_fp32.json")
    src = os.path.join(ROOT, "paper_1807_05117_amd", "csrc", "bl_transport.hip")
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("transport_source_sha256") != digest or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["bytes_per_launch"]


# the brain-shaped instance: 160x192x160, five tissue classes, band 40x48x40, Nt = 10
C3 = dict(grid=(160, 192, 160), band=(40, 48, 40), nt=10, disp=6.0, ncls=5)
BF16_DENSE_PEAK_TFLOPS = 2500.0


def zstage_rates(kern, grid, band, precision):
    """The z stages of the transforms (classes 3, 4, timed inside Gauss-Newton products):
    algorithmic rate of the stage's real products (2 flops per multiply-add: a
    [nz x 2 kzh] x [2 kzh x nx ny] product per component, 3 components) and, for the mixed
    form, the rate the matrix cores issue (3 split BF16 products per term, tiles padded to
    the 32 x 32 x 16 instruction) against the dense BF16 peak."""
    nq, nz, kzh, C = grid[0] * grid[1], grid[2], band[2] // 2, 3
    nq32 = (nq + 31) // 32 * 32
    out = {}
    for k, nm in ((3, "iota_z"), (4, "pi_z")):
        n, ms = kern.get(k, (0, 0.0))
        if not n:
            continue
        avg = ms / 1000.0 / n
        rec = {"avg_us": avg * 1e6,
               "tflops_algorithmic": 4.0 * nz * kzh * nq * C / avg / 1e12}
        if precision == B.BL_MIXED:
            if k == 3:
                kp = (2 * kzh + 15) // 16 * 16
                issued = 3 * 2.0 * ((nz + 31) // 32 * 32) * kp * nq32 * C
            else:
                jt = (2 * kzh + 31) // 32
                issued = 3 * 2.0 * (32 * jt) * ((nz + 15) // 16 * 16) * nq32 * C
            rec["mfma_issued_tflops"] = issued / avg / 1e12
            rec["mfma_util_of_bf16_dense_peak"] = issued / avg / 1e12 / BF16_DENSE_PEAK_TFLOPS
        out[nm + "_rates"] = rec
    return out


def rel_errs(got, ref, lv=None):
    """2-norm error relative to |ref| (gradient: to |L v| + |ref - L v|), and the largest entry
    error relative to the largest reference entry"""
    got = np.asarray(got, np.complex128)
    d = np.linalg.norm((got - ref).ravel())
    den = (np.linalg.norm(lv.ravel()) + np.linalg.norm((ref - lv).ravel())) if lv is not None \
        else np.linalg.norm(ref.ravel())
    return {"rel_2norm": float(d / den),
            "rel_maxabs": float(np.abs(got - ref).max() / np.abs(ref).max())}


def c3_leg(reps, with_oracle):
    """160x192x160 (band 40x48x40, Nt = 10, five tissue classes): plain FP32 and mixed form,
    registrations/min, Hv/s, the z stages' GB/s and matrix-core rate, and -- with the oracle --
    the gradient's and the product's errors against the FP64 oracle at a mid-optimisation
    velocity for both precisions."""
    size = dict(C3)
    ncls = size.pop("ncls")
    progress("C3 160x192x160: inputs")
    inputs = make_inputs(0, ncls=ncls, **size)
    I0, I1, vs = inputs
    grid, band, nt = size["grid"], size["band"], size["nt"]
    out = {"workload": "160x192x160 5-class shell phantom, 6 vox, band 40x48x40, Nt = 10"}
    gen = np.random.default_rng(7)
    dv = (gen.standard_normal(vs.shape) + 1j * gen.standard_normal(vs.shape)).astype(np.complex64)
    vh = (0.5 * vs).astype(np.complex64)
    gh = {}
    for name, prec in (("fp32", B.BL_FP32), ("mixed", B.BL_MIXED)):
        progress(f"C3: {name}")
        r = gpu_leg(3, 1, *reps, precision=prec, inputs=inputs, size=size)
        kern = kernel_table(r["kern"], grid, band, nt)
        kern.update(zstage_rates(r["kern"], grid, band, prec))
        out[name] = {"registrations_per_min": 60000.0 / (1000.0 * r["elapsed"] / 3),
                     "hv_per_s": r["hv_s"], "hv_p50_ms": percentile(r["hv_lat"], 50),
                     "gradients_per_s": r["grad_s"], "gn_iters": r["stats"]["gn_iters"],
                     "hessvecs": r["stats"]["hessvecs"],
                     "final_mse_rel": r["stats"]["mse_rel"][-1], "kernels": kern}
        p = B.make_problem(3, grid, band, nt, precision=prec)
        g, _ = B.bl_lddmm_gradient(p, I0, I1, vh)
        H = B.bl_lddmm_hessvec(p, I0, I1, vh, dv)
        gh[name] = (g, H)
    if with_oracle:
        from threadpoolctl import threadpool_limits

        import oracle as O

        progress("C3: FP64 oracle gradient and product (host)")
        with threadpool_limits(limits=1):
            prob = O.Problem(3, grid, band, nt)
            st = O.evaluate(vh.astype(np.complex128), I0.astype(np.float64),
                            I1.astype(np.float64), prob)
            gref = O.gradient(st)
            dvp = O.project(dv.astype(np.complex128), prob)
            Href = O.hessvec(st, dvp)
            lv = O.L_hat(prob)[None] * O.project(vh.astype(np.complex128), prob)
        out["errors_vs_fp64_oracle"] = {
            name: {"gradient": rel_errs(g, gref, lv), "hessvec": rel_errs(H, Href)}
            for name, (g, H) in gh.items()}
    return out


def hbm_resident_leg():
    """The transports on fields that do not fit the last-level cache: one registration and a
    few products at 256^3 (band 64^3, Nt = 20), per-class HIP-event timing."""
    size = dict(LARGE)
    ncls = size.pop("ncls")
    progress("256^3: inputs")
    inputs = make_inputs(0, ncls=ncls, **size)
    r = gpu_leg(1, 0, 10, 3, 2, inputs=inputs, size=size)
    return {"workload": "256^3 6-class shell phantom, 8 vox, band 64^3, Nt = 20",
            "kernels": kernel_table(r["kern"], size["grid"], size["band"], size["nt"]),
            "transport_voxels_per_thread": r["shapes"], "hv_per_s": r["hv_s"]}


def large_main(steps, warmup, reps):
    """256^3 single instance (band 64^3, Nt = 20): plain FP32 and the mixed form on the same
    pair, registrations/min, Hv/s, final mismatch, and the transports' HBM GB/s from HIP-event
    timing.  Printed as one JSON line; not the default benchmark."""
    size = dict(LARGE)
    ncls = size.pop("ncls")
    progress("large instance: inputs")
    inputs = make_inputs(0, ncls=ncls, **size)
    out = {"metric": "registrations/min and GN Hv/s at 256^3, plain FP32 vs mixed form",
           "workload": "256^3 6-class shell phantom, 8 vox, band 64^3, Nt = 20, 10 GN x <= 10 PCG",
           "data": "synthetic", "n_gpus": 1}
    for name, prec in (("fp32", B.BL_FP32), ("mixed", B.BL_MIXED)):
        progress(f"large instance: {name}")
        r = gpu_leg(steps, warmup, *reps, precision=prec, inputs=inputs, size=size)
        kern = kernel_table(r["kern"], size["grid"], size["band"], size["nt"])
        kern.update(zstage_rates(r["kern"], size["grid"], size["band"], prec))
        out[name] = {"registrations_per_min": 60000.0 / (1000.0 * r["elapsed"] / steps),
                     "hv_per_s": r["hv_s"], "hv_p50_ms": percentile(r["hv_lat"], 50),
                     "gradients_per_s": r["grad_s"], "gn_iters": r["stats"]["gn_iters"],
                     "hessvecs": r["stats"]["hessvecs"],
                     "final_mse_rel": r["stats"]["mse_rel"][-1], "kernels": kern,
                     "warped": r["warped"]}
    wf, wm = out["fp32"].pop("warped"), out["mixed"].pop("warped")
    out["warped_max_abs_diff_mixed_vs_fp32"] = float(np.abs(wf - wm).max())
    print(json.dumps(out), flush=True)


def headline_line(args, r):
    """The JSON line of the headline leg (128^3 FP32 registrations and products)."""
    ms_step = 1000.0 * r["elapsed"] / args.steps
    M = GRID[0] * GRID[1] * GRID[2]
    # dominant kernel: largest total time among the transport step kernels
    kc = max(KCLASS, key=lambda k: r["kern"][k][1])
    n_launch, ms_tot = r["kern"][kc]
    name, bpv = KCLASS[kc]
    avg_s = ms_tot / 1000.0 / max(n_launch, 1)
    achieved = bpv * M / avg_s / 1e9
    hv_bytes = (64 * NT + 36) * M
    return {
        "metric": "GN Hessian-vec products/s and registrations/min at 128^3; p50/p99 latency",
        "value": 60000.0 / ms_step,
        "unit": "registrations/min",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "registration of a 128^3 3-class shell phantom to its warp "
                               "(6 vox), band 32^3, Nt=10, 10 GN x <=10 PCG",
                   "grid": list(GRID), "band": list(BAND), "nt": NT, "alpha": 1e-3, "s": 2,
                   "sigma": 1.0, "precision": "fp32", "parallelism": "single GPU"},
        "registration": {"p50_ms": 1000 * percentile(r["lat"], 50),
                         "p99_ms": 1000 * percentile(r["lat"], 99),
                         "gn_iters": r["stats"]["gn_iters"], "hessvecs": r["stats"]["hessvecs"],
                         "gradients": r["stats"]["gradients"],
                         "evaluations": r["stats"]["evaluations"],
                         "final_mse_rel": r["stats"]["mse_rel"][-1],
                         "status": r["stats"]["status"],
                         "inputs": "resident in HBM (device pointers)",
                         "host_pointer_calls_per_min": 60.0 / float(np.median(r["t_host"]))},
        "hv_per_s": r["hv_s"],
        "hv_p50_ms": percentile(r["hv_lat"], 50),
        "hv_p99_ms": percentile(r["hv_lat"], 99),
        "hv_hbm_gbs_algorithmic": hv_bytes * r["hv_s"] / 1e9,
        "gradients_per_s": r["grad_s"],
        "kernels": kernel_table(r["kern"], GRID, BAND, NT),
        "transport_voxels_per_thread": r["shapes"],
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_record(name),
                     "bytes_per_voxel": bpv, "avg_launch_us": avg_s * 1e6,
                     "llc_assisted": True,
                     "note": ("at 128^3 the fields one time step re-reads (offsets, dv) stay in "
                              "the 256 MiB last-level cache between steps; hbm_resident_256 "
                              "gives the same kernels on 256^3 fields, which do not"),
                     "copy_gbs": r["copy_gbs"], "frac_of_copy": achieved / r["copy_gbs"],
                     "inplace_rmw_gbs": r["rmw_gbs"],
                     "frac_of_inplace_rmw": achieved / r["rmw_gbs"]},
        "cpu_baseline": None,
    }


def model_record(r, steps, **extra):
    rec = dict(extra)
    rec.update({"registrations_per_min": 60000.0 / (1000.0 * r["elapsed"] / steps),
                "hv_per_s": r["hv_s"], "hv_p50_ms": percentile(r["hv_lat"], 50),
                "gradients_per_s": r["grad_s"], "gn_iters": r["stats"]["gn_iters"],
                "hessvecs": r["stats"]["hessvecs"], "final_mse_rel": r["stats"]["mse_rel"][-1],
                "status": r["stats"]["status"]})
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    ap.add_argument("--quick", action="store_true",
                    help="fewer Hessian-vector repetitions (for profiler passes)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--large", action="store_true",
                    help="the 256^3 single instance instead (plain FP32 vs mixed form)")
    ap.add_argument("--no-c3", action="store_true", help="skip the 160x192x160 leg")
    ap.add_argument("--no-hbm", action="store_true", help="skip the 256^3 transport timing")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline leg (128^3 FP32 registrations and products), for "
                         "profiler passes")
    ap.add_argument("--oracle-register", action="store_true",
                    help="also time one full FP64 oracle registration at 128^3 (minutes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the registration path has no multi-GPU mode "
              "(pairs are independent; see the design notes for how it would shard).",
              file=sys.stderr)
        sys.exit(2)
    B.load()
    if not B.device_available():
        raise RuntimeError("no HIP device visible")
    reps = (20, 5, 2) if args.quick else (200, 50, 20)
    if args.large:
        large_main(args.steps, args.warmup, (20, 5, 3) if args.quick else (50, 20, 5))
        return
    r = gpu_leg(args.steps, args.warmup, *reps)
    line = headline_line(args, r)
    if args.headline_only:
        print(json.dumps(line), flush=True)
        return
    half = max(1, args.steps // 2)
    progress("mixed-precision form")
    rm = gpu_leg(half, 1, *reps, precision=B.BL_MIXED, inputs=r["inputs"])
    line["mixed"] = model_record(
        rm, half, precision="bf16 split hi/lo MFMA band<->grid z contractions, fp32 "
                            "transports, fp64 reductions",
        hv_p99_ms=percentile(rm["hv_lat"], 99), final_mse_rel_fp32=r["stats"]["mse_rel"][-1],
        warped_max_abs_diff_vs_fp32=float(np.abs(rm["warped"] - r["warped"]).max()))
    progress("incompressible H1 model")
    ri = gpu_leg(half, 1, *reps, model=dict(alpha=5e-3, s=1, gamma=1))
    line["incompressible_h1"] = model_record(
        ri, half, model="gamma = 1, s = 1, alpha = 5e-3 (divergence-free velocities, H1 "
                        "regulariser), same grid, band, Nt, FP32")
    progress("full Newton Hessian")
    rn = gpu_leg(half, 1, *reps, model=dict(newton=True), inputs=r["inputs"])
    line["full_newton"] = model_record(
        rn, half, hessian="full Newton products (adjoint source and lambda grad dm kept)")
    progress("non-stationary velocity")
    I0r, I1r, vsr = r["inputs"]
    rns = gpu_leg(half, 1, *reps, model=dict(nonstationary=True),
                  inputs=(I0r, I1r, np.stack([vsr] * (NT + 1))))
    line["nonstationary"] = model_record(
        rns, half, velocity=f"one band field per time node ({NT + 1} nodes)")
    progress("deformation state equation")
    rd = gpu_leg(half, 1, *reps, model=dict(deformation=True), inputs=r["inputs"])
    line["deformation_state"] = model_record(
        rd, half, method="band deformation state equation: RK4 on the band displacement, "
                         "truncated convolutions on a 48^3 product grid, Gauss-Newton products")
    if not args.no_hbm:
        B.bl_lddmm_release_cached()
        line["roofline"]["hbm_resident_256"] = hbm_resident_leg()
    if not args.no_c3:
        B.bl_lddmm_release_cached()
        line["c3"] = c3_leg(reps, not args.no_cpu)
    if not args.no_serve:
        B.bl_lddmm_release_cached()
        line["serving"] = serve_leg()
    if not args.no_cpu:
        progress("oracle baseline on the host")
        line["cpu_baseline"] = cpu_leg(r["stats"])
        if args.oracle_register:
            line["cpu_baseline"]["full_registration"] = oracle_register_leg()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
