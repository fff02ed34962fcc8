"""Mutation check of the oracle's pins: each plausible mistake (a dropped term, a wrong sign,
factor or index) is planted in a fresh copy of the oracle's source, and at least one pin
must then fail.  The pins here are compact versions of those in test_oracle_pins.py that
take the (possibly mutated) module as an argument; their expected values come from
brute-force sums, numpy.fft, closed forms and exact permutation cases, never from the oracle.
"""
import cmath
import itertools
import math
import os
import sys
import types

import numpy as np
import pytest

from paper_1807_05117_amd import phantoms

SRC = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "oracle", "bl_oracle.py")).read()


_serial = itertools.count()


def load(src):
    """a fresh module built from the (possibly mutated) oracle source text"""
    name = f"_oracle_copy_{next(_serial)}"
    mod = types.ModuleType(name)
    sys.modules[name] = mod  # dataclasses look their module up
    try:
        exec(compile(src, name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def rand_band(O, prob, seed):
    return O.project(phantoms.random_band_direction(seed, prob.dim, prob.k), prob)


def fft_pi(f, prob):
    F = np.fft.fftn(f) / prob.M
    idx = np.meshgrid(*[np.mod(np.arange(K) - K // 2, N) for K, N in zip(prob.bshape, prob.shape)],
                      indexing="ij")
    out = F[tuple(idx)].copy()
    for a in range(prob.dim):
        sl = [slice(None)] * prob.dim
        sl[a] = 0
        out[tuple(sl)] = 0
    return out


def np_grad(f, prob):
    h = 1.0 / prob.nref
    fp = np.pad(f, 1, mode="wrap")
    inner = tuple(slice(1, -1) for _ in range(prob.dim))
    return [np.gradient(fp, h, axis=prob.dim - 1 - j)[inner] for j in range(prob.dim)]


# ------------------------------------------------------------------------------ pins
def pin_bruteforce_dft(O):
    prob = O.Problem(3, (6, 4, 4), (4, 2, 4), 2)
    rng = np.random.default_rng(0)
    vh = rng.standard_normal(prob.bshape) + 1j * rng.standard_normal(prob.bshape)
    f = rng.standard_normal(prob.shape)
    ri = np.zeros(prob.shape, complex)
    rp = np.zeros(prob.bshape, complex)
    for idx in np.ndindex(prob.shape):
        for kidx in np.ndindex(prob.bshape):
            ph = sum((kidx[::-1][j] - prob.k[j] // 2) * idx[::-1][j] / prob.n[j] for j in range(3))
            e = cmath.exp(2j * math.pi * ph)
            ri[idx] += vh[kidx] * e
            rp[kidx] += f[idx] / e
    rp /= prob.M
    rp[0], rp[:, 0], rp[:, :, 0] = 0, 0, 0
    return (np.allclose(O.iota(vh, prob), ri.real, atol=1e-12)
            and np.allclose(O.pi_(f, prob), rp, atol=1e-12))


def pin_projection(O):
    prob = O.Problem(3, (8, 6, 6), (4, 4, 2), 2)
    raw = phantoms.random_band_direction(1, 3, prob.k)
    p = O.project(raw, prob)
    blk = p[:, 1:, 1:, 1:]
    return np.allclose(blk, np.conj(blk[:, ::-1, ::-1, ::-1])) and np.allclose(O.project(p, prob), p)


def pin_symbol_fd(O):
    kv, alpha, s = (3, -2), 1e-3, 2
    N = 256
    prob = O.Problem(2, (N, 3 * N // 4), (8, 8), 4, alpha=alpha, s=s)
    vh = np.zeros((2,) + prob.bshape, complex)
    ip = tuple(kv[j] + 4 for j in (1, 0))
    im = tuple(-kv[j] + 4 for j in (1, 0))
    vh[(0,) + ip] = 0.5 + 0.25j
    vh[(0,) + im] = 0.5 - 0.25j
    f = O.iota(vh[0], prob)
    g = f.copy()
    h = 1.0 / prob.nref
    for _ in range(s):
        g = g - alpha * sum((np.roll(g, 1, a) - 2 * g + np.roll(g, -1, a)) / h ** 2 for a in (0, 1))
    return np.max(np.abs(g - O.L_hat(prob)[ip] * f)) / np.max(np.abs(f)) < 1e-3


def pin_divergence(O):
    prob = O.Problem(3, (20, 16, 12), (8, 8, 6), 4)
    vh = np.zeros((3,) + prob.bshape, complex)
    kv, c = (2, -1, 1), 0.3 - 0.7j
    vh[(0,) + tuple(kv[j] + prob.k[j] // 2 for j in (2, 1, 0))] = c
    vh[(0,) + tuple(-kv[j] + prob.k[j] // 2 for j in (2, 1, 0))] = np.conj(c)
    r = O.iota(O.div_band(vh, prob), prob)
    zz, yy, xx = np.meshgrid(*[np.arange(N) / prob.nref for N in prob.shape], indexing="ij")
    q = [kv[j] * prob.nref / prob.n[j] for j in range(3)]
    ph = 2 * np.pi * (q[0] * xx + q[1] * yy + q[2] * zz)
    ref = 2 * np.real(c * 2j * np.pi * q[0] * np.exp(1j * ph))
    return np.allclose(r, ref, atol=1e-10 * np.abs(ref).max())


def pin_roll_and_identity(O):
    nt = 8
    prob = O.Problem(3, (16, 16, 16), (4, 4, 4), nt)
    I0 = np.random.default_rng(2).standard_normal(prob.shape)
    geo0 = O.setup(np.zeros((3,) + prob.bshape, complex), prob)
    if not np.array_equal(O.forward_state(I0, geo0["X"], prob)[-1], I0):
        return False
    vh = np.zeros((3,) + prob.bshape, complex)
    u = (1, -1, 2)
    for j in range(3):
        vh[(j, 2, 2, 2)] = u[j] * nt / prob.nref
    geo = O.setup(vh, prob)
    mT = O.forward_state(I0, geo["X"], prob)[-1]
    shift = tuple(nt * u[2 - a] for a in range(3))
    return np.array_equal(mT, np.roll(I0, shift, axis=(0, 1, 2))) and np.all(geo["a"] == 1)


def pin_interp_half_voxel(O):
    prob = O.Problem(2, (10, 8), (4, 4), 1)
    f = np.random.default_rng(3).standard_normal(prob.shape)
    off = [np.full(prob.shape, 0.25), np.zeros(prob.shape)]
    return np.allclose(O.interp(f, off, prob), 0.75 * f + 0.25 * np.roll(f, -1, axis=1))


def _zero_state(O):
    prob = O.Problem(3, (12, 10, 8), (4, 4, 4), 5, sigma=0.7, alpha=2e-3, s=1)
    rng = np.random.default_rng(4)
    I0, I1 = rng.standard_normal(prob.shape), rng.standard_normal(prob.shape)
    return prob, I0, I1, O.evaluate(np.zeros((3,) + prob.bshape, complex), I0, I1, prob)


def pin_gradient_closed_form(O):
    prob, I0, I1, st = _zero_state(O)
    gI = np_grad(I0, prob)
    lam = -(2.0 / prob.sigma ** 2) * (I0 - I1)
    ref = np.stack([fft_pi(lam * gI[j], prob) for j in range(3)])
    return np.allclose(O.gradient(st), ref, atol=1e-12 * np.abs(ref).max())


def pin_hessvec_closed_form(O):
    prob, I0, I1, st = _zero_state(O)
    d = rand_band(O, prob, 5)
    gI = np_grad(I0, prob)
    dv = [O.iota(d[j], prob) for j in range(3)]
    s_ = sum(gI[j] * dv[j] for j in range(3))
    ell = [N / prob.nref for N in prob.shape]
    kk = np.meshgrid(*[(np.arange(K) - K // 2) / l for K, l in zip(prob.bshape, ell)], indexing="ij")
    Lh = (1 + 4 * np.pi ** 2 * prob.alpha * sum(q ** 2 for q in kk)) ** prob.s
    ref = np.stack([Lh * d[j] + (2 / prob.sigma ** 2) * fft_pi(s_ * gI[j], prob) for j in range(3)])
    return np.allclose(O.hessvec(st, d), ref, atol=1e-11 * np.abs(ref).max())


def _smooth_pair(O):
    prob = O.Problem(2, (48, 48), (8, 8), 6)
    yy, xx = np.meshgrid(np.arange(48) / 48, np.arange(48) / 48, indexing="ij")
    I0 = np.cos(2 * np.pi * xx) * np.sin(2 * np.pi * (xx + 2 * yy))
    return prob, I0


def _velocity(O, prob, seed, disp):
    vh = O.project(phantoms.raw_band_velocity(seed, prob.dim, prob.k), prob)
    return vh * (disp / O.max_displacement_voxels(vh, prob))


def pin_gradient_fd(O):
    """central differences of the energy at a velocity of one voxel, on a smooth pair: the
    gap between optimise-then-discretise gradient and discrete derivative is about 2 %"""
    prob, I0 = _smooth_pair(O)
    yy, xx = np.meshgrid(np.arange(48) / 48, np.arange(48) / 48, indexing="ij")
    I1 = np.cos(2 * np.pi * (xx - 0.03)) * np.sin(2 * np.pi * (xx + 2 * yy + 0.05))
    vh = _velocity(O, prob, 6, 1.0)
    g = O.gradient(O.evaluate(vh, I0, I1, prob))
    ok = True
    for seed in (7, 8, 9):
        w = _velocity(O, prob, seed, 1.0)
        w /= np.sqrt(np.vdot(w, w).real)
        eps = 1e-5
        fd = (O.evaluate(vh + eps * w, I0, I1, prob).E - O.evaluate(vh - eps * w, I0, I1, prob).E) / (2 * eps)
        ok &= abs(fd - float(np.real(np.vdot(g, w)))) <= 0.05 * abs(fd)
    return ok


def pin_hessvec_fd_zero_residual(O):
    """at zero residual the Gauss-Newton product equals the derivative of the gradient up to
    the discretisation gap (6 % here)"""
    prob, I0 = _smooth_pair(O)
    vh = _velocity(O, prob, 9, 1.0)
    I1 = O.warp(I0, vh, prob)
    st = O.evaluate(vh, I0, I1, prob)
    d = _velocity(O, prob, 10, 1.0)
    H = O.hessvec(st, d)
    eps = 1e-4
    fd = (O.gradient(O.evaluate(vh + eps * d, I0, I1, prob))
          - O.gradient(O.evaluate(vh - eps * d, I0, I1, prob))) / (2 * eps)
    return np.linalg.norm((fd - H).ravel()) <= 0.1 * np.linalg.norm(H.ravel())


def pin_energy_regulariser(O):
    """with I0 = I1 constant the data term vanishes for every velocity (trilinear transport
    keeps a constant), so E is the regulariser alone, whose derivative along w is the real
    band inner product of L^ v~ and w"""
    prob = O.Problem(2, (40, 32), (8, 8), 4, alpha=0.05, s=1)
    I = np.full(prob.shape, 0.3)
    vh = _velocity(O, prob, 14, 2.0)
    st = O.evaluate(vh, I, I, prob)
    ell = [N / prob.nref for N in prob.shape]
    kk = np.meshgrid(*[(np.arange(K) - K // 2) / l for K, l in zip(prob.bshape, ell)], indexing="ij")
    Lh = 1 + 4 * np.pi ** 2 * prob.alpha * sum(q ** 2 for q in kk)
    E_ref = 0.5 * float(np.sum(Lh[None] * np.abs(vh) ** 2))
    w = _velocity(O, prob, 15, 1.0)
    eps = 1e-4
    fd = (O.evaluate(vh + eps * w, I, I, prob).E - O.evaluate(vh - eps * w, I, I, prob).E) / (2 * eps)
    return (abs(st.E - E_ref) <= 1e-12 * E_ref
            and abs(fd - float(np.real(np.vdot(O.gradient(st), w)))) <= 1e-8 * abs(fd))


def pin_incremental_adjoint_is_the_adjoint(O):
    """under the Gauss-Newton rule the incremental adjoint solves the adjoint equation with the
    incremental state as final residual: with I1' = m(1) - dm(1) the gradient's data part equals
    the Hessian product's data part exactly.  dm(1) is stepped here from the incremental state
    equation (Heun along the forward characteristic)."""
    prob = O.Problem(2, (32, 32), (8, 8), 4, sigma=0.9)
    yy, xx = np.meshgrid(np.arange(32) / 32, np.arange(32) / 32, indexing="ij")
    I0 = np.cos(2 * np.pi * xx) * np.sin(2 * np.pi * (xx + 2 * yy))
    vh = _velocity(O, prob, 16, 2.0)
    st = O.evaluate(vh, I0, I0, prob)
    d = _velocity(O, prob, 17, 1.0)
    dv = [O.iota(d[j], prob) for j in range(2)]
    f = [-sum(g * u for g, u in zip(O.grad_c(m, prob), dv)) for m in st.m]
    dm = np.zeros(prob.shape)
    for n in range(prob.nt):
        dm = O.interp(dm + 0.5 * prob.dt * f[n], st.geo["X"], prob) + 0.5 * prob.dt * f[n + 1]
    Lh = O.L_hat(prob)[None]
    lhs = O.hessvec(st, d) - Lh * d
    rhs = O.gradient(O.evaluate(vh, I0, st.m[-1] - dm, prob)) - Lh * st.geo["vh"]
    return np.allclose(lhs, rhs, rtol=0, atol=1e-10 * np.abs(lhs).max())


def pin_symmetry_shift(O):
    nt = 8
    prob = O.Problem(2, (24, 24), (8, 8), nt, sigma=0.8)
    vh = np.zeros((2,) + prob.bshape, complex)
    vh[(0, 4, 4)] = nt / prob.nref
    vh[(1, 4, 4)] = -nt / prob.nref
    I0 = phantoms.blobs_2d(3, 24)
    st = O.evaluate(vh, I0, np.roll(I0, 3, axis=0), prob)
    d1, d2 = rand_band(O, prob, 11), rand_band(O, prob, 12)
    a = np.vdot(O.hessvec(st, d1), d2).real
    b = np.vdot(d1, O.hessvec(st, d2)).real
    return abs(a - b) <= 1e-10 * (abs(a) + abs(b))


def pin_characteristics(O):
    """departure offsets and the adjoint's reaction factor against the exact flow of a field
    v_x(x) of one Fourier mode, integrated by fine RK4: X is the displacement over one step
    backward in time, Y over one step forward, and the factor is exp of the integral of
    dv_x/dx along the forward path.  Heun's local error is third order, so at 16 steps it
    sits far below a dropped term, a sign error or a predictor taken at the wrong point."""
    prob = O.Problem(2, (64, 64), (8, 8), 16)
    c = 0.1 * (1.0 - 0.5j)
    vh = np.zeros((2,) + prob.bshape, complex)
    vh[(0, 4, 5)] = c
    vh[(0, 4, 3)] = np.conj(c)
    geo = O.setup(vh, prob)
    v = lambda x: 2 * np.real(c * np.exp(2j * np.pi * x))
    r = lambda x: 2 * np.real(2j * np.pi * c * np.exp(2j * np.pi * x))
    x0 = np.arange(64) / 64.0
    ok = True
    for sign, key in ((1.0, "Y"), (-1.0, "X")):
        x, acc, h = x0.copy(), np.zeros(64), sign * prob.dt / 200
        for _ in range(200):
            k1 = v(x); k2 = v(x + h / 2 * k1); k3 = v(x + h / 2 * k2); k4 = v(x + h * k3)
            acc += h / 6 * (r(x) + 2 * r(x + h / 2 * k1) + 2 * r(x + h / 2 * k2) + r(x + h * k3))
            x = x + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        disp = (x - x0) * prob.nref
        ok &= np.max(np.abs(geo[key][0] - disp[None, :])) < 5e-3 * np.max(np.abs(disp))
        ok &= np.max(np.abs(geo[key][1])) == 0
        if key == "Y":
            exact = np.exp(acc)
            ok &= np.max(np.abs(geo["a"] - exact[None, :])) < 0.01 * np.max(np.abs(exact - 1))
    return ok


def pin_solver(O):
    prob = O.Problem(2, (24, 20), (8, 8), 4)
    I0 = np.full(prob.shape, 0.5)
    I1 = np.random.default_rng(13).standard_normal(prob.shape)
    v0 = O.project(phantoms.raw_band_velocity(61, 2, prob.k), prob)
    v0 *= 2.0 / O.max_displacement_voxels(v0, prob)
    vh, mT, stats = O.register(I0, I1, v0, prob, O.SolverOpts(max_gn=3, max_pcg=5))
    return (stats["pcg_iters"] == [1] and stats["status"] == O.CONVERGED
            and np.max(np.abs(vh)) <= 1e-12 * np.max(np.abs(v0)))


def _div_free_problem(O):
    prob = O.Problem(3, (20, 16, 12), (8, 8, 6), 4, alpha=5e-3, s=1, gamma=1)
    yy = np.arange(16)[None, :, None] / 16
    zz = np.arange(12)[:, None, None] / 12
    xx = np.arange(20)[None, None, :] / 20
    I0 = np.cos(2 * np.pi * xx) * np.sin(2 * np.pi * (yy + zz)) + 0.3 * np.sin(2 * np.pi * zz)
    return prob, I0


def pin_incompressible_projection(O):
    """gamma = 1: the projection of an arbitrary band vector is divergence-free to rounding
    (spectral divergence of the projected vector), idempotent, and leaves a velocity built as
    a spectral curl unchanged"""
    prob, _ = _div_free_problem(O)
    raw = phantoms.random_band_direction(21, 3, prob.k)
    p = O.project(raw, prob)
    div = O.div_band(p, prob)
    ok = np.max(np.abs(div)) <= 1e-12 * np.max(np.abs(p)) * 2 * np.pi * max(prob.k)
    ok &= np.allclose(O.project(p, prob), p, rtol=0, atol=1e-13 * np.abs(p).max())
    # curl of a potential: (q2 a3 - q3 a2, ...) is divergence-free by construction
    q = [2 * np.pi * x for x in O._kl(prob)]
    a = O.project(phantoms.random_band_direction(22, 3, prob.k), O.Problem(3, prob.n, prob.k, 4))
    c = np.stack([q[1] * a[2] - q[2] * a[1], q[2] * a[0] - q[0] * a[2], q[0] * a[1] - q[1] * a[0]])
    c = O.project(c, O.Problem(3, prob.n, prob.k, 4))
    ok &= np.allclose(O.project(c, prob), c, rtol=0, atol=1e-12 * np.abs(c).max())
    return ok


def pin_incompressible_gradient(O):
    """gamma = 1: the gradient is divergence-free, the reaction factor of an incompressible
    flow is 1, and central differences of E along divergence-free directions match <g, w>"""
    prob, I0 = _div_free_problem(O)
    vh = O.project(phantoms.raw_band_velocity(23, 3, prob.k), prob)
    vh *= 1.0 / O.max_displacement_voxels(vh, prob)
    I1 = np.roll(I0, 1, axis=2)
    st = O.evaluate(vh, I0, I1, prob)
    g = O.gradient(st)
    ok = np.max(np.abs(O.div_band(g, prob))) <= 1e-10 * np.abs(g).max() * 2 * np.pi * max(prob.k)
    ok &= np.max(np.abs(st.geo["a"] - 1)) < 1e-12
    for seed in (24, 25):
        w = O.project(phantoms.raw_band_velocity(seed, 3, prob.k), prob)
        w /= np.sqrt(np.vdot(w, w).real)
        eps = 1e-5
        fd = (O.evaluate(vh + eps * w, I0, I1, prob).E - O.evaluate(vh - eps * w, I0, I1, prob).E) / (2 * eps)
        ok &= abs(fd - float(np.real(np.vdot(g, w)))) <= 0.1 * abs(fd)   # the optimise-then-discretise gap is ~7% on this coarse grid
    return ok


def pin_newton_symmetric_on_permutations(O):
    nt = 8
    prob = O.Problem(2, (32, 32), (8, 8), nt, sigma=0.8)
    vh = np.zeros((2,) + prob.bshape, complex)
    vh[(0, 4, 4)] = nt / prob.nref
    vh[(1, 4, 4)] = -nt / prob.nref
    I0 = phantoms.blobs_2d(3, 32)
    st = O.evaluate(vh, I0, np.roll(I0, 2, axis=0) + 0.1, prob)
    d1, d2 = rand_band(O, prob, 11), rand_band(O, prob, 12)
    a = np.vdot(O.hessvec_newton(st, d1), d2).real
    b = np.vdot(d1, O.hessvec_newton(st, d2)).real
    return abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def pin_newton_closed_form(O):
    """v = 0: H dv = L^ dv + pi((-(2/sigma^2) f + s/2) grad I0 + (lambda/2) grad f)"""
    prob = O.Problem(3, (12, 10, 8), (4, 4, 4), 5, sigma=0.7, alpha=2e-3, s=1)
    rng = np.random.default_rng(4)
    I0, I1 = rng.standard_normal(prob.shape), rng.standard_normal(prob.shape)
    st = O.evaluate(np.zeros((3,) + prob.bshape, complex), I0, I1, prob)
    d = rand_band(O, prob, 5)
    F = np.zeros(prob.shape, complex)
    idx = np.meshgrid(*[np.mod(np.arange(K) - K // 2, N) for K, N in zip(prob.bshape, prob.shape)],
                      indexing="ij")
    dv = []
    for j in range(3):
        F[...] = 0
        F[tuple(idx)] = d[j]
        dv.append((np.fft.ifftn(F) * prob.M).real)
    gI = np_grad(I0, prob)
    c = 2.0 / prob.sigma ** 2
    lam = -c * (I0 - I1)
    f = -sum(gI[j] * dv[j] for j in range(3))
    s_ = sum(np_grad(lam * dv[j], prob)[j] for j in range(3))
    gf = np_grad(f, prob)
    ell = [N / prob.nref for N in prob.shape]
    kk = np.meshgrid(*[(np.arange(K) - K // 2) / l for K, l in zip(prob.bshape, ell)], indexing="ij")
    Lh = (1 + 4 * np.pi ** 2 * prob.alpha * sum(q ** 2 for q in kk)) ** prob.s
    ref = np.stack([Lh * d[j] + fft_pi((-c * f + 0.5 * s_) * gI[j] + 0.5 * lam * gf[j], prob)
                    for j in range(3)])
    return np.allclose(O.hessvec_newton(st, d), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def pin_ns_characteristics(O):
    """non-stationary Heun offsets of the first step against the exact flow of
    v_x(x, t) = (1 + 4t) v(x) of one Fourier mode (fine RK4): X^0 is the displacement from t_1
    back to 0, Y^0 from 0 to t_1.  Heun's local error is third order (0.1% here); a predictor
    taken with the wrong node's velocity is off by 0.4%."""
    prob = O.Problem(2, (64, 64), (8, 8), 16)
    c = 0.06 * (1.0 - 0.5j)
    V = np.zeros((prob.nt + 1, 2) + prob.bshape, complex)
    for n in range(prob.nt + 1):
        s_ = 1.0 + 4.0 * n * prob.dt
        V[n, 0, 4, 5] = s_ * c
        V[n, 0, 4, 3] = s_ * np.conj(c)
    geo = O.ns_setup(V, prob)
    v = lambda x, t: (1.0 + 4.0 * t) * 2 * np.real(c * np.exp(2j * np.pi * x))
    x0 = np.arange(64) / 64.0
    ok = True
    for key, t0, t1 in (("Y", 0.0, prob.dt), ("X", prob.dt, 0.0)):
        x, t, h = x0.copy(), t0, (t1 - t0) / 200
        for _ in range(200):
            k1 = v(x, t); k2 = v(x + h / 2 * k1, t + h / 2); k3 = v(x + h / 2 * k2, t + h / 2)
            k4 = v(x + h * k3, t + h)
            x, t = x + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4), t + h
        disp = (x - x0) * prob.nref
        ok &= np.max(np.abs(geo[key][0][0][0] - disp)) < 2e-3 * np.max(np.abs(disp))
    return ok


def pin_ns_stationary_limit(O):
    prob = O.Problem(2, (24, 20), (8, 8), 4, sigma=0.8)
    I0 = phantoms.blobs_2d(7, 24)[:20, :24]
    vh = O.project(phantoms.raw_band_velocity(1, 2, prob.k), prob)
    vh *= 1.5 / O.max_displacement_voxels(vh, prob)
    I1 = np.roll(I0, 1, axis=0)
    st, sn = O.evaluate(vh, I0, I1, prob), O.ns_evaluate(np.stack([vh] * 5), I0, I1, prob)
    w = O.trapezoid_weights(prob.nt)
    g = O.gradient(st)
    gs = sum(w[n] * O.ns_gradient(sn)[n] for n in range(5))
    d = rand_band(O, prob, 3)
    H = O.hessvec(st, d)
    Hs = sum(w[n] * O.ns_hessvec(sn, np.stack([d] * 5))[n] for n in range(5))
    return (abs(sn.E - st.E) <= 1e-12 * st.E and np.allclose(gs, g, rtol=0, atol=1e-12 * np.abs(g).max())
            and np.allclose(Hs, H, rtol=0, atol=1e-12 * np.abs(H).max()))


def pin_mse_rel(O):
    """MSE_rel (reading R-MSE) on the hand-worked 2 x 2 example (100 / 13) and exactly 100 %
    at the zero initial guess of a registration"""
    I0 = np.array([[0.5, 0.0], [1.0, 1.0]])
    I1 = np.array([[2.0, 0.0], [1.0, 0.0]])
    mT = np.array([[2.0, 0.5], [1.0, 0.0]])
    if abs(O.mse_rel(mT, I0, I1) - 100.0 / 13.0) > 1e-13:
        return False
    prob = O.Problem(2, (16, 12), (8, 4), 4)
    J0 = phantoms.blobs_2d(3, 16)[:12, :16]
    _, _, stats = O.register(J0, np.roll(J0, 1, axis=1), np.zeros((2,) + prob.bshape, complex),
                             prob, O.SolverOpts(max_gn=1, max_pcg=2))
    return abs(stats["mse_rel"][0] - 100.0) <= 4e-14


PINS = [pin_bruteforce_dft, pin_projection, pin_symbol_fd, pin_divergence, pin_roll_and_identity,
        pin_interp_half_voxel, pin_gradient_closed_form, pin_hessvec_closed_form, pin_gradient_fd,
        pin_hessvec_fd_zero_residual, pin_energy_regulariser,
        pin_incremental_adjoint_is_the_adjoint, pin_symmetry_shift, pin_characteristics, pin_solver,
        pin_incompressible_projection, pin_incompressible_gradient, pin_newton_symmetric_on_permutations,
        pin_newton_closed_form, pin_ns_characteristics, pin_ns_stationary_limit, pin_mse_rel]


def run_pins(O):
    failed = []
    for pin in PINS:
        try:
            ok = bool(pin(O))
        except Exception:
            ok = False
        if not ok:
            failed.append(pin.__name__)
    return failed


def test_pins_pass_on_the_unmodified_oracle():
    assert run_pins(load(SRC)) == []


MUTATIONS = [
    ("iota exponent sign", "E = [_emat(prob.n[j], prob.k[j], +1.0) for j in range(prob.dim)]",
     "E = [_emat(prob.n[j], prob.k[j], -1.0) for j in range(prob.dim)]"),
    ("pi without 1/M", "return zero_unpaired(out / prob.M, prob)", "return zero_unpaired(out, prob)"),
    ("projection without conj", "out[inner] = 0.5 * (w + np.conj(w[rev]))", "out[inner] = 0.5 * (w + w[rev])"),
    ("symbol 2 pi^2", "(1.0 + 4.0 * np.pi ** 2 * prob.alpha * q)", "(1.0 + 2.0 * np.pi ** 2 * prob.alpha * q)"),
    ("symbol k*l", "out.append(grids[prob.axis(j)] / lj)", "out.append(grids[prob.axis(j)] * lj)"),
    ("divergence without 2 pi", "return sum(2j * np.pi * kl[j] * vh[j] for j in range(prob.dim))",
     "return sum(1j * kl[j] * vh[j] for j in range(prob.dim))"),
    ("forward offset sign", "X = [-0.5 * (u[j] + interp(u[j], neg_u, prob)) for j in range(d)]",
     "X = [0.5 * (u[j] + interp(u[j], neg_u, prob)) for j in range(d)]"),
    ("Heun reaction without predictor", "a = 1.0 + 0.5 * prob.dt * (R + (1.0 + prob.dt * R) * r)",
     "a = 1.0 + 0.5 * prob.dt * (R + r)"),
    ("reaction sign", "a = 1.0 + 0.5 * prob.dt * (R + (1.0 + prob.dt * R) * r)",
     "a = 1.0 - 0.5 * prob.dt * (R + (1.0 + prob.dt * R) * r)"),
    ("interpolation weights swapped", "w = w * (frac[a] if corner[a] else 1.0 - frac[a])",
     "w = w * (1.0 - frac[a] if corner[a] else frac[a])"),
    ("central difference scale", "* (prob.nref / 2.0))", "* prob.nref)"),
    ("adjoint final-condition sign", "lam = -(2.0 / prob.sigma ** 2) * (st.m[-1] - st.I1)",
     "lam = (2.0 / prob.sigma ** 2) * (st.m[-1] - st.I1)"),
    ("gradient end weight", "b = [w[-1] * lam * gm[j] for j in range(d)]", "b = [w[1] * lam * gm[j] for j in range(d)]"),
    ("regulariser without 1/2", "reg = 0.5 * float(np.sum(Lh[None] * np.abs(vh) ** 2))",
     "reg = float(np.sum(Lh[None] * np.abs(vh) ** 2))"),
    ("incremental source dropped at n+1", "dm = interp(dm + 0.5 * dt * fn, X, prob) + 0.5 * dt * fn1",
     "dm = interp(dm + 0.5 * dt * fn, X, prob)"),
    ("incremental adjoint without reaction", "dlam = st.geo[\"a\"] * interp(dlam, st.geo[\"Y\"], prob)",
     "dlam = interp(dlam, st.geo[\"Y\"], prob)"),
    ("incremental adjoint wrong characteristic", "dlam = st.geo[\"a\"] * interp(dlam, st.geo[\"Y\"], prob)",
     "dlam = st.geo[\"a\"] * interp(dlam, st.geo[\"X\"], prob)"),
    ("Hessian regulariser missing", "np.stack([Lh * dvh[j] + pi_(Hb[j], prob) for j in range(d)])",
     "np.stack([pi_(Hb[j], prob) for j in range(d)])"),
    ("incompressible projection sign", "return np.stack([vh[j] - q[j] * s * inv for j in range(prob.dim)])",
     "return np.stack([vh[j] + q[j] * s * inv for j in range(prob.dim)])"),
    ("incompressible projection ignores the axis lengths", "q = [2.0 * np.pi * x for x in _kl(prob)]",
     "q = [2.0 * np.pi * x * (prob.n[j] / prob.nref) for j, x in enumerate(_kl(prob))]"),
    ("incompressible gradient not projected", "return leray(g, prob) if prob.gamma == 1 else g",
     "return g"),
    ("update sign", "st_try = evaluate(vh + eps * delta, I0, I1, prob)",
     "st_try = evaluate(vh - eps * delta, I0, I1, prob)"),
    ("trapezoid end weight not halved", "    w[0] *= 0.5\n", "    w[0] *= 1.0\n"),
    ("state along the backward characteristic", "m.append(interp(m[-1], X, prob))",
     "m.append(interp(m[-1], [-x for x in X], prob))"),
    ("backward offset predictor at the wrong point", "Y = [0.5 * (u[j] + interp(u[j], u, prob)) for j in range(d)]",
     "Y = [0.5 * (u[j] + interp(u[j], neg_u, prob)) for j in range(d)]"),
    ("Newton source sign", "src = [div_c([lam[n] * dv[j] for j in range(d)], prob) for n in range(prob.nt + 1)]",
     "src = [-div_c([lam[n] * dv[j] for j in range(d)], prob) for n in range(prob.nt + 1)]"),
    ("Newton drops lambda grad dm", "Hb[j] += w[n] * (dlam * gm[j] + lam[n] * gdm[j])",
     "Hb[j] += w[n] * (dlam * gm[j])"),
    ("Newton source half weights at both ends",
     "q = a * interp(q + 0.5 * dt * src[n + 1], Y, prob) + (0.5 * dt * src[n] if n > 0 else 0.0)",
     "q = a * interp(q + 0.5 * dt * src[n + 1], Y, prob) + 0.5 * dt * src[n]"),
    ("central divergence sign", "out += (np.roll(u[j], -1, axis=ax) - np.roll(u[j], 1, axis=ax)) * (prob.nref / 2.0)",
     "out += (np.roll(u[j], 1, axis=ax) - np.roll(u[j], -1, axis=ax)) * (prob.nref / 2.0)"),
    ("non-stationary predictor velocity swapped",
     "X.append([-0.5 * (u[n + 1][j] + interp(u[n][j], back, prob)) for j in range(d)])",
     "X.append([-0.5 * (u[n][j] + interp(u[n + 1][j], back, prob)) for j in range(d)])"),
    ("non-stationary regulariser without time weights",
     "reg = 0.5 * sum(w[n] * float(np.sum(Lh[None] * np.abs(geo[\"vh\"][n]) ** 2))",
     "reg = 0.5 * sum(float(np.sum(Lh[None] * np.abs(geo[\"vh\"][n]) ** 2))"),
    ("preconditioner inverted", "z = r / Lh[None]\n        p = z.copy()", "z = r * Lh[None]\n        p = z.copy()"),
    ("MSE_rel over |I1|^2", "den = float(np.sum((np.asarray(I0, np.float64) - I1) ** 2))",
     "den = float(np.sum(np.asarray(I1, np.float64) ** 2))"),
    ("MSE_rel over |I0|^2", "den = float(np.sum((np.asarray(I0, np.float64) - I1) ** 2))",
     "den = float(np.sum(np.asarray(I0, np.float64) ** 2))"),
    ("MSE_rel without the percent factor", "return 100.0 * num / den if den > 0 else 0.0",
     "return num / den if den > 0 else 0.0"),
    ("MSE_rel residual against the source", "num = float(np.sum((np.asarray(mT, np.float64) - I1) ** 2))",
     "num = float(np.sum((np.asarray(mT, np.float64) - I0) ** 2))"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new):
    assert SRC.count(old) >= 1, f"mutation anchor not found: {name}"
    failed = run_pins(load(SRC.replace(old, new, 1)))
    assert failed, f"no pin caught the mutation '{name}'"
