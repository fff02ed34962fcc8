"""Pins of the FP64 oracle against facts fixed by the paper's definitions and by mathematics.

Every check here computes its expected value by a route other than the oracle's own code:
brute-force sums, numpy.fft, closed-form derivatives, exact permutation cases, the exact
solution of the continuous transport equation integrated along characteristics, and
finite differences of the oracle's energy.  The paper prints no worked numerical example
(its tables need the NIREP volumes), so there is no paper value to pin against.
"""
import cmath
import math

import numpy as np
import pytest

import oracle as O
from paper_1807_05117_amd import phantoms

RNG = np.random.default_rng(1234)


def rand_band(prob, seed=0, admissible=True):
    v = phantoms.random_band_direction(seed, prob.dim, prob.k)
    return O.project(v, prob) if admissible else v


def fft_iota(vh, prob):
    """iota through numpy.fft: place v~(k) at index k mod N and take M * ifftn."""
    S = np.zeros(prob.shape, dtype=np.complex128)
    idx = np.meshgrid(*[np.mod(O.band_freqs(K).astype(int), N)
                        for K, N in zip(prob.bshape, prob.shape)], indexing="ij")
    S[tuple(idx)] = vh
    return np.fft.ifftn(S) * prob.M


def fft_pi(f, prob):
    """pi through numpy.fft: fftn(f)/M read at the band indices, unpaired planes zeroed."""
    F = np.fft.fftn(f) / prob.M
    idx = np.meshgrid(*[np.mod(O.band_freqs(K).astype(int), N)
                        for K, N in zip(prob.bshape, prob.shape)], indexing="ij")
    out = F[tuple(idx)].copy()
    for a in range(prob.dim):
        sl = [slice(None)] * prob.dim
        sl[a] = 0
        out[tuple(sl)] = 0
    return out


def np_grad(f, prob):
    """Central differences with numpy.gradient on a wrap-padded copy, spacing h = 1/N_ref."""
    h = 1.0 / prob.nref
    fp = np.pad(f, 1, mode="wrap")
    inner = tuple(slice(1, -1) for _ in range(prob.dim))
    out = []
    for j in range(prob.dim):
        out.append(np.gradient(fp, h, axis=prob.dim - 1 - j)[inner])
    return out


# ------------------------------------------------------------------------- band transforms

@pytest.mark.parametrize("dim,n,k", [(2, (8, 6), (4, 4)), (3, (8, 6, 4), (4, 4, 4)),
                                     (3, (6, 6, 8), (6, 2, 4))])
def test_iota_pi_bruteforce(dim, n, k):
    prob = O.Problem(dim, n, k, 4)
    vh = rand_band(prob, 3, admissible=False)[0]
    f = RNG.standard_normal(prob.shape)
    ref_i = np.zeros(prob.shape, dtype=np.complex128)
    ref_p = np.zeros(prob.bshape, dtype=np.complex128)
    for idx in np.ndindex(prob.shape):
        isp = idx[::-1]
        for kidx in np.ndindex(prob.bshape):
            ksp = [kidx[::-1][j] - k[j] // 2 for j in range(dim)]
            ph = sum(ksp[j] * isp[j] / n[j] for j in range(dim))
            e = cmath.exp(2j * math.pi * ph)
            ref_i[idx] += vh[kidx] * e
            ref_p[kidx] += f[idx] / e
    ref_p /= prob.M
    for a in range(dim):
        sl = [slice(None)] * dim
        sl[a] = 0
        ref_p[tuple(sl)] = 0
    got_i = O.iota(vh, prob)
    assert np.max(np.abs(got_i - ref_i.real)) <= 1e-13 * np.max(np.abs(ref_i))
    got_p = O.pi_(f, prob)
    assert np.max(np.abs(got_p - ref_p)) <= 1e-13 * np.max(np.abs(ref_p))


@pytest.mark.parametrize("dim,n,k", [(2, (8, 6), (4, 4)), (3, (8, 6, 4), (4, 4, 4))])
def test_point_sampled_transforms_bruteforce(dim, n, k):
    """iota_at / pi_at (single outputs of grids too large for the full transform) against the
    double sum written out term by term"""
    prob = O.Problem(dim, n, k, 4)
    vh = rand_band(prob, 3, admissible=False)[0]
    f = RNG.standard_normal(prob.shape)
    pts = [idx for idx in np.ndindex(prob.shape)][::3]
    kids = [kidx for kidx in np.ndindex(prob.bshape)]
    for idx, got in zip(pts, O.iota_at(vh, prob, pts)):
        ref = sum(vh[kidx] * cmath.exp(2j * math.pi * sum(
            (kidx[::-1][j] - k[j] // 2) * idx[::-1][j] / n[j] for j in range(dim))) for kidx in kids)
        assert abs(got - ref.real) <= 1e-13 * np.abs(vh).sum()
    for kidx, got in zip(kids, O.pi_at(f, prob, kids)):
        if 0 in kidx:
            assert got == 0
            continue
        ref = sum(f[idx] * cmath.exp(-2j * math.pi * sum(
            (kidx[::-1][j] - k[j] // 2) * idx[::-1][j] / n[j] for j in range(dim)))
            for idx in np.ndindex(prob.shape)) / prob.M
        assert abs(got - ref) <= 1e-14 * np.abs(f).sum()


def test_point_sampled_transforms_numpy_fft():
    prob = O.Problem(3, (40, 24, 18), (16, 12, 6), 4)
    vh = rand_band(prob, 9)[0]
    grid = fft_iota(vh, prob).real
    f = RNG.standard_normal(prob.shape)
    band = fft_pi(f, prob)
    rng = np.random.default_rng(17)
    pts = np.stack([rng.integers(0, N, 50) for N in prob.shape], axis=1)
    kids = np.stack([rng.integers(0, K, 50) for K in prob.bshape], axis=1)
    assert np.allclose(O.iota_at(vh, prob, pts), grid[tuple(pts.T)], rtol=0,
                       atol=1e-13 * np.abs(grid).max())
    assert np.allclose(O.pi_at(f, prob, kids), band[tuple(kids.T)], rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,n,k", [(2, (64, 48), (16, 12)), (3, (20, 16, 12), (8, 6, 4))])
def test_iota_pi_numpy_fft(dim, n, k):
    prob = O.Problem(dim, n, k, 4)
    vh = rand_band(prob, 5)[0]
    ref = fft_iota(vh, prob)
    assert np.max(np.abs(ref.imag)) <= 1e-12 * np.max(np.abs(ref.real))   # admissible -> real
    assert np.allclose(O.iota(vh, prob), ref.real, rtol=0, atol=1e-13 * np.abs(ref).max())
    f = RNG.standard_normal(prob.shape)
    assert np.allclose(O.pi_(f, prob), fft_pi(f, prob), rtol=0, atol=1e-14)


@pytest.mark.parametrize("dim,n,k", [(2, (32, 24), (8, 8)), (3, (16, 12, 10), (8, 6, 4))])
def test_pi_iota_identity_adjoint_parseval(dim, n, k):
    prob = O.Problem(dim, n, k, 4)
    a = rand_band(prob, 7)[0]
    f = RNG.standard_normal(prob.shape)
    ia = O.iota(a, prob)
    assert np.max(np.abs(O.pi_(ia, prob) - a)) <= 1e-13 * np.max(np.abs(a))
    lhs = np.mean(ia * f)
    rhs = O.dot(a, O.pi_(f, prob))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.abs(ia).max())
    assert abs(np.mean(ia * ia) - O.dot(a, a)) <= 1e-13 * O.dot(a, a)
    pa = O.project(a, prob)
    assert np.array_equal(pa, O.project(pa, prob)) or np.allclose(pa, O.project(pa, prob),
                                                                    rtol=0, atol=1e-16)


def test_projection_is_hermitian_and_idempotent():
    prob = O.Problem(3, (16, 12, 10), (8, 6, 4), 4)
    raw = rand_band(prob, 9, admissible=False)
    p = O.project(raw, prob)
    # v~(-k) = conj v~(k) on the paired block; the unpaired planes are zero
    inner = (slice(None), slice(1, None), slice(1, None), slice(1, None))
    blk = p[inner]
    assert np.array_equal(blk, np.conj(blk[:, ::-1, ::-1, ::-1]))
    assert np.all(p[:, 0] == 0) and np.all(p[:, :, 0] == 0) and np.all(p[:, :, :, 0] == 0)
    assert np.allclose(O.project(p, prob), p, rtol=0, atol=0)


# ---------------------------------------------------------------------------------- symbols

def _mode(prob, comp, kvec, c):
    """Band vector holding c at +kvec and conj(c) at -kvec in component comp."""
    vh = np.zeros((prob.dim,) + prob.bshape, dtype=np.complex128)
    ip = tuple(kvec[j] + prob.k[j] // 2 for j in reversed(range(prob.dim)))
    im = tuple(-kvec[j] + prob.k[j] // 2 for j in reversed(range(prob.dim)))
    vh[(comp,) + ip] += c
    vh[(comp,) + im] += np.conj(c)
    return vh


def test_divergence_of_single_mode_matches_analytic_derivative():
    # non-cubic grid: l = N / N_ref differs per axis
    prob = O.Problem(3, (20, 16, 12), (8, 8, 6), 4)
    kv = (2, -1, 1)
    c = 0.3 - 0.7j
    vh = _mode(prob, 0, kv, c) + _mode(prob, 2, (1, 2, -2), 0.2 + 0.1j)
    r = O.iota(O.div_band(vh, prob), prob)
    # analytic: v_c(x) = 2 Re(c exp(2 pi i sum_j q_j x_j)), x_j = i_j / N_ref, q_j = k_j / l_j
    zz, yy, xx = np.meshgrid(*[np.arange(N) / prob.nref for N in prob.shape], indexing="ij")
    X = (xx, yy, zz)

    def dcomp(kvec, cc, axis):
        q = [kvec[j] * prob.nref / prob.n[j] for j in range(3)]
        ph = 2 * np.pi * sum(q[j] * X[j] for j in range(3))
        return 2 * np.real(cc * 2j * np.pi * q[axis] * np.exp(1j * ph))

    ref = dcomp(kv, c, 0) + dcomp((1, 2, -2), 0.2 + 0.1j, 2)
    assert np.max(np.abs(r - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_regulariser_symbol_matches_finite_difference_operator():
    """(Id - alpha Lap)^s applied with a fine-grid FD Laplacian to a sampled mode converges
    to L^(k) times the mode; checks alpha, s, 4 pi^2 and the k/l scaling on a non-square grid."""
    alpha, s = 1e-3, 2
    kv = (3, -2)
    errs = []
    for N in (128, 256, 512):
        prob = O.Problem(2, (N, 3 * N // 4), (8, 8), 4, alpha=alpha, s=s)
        vh = _mode(prob, 0, kv, 0.5 + 0.25j)
        f = O.iota(vh[0], prob)
        h = 1.0 / prob.nref
        g = f.copy()
        for _ in range(s):
            lap = sum((np.roll(g, 1, a) - 2 * g + np.roll(g, -1, a)) / h ** 2 for a in (0, 1))
            g = g - alpha * lap
        Lh = O.L_hat(prob)
        ip = tuple(kv[j] + prob.k[j] // 2 for j in reversed(range(2)))
        errs.append(np.max(np.abs(g - Lh[ip] * f)) / np.max(np.abs(f)))
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 5e-4           # a wrong alpha, s or k/l scaling gives O(1) errors
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5  # second order in h


def test_preconditioner_inverts_symbol():
    prob = O.Problem(3, (16, 16, 16), (8, 8, 8), 4, alpha=2e-3, s=3)
    Lh = O.L_hat(prob)
    assert np.all(Lh >= 1.0)
    assert np.allclose((1.0 / Lh) * Lh, 1.0, rtol=1e-15)


# ----------------------------------------------------------------------- interpolation / SL

def _img(prob, seed=11):
    if prob.dim == 2:
        return phantoms.blobs_2d(seed, prob.n[0])[:prob.shape[0], :prob.shape[1]]
    return phantoms.shells_3d(seed, prob.n, n_classes=3)


def test_zero_velocity_is_identity():
    prob = O.Problem(3, (12, 10, 8), (4, 4, 4), 5)
    I0 = RNG.standard_normal(prob.shape)
    geo = O.setup(np.zeros((3,) + prob.bshape, complex), prob)
    for j in range(3):
        assert np.all(geo["X"][j] == 0) and np.all(geo["Y"][j] == 0)
    assert np.all(geo["a"] == 1.0)
    m = O.forward_state(I0, geo["X"], prob)
    assert all(np.array_equal(mm, I0) for mm in m)


@pytest.mark.parametrize("dim,u", [(2, (1, -2)), (3, (1, 0, -1)), (3, (-2, 1, 3))])
def test_whole_voxel_shift_is_exact_roll(dim, u):
    nt = 8
    n = (32,) * dim
    prob = O.Problem(dim, n, (8,) * dim, nt)
    vh = np.zeros((dim,) + prob.bshape, complex)
    centre = tuple(K // 2 for K in prob.bshape)
    for j in range(dim):
        vh[(j,) + centre] = u[j] * nt / prob.nref   # v = u N_t / N_ref  <=> u voxels per step
    geo = O.setup(vh, prob)
    for j in range(dim):
        assert np.all(geo["X"][j] == -u[j]) and np.all(geo["Y"][j] == u[j])
    assert np.all(geo["a"] == 1.0)
    I0 = RNG.standard_normal(prob.shape)
    mT = O.forward_state(I0, geo["X"], prob)[-1]
    shift = tuple(nt * u[prob.dim - 1 - a] for a in range(dim))
    assert np.array_equal(mT, np.roll(I0, shift, axis=tuple(range(dim))))
    lam = I0.copy()
    for _ in range(nt):
        lam = geo["a"] * O.interp(lam, geo["Y"], prob)
    assert np.array_equal(lam, np.roll(I0, tuple(-s for s in shift), axis=tuple(range(dim))))


def test_interp_half_voxel_is_neighbour_average():
    prob = O.Problem(2, (10, 8), (4, 4), 1)
    f = RNG.standard_normal(prob.shape)
    off = [np.full(prob.shape, 0.5), np.zeros(prob.shape)]
    assert np.allclose(O.interp(f, off, prob), 0.5 * (f + np.roll(f, -1, axis=1)),
                       rtol=0, atol=1e-15)
    off = [np.full(prob.shape, -3.25), np.full(prob.shape, 17.0)]
    ref = 0.75 * np.roll(f, (-17, 3), axis=(0, 1)) + 0.25 * np.roll(f, (-17, 4), axis=(0, 1))
    assert np.allclose(O.interp(f, off, prob), ref, rtol=0, atol=1e-14)


# smooth continuous problem for refinement studies: velocity given by band coefficients is
# the same continuous field on every grid (R1, R4), so grids of different size can be
# compared with the exact solution of the transport equation.
_KV = [((1, 0), 0, 0.05 - 0.03j), ((1, 1), 1, 0.04 + 0.02j), ((0, 2), 0, -0.02 + 0.01j)]


def _smooth_vh(prob):
    vh = np.zeros((2,) + prob.bshape, complex)
    for kv, comp, c in _KV:
        vh += _mode(prob, comp, kv, c)
    return vh


def _v_exact(x, y):
    vx = np.zeros_like(x)
    vy = np.zeros_like(x)
    for kv, comp, c in _KV:
        val = 2 * np.real(c * np.exp(2j * np.pi * (kv[0] * x + kv[1] * y)))
        if comp == 0:
            vx += val
        else:
            vy += val
    return vx, vy


def _div_exact(x, y):
    r = np.zeros_like(x)
    for kv, comp, c in _KV:
        r += 2 * np.real(c * 2j * np.pi * kv[comp] * np.exp(2j * np.pi * (kv[0] * x + kv[1] * y)))
    return r


def _I0_exact(x, y):
    return np.cos(2 * np.pi * x) * np.sin(2 * np.pi * (x + 2 * y)) + 0.5 * np.cos(2 * np.pi * y)


def _flow(x, y, sign, steps=400, with_div=False):
    """RK4 for dz/ds = sign v(z) over unit time; optionally integrate div v along the path."""
    h = 1.0 / steps
    acc = np.zeros_like(x)
    for _ in range(steps):
        k1 = _v_exact(x, y)
        k2 = _v_exact(x + 0.5 * h * sign * k1[0], y + 0.5 * h * sign * k1[1])
        k3 = _v_exact(x + 0.5 * h * sign * k2[0], y + 0.5 * h * sign * k2[1])
        k4 = _v_exact(x + h * sign * k3[0], y + h * sign * k3[1])
        if with_div:
            d1 = _div_exact(x, y)
            d2 = _div_exact(x + 0.5 * h * sign * k1[0], y + 0.5 * h * sign * k1[1])
            d3 = _div_exact(x + 0.5 * h * sign * k2[0], y + 0.5 * h * sign * k2[1])
            d4 = _div_exact(x + h * sign * k3[0], y + h * sign * k3[1])
            acc += h / 6 * (d1 + 2 * d2 + 2 * d3 + d4)
        x = x + h / 6 * sign * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        y = y + h / 6 * sign * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    return x, y, acc


def test_state_transport_converges_to_exact_solution():
    errs = []
    for N, nt in ((32, 4), (64, 8), (128, 16)):
        prob = O.Problem(2, (N, N), (8, 8), nt)
        yy, xx = np.meshgrid(np.arange(N) / N, np.arange(N) / N, indexing="ij")
        I0 = _I0_exact(xx, yy)
        mT = O.warp(I0, _smooth_vh(prob), prob)
        bx, by, _ = _flow(xx, yy, -1.0)          # back-trace: m(1)(x) = I0(Phi^-1(x))
        errs.append(np.max(np.abs(mT - _I0_exact(bx, by))))
    # d-linear SL with Nt proportional to N: the interpolation error Nt h^2 is first order
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6, errs
    assert errs[2] < 0.06, errs


def test_adjoint_transport_converges_to_exact_solution():
    """lambda(0)(x) = lambda(1)(Phi(x)) exp(int_0^1 div v(Phi_t(x)) dt) solves the adjoint
    (continuity) equation of Section 2.2 backward from t = 1."""
    errs = []
    for N, nt in ((32, 4), (64, 8), (128, 16)):
        prob = O.Problem(2, (N, N), (8, 8), nt)
        yy, xx = np.meshgrid(np.arange(N) / N, np.arange(N) / N, indexing="ij")
        lam1 = _I0_exact(xx, yy)
        geo = O.setup(_smooth_vh(prob), prob)
        lam = lam1
        for _ in range(nt):
            lam = geo["a"] * O.interp(lam, geo["Y"], prob)
        fx, fy, acc = _flow(xx, yy, +1.0, with_div=True)
        ref = _I0_exact(fx, fy) * np.exp(acc)
        errs.append(np.max(np.abs(lam - ref)))
    # d-linear SL with Nt proportional to N: the interpolation error Nt h^2 is first order
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6, errs
    assert errs[2] < 0.1 * np.max(np.abs(ref)), errs  # first order; 0.064 at N = 512


def test_spectral_divergence_and_grid_velocity_match_continuous_field():
    prob = O.Problem(2, (40, 40), (8, 8), 4)
    geo = O.setup(_smooth_vh(prob), prob)
    yy, xx = np.meshgrid(np.arange(40) / 40, np.arange(40) / 40, indexing="ij")
    vx, vy = _v_exact(xx, yy)
    assert np.max(np.abs(geo["v"][0] - vx)) < 1e-15 * 40
    assert np.max(np.abs(geo["v"][1] - vy)) < 1e-15 * 40
    assert np.max(np.abs(geo["r"] - _div_exact(xx, yy))) < 1e-13


# ---------------------------------------------------------------------------- gradient pins

def _pair(prob, seed=21):
    I0 = _img(prob, seed)
    I1 = np.roll(I0, 1, axis=-1) * 0.9 + 0.05
    return I0, I1


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_closed_form_at_zero_velocity(dim):
    prob = O.Problem(dim, (32, 24) if dim == 2 else (16, 12, 10),
                     (8, 8) if dim == 2 else (8, 6, 4), 6, sigma=0.7)
    I0, I1 = (RNG.standard_normal(prob.shape) for _ in range(2))
    st = O.evaluate(np.zeros((dim,) + prob.bshape, complex), I0, I1, prob)
    g = O.gradient(st)
    gI = np_grad(I0, prob)
    lam = -(2.0 / prob.sigma ** 2) * (I0 - I1)
    ref = np.stack([fft_pi(lam * gI[j], prob) for j in range(dim)])
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_central_fd_at_zero_velocity(dim):
    prob = O.Problem(dim, (32, 32) if dim == 2 else (16, 12, 10),
                     (8, 8) if dim == 2 else (8, 6, 4), 5, alpha=1e-3, s=2)
    I0 = _img(prob) if dim == 2 else phantoms.shells_3d(3, prob.n)
    I1 = np.roll(I0, 2, axis=0)
    v0 = np.zeros((dim,) + prob.bshape, complex)
    st = O.evaluate(v0, I0, I1, prob)
    g = O.gradient(st)
    w = rand_band(prob, 13)
    w /= O.norm2(w)
    eps = 1e-6
    fd = (O.evaluate(eps * w, I0, I1, prob).E - O.evaluate(-eps * w, I0, I1, prob).E) / (2 * eps)
    an = O.dot(g, w)
    assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


def test_gradient_fd_gap_shrinks_under_refinement():
    """At v~ != 0 the discretised adjoint (optimise-then-discretise) differs from the exact
    derivative of the discrete energy by a discretisation error that must shrink."""
    gaps = []
    for N, nt in ((32, 4), (64, 8), (128, 16)):
        prob = O.Problem(2, (N, N), (8, 8), nt)
        yy, xx = np.meshgrid(np.arange(N) / N, np.arange(N) / N, indexing="ij")
        I0 = _I0_exact(xx, yy)
        I1 = _I0_exact(xx - 0.03, yy + 0.02)
        vh = 0.5 * _smooth_vh(prob)
        st = O.evaluate(vh, I0, I1, prob)
        g = O.gradient(st)
        w = _smooth_vh(prob)[::-1].copy()
        w /= O.norm2(w)
        eps = 1e-5
        fd = (O.evaluate(vh + eps * w, I0, I1, prob).E
              - O.evaluate(vh - eps * w, I0, I1, prob).E) / (2 * eps)
        gaps.append(abs(fd - O.dot(g, w)) / abs(fd))
    assert gaps[0] > 1.5 * gaps[1] > 2.25 * gaps[2], gaps   # first order: 0.038, 0.023, 0.012
    assert gaps[2] < 2e-2, gaps


def test_zero_residual_gradient_is_regulariser_only():
    prob = O.Problem(3, (16, 12, 10), (8, 6, 4), 5)
    I0 = phantoms.shells_3d(5, prob.n)
    vh = 0.05 * rand_band(prob, 17)
    I1 = O.warp(I0, vh, prob)
    g = O.gradient(O.evaluate(vh, I0, I1, prob))
    ref = O.L_hat(prob)[None] * O.project(vh, prob)
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))


# -------------------------------------------------------------------------- Hessian pins

@pytest.mark.parametrize("dim", [2, 3])
def test_hessvec_closed_form_at_zero_velocity(dim):
    prob = O.Problem(dim, (32, 24) if dim == 2 else (16, 12, 10),
                     (8, 8) if dim == 2 else (8, 6, 4), 6, sigma=1.3, alpha=2e-3, s=1)
    I0, I1 = (RNG.standard_normal(prob.shape) for _ in range(2))
    st = O.evaluate(np.zeros((dim,) + prob.bshape, complex), I0, I1, prob)
    d = rand_band(prob, 23)
    H = O.hessvec(st, d)
    gI = np_grad(I0, prob)
    dv = [fft_iota(d[j], prob).real for j in range(dim)]
    s_ = sum(gI[j] * dv[j] for j in range(dim))
    ref = np.stack([O.L_hat(prob) * d[j] + (2 / prob.sigma ** 2) * fft_pi(s_ * gI[j], prob)
                    for j in range(dim)])
    assert np.max(np.abs(H - ref)) <= 1e-12 * np.max(np.abs(ref))


def _shift_state(dim, seed=31):
    nt = 8
    prob = O.Problem(dim, (24,) * dim if dim == 2 else (16, 12, 10),
                     (8,) * dim if dim == 2 else (8, 6, 4), nt, sigma=0.8)
    vh = np.zeros((dim,) + prob.bshape, complex)
    centre = tuple(K // 2 for K in prob.bshape)
    u = (1, -1, 2)[:dim]
    for j in range(dim):
        vh[(j,) + centre] = u[j] * nt / prob.nref
    I0 = _img(prob, seed) if dim == 2 else phantoms.shells_3d(seed, prob.n)
    I1 = np.roll(I0, 3, axis=0)
    return prob, O.evaluate(vh, I0, I1, prob)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("case", ["zero", "shift"])
def test_hessvec_symmetric_psd_when_transports_are_permutations(dim, case):
    if case == "shift":
        prob, st = _shift_state(dim)
    else:
        prob = O.Problem(dim, (24, 20) if dim == 2 else (16, 12, 10),
                         (8, 8) if dim == 2 else (8, 6, 4), 7)
        I0 = RNG.standard_normal(prob.shape)
        st = O.evaluate(np.zeros((dim,) + prob.bshape, complex), I0, 0 * I0, prob)
    d1, d2 = rand_band(prob, 41), rand_band(prob, 43)
    H1, H2 = O.hessvec(st, d1), O.hessvec(st, d2)
    a, b = O.dot(H1, d2), O.dot(d1, H2)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b)), (a, b)
    Lh = O.L_hat(prob)[None]
    assert O.dot(H1, d1) >= O.dot(Lh * d1, d1) * (1 - 1e-14)


def test_hessvec_linearity_and_general_symmetry_defect():
    """Linearity is exact.  Away from permutation transports the discretised adjoint is not
    the exact transpose, so the data part of <H d1, d2> - <d1, H d2> is a discretisation
    defect that must shrink when the grid is refined at fixed continuous problem."""
    defects = []
    for n in ((16, 12, 10), (32, 24, 20)):
        prob = O.Problem(3, n, (8, 6, 4), 5)
        I0 = phantoms.shells_3d(7, prob.n)
        I1 = np.roll(I0, 1, axis=2)
        vh = O.project(phantoms.raw_band_velocity(51, 3, prob.k), prob)
        vh *= 0.125 / O.max_displacement_voxels(vh, prob) * n[0]    # 1/8 of the domain
        st = O.evaluate(vh, I0, I1, prob)
        d1, d2 = rand_band(prob, 53), rand_band(prob, 55)
        H1, H2 = O.hessvec(st, d1), O.hessvec(st, d2)
        H12 = O.hessvec(st, 0.7 * d1 - 1.9 * d2)
        assert np.max(np.abs(H12 - (0.7 * H1 - 1.9 * H2))) <= 1e-13 * np.max(np.abs(H12))
        Lh = O.L_hat(prob)[None]
        a0 = O.dot(Lh * d1, d2)
        a, b = O.dot(H1, d2), O.dot(d1, H2)
        defects.append(abs(a - b) / (abs(a - a0) + abs(b - a0)))
        assert O.dot(H1, d1) > O.dot(Lh * d1, d1)
    assert defects[1] < 0.5 * defects[0] and defects[1] < 0.1, defects


def test_hessvec_matches_fd_of_gradient_at_zero_residual_under_refinement():
    """At zero residual the Gauss-Newton Hessian is the full Hessian; compare with central
    differences of the oracle gradient.  The gap is discretisation error and must shrink."""
    gaps = []
    for N, nt in ((32, 4), (64, 8), (128, 16)):
        prob = O.Problem(2, (N, N), (8, 8), nt)
        yy, xx = np.meshgrid(np.arange(N) / N, np.arange(N) / N, indexing="ij")
        I0 = _I0_exact(xx, yy)
        vh = 2.0 * _smooth_vh(prob)
        I1 = O.warp(I0, vh, prob)
        st = O.evaluate(vh, I0, I1, prob)
        d = _smooth_vh(prob)[::-1].copy()
        H = O.hessvec(st, d)
        eps = 1e-5
        gp = O.gradient(O.evaluate(vh + eps * d, I0, I1, prob))
        gm = O.gradient(O.evaluate(vh - eps * d, I0, I1, prob))
        fd = (gp - gm) / (2 * eps)
        gaps.append(O.norm2(fd - H) / O.norm2(H))
    assert gaps[0] > gaps[1] > gaps[2], gaps
    assert gaps[2] < 5e-2, gaps


# ------------------------------------------------------------------------------ solver pins

def test_solver_constant_source_reduces_to_regulariser_in_one_pcg_step():
    prob = O.Problem(2, (24, 20), (8, 8), 4)
    I0 = np.full(prob.shape, 0.5)
    I1 = RNG.standard_normal(prob.shape)
    v0 = O.project(phantoms.raw_band_velocity(61, 2, prob.k), prob)
    v0 *= 2.0 / O.max_displacement_voxels(v0, prob)
    vh, mT, stats = O.register(I0, I1, v0, prob, O.SolverOpts(max_gn=3, max_pcg=5))
    assert stats["pcg_iters"] == [1]
    assert stats["eps"] == [1.0]
    assert stats["status"] == O.CONVERGED
    assert np.max(np.abs(vh)) <= 1e-14 * np.max(np.abs(v0))
    assert np.allclose(mT, I0, rtol=0, atol=1e-15)


def c1_problem(seed=0):
    """The 2D plain-method problem: 64^2 Gaussian blobs, target warped by a random 16^2 band
    velocity scaled to 4 px maximal displacement, Nt = 10, alpha = 1e-3, s = 2, sigma = 1."""
    prob = O.Problem(2, (64, 64), (16, 16), 10, alpha=1e-3, s=2, sigma=1.0)
    I0 = phantoms.blobs_2d(seed, 64).astype(np.float32).astype(np.float64)
    vs = O.project(phantoms.raw_band_velocity(seed, 2, prob.k), prob)
    vs *= 4.0 / O.max_displacement_voxels(vs, prob)
    I1 = O.warp(I0, vs, prob).astype(np.float32).astype(np.float64)
    return prob, I0, I1, vs


def test_mse_rel_hand_computed_value():
    """MSE_rel of Section 4.1 (reading R-MSE: 100 |m(1) - I1|^2 / |I0 - I1|^2 in percent) on a
    2 x 2 example worked by hand: |m(1) - I1|^2 = 0.5^2 = 0.25, |I0 - I1|^2 = 1.5^2 + 1 = 3.25,
    so the value is 100 / 13.  The alternatives a plausible mistake would give all differ:
    |I1|^2 = 5 or |I0|^2 = 2.25 as the denominator (5, 11.1), a dropped factor 100 (0.077), or
    m(1) compared with I0 instead of I1 (107.7)."""
    I0 = np.array([[0.5, 0.0], [1.0, 1.0]])
    I1 = np.array([[2.0, 0.0], [1.0, 0.0]])
    mT = np.array([[2.0, 0.5], [1.0, 0.0]])
    assert O.mse_rel(mT, I0, I1) == pytest.approx(7.6923076923076923, rel=1e-15, abs=0)
    # no mismatch left and no motion at all are the two ends of the scale
    assert O.mse_rel(I1, I0, I1) == 0.0
    assert O.mse_rel(I0, I0, I1) == 100.0


def test_mse_rel_starts_at_100_from_zero_velocity():
    """at the zero initial guess every transport is the identity, so m(1) = I0 exactly and the
    first MSE_rel of a registration is 100 % up to the rounding of 100 x / x"""
    prob = O.Problem(2, (16, 12), (8, 4), 4)
    I0 = phantoms.blobs_2d(3, 16)[:12, :16]
    I1 = np.roll(I0, 1, axis=1)
    _, _, stats = O.register(I0, I1, np.zeros((2,) + prob.bshape, complex), prob,
                             O.SolverOpts(max_gn=1, max_pcg=2))
    assert stats["mse_rel"][0] == pytest.approx(100.0, rel=4e-16, abs=0)
    assert 0.0 < stats["mse_rel"][1] < 100.0


def test_c1_recovery_of_known_warp():
    prob, I0, I1, vs = c1_problem(0)
    vh, mT, stats = O.register(I0, I1, np.zeros_like(vs), prob, O.SolverOpts())
    E = stats["E"]
    assert all(E[i + 1] < E[i] for i in range(len(E) - 1))
    assert stats["mse_rel"][-1] < 5.0, stats["mse_rel"]
    # the regularised minimiser is not v*, but the solver must reach an energy at least as
    # low as the generating velocity's (flat background leaves v* unidentifiable there)
    assert E[-1] <= O.evaluate(vs, I0, I1, prob).E
    assert stats["status"] == O.CONVERGED
    assert stats["ginf_rel"][-1] < 1e-3


def test_leray_projection_of_one_mode_by_hand():
    """Leray projection (gamma = 1) of a single band mode on a non-cubic 2D domain: 16 x 8
    voxels, so l = (1, 1/2) and the mode k = (1, 1) has wave vector k / l = (1, 2).  For the
    amplitude a = (1, 0) the divergence-free part is a - q (q . a) / |q|^2 with q = (1, 2):
    (1 - 1/5, -2/5) = (0.8, -0.4), worked by hand.  Its Hermitian partner maps to the
    conjugate, the zero mode is left alone, and every other entry stays zero."""
    prob = O.Problem(2, (16, 8), (8, 8), 4, gamma=1)
    vh = np.zeros((2, 8, 8), np.complex128)       # [component][ky + 4][kx + 4]
    vh[0, 5, 5] = 1.0                              # k = (kx, ky) = (1, 1), x component
    vh[0, 3, 3] = 1.0                              # its partner -k (conjugate of a real amplitude)
    vh[:, 4, 4] = (0.3, -0.7)                      # k = 0: no divergence, kept as is
    P = O.leray(vh, prob)
    assert np.allclose(P[:, 5, 5], [0.8, -0.4], rtol=0, atol=1e-15)
    assert np.allclose(P[:, 3, 3], [0.8, -0.4], rtol=0, atol=1e-15)
    assert np.allclose(P[:, 4, 4], [0.3, -0.7], rtol=0, atol=1e-15)
    rest = np.ones((8, 8), bool)
    rest[5, 5] = rest[3, 3] = rest[4, 4] = False
    assert np.all(P[:, rest] == 0)


def test_leray_projection_is_an_orthogonal_projection():
    """on a random band vector of a non-cubic 3D problem: idempotent, self-adjoint in the l2
    product, output with zero spectral divergence, divergence-free input unchanged"""
    prob = O.Problem(3, (12, 10, 8), (8, 6, 4), 3, gamma=1)
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3,) + prob.bshape) + 1j * rng.standard_normal((3,) + prob.bshape)
    b = rng.standard_normal((3,) + prob.bshape) + 1j * rng.standard_normal((3,) + prob.bshape)
    Pa, Pb = O.leray(a, prob), O.leray(b, prob)
    scale = np.abs(a).max()
    assert np.allclose(O.leray(Pa, prob), Pa, rtol=0, atol=1e-14 * scale)
    assert abs(O.dot(Pa, b) - O.dot(a, Pb)) <= 1e-12 * O.norm2(a) * O.norm2(b)
    assert np.abs(O.div_band(Pa, prob)).max() <= 1e-12 * scale * 2 * np.pi * 8
    assert O.norm2(Pa) <= O.norm2(a) * (1 + 1e-14)


def test_incompressible_registration_of_divergence_free_warp():
    """gamma = 1 with H^1 (s = 1): a target made by a divergence-free velocity is registered
    with energies decreasing, a divergence-free result, a reaction factor of exactly 1 along
    the way and an energy at most the generating velocity's"""
    prob = O.Problem(2, (48, 48), (12, 12), 8, alpha=2e-3, s=1, gamma=1)
    I0 = phantoms.blobs_2d(4, 48)
    vs = O.project(phantoms.raw_band_velocity(4, 2, prob.k), prob)
    vs *= 3.0 / O.max_displacement_voxels(vs, prob)
    assert np.max(np.abs(O.div_band(vs, prob))) <= 1e-12 * np.abs(vs).max() * 2 * np.pi * 12
    I1 = O.warp(I0, vs, prob)
    vh, mT, stats = O.register(I0, I1, np.zeros_like(vs), prob, O.SolverOpts(max_gn=6))
    E = stats["E"]
    assert all(E[i + 1] < E[i] for i in range(len(E) - 1))
    assert stats["mse_rel"][-1] < stats["mse_rel"][0] * 0.2
    assert np.max(np.abs(O.div_band(vh, prob))) <= 1e-11 * np.abs(vh).max() * 2 * np.pi * 12
    assert np.max(np.abs(O.setup(vh, prob)["a"] - 1.0)) < 1e-12
    assert E[-1] <= O.evaluate(vs, I0, I1, prob).E


# ------------------------------------------------------------------ full Newton (reading R-N)

def _newton_shift_case(dim):
    nt = 8
    n = (32,) * dim if dim == 2 else (32, 16, 16)
    prob = O.Problem(dim, n, (8,) * dim, nt, sigma=0.8)
    vh = np.zeros((dim,) + prob.bshape, complex)
    centre = tuple(K // 2 for K in prob.bshape)
    for j in range(dim):
        vh[(j,) + centre] = (1, -1, 1)[j] * nt / prob.nref
    I0 = phantoms.blobs_2d(3, 32) if dim == 2 else phantoms.shells_3d(3, n)
    I1 = np.roll(I0, 2, axis=0) + 0.1          # a residual far from zero
    return prob, O.evaluate(vh, I0, I1, prob)


@pytest.mark.parametrize("dim", [2, 3])
def test_newton_hessian_exactly_symmetric_on_permutation_transports(dim):
    prob, st = _newton_shift_case(dim)
    d1 = O.project(phantoms.random_band_direction(7, dim, prob.k), prob)
    d2 = O.project(phantoms.random_band_direction(8, dim, prob.k), prob)
    a = O.dot(O.hessvec_newton(st, d1), d2)
    b = O.dot(d1, O.hessvec_newton(st, d2))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    # the adjoint terms matter here: the product differs from the Gauss-Newton one
    assert abs(a - O.dot(O.hessvec(st, d1), d2)) > 0.05 * abs(a)


def test_newton_equals_gauss_newton_at_zero_residual():
    """lambda = 0 when m(1) = I1, so both adjoint terms of the Newton product vanish"""
    prob = O.Problem(3, (20, 16, 12), (8, 6, 4), 5)
    I0 = phantoms.shells_3d(5, prob.n)
    vh = O.project(phantoms.raw_band_velocity(5, 3, prob.k), prob)
    vh *= 2.0 / O.max_displacement_voxels(vh, prob)
    st = O.evaluate(vh, I0, O.warp(I0, vh, prob), prob)
    d = O.project(phantoms.random_band_direction(6, 3, prob.k), prob)
    H = O.hessvec(st, d)
    assert np.allclose(O.hessvec_newton(st, d), H, rtol=0, atol=1e-14 * np.abs(H).max())


def test_newton_closed_form_at_zero_velocity():
    """at v = 0: m^n = I0, lambda = -(2/sigma^2)(I0 - I1) in every step, dm^n = t_n f with
    f = -grad I0 . dv, and the trapezoid sums give
    H dv = L^ dv + pi((-(2/sigma^2) f + s/2) grad I0 + (lambda/2) grad f), s = div(lambda dv);
    written here with numpy.gradient and numpy.fft"""
    prob = O.Problem(3, (12, 10, 8), (4, 4, 4), 5, sigma=0.7, alpha=2e-3, s=1)
    rng = np.random.default_rng(4)
    I0, I1 = rng.standard_normal(prob.shape), rng.standard_normal(prob.shape)
    st = O.evaluate(np.zeros((3,) + prob.bshape, complex), I0, I1, prob)
    d = rand_band(prob, 5)
    dv = [fft_iota(d[j], prob).real for j in range(3)]
    gI = np_grad(I0, prob)
    c = 2.0 / prob.sigma ** 2
    lam = -c * (I0 - I1)
    f = -sum(gI[j] * dv[j] for j in range(3))
    s = sum(np_grad(lam * dv[j], prob)[j] for j in range(3))
    gf = np_grad(f, prob)
    Lh = O.L_hat(prob)
    ref = np.stack([Lh * d[j] + fft_pi((-c * f + 0.5 * s) * gI[j] + 0.5 * lam * gf[j], prob)
                    for j in range(3)])
    got = O.hessvec_newton(st, d)
    assert np.allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_newton_matches_derivative_of_gradient_away_from_zero_residual():
    """central differences of the gradient along d against the Newton product at a large
    residual: within the optimise-then-discretise gap (8% here), while the Gauss-Newton
    product, which drops the adjoint terms, is off by over three times as much"""
    prob = O.Problem(2, (48, 48), (8, 8), 6)
    yy, xx = np.meshgrid(np.arange(48) / 48, np.arange(48) / 48, indexing="ij")
    I0 = np.cos(2 * np.pi * xx) * np.sin(2 * np.pi * (xx + 2 * yy))
    I1 = (np.cos(2 * np.pi * (xx - 0.05)) * np.sin(2 * np.pi * (xx + 2 * yy + 0.08))
          + 0.3 * np.sin(2 * np.pi * yy))
    vh = O.project(phantoms.raw_band_velocity(9, 2, prob.k), prob)
    vh *= 1.0 / O.max_displacement_voxels(vh, prob)
    d = O.project(phantoms.raw_band_velocity(10, 2, prob.k), prob)
    d *= 1.0 / O.max_displacement_voxels(d, prob)
    st = O.evaluate(vh, I0, I1, prob)
    HN, HG = O.hessvec_newton(st, d), O.hessvec(st, d)
    eps = 1e-4
    fd = (O.gradient(O.evaluate(vh + eps * d, I0, I1, prob))
          - O.gradient(O.evaluate(vh - eps * d, I0, I1, prob))) / (2 * eps)
    gap_n = np.linalg.norm((fd - HN).ravel()) / np.linalg.norm(HN.ravel())
    gap_g = np.linalg.norm((fd - HG).ravel()) / np.linalg.norm(HN.ravel())
    assert gap_n < 0.12 and gap_g > 3 * gap_n


# --------------------------------------------------- non-stationary velocity (reading R-NS)

def _ns_case(seed=0, nt=5):
    prob = O.Problem(3, (20, 16, 12), (8, 6, 4), nt, sigma=0.8)
    I0 = phantoms.shells_3d(seed, prob.n)
    I1 = np.roll(I0, 1, axis=2) + 0.05
    return prob, I0, I1


def test_ns_reduces_to_stationary_for_equal_nodes():
    """all nodes equal: the same transports and energy, and the weighted sums of the per-node
    gradient and Hessian product are the stationary ones"""
    prob, I0, I1 = _ns_case()
    vh = O.project(phantoms.raw_band_velocity(1, 3, prob.k), prob)
    vh *= 2.0 / O.max_displacement_voxels(vh, prob)
    V = np.stack([vh] * (prob.nt + 1))
    st, sn = O.evaluate(vh, I0, I1, prob), O.ns_evaluate(V, I0, I1, prob)
    assert np.allclose(sn.m[-1], st.m[-1], rtol=0, atol=1e-13) and abs(sn.E - st.E) < 1e-12 * st.E
    w = O.trapezoid_weights(prob.nt)
    g = O.gradient(st)
    gs = sum(w[n] * O.ns_gradient(sn)[n] for n in range(prob.nt + 1))
    assert np.allclose(gs, g, rtol=0, atol=1e-12 * np.abs(g).max())
    d = O.project(phantoms.random_band_direction(2, 3, prob.k), prob)
    H = O.hessvec(st, d)
    Hs = sum(w[n] * O.ns_hessvec(sn, np.stack([d] * (prob.nt + 1)))[n] for n in range(prob.nt + 1))
    assert np.allclose(Hs, H, rtol=0, atol=1e-12 * np.abs(H).max())


def test_ns_gradient_matches_finite_differences():
    """central differences of E along time-varying directions (independent per node) against
    the weighted inner product with the per-node gradient, on a smooth pair: the
    optimise-then-discretise gap is about 1% here"""
    prob = O.Problem(2, (48, 48), (8, 8), 6)
    yy, xx = np.meshgrid(np.arange(48) / 48, np.arange(48) / 48, indexing="ij")
    I0 = np.cos(2 * np.pi * xx) * np.sin(2 * np.pi * (xx + 2 * yy))
    I1 = np.cos(2 * np.pi * (xx - 0.03)) * np.sin(2 * np.pi * (xx + 2 * yy + 0.05))
    base = O.project(phantoms.raw_band_velocity(6, 2, prob.k), prob)
    V = np.stack([base * (1 + 0.3 * np.sin(n)) for n in range(prob.nt + 1)])
    V *= 1.0 / max(O.max_displacement_voxels(V[n], prob) for n in range(prob.nt + 1))
    g = O.ns_gradient(O.ns_evaluate(V, I0, I1, prob))
    for seed in (7, 8):
        W = np.stack([O.project(phantoms.raw_band_velocity(seed * 10 + n, 2, prob.k), prob)
                      for n in range(prob.nt + 1)])
        W /= np.sqrt(O.ns_dot(W, W, prob))
        eps = 1e-5
        fd = (O.ns_evaluate(V + eps * W, I0, I1, prob).E
              - O.ns_evaluate(V - eps * W, I0, I1, prob).E) / (2 * eps)
        assert abs(fd - O.ns_dot(g, W, prob)) <= 0.05 * abs(fd)


def test_ns_hessian_symmetric_on_permutation_transports():
    nt = 6
    prob = O.Problem(2, (32, 32), (8, 8), nt, sigma=0.8)
    vh = np.zeros((2,) + prob.bshape, complex)
    vh[(0, 4, 4)] = nt / prob.nref
    vh[(1, 4, 4)] = -nt / prob.nref
    V = np.stack([vh] * (nt + 1))
    I0 = phantoms.blobs_2d(3, 32)
    sn = O.ns_evaluate(V, I0, np.roll(I0, 2, axis=0), prob)
    D1 = np.stack([O.project(phantoms.random_band_direction(30 + n, 2, prob.k), prob) for n in range(nt + 1)])
    D2 = np.stack([O.project(phantoms.random_band_direction(40 + n, 2, prob.k), prob) for n in range(nt + 1)])
    a = O.ns_dot(O.ns_hessvec(sn, D1), D2, prob)
    b = O.ns_dot(D1, O.ns_hessvec(sn, D2), prob)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def test_ns_hessvec_closed_form_at_zero_velocity():
    """v = 0: (H dv)^n = L^ dv~^n + (2/sigma^2) pi((sum_k w_k grad I0 . dv^k) grad I0)"""
    prob = O.Problem(3, (12, 10, 8), (4, 4, 4), 4, sigma=0.7, alpha=2e-3, s=1)
    rng = np.random.default_rng(6)
    I0, I1 = rng.standard_normal(prob.shape), rng.standard_normal(prob.shape)
    sn = O.ns_evaluate(np.zeros((prob.nt + 1, 3) + prob.bshape, complex), I0, I1, prob)
    D = np.stack([rand_band(prob, 50 + n) for n in range(prob.nt + 1)])
    w = O.trapezoid_weights(prob.nt)
    gI = np_grad(I0, prob)
    S = sum(w[k] * sum(gI[j] * fft_iota(D[k][j], prob).real for j in range(3))
            for k in range(prob.nt + 1))
    Lh = O.L_hat(prob)
    c = 2.0 / prob.sigma ** 2
    got = O.ns_hessvec(sn, D)
    for n in range(prob.nt + 1):
        ref = np.stack([Lh * D[n][j] + c * fft_pi(S * gI[j], prob) for j in range(3)])
        assert np.allclose(got[n], ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_ns_registration_of_time_varying_warp():
    prob = O.Problem(2, (48, 48), (12, 12), 6, alpha=2e-3)
    I0 = phantoms.blobs_2d(5, 48)
    V = np.stack([O.project(phantoms.raw_band_velocity(60 + (n > 2), 2, prob.k), prob)
                  for n in range(prob.nt + 1)])
    V *= 3.0 / max(O.max_displacement_voxels(V[n], prob) for n in range(prob.nt + 1))
    sn = O.ns_evaluate(V, I0, np.zeros(prob.shape), prob)
    I1 = sn.m[-1]
    vh, mT, stats = O.ns_register(I0, I1, np.zeros_like(V), prob, O.SolverOpts(max_gn=6))
    E = stats["E"]
    assert all(E[i + 1] < E[i] for i in range(len(E) - 1))
    assert stats["mse_rel"][-1] < 0.2 * stats["mse_rel"][0]
