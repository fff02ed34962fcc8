"""Pins of the deformation-state oracle, written as functions of the oracle module so that the
mutation check can run them on planted-mistake copies.  Expected values come from routes other
than the oracle's code: the double sum that defines the truncated convolution, the exact
inverse flow of an analytic velocity integrated along its characteristics, closed forms for
constant and zero velocities through numpy.fft and numpy.gradient, exact symmetry of a
Gauss-Newton Hessian, and finite differences of the oracle's own energy and gradient.

Each check returns an error (or defect) measure; the callers hold it to a bound."""
import numpy as np

import oracle.bl_oracle as O
from paper_1807_05117_amd import phantoms


# --------------------------------------------------------------------------- references

def conv_bruteforce(a, b, prob):
    """sum over band index pairs k' + k'' = k of a(k') b(k''), k in the band, unpaired
    planes zeroed afterwards"""
    K = prob.bshape
    half = [k // 2 for k in K]
    out = np.zeros(K, dtype=np.complex128)
    for i1 in np.ndindex(*K):
        if a[i1] == 0:
            continue
        for i2 in np.ndindex(*K):
            t = tuple(i1[x] + i2[x] - half[x] for x in range(len(K)))
            if all(0 <= t[x] < K[x] for x in range(len(K))):
                out[t] += a[i1] * b[i2]
    for ax in range(len(K)):
        sl = [slice(None)] * len(K)
        sl[ax] = 0
        out[tuple(sl)] = 0
    return out


def fft_iota(vh, prob):
    S = np.zeros(prob.shape, dtype=np.complex128)
    idx = np.meshgrid(*[np.mod(np.arange(K) - K // 2, N) for K, N in zip(prob.bshape, prob.shape)],
                      indexing="ij")
    S[tuple(idx)] = vh
    return (np.fft.ifftn(S) * prob.M).real


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
    fp = np.pad(f, 1, mode="wrap")
    inner = tuple(slice(1, -1) for _ in range(prob.dim))
    return [np.gradient(fp, 1.0 / prob.nref, axis=prob.dim - 1 - j)[inner] for j in range(prob.dim)]


def symbol(prob):
    ell = [N / prob.nref for N in prob.shape]
    kk = np.meshgrid(*[(np.arange(K) - K // 2) / l for K, l in zip(prob.bshape, ell)], indexing="ij")
    return (1 + 4 * np.pi ** 2 * prob.alpha * sum(q * q for q in kk)) ** prob.s


def theta(prob, v):
    """2 pi sum_j k_j v_j / l_j on the band, v in spatial order (domain units)"""
    ell = [N / prob.nref for N in prob.shape]           # numpy order
    kk = np.meshgrid(*[(np.arange(K) - K // 2) / l for K, l in zip(prob.bshape, ell)], indexing="ij")
    return 2 * np.pi * sum(kk[prob.dim - 1 - j] * v[j] for j in range(prob.dim))


def modes_field(prob, terms):
    """band velocity with v_c += 2 Re(a exp(2 pi i sum_j k_j x_j / l_j)) for each (c, k, a),
    k in spatial order; and the same velocity as a function of points in domain units"""
    vh = np.zeros((prob.dim,) + prob.bshape, dtype=np.complex128)
    for c, k, a in terms:
        idx = tuple(K // 2 + k[prob.dim - 1 - ax] for ax, K in enumerate(prob.bshape))
        neg = tuple(K // 2 - k[prob.dim - 1 - ax] for ax, K in enumerate(prob.bshape))
        vh[(c,) + idx] += a
        vh[(c,) + neg] += np.conj(a)
    ell = [N / prob.nref for N in prob.n]

    def vel(X):
        out = [np.zeros_like(X[0]) for _ in range(prob.dim)]
        for c, k, a in terms:
            ph = 2 * np.pi * sum(k[j] * X[j] / ell[j] for j in range(prob.dim))
            out[c] = out[c] + 2 * np.real(a * np.exp(1j * ph))
        return out
    return vh, vel


def inverse_flow(prob, vel, steps=400):
    """phi(1)(x) - x at the grid points: dY/dtau = -v(Y), Y(0) = x, tau in [0, 1], by RK4 with
    many small steps; spatial order, domain units"""
    grids = np.meshgrid(*[np.arange(N) / prob.nref for N in prob.shape], indexing="ij")
    x0 = [grids[prob.dim - 1 - j] for j in range(prob.dim)]
    Y = [g.copy() for g in x0]
    h = 1.0 / steps
    for _ in range(steps):
        k1 = vel(Y)
        k2 = vel([Y[j] - 0.5 * h * k1[j] for j in range(prob.dim)])
        k3 = vel([Y[j] - 0.5 * h * k2[j] for j in range(prob.dim)])
        k4 = vel([Y[j] - h * k3[j] for j in range(prob.dim)])
        Y = [Y[j] - h / 6 * (k1[j] + 2 * k2[j] + 2 * k3[j] + k4[j]) for j in range(prob.dim)]
    return [Y[j] - x0[j] for j in range(prob.dim)]


def rand_adm(prob, seed):
    return O.project(phantoms.random_band_direction(seed, prob.dim, prob.k), prob)


def blob_case(n=32, k=12, nt=6, disp=3.0):
    prob = O.Problem(2, (n, n), (k, k), nt)
    I0 = phantoms.blobs_2d(0, n)
    vs = O.project(phantoms.raw_band_velocity(0, 2, prob.k), prob)
    vs *= disp / O.max_displacement_voxels(vs, prob)
    return prob, I0, vs


# ------------------------------------------------------------------------------- checks

def check_star_bruteforce(D):
    err = 0.0
    for prob in (O.Problem(2, (8, 6), (4, 6), 2), O.Problem(3, (8, 6, 4), (4, 6, 4), 2)):
        a = O.project(phantoms.random_band_direction(1, prob.dim, prob.k)[0], prob)
        b = O.project(phantoms.random_band_direction(2, prob.dim, prob.k)[1], prob)
        ref = conv_bruteforce(a, b, prob)
        err = max(err, np.abs(D.star(a, b, prob) - ref).max() / np.abs(ref).max())
    return err


def check_transposes(D):
    """<D~a * v, c> = -<a, div~(c * v)> and <D~U * b, c> = <b, (D~U)^T * c> on a non-cubic grid"""
    prob = O.Problem(3, (12, 10, 8), (6, 6, 4), 2)
    a, v, c, U, b = (rand_adm(prob, s) for s in range(5))
    l1, r1 = O.dot(D.conv_D(a, v, prob), c), -O.dot(a, D.adj_A(c, v, prob))
    l2, r2 = O.dot(D.conv_D(U, b, prob), c), O.dot(b, D.conv_DT(U, c, prob))
    return max(abs(l1 - r1) / abs(l1), abs(l2 - r2) / abs(l2))


FLOW_2D = [(0, (0, 1), 0.04), (1, (1, 0), -0.03j), (0, (1, 1), 0.01), (1, (2, -1), 0.006 + 0.004j)]
FLOW_3D = [(0, (0, 1, 0), 0.03), (1, (0, 0, 1), -0.02j), (2, (1, 0, 0), 0.025),
           (0, (1, 0, 1), 0.008j), (2, (0, 1, 1), 0.01)]


def check_inverse_flow(D, dim=2, nt=10):
    """max |iota(u~(1)) - (phi(1) - id)| relative to the largest displacement"""
    if dim == 2:
        prob = O.Problem(2, (32, 32), (16, 16), nt)
        terms = FLOW_2D
    else:
        prob = O.Problem(3, (16, 24, 20), (12, 12, 12), nt)
        terms = FLOW_3D
    vh, vel = modes_field(prob, terms)
    ref = inverse_flow(prob, vel)
    u1, _ = D.def_forward(vh, prob)
    scale = max(np.abs(r).max() for r in ref)
    return max(np.abs(O.iota(u1[j], prob) - ref[j]).max() for j in range(dim)) / scale


def check_constant_velocity(D):
    """whole-voxel constant velocity: u(1) = -v, m(1) an exact roll; gradient and GN product
    against their continuous closed forms (numpy.fft), the adjoint and incremental states being
    pure phase rotations exp(i theta t)"""
    prob = O.Problem(2, (16, 16), (8, 8), 16)
    I0 = phantoms.blobs_2d(3, 16)
    I1 = phantoms.blobs_2d(4, 16)
    vox = (1, -1)
    vh = np.zeros((2,) + prob.bshape, dtype=np.complex128)
    c = tuple(K // 2 for K in prob.bshape)
    for j in range(2):
        vh[(j,) + c] = vox[j] / prob.nref
    st = D.def_evaluate(vh, I0, I1, prob)
    err_u = np.abs(st.u1 + vh).max() * prob.nref
    shift = tuple(vox[prob.dim - 1 - a] for a in range(prob.dim))
    err_m = np.abs(st.m1 - np.roll(I0, shift, axis=(0, 1))).max()
    th = theta(prob, [vox[j] / prob.nref for j in range(2)])
    with np.errstate(invalid="ignore", divide="ignore"):
        fwd = np.where(th == 0, 1.0, (np.exp(1j * th) - 1) / (1j * th))     # int_0^1 e^{i th (1-t)}
    gI = [np.roll(x, shift, axis=(0, 1)) for x in np_grad(I0, prob)]
    lam = -2.0 * (np.roll(I0, shift, axis=(0, 1)) - I1)
    rho1 = np.stack([fft_pi(lam * gI[j], prob) for j in range(2)])
    g_ref = symbol(prob)[None] * vh + fwd[None] * rho1
    e_g = np.linalg.norm(D.def_gradient(st) - g_ref) / np.linalg.norm(g_ref)
    dv = rand_adm(prob, 9)
    du1 = -np.conj(fwd)[None] * dv                                        # -int e^{-i th (1-s)} ds dv
    dm = sum(gI[j] * fft_iota(du1[j], prob) for j in range(2))
    drho = np.stack([fft_pi(-2.0 * dm * gI[j], prob) for j in range(2)])
    H_ref = symbol(prob)[None] * dv + fwd[None] * drho
    e_h = np.linalg.norm(D.def_hessvec(st, dv) - H_ref) / np.linalg.norm(H_ref)
    return max(err_u, err_m), e_g, e_h


def check_zero_velocity(D, dim=2):
    if dim == 2:
        prob = O.Problem(2, (24, 16), (8, 6), 4)
        I0, I1 = phantoms.blobs_2d(5, 24)[:16], phantoms.blobs_2d(6, 24)[:16]
    else:
        prob = O.Problem(3, (12, 10, 8), (6, 6, 4), 3)
        I0 = phantoms.shells_3d(0, prob.n, n_classes=3)
        I1 = phantoms.shells_3d(1, prob.n, n_classes=3)
    st = D.def_evaluate(np.zeros((dim,) + prob.bshape), I0, I1, prob)
    gI = np_grad(I0, prob)
    lam = -2.0 * (I0 - I1)
    g_ref = np.stack([fft_pi(lam * gI[j], prob) for j in range(dim)])
    e_g = np.linalg.norm(D.def_gradient(st) - g_ref) / np.linalg.norm(g_ref)
    dv = rand_adm(prob, 3)
    s = sum(gI[j] * fft_iota(dv[j], prob) for j in range(dim))
    H_ref = np.stack([symbol(prob) * dv[j] + 2.0 * fft_pi(s * gI[j], prob) for j in range(dim)])
    e_h = np.linalg.norm(D.def_hessvec(st, dv) - H_ref) / np.linalg.norm(H_ref)
    return e_g, e_h


def check_symmetry(D, dim=2):
    """(defect of <H a, b> = <a, H b>, min of <a, H a> / <a, L a>) at a realistic velocity"""
    if dim == 2:
        prob, I0, vs = blob_case()
        I1 = phantoms.blobs_2d(1, 32)
    else:
        prob = O.Problem(3, (12, 10, 8), (6, 6, 4), 4)
        I0 = phantoms.shells_3d(0, prob.n, n_classes=3)
        I1 = phantoms.shells_3d(1, prob.n, n_classes=3)
        vs = O.project(phantoms.raw_band_velocity(0, 3, prob.k), prob)
        vs *= 2.0 / O.max_displacement_voxels(vs, prob)
    st = D.def_evaluate(vs, I0, I1, prob)
    a, b = rand_adm(prob, 11), rand_adm(prob, 12)
    Ha, Hb = D.def_hessvec(st, a), D.def_hessvec(st, b)
    x, y = O.dot(Ha, b), O.dot(a, Hb)
    Lh = symbol(prob)[None]
    pos = min(O.dot(a, Ha) / O.dot(a, Lh * a), O.dot(b, Hb) / O.dot(b, Lh * b))
    return abs(x - y) / (abs(x) + abs(y)), pos


def check_fd_gradient(D, eps=1e-3):
    prob, I0, vs = blob_case()
    I1 = D.def_warp(I0, vs, prob)
    vh = 0.5 * vs
    st = D.def_evaluate(vh, I0, I1, prob)
    w = rand_adm(prob, 5)
    w *= 0.3 * np.abs(vs).max() / np.abs(w).max()
    fd = (D.def_evaluate(vh + eps * w, I0, I1, prob).E
          - D.def_evaluate(vh - eps * w, I0, I1, prob).E) / (2 * eps)
    an = O.dot(D.def_gradient(st), w)
    return abs(fd - an) / abs(an)


def check_fd_hessian_zero_residual(D, eps=1e-3):
    prob, I0, vs = blob_case()
    vh = 0.5 * vs
    I1 = D.def_warp(I0, vh, prob)
    st = D.def_evaluate(vh, I0, I1, prob)
    w = rand_adm(prob, 5)
    w *= 0.3 * np.abs(vs).max() / np.abs(w).max()
    Hw = D.def_hessvec(st, w)
    fd = (D.def_gradient(D.def_evaluate(vh + eps * w, I0, I1, prob))
          - D.def_gradient(D.def_evaluate(vh - eps * w, I0, I1, prob))) / (2 * eps)
    return np.linalg.norm(fd - Hw) / np.linalg.norm(Hw)


def check_state_map_derivatives(D, eps=1e-5):
    """du~(1) against central differences of the state map u~(1)(v~), and minus the transpose
    against du~(1) through <w, def_transpose(c)> = -<du~(1)(w), c>: (linearisation error,
    finite-difference error of the transpose, exact transpose defect)"""
    prob = O.Problem(2, (24, 24), (12, 10), 5)
    vh = O.project(phantoms.raw_band_velocity(2, 2, prob.k), prob)
    vh *= 3.0 / O.max_displacement_voxels(vh, prob)
    I0 = phantoms.blobs_2d(0, 24)
    st = D.def_evaluate(vh, I0, I0, prob)
    w = rand_adm(prob, 21)
    w *= np.abs(vh).max() / np.abs(w).max()
    c = rand_adm(prob, 22)
    fd = (D.def_forward(vh + eps * w, prob)[0] - D.def_forward(vh - eps * w, prob)[0]) / (2 * eps)
    du = D.def_incremental(st, w)
    e_lin = np.linalg.norm(du - fd) / np.linalg.norm(fd)
    t = O.dot(w, D.def_transpose(st, c))
    e_fd = abs(t + O.dot(fd, c)) / abs(t)
    e_tr = abs(t + O.dot(du, c)) / abs(t)
    return e_lin, e_fd, e_tr
