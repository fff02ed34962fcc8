"""Plain FP64 NumPy oracle of band-limited PDE-LDDMM on the state equation.

TEST INFRASTRUCTURE ONLY: used by the tests, by the smoke check and by the benchmark's CPU
baseline leg.  Nothing in the product library imports, links or runs it, and it shares no
code with the GPU path.

What is computed (paper: Hernandez, "Newton-Krylov optimization in PDE-constrained
diffeomorphic registration parameterized in the space of band-limited vector fields"):

  * the band-limited energy of the state-equation method (Section 3.2, equation BLEnergy),
        E(v~) = 1/2 <L~ v~, v~>_l2 + sigma^-2 || m(1) - I1 ||^2,
    with m transported by the state equation d_t m + grad m . iota(v~) = 0, m(0) = I0
    (Section 2.2, equation StateEquation);
  * its gradient L~ v~ + pi( int lambda grad m dt ) with the adjoint
    -d_t lambda - div(lambda v) = 0, lambda(1) = -(2/sigma^2)(m(1) - I1)
    (Section 2.2, equations FirstOrder1-4; Section 3.2 gradient);
  * the Gauss-Newton Hessian-vector product L~ dv~ + pi( int dlambda grad m dt ) with the
    incremental state d_t dm + grad dm . v + grad m . dv = 0, dm(0) = 0 and the incremental
    adjoint -d_t dlambda - div(dlambda v) = 0, dlambda(1) = -(2/sigma^2) dm(1)
    (Section 2.2, second-order system; Section 3.2 equation BLHessianStateEquation with the
    Gauss-Newton rule of Section 3.4, which drops the residual-proportional terms);
  * the reduced-space Gauss-Newton-Krylov solver with PCG preconditioned by K~ = L~^-1
    (Section 2.4 equations Newton and KKT; Section 3.4 equations BLNewton and BLKKT).

Readings taken where the paper is silent or garbled (each is also listed in the design
notes):
  R1  periodic domain, isotropic voxels of size h = 1/N_ref with N_ref = max_j N_j, so the
      domain is prod_j [0, l_j) with l_j = N_j / N_ref;
  R2  unit-volume inner products <f, g> = (1/M) sum_i f_i g_i, M = prod_j N_j, and
      <a, b>_l2 = Re sum conj(a) b over the full centred band;
  R3  band B = prod_j {-K_j/2, ..., K_j/2 - 1}; admissible coefficients are Hermitian with
      the unpaired plane k_j = -K_j/2 set to zero;
  R4  iota(v~)(x_i) = Re sum_k v~(k) exp(2 pi i sum_j k_j i_j / N_j),
      pi(f)(k) = (1/M) sum_i f_i exp(-2 pi i sum_j k_j i_j / N_j), zero on unpaired planes;
  R5  L^(k) = (1 + 4 pi^2 alpha sum_j (k_j / l_j)^2)^s, K^ = 1 / L^;
  R7  E uses the 1/2 of equation BLEnergy on the regulariser only;
  R8  stationary v~ (the "St." rows of Table 1);
  R9  semi-Lagrangian steps, Nt uniform steps, RK2 (Heun) departure points, periodic
      d-linear interpolation, offsets in voxel units;
  R10 grad by periodic second-order central differences;
  R11 div v spectral, r = iota(sum_j 2 pi i (k_j / l_j) v~_j);
  R12 adjoint reaction along the backward characteristic by Heun:
      lambda^n = a * Interp(lambda^{n+1}, i + Y), a = 1 + dt/2 [R + (1 + dt R) r];
  R13 trapezoid weights in time; trapezoid along characteristics for the dm source;
  R-GN Gauss-Newton = the Eulerian incremental system with every residual-proportional
      term dropped (symmetric positive definite);
  R-LS update v~ <- v~ + eps dv~ (Hdv~ = -g is a descent direction), Armijo backtracking;
  R-PCG dv~_0 = 0, at most max_pcg steps, forcing eta = min(0.5, sqrt(|g| / |g_0|));
  R-gamma gamma = 1 (incompressible flow, Section 2.2 constraint, Section 3.2 band form):
      v~ restricted to divergence-free band vectors; the multiplier terms of the gradient and
      Hessian make them divergence-free, i.e. both are the per-index orthogonal projections
      I - q q^T / |q|^2 (q_j = 2 pi k_j / l_j) of the gamma = 0 expressions; inputs projected;
  R-N  full Newton: the incremental adjoint's source div(lambda dv) by the trapezoid rule along
      the backward characteristic with its own-time half weight at t = 1 (see hessvec_newton);
  R-NS non-stationary velocity: one band field per time node, trapezoid-weighted regulariser
      and inner product, Heun steps with the velocity at both ends of a step (see ns_setup).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Problem", "band_freqs", "project", "zero_unpaired", "iota", "pi_", "L_hat",
    "div_band", "leray", "iota_at", "pi_at", "interp", "grad_c", "trapezoid_weights", "setup", "forward_state",
    "energy", "State", "evaluate", "gradient", "hessvec", "adjoint", "div_c", "hessvec_newton",
    "warp", "dot", "norm2",
    "norm_inf", "mse_rel", "register", "SolverOpts", "CONVERGED", "MAXITER", "STALLED",
    "max_displacement_voxels", "ns_project", "ns_dot", "ns_setup", "ns_evaluate", "ns_gradient",
    "ns_hessvec", "ns_register",
]

CONVERGED, MAXITER, STALLED = 0, 1, 2


@dataclass(frozen=True)
class Problem:
    """Grid, band and weights of one registration problem (Section 3.2 statement).

    n, k are given in spatial order (x, y[, z]); arrays use NumPy order ([z,] y, x).
    """
    dim: int
    n: tuple
    k: tuple
    nt: int
    alpha: float = 1e-3
    s: int = 2
    sigma: float = 1.0
    gamma: int = 0

    def __post_init__(self):
        if self.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if len(self.n) != self.dim or len(self.k) != self.dim:
            raise ValueError("n and k need dim entries")
        for nj, kj in zip(self.n, self.k):
            if kj < 2 or kj % 2 or kj > nj:
                raise ValueError("band sizes must be even, >= 2 and <= grid size")
        if self.nt < 1 or self.sigma <= 0 or self.alpha < 0 or self.s < 0:
            raise ValueError("bad nt / sigma / alpha / s")
        if self.gamma not in (0, 1):
            raise ValueError("gamma must be 0 or 1")

    @property
    def shape(self):
        return tuple(int(v) for v in reversed(self.n))

    @property
    def bshape(self):
        return tuple(int(v) for v in reversed(self.k))

    @property
    def nref(self):
        return int(max(self.n))

    @property
    def M(self):
        return int(np.prod(self.n))

    @property
    def dt(self):
        return 1.0 / self.nt

    def axis(self, j):
        """NumPy axis of spatial axis j (j = 0 is x)."""
        return self.dim - 1 - j


# ----------------------------------------------------------------------------- band helpers

def band_freqs(K: int) -> np.ndarray:
    """Integer frequencies of a centred band axis of size K: -K/2, ..., K/2 - 1 (R3)."""
    return np.arange(K, dtype=np.float64) - K // 2


def zero_unpaired(vh: np.ndarray, prob: Problem) -> np.ndarray:
    """Set the unpaired planes k_j = -K_j/2 (index 0 on every band axis) to zero (R3)."""
    out = np.array(vh, dtype=np.complex128, copy=True)
    lead = out.ndim - prob.dim
    for a in range(prob.dim):
        sl = [slice(None)] * out.ndim
        sl[lead + a] = 0
        out[tuple(sl)] = 0.0
    return out


def project(vh: np.ndarray, prob: Problem) -> np.ndarray:
    """Projection onto admissible coefficients: (v~(k) + conj v~(-k)) / 2 on paired
    indices, zero on unpaired planes (R3).  Works on one component or on a stack; a velocity
    stack (dim components) of an incompressible problem (gamma = 1) is then also made
    divergence-free (leray, reading R-gamma)."""
    vh = np.asarray(vh, dtype=np.complex128)
    out = np.zeros_like(vh)
    lead = vh.ndim - prob.dim
    inner = (slice(None),) * lead + (slice(1, None),) * prob.dim
    rev = (slice(None),) * lead + (slice(None, None, -1),) * prob.dim
    w = vh[inner]
    out[inner] = 0.5 * (w + np.conj(w[rev]))
    if prob.gamma == 1 and lead == 1 and vh.shape[0] == prob.dim:
        out = leray(out, prob)
    return out


def leray(vh: np.ndarray, prob: Problem) -> np.ndarray:
    """Orthogonal projection of a band velocity (dim components) onto the divergence-free
    band vectors, per index k: v~ - q (q . v~) / |q|^2 with q_j = 2 pi k_j / l_j, the symbol of
    the spectral divergence up to the factor i; identity at k = 0 (reading R-gamma: the
    multiplier term gamma grad~ p~ of the gradient and Hessian of Section 3.2 is what makes
    them divergence-free, i.e. these projections)."""
    vh = np.asarray(vh, dtype=np.complex128)
    q = [2.0 * np.pi * x for x in _kl(prob)]
    qq = sum(x * x for x in q)
    s = sum(q[j] * vh[j] for j in range(prob.dim))
    inv = np.divide(1.0, qq, out=np.zeros_like(qq), where=qq > 0)
    return np.stack([vh[j] - q[j] * s * inv for j in range(prob.dim)])


def _emat(N: int, K: int, sign: float) -> np.ndarray:
    """(N, K) matrix exp(sign 2 pi i k i / N) for grid index i and centred frequency k."""
    i = np.arange(N, dtype=np.float64)[:, None]
    k = band_freqs(K)[None, :]
    return np.exp(sign * 2j * np.pi * i * k / N)


def iota(vh: np.ndarray, prob: Problem) -> np.ndarray:
    """Band -> grid, one component (Section 3.1, inclusion iota; normalisation R4).

    iota(v~)(x_i) = Re sum_{k in B} v~(k) exp(2 pi i sum_j k_j i_j / N_j).  The exponential
    of the sum is the product of the per-axis exponentials, so the sum is written as one
    einsum over the per-axis matrices.
    """
    vh = np.asarray(vh, dtype=np.complex128)
    E = [_emat(prob.n[j], prob.k[j], +1.0) for j in range(prob.dim)]
    if prob.dim == 2:
        out = np.einsum("yb,xa,ba->yx", E[1], E[0], vh, optimize=True)
    else:
        out = np.einsum("zc,yb,xa,cba->zyx", E[2], E[1], E[0], vh, optimize=True)
    return out.real.copy()


def pi_(f: np.ndarray, prob: Problem) -> np.ndarray:
    """Grid -> band, one component (Section 3.1, projection pi; normalisation R4).

    pi(f)(k) = (1/M) sum_i f_i exp(-2 pi i sum_j k_j i_j / N_j), zero on unpaired planes.
    """
    f = np.asarray(f, dtype=np.float64)
    E = [np.conj(_emat(prob.n[j], prob.k[j], +1.0)) for j in range(prob.dim)]
    if prob.dim == 2:
        out = np.einsum("yb,xa,yx->ba", E[1], E[0], f, optimize=True)
    else:
        out = np.einsum("zc,yb,xa,zyx->cba", E[2], E[1], E[0], f, optimize=True)
    return zero_unpaired(out / prob.M, prob)


def iota_at(vh: np.ndarray, prob: Problem, points) -> np.ndarray:
    """iota of one component at selected grid points only (same definition as iota, R4).

    points: integer array (P, dim) of NumPy-order grid indices ([z,] y, x).  Used to check
    single outputs of grids too large for the full transform.
    """
    vh = np.asarray(vh, dtype=np.complex128)
    pts = np.asarray(points, dtype=np.int64).reshape(-1, prob.dim)
    out = np.empty(len(pts))
    for p, idx in enumerate(pts):
        acc = vh
        for a in range(prob.dim - 1, -1, -1):  # contract the last band axis first
            N, K = prob.shape[a], prob.bshape[a]
            e = np.exp(2j * np.pi * idx[a] * band_freqs(K) / N)
            acc = acc @ e
        out[p] = acc.real
    return out


def pi_at(f: np.ndarray, prob: Problem, kidx) -> np.ndarray:
    """pi of one grid field at selected band indices only (same definition as pi_, R4).

    kidx: integer array (P, dim) of NumPy-order band indices (index j <-> k = j - K/2);
    entries on an unpaired plane are zero.
    """
    f = np.asarray(f, dtype=np.float64)
    ks = np.asarray(kidx, dtype=np.int64).reshape(-1, prob.dim)
    out = np.empty(len(ks), dtype=np.complex128)
    for p, kk in enumerate(ks):
        if np.any(kk == 0):
            out[p] = 0.0
            continue
        acc = f
        for a in range(prob.dim - 1, -1, -1):
            N, K = prob.shape[a], prob.bshape[a]
            e = np.exp(-2j * np.pi * np.arange(N) * (kk[a] - K // 2) / N)
            acc = acc @ e
        out[p] = acc / prob.M
    return out


def _kl(prob: Problem):
    """Per spatial axis j: k_j / l_j broadcast over the band (NumPy order), l_j = N_j/N_ref."""
    grids = np.meshgrid(*[band_freqs(K) for K in prob.bshape], indexing="ij")
    out = []
    for j in range(prob.dim):
        lj = prob.n[j] / prob.nref
        out.append(grids[prob.axis(j)] / lj)
    return out


def L_hat(prob: Problem) -> np.ndarray:
    """Fourier symbol of L = (Id - alpha Lap)^s (Section 2.1; projected operator L~ of
    Section 3.1): (1 + 4 pi^2 alpha sum_j (k_j / l_j)^2)^s (R5)."""
    kl = _kl(prob)
    q = sum(x * x for x in kl)
    return (1.0 + 4.0 * np.pi ** 2 * prob.alpha * q) ** prob.s


def div_band(vh: np.ndarray, prob: Problem) -> np.ndarray:
    """Spectral divergence (projected operator of Section 3.1, R11): sum_j 2 pi i (k_j/l_j) v~_j."""
    kl = _kl(prob)
    return sum(2j * np.pi * kl[j] * vh[j] for j in range(prob.dim))


# --------------------------------------------------------------------------- grid helpers

def interp(f: np.ndarray, off, prob: Problem) -> np.ndarray:
    """Periodic d-linear interpolation of f at the points i + off (voxel units) (R9).

    off is a sequence of dim arrays in spatial order (off[0] is the x offset).
    """
    shape = f.shape
    idx = np.indices(shape, dtype=np.float64)
    base, frac = [], []
    for a in range(prob.dim):
        p = idx[a] + off[prob.dim - 1 - a]
        p0 = np.floor(p)
        base.append(p0.astype(np.int64))
        frac.append(p - p0)
    out = np.zeros(shape, dtype=np.float64)
    for corner in itertools.product((0, 1), repeat=prob.dim):
        w = np.ones(shape, dtype=np.float64)
        ind = []
        for a in range(prob.dim):
            ind.append(np.mod(base[a] + corner[a], shape[a]))
            w = w * (frac[a] if corner[a] else 1.0 - frac[a])
        out += w * f[tuple(ind)]
    return out


def grad_c(f: np.ndarray, prob: Problem):
    """Periodic central differences (f(i + e_j) - f(i - e_j)) / (2h), h = 1/N_ref (R10).

    Returns dim arrays in spatial order."""
    out = []
    for j in range(prob.dim):
        ax = prob.axis(j)
        out.append((np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) * (prob.nref / 2.0))
    return out


def trapezoid_weights(nt: int) -> np.ndarray:
    """Trapezoid weights on t_n = n/nt: dt/2 at both ends, dt inside (R13)."""
    w = np.full(nt + 1, 1.0 / nt)
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


# ------------------------------------------------------------------------------- the path

def setup(vh: np.ndarray, prob: Problem) -> dict:
    """Velocity on the grid, its divergence, departure offsets and adjoint reaction factor.

    v = iota(v~); r = iota(div~ v~); u = dt N_ref v (voxels per step);
    X = -(u + Interp(u, i - u)) / 2  (forward characteristic, Heun),
    Y = +(u + Interp(u, i + u)) / 2  (backward characteristic, Heun),
    a = 1 + dt/2 [R + (1 + dt R) r] with R = Interp(r, i + Y)          (R9, R11, R12).
    """
    vh = project(vh, prob)
    d = prob.dim
    v = [iota(vh[j], prob) for j in range(d)]
    r = iota(div_band(vh, prob), prob)
    u = [prob.dt * prob.nref * v[j] for j in range(d)]
    neg_u = [-x for x in u]
    X = [-0.5 * (u[j] + interp(u[j], neg_u, prob)) for j in range(d)]
    Y = [0.5 * (u[j] + interp(u[j], u, prob)) for j in range(d)]
    R = interp(r, Y, prob)
    a = 1.0 + 0.5 * prob.dt * (R + (1.0 + prob.dt * R) * r)
    return {"vh": vh, "v": v, "r": r, "X": X, "Y": Y, "a": a}


def forward_state(I0: np.ndarray, X, prob: Problem):
    """State equation by semi-Lagrangian steps: m^0 = I0, m^{n+1} = Interp(m^n, i + X)
    (Section 2.2 StateEquation; Section 3.2 constraint with iota(v~))."""
    m = [np.asarray(I0, dtype=np.float64)]
    for _ in range(prob.nt):
        m.append(interp(m[-1], X, prob))
    return m


def energy(vh: np.ndarray, mT: np.ndarray, I1: np.ndarray, prob: Problem) -> float:
    """E = 1/2 sum_c sum_k L^ |v~_c|^2 + sigma^-2 (1/M) sum (m(1) - I1)^2 (Section 3.2,
    equation BLEnergy; R2, R7)."""
    Lh = L_hat(prob)
    reg = 0.5 * float(np.sum(Lh[None] * np.abs(vh) ** 2))
    res = mT - I1
    return reg + float(np.mean(res * res)) / prob.sigma ** 2


@dataclass
class State:
    prob: Problem
    I0: np.ndarray
    I1: np.ndarray
    geo: dict
    m: list
    E: float


def evaluate(vh, I0, I1, prob: Problem) -> State:
    """Setup, forward state and energy at v~ (projected first)."""
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    geo = setup(vh, prob)
    m = forward_state(I0, geo["X"], prob)
    return State(prob, I0, I1, geo, m, energy(geo["vh"], m[-1], I1, prob))


def gradient(st: State) -> np.ndarray:
    """g~ = L^ v~ + pi(b), b = sum_n w_n lambda^n grad m^n (Section 3.2 gradient, R12, R13).

    lambda^Nt = -(2/sigma^2)(m^Nt - I1) (Section 2.2 final condition),
    lambda^n = a Interp(lambda^{n+1}, i + Y).
    """
    prob, d = st.prob, st.prob.dim
    w = trapezoid_weights(prob.nt)
    lam = -(2.0 / prob.sigma ** 2) * (st.m[-1] - st.I1)
    gm = grad_c(st.m[-1], prob)
    b = [w[-1] * lam * gm[j] for j in range(d)]
    for n in range(prob.nt - 1, -1, -1):
        lam = st.geo["a"] * interp(lam, st.geo["Y"], prob)
        gm = grad_c(st.m[n], prob)
        for j in range(d):
            b[j] += w[n] * lam * gm[j]
    Lh = L_hat(prob)
    return _constrained(np.stack([Lh * st.geo["vh"][j] + pi_(b[j], prob) for j in range(d)]), prob)


def hessvec(st: State, dvh: np.ndarray) -> np.ndarray:
    """Gauss-Newton Hessian-vector product (Section 3.2 BLHessianStateEquation with the
    Gauss-Newton rule of Section 3.4, reading R-GN):

      dv = iota(dv~), f^n = -grad m^n . dv;
      dm^0 = 0, dm^{n+1} = Interp(dm^n + dt/2 f^n, i + X) + dt/2 f^{n+1};
      dlambda^Nt = -(2/sigma^2) dm^Nt, dlambda^n = a Interp(dlambda^{n+1}, i + Y);
      H dv~ = L^ dv~ + pi(sum_n w_n dlambda^n grad m^n).
    """
    prob, d = st.prob, st.prob.dim
    dvh = project(dvh, prob)
    dv = [iota(dvh[j], prob) for j in range(d)]
    dt = prob.dt

    def f(n):
        gm = grad_c(st.m[n], prob)
        return -sum(gm[j] * dv[j] for j in range(d))

    X = st.geo["X"]
    dm = np.zeros(prob.shape)
    fn = f(0)
    for n in range(prob.nt):
        fn1 = f(n + 1)
        dm = interp(dm + 0.5 * dt * fn, X, prob) + 0.5 * dt * fn1
        fn = fn1
    w = trapezoid_weights(prob.nt)
    dlam = -(2.0 / prob.sigma ** 2) * dm
    gm = grad_c(st.m[-1], prob)
    Hb = [w[-1] * dlam * gm[j] for j in range(d)]
    for n in range(prob.nt - 1, -1, -1):
        dlam = st.geo["a"] * interp(dlam, st.geo["Y"], prob)
        gm = grad_c(st.m[n], prob)
        for j in range(d):
            Hb[j] += w[n] * dlam * gm[j]
    Lh = L_hat(prob)
    return _constrained(np.stack([Lh * dvh[j] + pi_(Hb[j], prob) for j in range(d)]), prob)


def adjoint(st: State) -> list:
    """The adjoint at every time step (Section 2.2 adjoint equation and final condition,
    reading R12): lambda^Nt = -(2/sigma^2)(m^Nt - I1), lambda^n = a Interp(lambda^{n+1}, i + Y).
    Returns [lambda^0, ..., lambda^Nt]."""
    prob = st.prob
    lam = [None] * (prob.nt + 1)
    lam[-1] = -(2.0 / prob.sigma ** 2) * (st.m[-1] - st.I1)
    for n in range(prob.nt - 1, -1, -1):
        lam[n] = st.geo["a"] * interp(lam[n + 1], st.geo["Y"], prob)
    return lam


def div_c(u, prob: Problem) -> np.ndarray:
    """Central-difference divergence sum_j (u_j(i + e_j) - u_j(i - e_j)) / (2h) of dim fields
    in spatial order: minus the transpose of grad_c (R10), periodic."""
    out = np.zeros(prob.shape)
    for j in range(prob.dim):
        ax = prob.axis(j)
        out += (np.roll(u[j], -1, axis=ax) - np.roll(u[j], 1, axis=ax)) * (prob.nref / 2.0)
    return out


def hessvec_newton(st: State, dvh: np.ndarray) -> np.ndarray:
    """Full Newton Hessian-vector product: the second-order system of Section 2.2 and the
    Hessian of Section 3.2 equation BLHessianStateEquation with both adjoint terms kept
    (reading R-N):

      dm^n as in the Gauss-Newton product, every time step kept;
      s^n = div(lambda^n dv)      (the source -div(lambda dv) of the incremental adjoint);
      q^Nt = -(2/sigma^2) dm^Nt,
      q^n = a Interp(q^{n+1} + dt/2 s^{n+1}, i + Y) + dt/2 s^n   (0 < n < Nt),
      q^0 = a Interp(q^1 + dt/2 s^1, i + Y),
      dlambda^n = q^n for n < Nt, dlambda^Nt = q^Nt + dt/2 s^Nt;
      H dv~ = L^ dv~ + pi(sum_n w_n [dlambda^n grad m^n + lambda^n grad dm^n]).
    The source is integrated by the trapezoid rule along the backward characteristic, with its
    own-time half weight moved from t = 0 to t = 1: the mirror of dm^n, which has its own-time
    half weight at every n >= 1 and none at 0.  With the trapezoid weights w_n of the Hessian
    sum this pairs every term of lambda grad dm with its transpose in dlambda grad m, so the
    product is exactly symmetric when the transports are permutations (pinned); the moved
    half weights change the sum by O(dt^2).
    """
    prob, d = st.prob, st.prob.dim
    dvh = project(dvh, prob)
    dv = [iota(dvh[j], prob) for j in range(d)]
    dt = prob.dt
    X, Y, a = st.geo["X"], st.geo["Y"], st.geo["a"]

    def f(n):
        gm = grad_c(st.m[n], prob)
        return -sum(gm[j] * dv[j] for j in range(d))

    dm = [np.zeros(prob.shape)]
    fn = f(0)
    for n in range(prob.nt):
        fn1 = f(n + 1)
        dm.append(interp(dm[-1] + 0.5 * dt * fn, X, prob) + 0.5 * dt * fn1)
        fn = fn1
    lam = adjoint(st)
    src = [div_c([lam[n] * dv[j] for j in range(d)], prob) for n in range(prob.nt + 1)]
    w = trapezoid_weights(prob.nt)
    q = -(2.0 / prob.sigma ** 2) * dm[-1]
    Hb = [np.zeros(prob.shape) for _ in range(d)]
    for n in range(prob.nt, -1, -1):
        if n < prob.nt:
            q = a * interp(q + 0.5 * dt * src[n + 1], Y, prob) + (0.5 * dt * src[n] if n > 0 else 0.0)
        dlam = q + 0.5 * dt * src[n] if n == prob.nt else q
        gm = grad_c(st.m[n], prob)
        gdm = grad_c(dm[n], prob)
        for j in range(d):
            Hb[j] += w[n] * (dlam * gm[j] + lam[n] * gdm[j])
    Lh = L_hat(prob)
    return _constrained(np.stack([Lh * dvh[j] + pi_(Hb[j], prob) for j in range(d)]), prob)


def _constrained(g: np.ndarray, prob: Problem) -> np.ndarray:
    """gamma = 1: the gradient or Hessian product with its multiplier term, i.e. the
    divergence-free part (reading R-gamma); gamma = 0: unchanged."""
    return leray(g, prob) if prob.gamma == 1 else g


def warp(I0, vh, prob: Problem) -> np.ndarray:
    """m(1) = I0 transported by the stationary band-limited velocity v~."""
    geo = setup(vh, prob)
    return forward_state(np.asarray(I0, dtype=np.float64), geo["X"], prob)[-1]


def max_displacement_voxels(vh, prob: Problem) -> float:
    """max_i |iota(v~)(x_i)|_2 * N_ref: the largest displacement over unit time, in voxels."""
    vh = project(vh, prob)
    v = [iota(vh[j], prob) for j in range(prob.dim)]
    return float(np.sqrt(sum(x * x for x in v)).max() * prob.nref)


# -------------------------------------------------------------------------------- solver

def dot(a, b) -> float:
    """<a, b>_l2 = Re sum conj(a) b (R2)."""
    return float(np.real(np.vdot(np.asarray(a).ravel(), np.asarray(b).ravel())))


def norm2(a) -> float:
    return math.sqrt(max(dot(a, a), 0.0))


def norm_inf(a) -> float:
    return float(np.abs(a).max()) if np.size(a) else 0.0


def mse_rel(mT, I0, I1) -> float:
    """100 |m(1) - I1|^2 / |I0 - I1|^2 in percent (reading R-MSE of the metric named in
    Section 4.1)."""
    den = float(np.sum((np.asarray(I0, np.float64) - I1) ** 2))
    num = float(np.sum((np.asarray(mT, np.float64) - I1) ** 2))
    return 100.0 * num / den if den > 0 else 0.0


@dataclass
class SolverOpts:
    max_gn: int = 10
    max_pcg: int = 10
    gtol: float = 1e-3          # stop when |g|_inf,rel < gtol
    c1: float = 1e-4            # Armijo constant
    max_halvings: int = 10
    newton: bool = False        # full Newton products (reading R-N) instead of Gauss-Newton


def register(I0, I1, vh0, prob: Problem, opts: SolverOpts = SolverOpts(), on_iteration=None):
    """Reduced-space Gauss-Newton-Krylov registration in the band (Section 3.4):
    PCG with preconditioner K^ = 1/L^ on H dv~ = -g~, then v~ <- v~ + eps dv~ with Armijo
    backtracking (readings R-LS, R-PCG).

    Returns (v~, m(1), stats) with stats a dict of per-iteration lists.  on_iteration (if not
    None) is called with stats after every accepted iteration (progress reports only).
    """
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    Lh = L_hat(prob)
    vh = project(vh0, prob)
    st = evaluate(vh, I0, I1, prob)
    g = gradient(st)
    g0n = norm2(g)
    ginf0 = norm_inf(g)
    stats = {"E": [st.E], "mse_rel": [mse_rel(st.m[-1], I0, I1)], "ginf_rel": [1.0],
             "pcg_iters": [], "ls_trials": [], "eps": [], "status": MAXITER, "gn_iters": 0,
             "hessvecs": 0, "gradients": 1, "evaluations": 1}
    if ginf0 == 0.0:
        stats["status"] = CONVERGED
        stats["ginf_rel"][0] = 0.0
        return vh, st.m[-1], stats
    for _ in range(opts.max_gn):
        if norm_inf(g) / ginf0 < opts.gtol:
            stats["status"] = CONVERGED
            break
        gn = norm2(g)
        eta = min(0.5, math.sqrt(gn / g0n))
        delta = np.zeros_like(vh)
        r = -g
        z = r / Lh[None]
        p = z.copy()
        rz = dot(r, z)
        iters = 0
        for _j in range(opts.max_pcg):
            Hp = hessvec_newton(st, p) if opts.newton else hessvec(st, p)
            stats["hessvecs"] += 1
            pHp = dot(p, Hp)
            if pHp <= 0.0:
                if iters == 0:
                    delta = z.copy()
                break
            alpha = rz / pHp
            delta = delta + alpha * p
            r = r - alpha * Hp
            iters += 1
            if norm2(r) <= eta * gn:
                break
            z = r / Lh[None]
            rz_new = dot(r, z)
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
        stats["pcg_iters"].append(iters)
        slope = dot(g, delta)
        eps = 1.0
        accepted = False
        trials = 0
        for _t in range(opts.max_halvings + 1):
            trials += 1
            st_try = evaluate(vh + eps * delta, I0, I1, prob)
            stats["evaluations"] += 1
            if st_try.E <= st.E + opts.c1 * eps * slope:
                accepted = True
                break
            eps *= 0.5
        stats["ls_trials"].append(trials)
        if not accepted:
            stats["status"] = STALLED
            stats["eps"].append(0.0)
            break
        stats["eps"].append(eps)
        vh = st_try.geo["vh"]
        st = st_try
        g = gradient(st)
        stats["gradients"] += 1
        stats["gn_iters"] += 1
        stats["E"].append(st.E)
        stats["mse_rel"].append(mse_rel(st.m[-1], I0, I1))
        stats["ginf_rel"].append(norm_inf(g) / ginf0)
        if on_iteration is not None:
            on_iteration(stats)
    else:
        stats["status"] = MAXITER
        if norm_inf(g) / ginf0 < opts.gtol:
            stats["status"] = CONVERGED
    return vh, st.m[-1], stats


# ---------------------------------------------------------- non-stationary velocity (R-NS)
#
# The velocity is a band field per time node t_n = n dt, n = 0..Nt: an array of shape
# (Nt + 1, dim, band...).  Reading R-NS: the regulariser is integrated by the trapezoid rule,
# E = 1/2 sum_n w_n <L~ v~^n, v~^n> + sigma^-2 |m(1) - I1|^2; the Heun characteristic of the
# step t_n -> t_{n+1} takes the velocity at its two ends; gradients and Hessian products are
# the pointwise-in-time expressions of Section 2.2 / 3.2 (FirstOrder4 with v_t), i.e. the
# representers in the trapezoid-weighted inner product <a, b>_w = sum_n w_n <a^n, b^n>, which
# the solver uses for every dot product and norm.

def ns_project(vh, prob: Problem) -> np.ndarray:
    return np.stack([project(vh[n], prob) for n in range(prob.nt + 1)])


def ns_dot(a, b, prob: Problem) -> float:
    """<a, b>_w = sum_n w_n <a^n, b^n>_l2 (trapezoid weights in time, R-NS)."""
    w = trapezoid_weights(prob.nt)
    return float(sum(w[n] * dot(a[n], b[n]) for n in range(prob.nt + 1)))


def ns_setup(vh, prob: Problem) -> dict:
    """Per-node velocities and divergences; per step n (t_n -> t_{n+1}) the Heun offsets with
    the velocity at the step's two ends (R9 with a time-dependent velocity, R-NS):
      X^n = -(u^{n+1} + Interp(u^n, i - u^{n+1})) / 2     (end point i at t_{n+1}),
      Y^n = +(u^n + Interp(u^{n+1}, i + u^n)) / 2         (start point i at t_n),
      a^n = 1 + dt/2 [R + (1 + dt R) r^n],  R = Interp(r^{n+1}, i + Y^n)   (R12)."""
    vh = ns_project(vh, prob)
    d, nt = prob.dim, prob.nt
    v = [[iota(vh[n][j], prob) for j in range(d)] for n in range(nt + 1)]
    r = [iota(div_band(vh[n], prob), prob) for n in range(nt + 1)]
    u = [[prob.dt * prob.nref * v[n][j] for j in range(d)] for n in range(nt + 1)]
    X, Y, a = [], [], []
    for n in range(nt):
        back = [-x for x in u[n + 1]]
        X.append([-0.5 * (u[n + 1][j] + interp(u[n][j], back, prob)) for j in range(d)])
        Yn = [0.5 * (u[n][j] + interp(u[n + 1][j], u[n], prob)) for j in range(d)]
        R = interp(r[n + 1], Yn, prob)
        Y.append(Yn)
        a.append(1.0 + 0.5 * prob.dt * (R + (1.0 + prob.dt * R) * r[n]))
    return {"vh": vh, "v": v, "r": r, "X": X, "Y": Y, "a": a}


def ns_evaluate(vh, I0, I1, prob: Problem) -> State:
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    geo = ns_setup(vh, prob)
    m = [I0]
    for n in range(prob.nt):
        m.append(interp(m[-1], geo["X"][n], prob))
    Lh = L_hat(prob)
    w = trapezoid_weights(prob.nt)
    reg = 0.5 * sum(w[n] * float(np.sum(Lh[None] * np.abs(geo["vh"][n]) ** 2))
                    for n in range(prob.nt + 1))
    res = m[-1] - I1
    return State(prob, I0, I1, geo, m, reg + float(np.mean(res * res)) / prob.sigma ** 2)


def ns_gradient(st: State) -> np.ndarray:
    """g^n = L^ v~^n + pi(lambda^n grad m^n), lambda^Nt = -(2/sigma^2)(m^Nt - I1),
    lambda^n = a^n Interp(lambda^{n+1}, i + Y^n)."""
    prob, d = st.prob, st.prob.dim
    lam = -(2.0 / prob.sigma ** 2) * (st.m[-1] - st.I1)
    Lh = L_hat(prob)
    g = [None] * (prob.nt + 1)
    for n in range(prob.nt, -1, -1):
        if n < prob.nt:
            lam = st.geo["a"][n] * interp(lam, st.geo["Y"][n], prob)
        gm = grad_c(st.m[n], prob)
        g[n] = _constrained(np.stack([Lh * st.geo["vh"][n][j] + pi_(lam * gm[j], prob)
                                      for j in range(d)]), prob)
    return np.stack(g)


def ns_hessvec(st: State, dvh) -> np.ndarray:
    """Gauss-Newton product per node (R-GN, R-NS): dv^n = iota(dv~^n), f^n = -grad m^n . dv^n,
    dm^{n+1} = Interp(dm^n + dt/2 f^n, i + X^n) + dt/2 f^{n+1}, dlambda^Nt = -(2/sigma^2) dm^Nt,
    dlambda^n = a^n Interp(dlambda^{n+1}, i + Y^n), (H dv~)^n = L^ dv~^n + pi(dlambda^n grad m^n)."""
    prob, d, dt = st.prob, st.prob.dim, st.prob.dt
    dvh = ns_project(dvh, prob)

    def f(n):
        gm = grad_c(st.m[n], prob)
        return -sum(gm[j] * iota(dvh[n][j], prob) for j in range(d))

    dm = np.zeros(prob.shape)
    fn = f(0)
    for n in range(prob.nt):
        fn1 = f(n + 1)
        dm = interp(dm + 0.5 * dt * fn, st.geo["X"][n], prob) + 0.5 * dt * fn1
        fn = fn1
    dlam = -(2.0 / prob.sigma ** 2) * dm
    Lh = L_hat(prob)
    out = [None] * (prob.nt + 1)
    for n in range(prob.nt, -1, -1):
        if n < prob.nt:
            dlam = st.geo["a"][n] * interp(dlam, st.geo["Y"][n], prob)
        gm = grad_c(st.m[n], prob)
        out[n] = _constrained(np.stack([Lh * dvh[n][j] + pi_(dlam * gm[j], prob)
                                        for j in range(d)]), prob)
    return np.stack(out)


def ns_register(I0, I1, vh0, prob: Problem, opts: SolverOpts = SolverOpts()):
    """The Gauss-Newton-Krylov solver of `register` on a non-stationary velocity, every dot
    product and 2-norm in the trapezoid-weighted inner product (R-NS); PCG preconditioner K^
    per node; the gradient's inf-norm over all nodes."""
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    Lh = L_hat(prob)
    vh = ns_project(vh0, prob)
    st = ns_evaluate(vh, I0, I1, prob)
    g = ns_gradient(st)
    wnorm = lambda x: math.sqrt(max(ns_dot(x, x, prob), 0.0))
    g0n, ginf0 = wnorm(g), norm_inf(g)
    stats = {"E": [st.E], "mse_rel": [mse_rel(st.m[-1], I0, I1)], "ginf_rel": [1.0],
             "pcg_iters": [], "ls_trials": [], "eps": [], "status": MAXITER, "gn_iters": 0,
             "hessvecs": 0, "gradients": 1, "evaluations": 1}
    if ginf0 == 0.0:
        stats["status"] = CONVERGED
        stats["ginf_rel"][0] = 0.0
        return vh, st.m[-1], stats
    for _ in range(opts.max_gn):
        if norm_inf(g) / ginf0 < opts.gtol:
            stats["status"] = CONVERGED
            break
        gn = wnorm(g)
        eta = min(0.5, math.sqrt(gn / g0n))
        delta = np.zeros_like(vh)
        r = -g
        z = r / Lh[None, None]
        p = z.copy()
        rz = ns_dot(r, z, prob)
        iters = 0
        for _j in range(opts.max_pcg):
            Hp = ns_hessvec(st, p)
            stats["hessvecs"] += 1
            pHp = ns_dot(p, Hp, prob)
            if pHp <= 0.0:
                if iters == 0:
                    delta = z.copy()
                break
            alpha = rz / pHp
            delta = delta + alpha * p
            r = r - alpha * Hp
            iters += 1
            if wnorm(r) <= eta * gn:
                break
            z = r / Lh[None, None]
            rz_new = ns_dot(r, z, prob)
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
        stats["pcg_iters"].append(iters)
        slope = ns_dot(g, delta, prob)
        eps, accepted, trials = 1.0, False, 0
        for _t in range(opts.max_halvings + 1):
            trials += 1
            st_try = ns_evaluate(vh + eps * delta, I0, I1, prob)
            stats["evaluations"] += 1
            if st_try.E <= st.E + opts.c1 * eps * slope:
                accepted = True
                break
            eps *= 0.5
        stats["ls_trials"].append(trials)
        if not accepted:
            stats["status"] = STALLED
            stats["eps"].append(0.0)
            break
        stats["eps"].append(eps)
        vh = st_try.geo["vh"]
        st = st_try
        g = ns_gradient(st)
        stats["gradients"] += 1
        stats["gn_iters"] += 1
        stats["E"].append(st.E)
        stats["mse_rel"].append(mse_rel(st.m[-1], I0, I1))
        stats["ginf_rel"].append(norm_inf(g) / ginf0)
    else:
        stats["status"] = MAXITER
        if norm_inf(g) / ginf0 < opts.gtol:
            stats["status"] = CONVERGED
    return vh, st.m[-1], stats
