"""Plain FP64 NumPy oracle of band-limited PDE-LDDMM on the deformation state equation.

TEST INFRASTRUCTURE ONLY: used by the tests, by the smoke check and by the benchmark's CPU
baseline leg.  Nothing in the product library imports, links or runs it, and it shares no
code with the GPU path.

What is computed (paper: Hernandez, arXiv 1807.05117, Section 3.3 with the continuous system
of Section 2.3 and the Gauss-Newton rule of Section 3.4):

  * E(v~) = 1/2 <L~ v~, v~>_l2 + sigma^-2 || m(1) - I1 ||^2 (Section 3.2, equation BLEnergy),
    where m(1) = I0 o phi(1) and the inverse map phi solves the band deformation state
    equation  d_t phi~ + D~phi~ * v~ = 0, phi(0) = id  (Section 3.3; * is the truncated
    convolution of Section 3.1);
  * its gradient  L~ v~ + int_0^1 D~phi~ * rho~ dt  with the band adjoint
    -d_t rho~ - div~(rho~ * v~) = 0 and rho(1) from lambda(1) = -(2/sigma^2)(m(1) - I1)
    (Section 3.3; Section 2.3 final condition);
  * the Gauss-Newton Hessian-vector product: incremental state
    d_t dphi~ + D~dphi~ * v~ + D~phi~ * dv~ = 0, dphi(0) = 0, incremental adjoint
    -d_t drho~ - div~(drho~ * v~) = 0 with drho(1) from dlambda(1) = -(2/sigma^2) dm(1),
    dm(1) = (grad I0 o phi(1)) . dphi(1), and H dv~ = L~ dv~ + int D~phi~ * drho~ dt: the
    terms div~(rho~ * dv~), lambda(1) d(grad m(1)) and D~dphi~ * rho~ are the ones the
    Gauss-Newton rule of Section 3.4 removes;
  * the Gauss-Newton-Krylov solver of Section 3.4 (the same as the state-equation oracle's).

Readings taken where the paper is silent (each is also listed in the design notes; R1-R11
and R-LS, R-PCG, R-gamma are those of the state-equation oracle):
  R-D1 the band state is the displacement u~ = phi~ - id of the inverse map (the identity
       is not band-limited); D~phi~ = I + D~u~, so the state equation reads
       d_t u~ = -v~ - D~u~ * v~, u~(0) = 0, with (D~a * b)_i = sum_j (d~_j a_i) * b_j and the
       spectral derivative d~_j = 2 pi i k_j / l_j (R11);
  R-D2 the truncated convolution of two admissible scalar band fields is
       (a * b)(k) = sum over k' + k'' = k of a(k') b(k''), for k in the band, zero on the
       unpaired planes; it equals pi(iota(a) iota(b)) on any grid with at least
       3 K_j / 2 - 2 points per axis (no product term aliases into the band); the oracle
       uses 2 K_j;
  R-D3 time: Nt uniform steps of the classical fourth-order Runge-Kutta method (explicit
       Heun is not stable for the purely oscillatory modes of this equation);
  R-D4 m(1) = Interp(I0, i + N_ref iota(u~(1))) (d-linear, R9); the gradient of m(1) in the
       final condition is read as (grad I0) o phi(1) = Interp(grad_c I0, i + N_ref iota(u~(1)))
       (R10), the derivative of the data term with respect to phi(1):
       rho~(1) = pi(lambda(1) (grad I0) o phi(1));
  R-D5 the adjoint, incremental state and the time integral of the gradient are the exact
       transpose and linearisation of the Runge-Kutta step.  For the stationary velocity
       this is the Runge-Kutta method on the band adjoint equation, with the integrand
       (I + D~u~)^T * rho~ summed at the four stages with weights dt (1, 2, 2, 1) / 6.
       The discrete Gauss-Newton Hessian is then exactly symmetric for every velocity;
  R8   stationary v~.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .bl_oracle import (CONVERGED, MAXITER, STALLED, Problem, SolverOpts, _constrained, _kl,
                        L_hat, dot, energy, grad_c, interp, iota, mse_rel, norm2, norm_inf, pi_,
                        project)

__all__ = [
    "product_problem", "star", "star_sum", "dband", "conv_D", "adj_A", "conv_DT",
    "def_forward", "DefState", "def_evaluate", "def_transpose", "def_incremental", "def_gradient",
    "def_hessvec", "def_warp",
    "def_register", "def_displacement",
]


# ----------------------------------------------------------------- truncated convolution

def product_problem(prob: Problem) -> Problem:
    """Grid of 2 K_j points per axis with the same band: where iota(a) iota(b) is formed
    (R-D2).  Only the index phases k_j i_j / N_j of iota and pi depend on it."""
    return Problem(prob.dim, tuple(2 * k for k in prob.k), prob.k, prob.nt)


def star(a, b, prob: Problem) -> np.ndarray:
    """a * b of two admissible scalar band fields (R-D2): pi(iota(a) iota(b)) on the
    product grid."""
    Q = product_problem(prob)
    return pi_(iota(a, Q) * iota(b, Q), Q)


def star_sum(pairs, prob: Problem) -> np.ndarray:
    """sum over (a, b) in pairs of a * b, as pi of the summed products (pi is linear)."""
    Q = product_problem(prob)
    acc = np.zeros(Q.shape)
    for a, b in pairs:
        acc += iota(a, Q) * iota(b, Q)
    return pi_(acc, Q)


def dband(a, prob: Problem, j: int) -> np.ndarray:
    """Spectral derivative along spatial axis j: 2 pi i (k_j / l_j) a (R11, R-D1)."""
    return 2j * np.pi * _kl(prob)[j] * a


def conv_D(a, b, prob: Problem) -> np.ndarray:
    """(D~a * b)_i = sum_j (d~_j a_i) * b_j for dim-component band fields a, b (R-D1)."""
    d = prob.dim
    return np.stack([star_sum([(dband(a[i], prob, j), b[j]) for j in range(d)], prob)
                     for i in range(d)])


def adj_A(rho, vh, prob: Problem) -> np.ndarray:
    """div~(rho~ * v~) per component: sum_j d~_j (rho_i * v_j), the operator of the band
    adjoint equation (Section 3.3)."""
    d = prob.dim
    return np.stack([sum(dband(star(rho[i], vh[j], prob), prob, j) for j in range(d))
                     for i in range(d)])


def conv_DT(U, kap, prob: Problem) -> np.ndarray:
    """(D~U)^T * kap: component j is sum_i (d~_j U_i) * kap_i (the gradient integrand's
    deformation term, Section 3.3 D~phi~ * rho~ without the identity)."""
    d = prob.dim
    return np.stack([star_sum([(dband(U[i], prob, j), kap[i]) for i in range(d)], prob)
                     for j in range(d)])


# ---------------------------------------------------------------------------- the path

def _rhs(u, vh, prob):
    """d_t u~ = -v~ - D~u~ * v~ (R-D1)."""
    return -vh - conv_D(u, vh, prob)


def def_forward(vh, prob: Problem):
    """Runge-Kutta steps of the band deformation state equation from u~(0) = 0 (R-D1, R-D3).
    Returns u~(1) and, per step, the four stage states (u_n, U2, U3, U4)."""
    h = prob.dt
    u = np.zeros((prob.dim,) + prob.bshape, dtype=np.complex128)
    stages = []
    for _ in range(prob.nt):
        U1 = u
        k1 = _rhs(U1, vh, prob)
        U2 = u + 0.5 * h * k1
        k2 = _rhs(U2, vh, prob)
        U3 = u + 0.5 * h * k2
        k3 = _rhs(U3, vh, prob)
        U4 = u + h * k3
        k4 = _rhs(U4, vh, prob)
        stages.append((U1, U2, U3, U4))
        u = u + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return u, stages


def def_displacement(u1, prob: Problem):
    """Voxel offsets N_ref iota(u~(1)) of the inverse map phi(1) = id + u(1), spatial order."""
    return [prob.nref * iota(u1[j], prob) for j in range(prob.dim)]


@dataclass
class DefState:
    prob: Problem
    I0: np.ndarray
    I1: np.ndarray
    vh: np.ndarray
    u1: np.ndarray
    stages: list
    m1: np.ndarray      # I0 o phi(1)
    gphi: list          # (grad I0) o phi(1), spatial order
    E: float


def def_evaluate(vh, I0, I1, prob: Problem) -> DefState:
    """State, warped image and energy at v~ (projected first; R-D1, R-D3, R-D4)."""
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    vh = project(vh, prob)
    u1, stages = def_forward(vh, prob)
    off = def_displacement(u1, prob)
    m1 = interp(I0, off, prob)
    gI = grad_c(I0, prob)
    gphi = [interp(gI[j], off, prob) for j in range(prob.dim)]
    return DefState(prob, I0, I1, vh, u1, stages, m1, gphi, energy(vh, m1, I1, prob))


def def_transpose(st: DefState, rho):
    """Minus the transpose of the Runge-Kutta state map dv~ -> du~(1), applied to the final
    cotangent rho~(1) (R-D5): per step, backwards,
        kap4 = h/6 rho,  kap3 = h/3 rho + h A kap4,  kap2 = h/3 rho + h/2 A kap3,
        kap1 = h/6 rho + h/2 A kap2,  rho <- rho + A (kap1 + kap2 + kap3 + kap4),
    with A = div~(. * v~), and the gradient integrand sum_s (I + D~U_s)^T * kap_s."""
    prob, vh, h = st.prob, st.vh, st.prob.dt
    acc = np.zeros_like(rho)
    for n in range(prob.nt - 1, -1, -1):
        U = st.stages[n]
        kap4 = (h / 6.0) * rho
        kap3 = (h / 3.0) * rho + h * adj_A(kap4, vh, prob)
        kap2 = (h / 3.0) * rho + (0.5 * h) * adj_A(kap3, vh, prob)
        kap1 = (h / 6.0) * rho + (0.5 * h) * adj_A(kap2, vh, prob)
        for Us, kap in zip(U, (kap1, kap2, kap3, kap4)):
            acc += kap + conv_DT(Us, kap, prob)
        rho = rho + adj_A(kap1 + kap2 + kap3 + kap4, vh, prob)
    return acc


def def_gradient(st: DefState) -> np.ndarray:
    """g~ = L^ v~ + int (I + D~u~)^T * rho~ dt, rho~(1) = pi(lambda(1) (grad I0) o phi(1)),
    lambda(1) = -(2/sigma^2)(m(1) - I1) (Section 3.3; R-D4, R-D5)."""
    prob, d = st.prob, st.prob.dim
    lam1 = -(2.0 / prob.sigma ** 2) * (st.m1 - st.I1)
    rho = np.stack([pi_(lam1 * st.gphi[j], prob) for j in range(d)])
    acc = def_transpose(st, rho)
    return _constrained(L_hat(prob)[None] * st.vh + acc, prob)


def def_incremental(st: DefState, dvh) -> np.ndarray:
    """du~(1): the Runge-Kutta state map linearised at v~ along dv~ (admissible), i.e. the
    steps of d_t du~ = -dv~ - D~du~ * v~ - D~u~ * dv~ with the stored stage states
    (Section 3.3 incremental state equation; R-D5)."""
    prob, h, vh = st.prob, st.prob.dt, st.vh

    def drhs(dU, U):
        return -dvh - conv_D(dU, vh, prob) - conv_D(U, dvh, prob)

    du = np.zeros_like(vh)
    for n in range(prob.nt):
        U1, U2, U3, U4 = st.stages[n]
        dk1 = drhs(du, U1)
        dk2 = drhs(du + 0.5 * h * dk1, U2)
        dk3 = drhs(du + 0.5 * h * dk2, U3)
        dk4 = drhs(du + h * dk3, U4)
        du = du + (h / 6.0) * (dk1 + 2.0 * dk2 + 2.0 * dk3 + dk4)
    return du


def def_hessvec(st: DefState, dvh) -> np.ndarray:
    """Gauss-Newton product (Section 3.3 second-order system, Section 3.4 rule):
    du~(1) from def_incremental, dm(1) = (grad I0) o phi(1) . iota(du~(1)),
    dlambda(1) = -(2/sigma^2) dm(1), drho~(1) = pi(dlambda(1) (grad I0) o phi(1)), then the
    transposed steps of the gradient."""
    prob, d = st.prob, st.prob.dim
    dvh = project(dvh, prob)
    du = def_incremental(st, dvh)
    dm1 = sum(st.gphi[j] * iota(du[j], prob) for j in range(d))
    dlam1 = -(2.0 / prob.sigma ** 2) * dm1
    drho = np.stack([pi_(dlam1 * st.gphi[j], prob) for j in range(d)])
    acc = def_transpose(st, drho)
    return _constrained(L_hat(prob)[None] * dvh + acc, prob)


def def_warp(I0, vh, prob: Problem) -> np.ndarray:
    """m(1) = I0 o phi(1) with phi from the band deformation state equation."""
    vh = project(vh, prob)
    u1, _ = def_forward(vh, prob)
    return interp(np.asarray(I0, dtype=np.float64), def_displacement(u1, prob), prob)


def def_register(I0, I1, vh0, prob: Problem, opts: SolverOpts = SolverOpts()):
    """The Gauss-Newton-Krylov solver of the state-equation oracle (Section 3.4; readings
    R-LS, R-PCG) on the deformation-state energy, gradient and Gauss-Newton product."""
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    Lh = L_hat(prob)
    vh = project(vh0, prob)
    st = def_evaluate(vh, I0, I1, prob)
    g = def_gradient(st)
    g0n, ginf0 = norm2(g), norm_inf(g)
    stats = {"E": [st.E], "mse_rel": [mse_rel(st.m1, I0, I1)], "ginf_rel": [1.0],
             "pcg_iters": [], "ls_trials": [], "eps": [], "status": MAXITER, "gn_iters": 0,
             "hessvecs": 0, "gradients": 1, "evaluations": 1}
    if ginf0 == 0.0:
        stats["status"] = CONVERGED
        stats["ginf_rel"][0] = 0.0
        return vh, st.m1, stats
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
            Hp = def_hessvec(st, p)
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
        eps, accepted, trials = 1.0, False, 0
        for _t in range(opts.max_halvings + 1):
            trials += 1
            st_try = def_evaluate(vh + eps * delta, I0, I1, prob)
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
        vh = st_try.vh
        st = st_try
        g = def_gradient(st)
        stats["gradients"] += 1
        stats["gn_iters"] += 1
        stats["E"].append(st.E)
        stats["mse_rel"].append(mse_rel(st.m1, I0, I1))
        stats["ginf_rel"].append(norm_inf(g) / ginf0)
    else:
        stats["status"] = MAXITER
        if norm_inf(g) / ginf0 < opts.gtol:
            stats["status"] = CONVERGED
    return vh, st.m1, stats
