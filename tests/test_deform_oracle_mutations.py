"""Mutation check of the deformation-state oracle's pins: each plausible mistake is planted in a
fresh copy of oracle/bl_deform.py, and at least one pin of deform_pin_checks.py must then fail
(the expected values there never come from the oracle)."""
import itertools
import os
import sys
import types

import pytest

import deform_pin_checks as P

SRC = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "oracle", "bl_deform.py")).read()
_serial = itertools.count()


def load(src):
    name = f"_deform_copy_{next(_serial)}"
    mod = types.ModuleType(name)
    sys.modules[name] = mod
    try:
        exec(compile(src.replace("from .bl_oracle import", "from oracle.bl_oracle import"),
                     name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


# (name, check, bound): a pin passes when every value it returns is within its bound
PINS = [
    ("star", lambda D: P.check_star_bruteforce(D) < 1e-12),
    ("transposes", lambda D: P.check_transposes(D) < 1e-12),
    ("zero velocity", lambda D: max(P.check_zero_velocity(D)) < 1e-10),
    ("constant velocity", lambda D: (lambda r: r[0] < 1e-12 and r[1] < 1e-5 and r[2] < 1e-5)(
        P.check_constant_velocity(D))),
    ("inverse flow", lambda D: P.check_inverse_flow(D) < 5e-5),
    ("state map derivatives", lambda D: max(P.check_state_map_derivatives(D)) < 1e-7),
    ("symmetry", lambda D: (lambda r: r[0] < 1e-12 and r[1] > 0.999)(P.check_symmetry(D))),
    ("fd gradient", lambda D: P.check_fd_gradient(D) < 0.02),
    ("fd hessian", lambda D: P.check_fd_hessian_zero_residual(D) < 0.06),
]

MUTATIONS = [
    ("velocity sign in the state equation", "return -vh - conv_D(u, vh, prob)",
     "return vh - conv_D(u, vh, prob)"),
    ("dropped convolution term", "return -vh - conv_D(u, vh, prob)", "return -vh + 0 * vh"),
    ("Runge-Kutta weights", "(k1 + 2.0 * k2 + 2.0 * k3 + k4)", "(2.0 * k1 + k2 + k3 + 2.0 * k4)"),
    ("third stage from the first slope", "U3 = u + 0.5 * h * k2", "U3 = u + 0.5 * h * k1"),
    ("derivative without 2 pi", "return 2j * np.pi * _kl(prob)[j] * a",
     "return 1j * _kl(prob)[j] * a"),
    ("derivative index swapped in D~a * b", "star_sum([(dband(a[i], prob, j), b[j])",
     "star_sum([(dband(a[j], prob, i), b[j])"),
    ("adjoint divergence along the wrong axis", "dband(star(rho[i], vh[j], prob), prob, j)",
     "dband(star(rho[i], vh[j], prob), prob, i)"),
    ("transposed deformation term not transposed", "star_sum([(dband(U[i], prob, j), kap[i])",
     "star_sum([(dband(U[j], prob, i), kap[i])"),
    ("product grid too small (aliasing)", "tuple(2 * k for k in prob.k)", "tuple(k for k in prob.k)"),
    ("adjoint stage coefficient", "kap3 = (h / 3.0) * rho + h * adj_A(kap4",
     "kap3 = (h / 3.0) * rho + 0.5 * h * adj_A(kap4"),
    ("identity dropped from (I + D~U)^T", "acc += kap + conv_DT(Us, kap, prob)",
     "acc += conv_DT(Us, kap, prob)"),
    ("adjoint propagation sign", "rho = rho + adj_A(kap1 + kap2 + kap3 + kap4, vh, prob)",
     "rho = rho - adj_A(kap1 + kap2 + kap3 + kap4, vh, prob)"),
    ("image gradient not composed with phi(1)", "gphi = [interp(gI[j], off, prob)",
     "gphi = [gI[j] + 0 * interp(gI[j], off, prob)"),
    ("offsets in domain units", "return [prob.nref * iota(u1[j], prob)",
     "return [iota(u1[j], prob)"),
    ("lambda sign", "lam1 = -(2.0 / prob.sigma ** 2) * (st.m1 - st.I1)",
     "lam1 = (2.0 / prob.sigma ** 2) * (st.m1 - st.I1)"),
    ("incremental source without D~u~ * dv~", "return -dvh - conv_D(dU, vh, prob) - conv_D(U, dvh, prob)",
     "return -dvh - conv_D(dU, vh, prob)"),
    ("incremental adjoint sign", "dlam1 = -(2.0 / prob.sigma ** 2) * dm1",
     "dlam1 = (2.0 / prob.sigma ** 2) * dm1"),
    ("stage states stored one step late", "stages.append((U1, U2, U3, U4))",
     "stages.append((U2, U2, U3, U4))"),
]


def test_mutations_are_distinct_and_apply():
    for name, old, new in MUTATIONS:
        assert SRC.count(old) == 1, name
        assert old != new


def test_unmutated_oracle_passes_every_pin():
    D = load(SRC)
    for pname, ok in PINS:
        assert ok(D), pname


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new):
    D = load(SRC.replace(old, new))
    for pname, ok in PINS:
        try:
            passed = ok(D)
        except Exception:           # a mistake that breaks the code is caught too
            passed = False
        if not passed:
            return
    pytest.fail(f"no pin catches: {name}")
