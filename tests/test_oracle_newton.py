"""Pins of the oracle's Newton globalisation (Sec. 6: Newton with cubic
backtracking) and of its CG-based Newton root.

The line search is driven on merit functions whose restriction to the search
line is a known polynomial f(l) with f'(0) = -2 f(0) (a Newton direction).
When f is quadratic, the quadratic model is exact, so the first backtracking
step must be the exact minimiser of f; when f is cubic, the cubic model
through f(0), f'(0) and two trial values is exact, so the second backtracking
step must be the exact local minimiser of f.  Both minimisers are written out
here by hand from the polynomial, not from the line search's formulas.
"""
import math

import numpy as np
import pytest

from oracle import bidomain, dd, newton
from workload import Mesh, workload


def _line_residual(phi, s):
    """resfun whose merit function along u = l s is phi(l): R = sqrt(2 phi)."""
    def resfun(u):
        lam = float(u @ s / (s @ s))
        val = phi(lam)
        return np.array([math.sqrt(2.0 * val) if val >= 0 and math.isfinite(val) else float("nan")])
    return resfun


def _run(phi, maxit=20):
    s = np.array([1.0])
    u0 = np.array([0.0])
    R0 = _line_residual(phi, s)(u0)
    trace = []
    un, Rn, lam, ok = newton.linesearch(_line_residual(phi, s), u0, s, R0, maxit=maxit, trace=trace)
    return lam, ok, trace


def test_full_step_accepted_when_armijo_holds():
    lam, ok, trace = _run(lambda l: 1.0 - 2.0 * l + 1.5 * l * l)
    assert ok and lam == 1.0 and trace == [1.0]


def test_quadratic_backtrack_is_exact_minimiser():
    # f = 1 - 2 l + 3 l^2: f(1) = 2 fails Armijo; minimiser l* = 1/3
    lam, ok, trace = _run(lambda l: 1.0 - 2.0 * l + 3.0 * l * l)
    assert ok
    assert trace[0] == 1.0
    assert lam == pytest.approx(1.0 / 3.0, rel=1e-14)
    assert len(trace) == 2


def test_cubic_backtrack_is_exact_local_minimiser():
    # f = 1 - 2 l + 9 l^2 - 6 l^3: f(1) = 2 fails; the quadratic through f(0),
    # f'(0), f(1) has its minimum at 1/3, where f = 10/9 still fails; f' = 0
    # gives l^2 - l + 1/9 = 0, local minimum l = (3 - sqrt 5) / 6, inside
    # [0.1, 0.5] of 1/3, where Armijo holds.
    lam, ok, trace = _run(lambda l: 1.0 - 2.0 * l + 9.0 * l * l - 6.0 * l ** 3)
    assert ok
    assert len(trace) == 3
    assert trace[1] == pytest.approx(1.0 / 3.0, rel=1e-14)
    assert lam == pytest.approx((3.0 - math.sqrt(5.0)) / 6.0, rel=1e-12)


def test_backtrack_clamped_to_tenth():
    # f = 1 - 2 l + 100 l^2: the quadratic minimiser 0.01 lies below 0.1 of
    # the previous step, so the clamp takes l = 0.1; f(0.1) = 1.8 fails and
    # the cubic model (exact for this quadratic) again asks for 0.01, clamped
    # to 0.1 * 0.1, where Armijo holds.
    lam, ok, trace = _run(lambda l: 1.0 - 2.0 * l + 100.0 * l * l)
    assert ok
    assert trace[1] == pytest.approx(0.1, rel=1e-15)
    assert lam == pytest.approx(0.01, rel=1e-12)


def test_non_finite_trial_is_halved_and_failure_reported():
    # f is not finite for l > 0.3: 1 -> 0.5 -> 0.25 by halving, then the
    # function is the quadratic above with minimiser 1/3 > 0.25: Armijo holds
    lam, ok, trace = _run(lambda l: float("inf") if l > 0.3 else 1.0 - 2.0 * l + 3.0 * l * l)
    assert ok and trace == [1.0, 0.5, 0.25] and lam == 0.25
    # a merit function that never decreases: no step passes within maxit
    lam, ok, trace = _run(lambda l: 1.0 + l, maxit=5)
    assert not ok and len(trace) == 5


def test_backtracking_newton_reaches_the_direct_root():
    """A long time step (tau = 0.3 ms, inside the 0.366 ms coercivity bound
    of Sec. 3c) from v near (v_th + v_p)/3, where dI_ion/dv is most negative:
    the reaction diagonal is small, the first Newton steps are long and the
    full step fails Armijo.  The globalised Newton (quadratic, then cubic
    steps) ends at the same root as the plain Newton with direct solves."""
    wl = workload("slab8_supra")
    prob = bidomain.Problem(wl.mesh, wl.physics, 0.3)
    dec = dd.Decomposition(wl.mesh)
    N = prob.N
    v = 37.67 + np.random.default_rng(3).uniform(-1, 1, N)
    z = np.zeros(N)
    st = newton.StepStats()
    vv, uu, _, st = newton.time_step(prob, dec, v, z, z, z, stats=st)
    assert min(st.lambdas) < 1.0
    # at least one step that is neither 1 nor a clamp value (a model minimiser)
    assert any(0.1 < l < 0.5 and abs(l - 0.25) > 1e-3 for l in st.lambdas), st.lambdas
    vr, ur, _, _ = bidomain.time_step_direct(prob, v, z, z, z)
    assert np.linalg.norm(vv - vr) / np.linalg.norm(vr) < 1e-10
    assert np.linalg.norm(uu - ur) / np.linalg.norm(ur) < 1e-10


@pytest.mark.parametrize("mesh", [workload("slab8").mesh,
                                  Mesh(11, 9, 10, 0.01, (0, 3, 7, 11), (0, 5, 9), (0, 4, 10))])
def test_cg_newton_root_equals_direct_root(mesh):
    """The CG-based Newton (Jacobi-preconditioned CG per Newton system) and
    the direct bordered solve reach the same root of R(u) = 0."""
    wl = workload("slab8")
    prob = bidomain.Problem(mesh, wl.physics, wl.solver.dt)
    N = prob.N
    rng = np.random.default_rng(5)
    vn = rng.uniform(-10, 40, N)
    w = rng.uniform(0, 0.1, N)
    Is = np.zeros(N)
    Is[:50] = 1e5
    a = bidomain.time_step_direct(prob, vn, np.zeros(N), w, Is)
    b = bidomain.time_step_direct(prob, vn, np.zeros(N), w, Is, linear="cg")
    for x, y in zip(a[:2], b[:2]):
        assert np.linalg.norm(x - y) / np.linalg.norm(x) < 1e-11
    R = prob.residual(b[0], b[1], vn, b[2], Is)
    assert np.linalg.norm(R) <= 1e-12 * b[3][0]
