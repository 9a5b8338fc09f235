"""Newton-Krylov time step with BDDC- or FETI-DP-preconditioned CG
(paper Sec. 3b-c, 4, 6).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings:
  * Initial guess u^n unless one is given; the stopping reference is
    ||R(u^n)|| whatever the guess (so a better guess is never judged more
    strictly): stop when ||R(u^k)|| <= rtol ||R(u^n)|| or ||R(u^k)|| <= atol.
  * Globalisation: a full step is accepted when it satisfies the Armijo test
    f(u + l s) <= f(u) + alpha l f'(0) on f = ||R||^2 / 2 with alpha = 1e-4 and
    f'(0) = -||R||^2; otherwise l is reduced by a quadratic (first) and then a
    cubic model, clamped to [0.1 l, 0.5 l].
  * After every update u_e is gauged to zero nodal mean.
  * The Krylov right-hand side has its u_e block projected to zero sum (the
    range of the singular Jacobian).
"""
from __future__ import annotations

import numpy as np

from . import ionic
from .bddc import BDDC
from .bidomain import gauge
from .fetidp import FETIDP
from .krylov import pcg


def project_range(b, N):
    b = b.copy()
    b[N:] -= b[N:].mean()
    return b


def linesearch(resfun, u, s, R, alpha=1e-4, maxit=20, trace=None):
    """Backtracking on f = ||R||^2/2 along the Newton direction s (Sec. 6,
    the nonlinear solver's cubic backtracking line search).

    f'(0) = R.(J s) = -||R||^2 for a Newton direction.  The full step is
    tried first; while the Armijo test f(l) <= f(0) + alpha l f'(0) fails, the
    next l minimises a model of f along s: after the first failure the
    quadratic through f(0), f'(0), f(1); after later failures the cubic
    through f(0), f'(0) and the last two trial values.  Each new l is kept in
    [0.1 l, 0.5 l] of the previous one.  A trial with a non-finite f is not
    modelled: l is halved.  Every l tried is appended to ``trace`` when one
    is given.  Returns (u_new, R_new, lambda, ok); ok is False when no l
    passed the test within ``maxit`` trials (the last trial is returned)."""
    f0 = 0.5 * R @ R
    g0 = -2.0 * f0
    lam = 1.0
    lam_prev = f_prev = None
    for _ in range(maxit):
        if trace is not None:
            trace.append(lam)
        un = u + lam * s
        Rn = resfun(un)
        f = 0.5 * Rn @ Rn
        if np.isfinite(f) and f <= f0 + alpha * lam * g0:
            return un, Rn, lam, True
        if not np.isfinite(f):
            lam = 0.5 * lam
            continue
        if lam_prev is None:
            lt = -g0 / (2.0 * (f - f0 - g0))
        else:
            r1 = f - f0 - lam * g0
            r2 = f_prev - f0 - lam_prev * g0
            a = (r1 / lam ** 2 - r2 / lam_prev ** 2) / (lam - lam_prev)
            b = (-lam_prev * r1 / lam ** 2 + lam * r2 / lam_prev ** 2) / (lam - lam_prev)
            if a == 0.0:
                lt = -g0 / (2.0 * b)
            else:
                disc = max(b * b - 3.0 * a * g0, 0.0)
                lt = (-b + np.sqrt(disc)) / (3.0 * a)
        lam_prev, f_prev = lam, f
        lam = min(max(lt, 0.1 * lam), 0.5 * lam)
    return un, Rn, lam, False


class StepStats:
    def __init__(self):
        self.newton_its = 0
        self.krylov_its = []
        self.res_hist = []
        self.conds = []
        self.lambdas = []


def solve_linear(prob, dec, v, w, b, method, krtol, kmaxit, scaling="deluxe"):
    """Solve J s = b with PCG preconditioned by BDDC, or by FETI-DP on the
    multiplier system followed by recovery.  Returns (s, KrylovResult)."""
    N = prob.N
    bd = BDDC(prob, dec, v, w, scaling=scaling)
    J = prob.jacobian(v, w)
    if method == "bddc":
        res = pcg(lambda x: J @ x, bd.apply, b, rtol=krtol, maxit=kmaxit,
                  project=lambda x: project_range(x, N))
        return res.x, res
    fd = FETIDP(bd)
    bp = project_range(b, N)
    g = fd.condense(bp)
    d = fd.rhs(g)
    res = pcg(fd.F, fd.precond, d, rtol=krtol, maxit=kmaxit)
    zG = fd.recover(g, res.x)
    return fd.expand(bp, zG), res


def time_step(prob, dec, v_n, ue_n, w_n, Is, method="bddc", rtol=1e-8, atol=0.0,
              krtol=1e-10, kmaxit=1000, maxit=20, guess=None, stats=None, scaling="deluxe"):
    """One decoupled BE step: Step 1 gating update, then Newton on Step 2."""
    N = prob.N
    st = stats if stats is not None else StepStats()
    w = ionic.step1(prob.ph, prob.tau, v_n, w_n)

    def resfun(u):
        return prob.residual(u[:N], u[N:], v_n, w, Is)

    u = np.concatenate([v_n, ue_n]) if guess is None else np.concatenate(guess)
    ref = np.linalg.norm(resfun(np.concatenate([v_n, ue_n])))
    R = resfun(u)
    st.res_hist.append(np.linalg.norm(R))
    for _ in range(maxit):
        if np.linalg.norm(R) <= max(rtol * ref, atol):
            break
        s, kres = solve_linear(prob, dec, u[:N], w, -R, method, krtol, kmaxit, scaling)
        st.krylov_its.append(kres.its)
        st.conds.append(kres.cond())
        u, R, lam, ok = linesearch(resfun, u, s, R)
        if not ok:
            raise RuntimeError("line search found no step that decreases ||R||")
        u[N:] = gauge(u[N:])
        st.lambdas.append(lam)
        st.newton_its += 1
        st.res_hist.append(np.linalg.norm(R))
    return u[:N].copy(), u[N:].copy(), w, st
