"""Backward-Euler Bidomain residual and Jacobian in the (v, u_e) unknowns,
and the direct-sparse Newton reference solution (paper Sec. 3b-c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Global vectors are blocked [v (N) ; u_e (N)].  The paper writes Step 2 as
F(u) = G in u = (u_i, u_e).  With u = T (v, u_e), T = [[I, I], [0, I]], the
oracle solves the congruent system T^T (F(T x) - G) = 0, i.e. its first row
is the u_i equation and its second row is the sum of the two equations.  The
stimulus is applied as a transmembrane current I_s (I_app^i = I_app^e = I_s),
which satisfies the compatibility condition by construction.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, ionic


class Problem:
    """Mesh, physics and assembled operators of one slab workload."""

    def __init__(self, mesh, physics, dt):
        self.mesh = mesh
        self.ph = physics
        self.tau = dt
        self.c = physics.chi * physics.Cm
        self.Ai, self.Ae, self.m = fem.assemble(mesh, physics)
        self.N = mesh.nnodes

    # -- paper block operators in (u_i, u_e) -------------------------------
    def _blocks(self):
        M = sp.diags(self.m)
        Mcal = sp.bmat([[M, -M], [-M, M]])                 # script M (Sec. 3a)
        Acal = sp.bmat([[self.Ai, None], [None, self.Ae]])  # script A (Sec. 3a)
        return M, Mcal, Acal

    def T(self):
        I = sp.identity(self.N)
        return sp.bmat([[I, I], [None, I]]).tocsr()

    def residual_paper(self, ui, ue, v_n, ue_n, w, Is):
        """F(u) - G of Step 2 (Sec. 3b) in (u_i, u_e), with G carrying the
        transmembrane stimulus tau [M I_s ; -M I_s]."""
        M, Mcal, Acal = self._blocks()
        u = np.concatenate([ui, ue])
        un = np.concatenate([v_n + ue_n, ue_n])
        v = ui - ue
        I = ionic.iion(self.ph, v, w)
        F = (self.c * Mcal + self.tau * Acal) @ u + self.tau * np.concatenate([M @ I, -(M @ I)])
        G = self.c * (Mcal @ un) + self.tau * np.concatenate([M @ Is, -(M @ Is)])
        return F - G

    def residual(self, v, ue, v_n, w, Is):
        """R(v, u_e) = T^T (F - G) evaluated at u = T (v, u_e)."""
        ue_n = np.zeros_like(v_n)          # G depends on u^n only through v^n
        Rp = self.residual_paper(v + ue, ue, v_n, ue_n, w, Is)
        return self.T().T @ Rp

    def jacobian(self, v, w):
        """J = T^T JF T with JF the Jacobian of F in (u_i, u_e) (Sec. 3c);
        the reaction term is diagonal because I_ion is evaluated at nodes and
        multiplied by the lumped mass."""
        M, Mcal, Acal = self._blocks()
        Dp = sp.diags(self.m * ionic.diion_dv(self.ph, v, w))
        JF = self.c * Mcal + self.tau * Acal + self.tau * sp.bmat([[Dp, -Dp], [-Dp, Dp]])
        T = self.T()
        return (T.T @ JF @ T).tocsr()

    def reaction_diag(self, v, w):
        """Lumped reaction diagonal m_l (chi C_m + tau dI_ion/dv(v_l, w_l)); its
        positivity is the hypothesis of the coercivity lemma (Sec. 3c)."""
        return self.m * (self.c + self.tau * ionic.diion_dv(self.ph, v, w))


def gauge(ue):
    """u_e is defined up to a constant; fix the arithmetic nodal mean to 0."""
    return ue - ue.mean()


def direct_newton_solve(J, R, N):
    """Solve J s = -R with the bordered system [[J, e], [e^T, 0]], e = (0, 1/N)
    on the u_e block, which removes the constant-u_e kernel."""
    e = np.concatenate([np.zeros(N), np.full(N, 1.0 / N)])
    K = sp.bmat([[J, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]]).tocsc()
    rhs = np.concatenate([-R, [0.0]])
    x = spla.spsolve(K, rhs)
    return x[:-1]


def cg_newton_solve(J, R, N, rtol=1e-14):
    """Solve J s = -R by conjugate gradients with the Jacobi preconditioner
    (SciPy), on the right-hand side with its u_e block projected to zero sum
    (the range of the singular Jacobian); s is gauged afterwards.  Used on
    meshes where a sparse direct factorisation of the 3-D stencil takes
    minutes; the Newton loop then checks the root by its own residual."""
    b = -R.copy()
    b[N:] -= b[N:].mean()
    Minv = sp.diags(1.0 / J.diagonal())
    s, info = spla.cg(J, b, rtol=rtol, atol=0.0, maxiter=50 * int(np.sqrt(J.shape[0])) + 1000, M=Minv)
    s[N:] -= s[N:].mean()
    return s


def time_step_direct(prob, v_n, ue_n, w_n, Is, rtol=1e-13, maxit=30, linear="direct"):
    """One decoupled Backward-Euler step (Sec. 3b) with Newton (Sec. 3c): the
    reference root of R(u) = 0.  Each Newton system is solved by the sparse
    direct bordered solve (linear="direct") or by Jacobi-preconditioned CG to
    relative 1e-14 (linear="cg"); either way Newton runs until
    ||R|| <= rtol ||R(u^n)|| or stops reducing it (round-off level)."""
    N = prob.N
    solve = {"direct": direct_newton_solve, "cg": cg_newton_solve}[linear]
    w = ionic.step1(prob.ph, prob.tau, v_n, w_n)
    v, ue = v_n.copy(), ue_n.copy()
    R = prob.residual(v, ue, v_n, w, Is)
    r0 = np.linalg.norm(R)
    hist = [r0]
    for _ in range(maxit):
        if hist[-1] <= rtol * r0 or hist[-1] == 0.0:
            break
        s = solve(prob.jacobian(v, w), R, N)
        v = v + s[:N]
        ue = gauge(ue + s[N:])
        R = prob.residual(v, ue, v_n, w, Is)
        hist.append(np.linalg.norm(R))
        if len(hist) > 2 and hist[-1] >= 0.5 * hist[-2]:
            break                           # no further progress: round-off level
    return v, ue, w, hist
