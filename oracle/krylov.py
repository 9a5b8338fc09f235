"""Preconditioned conjugate gradients with a Lanczos estimate of the
extreme eigenvalues (paper Sec. 4.1 and the condition numbers of Sec. 6).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings: zero initial guess; stop when the unpreconditioned residual
satisfies ||r_k||_2 <= rtol ||r_0||_2; beta by the Polak-Ribiere formula
beta_k = z_{k+1}.(r_{k+1} - r_k) / z_k.r_k (equal to Fletcher-Reeves in exact
arithmetic for a fixed SPD preconditioner); divergence when
||r_k|| > dtol ||r_0||.
"""
from __future__ import annotations

import numpy as np


class KrylovResult:
    def __init__(self, x, its, hist, alphas, betas, status):
        self.x = x
        self.its = its
        self.hist = hist
        self.alphas = alphas
        self.betas = betas
        self.status = status        # 0 converged, 1 maxit, 2 diverged

    def lanczos_extremes(self):
        """Extreme eigenvalues of the Lanczos tridiagonal built from the CG
        coefficients: T_kk = 1/a_k + b_{k-1}/a_{k-1}, T_k,k+1 = sqrt(b_k)/a_k."""
        a, b = self.alphas, self.betas
        k = len(a)
        if k == 0:
            return 1.0, 1.0
        T = np.zeros((k, k))
        for i in range(k):
            T[i, i] = 1.0 / a[i] + (b[i - 1] / a[i - 1] if i > 0 else 0.0)
            if i + 1 < k:
                T[i, i + 1] = T[i + 1, i] = np.sqrt(max(b[i], 0.0)) / a[i]
        ev = np.linalg.eigvalsh(T)
        return ev[0], ev[-1]

    def cond(self):
        lo, hi = self.lanczos_extremes()
        return hi / lo


def pcg(A, M, b, rtol=1e-10, maxit=1000, dtol=1e4, project=None):
    """PCG for A x = b with preconditioner M (callables)."""
    if project is not None:
        b = project(b)
    x = np.zeros_like(b)
    r = b.copy()
    r0 = np.linalg.norm(r)
    hist = [r0]
    alphas, betas = [], []
    if r0 == 0.0:
        return KrylovResult(x, 0, hist, alphas, betas, 0)
    z = M(r)
    p = z.copy()
    rz = r @ z
    status = 1
    its = 0
    for k in range(maxit):
        q = A(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r_old = r
        r = r - alpha * q
        its = k + 1
        alphas.append(alpha)
        rn = np.linalg.norm(r)
        hist.append(rn)
        if rn <= rtol * r0:
            status = 0
            break
        if rn > dtol * r0:
            status = 2
            break
        z = M(r)
        rz_new = z @ (r - r_old)
        beta = rz_new / rz
        rz = r @ z
        betas.append(beta)
        p = z + beta * p
    return KrylovResult(x, its, hist, alphas, betas, status)
