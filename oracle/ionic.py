"""Rogers-McCulloch ionic model (paper Sec. 2) and the Step-1 gating update
of the decoupled Backward Euler scheme (Sec. 3b).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The current per unit volume is chi times the membrane current
    I_ion(v, w) = G v (1 - v/v_th)(1 - v/v_p) + eta_1 v w,
and the gating right-hand side is R(v, w) = eta_2 (v/v_p - w).
"""
from __future__ import annotations


def iion(ph, v, w):
    """Volumetric ionic current chi * I_ion(v, w) (Sec. 2)."""
    return ph.chi * (ph.G * v * (1.0 - v / ph.vth) * (1.0 - v / ph.vp) + ph.eta1 * v * w)


def diion_dv(ph, v, w):
    """d(chi I_ion)/dv, by differentiating the cubic term by term."""
    cubic = (1.0 - v / ph.vth) * (1.0 - v / ph.vp) \
        - v / ph.vth * (1.0 - v / ph.vp) - v / ph.vp * (1.0 - v / ph.vth)
    return ph.chi * (ph.G * cubic + ph.eta1 * w)


def gating_rhs(ph, v, w):
    """R(v, w) = eta_2 (v/v_p - w) (Sec. 2)."""
    return ph.eta2 * (v / ph.vp - w)


def step1(ph, tau, v_n, w_n):
    """Step 1: solve w^{n+1} - tau R(v^n, w^{n+1}) = w^n (Sec. 3b).

    R is affine in w, so the equation is linear in w^{n+1}:
    w^{n+1} (1 + tau eta_2) = w^n + tau eta_2 v^n / v_p."""
    return (w_n + tau * ph.eta2 * v_n / ph.vp) / (1.0 + tau * ph.eta2)
