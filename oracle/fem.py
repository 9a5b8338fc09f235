"""Q1 finite elements on a structured box (paper Sec. 3a) and the
anisotropic conductivity tensors (Sec. 2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Nodes are numbered lexicographically, x fastest:
    node(i, j, k) = i + (nx+1) * (j + (ny+1) * k).
Element (ex, ey, ez) owns the 8 nodes (ex+a, ey+b, ez+c), local index
a + 2b + 4c.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def node_id(mesh, i, j, k):
    return i + (mesh.nx + 1) * (j + (mesh.ny + 1) * k)


def element_nodes(mesh, ex, ey, ez):
    return [node_id(mesh, ex + a, ey + b, ez + c)
            for c in (0, 1) for b in (0, 1) for a in (0, 1)]


def fibre_angle(physics, zc, Lz):
    """Fibres rotate linearly through the thickness (Sec. 6, 120 degrees in
    total), in the xy-plane; evaluated at an element centroid height zc."""
    return physics.theta0 + (physics.theta1 - physics.theta0) * zc / Lz


def conductivity(sig, theta):
    """D = sum_{l,t,n} sigma_* a_* a_*^T with the orthonormal fibre frame
    a_l = (cos, sin, 0), a_t = (-sin, cos, 0), a_n = (0, 0, 1) (Sec. 2; the
    printed formula omits the outer product)."""
    al = np.array([math.cos(theta), math.sin(theta), 0.0])
    at = np.array([-math.sin(theta), math.cos(theta), 0.0])
    an = np.array([0.0, 0.0, 1.0])
    return sig[0] * np.outer(al, al) + sig[1] * np.outer(at, at) + sig[2] * np.outer(an, an)


_GP = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))


def _q1_basis(s, t, u):
    """Values and reference gradients of the 8 trilinear basis functions at
    (s, t, u) in [0,1]^3."""
    val = np.empty(8)
    grad = np.empty((8, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                n = a + 2 * b + 4 * c
                fx = s if a else 1 - s
                fy = t if b else 1 - t
                fz = u if c else 1 - u
                dx = 1.0 if a else -1.0
                dy = 1.0 if b else -1.0
                dz = 1.0 if c else -1.0
                val[n] = fx * fy * fz
                grad[n] = (dx * fy * fz, fx * dy * fz, fx * fy * dz)
    return val, grad


def _sizes(h):
    """(hx, hy, hz) from a cube side or a 3-tuple of box sizes."""
    return (h, h, h) if np.isscalar(h) else tuple(h)


def element_stiffness(D, h):
    """{A}_nm = int_e grad(phi_n)^T D grad(phi_m) on a box element of sizes
    h = (hx, hy, hz) (or a cube of side h), with 2x2x2 Gauss quadrature
    (exact for constant D on a box): the map from the unit cube scales the
    gradients by 1/h_d per axis and the volume by hx hy hz."""
    hx, hy, hz = _sizes(h)
    A = np.zeros((8, 8))
    w = hx * hy * hz / 8.0
    for s in _GP:
        for t in _GP:
            for u in _GP:
                _, g = _q1_basis(s, t, u)
                g = g / np.array([hx, hy, hz])
                A += w * g @ D @ g.T
    return A


def element_mass(h):
    """Consistent Q1 element mass {M}_nm = int_e phi_n phi_m (2x2x2 Gauss) on
    a box element of sizes h = (hx, hy, hz) (or a cube of side h)."""
    hx, hy, hz = _sizes(h)
    Me = np.zeros((8, 8))
    w = hx * hy * hz / 8.0
    for s in _GP:
        for t in _GP:
            for u in _GP:
                v, _ = _q1_basis(s, t, u)
                Me += w * np.outer(v, v)
    return Me


def layer_stiffness(mesh, physics):
    """Per z-layer element stiffness matrices for the two media."""
    hs = mesh.spacing
    Lz = mesh.nz * hs[2]
    Ai, Ae = [], []
    for ez in range(mesh.nz):
        th = fibre_angle(physics, (ez + 0.5) * hs[2], Lz)
        Ai.append(element_stiffness(conductivity(physics.sigma_i, th), hs))
        Ae.append(element_stiffness(conductivity(physics.sigma_e, th), hs))
    return Ai, Ae


def elements(mesh, box=None):
    """Yield (ex, ey, ez) for the elements of the mesh or of the element box
    ((x0,x1),(y0,y1),(z0,z1)), half-open."""
    if box is None:
        box = ((0, mesh.nx), (0, mesh.ny), (0, mesh.nz))
    for ez in range(*box[2]):
        for ey in range(*box[1]):
            for ex in range(*box[0]):
                yield ex, ey, ez


def element_node_table(mesh, box=None):
    """(E, 8) node ids and (E,) z-layer of the elements of the mesh or box."""
    if box is None:
        box = ((0, mesh.nx), (0, mesh.ny), (0, mesh.nz))
    ez, ey, ex = np.meshgrid(np.arange(*box[2]), np.arange(*box[1]), np.arange(*box[0]),
                             indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    cols = []
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                cols.append(node_id(mesh, ex + a, ey + b, ez + c))
    return np.stack(cols, axis=1), ez


def assemble(mesh, physics, box=None):
    """Global (or box-restricted) stiffness A_i, A_e and lumped mass M.

    A = sum_e P_e^T A^e P_e over the elements; the lumped mass is the row sum
    of the consistent mass ("usual mass lumping", Sec. 3a).  Matrices are
    over all mesh nodes; rows of nodes outside the box are empty."""
    Ai_l, Ae_l = layer_stiffness(mesh, physics)
    Me = element_mass(mesh.spacing)
    en, lay = element_node_table(mesh, box)
    rows = np.repeat(en, 8, axis=1).ravel()          # (e, a, b) -> node a
    cols = np.tile(en, (1, 8)).ravel()               # (e, a, b) -> node b
    vi = np.stack(Ai_l)[lay].ravel()
    ve = np.stack(Ae_l)[lay].ravel()
    n = mesh.nnodes
    Ai = sp.csr_matrix((vi, (rows, cols)), shape=(n, n))
    Ae = sp.csr_matrix((ve, (rows, cols)), shape=(n, n))
    m = np.zeros(n)
    np.add.at(m, en.ravel(), np.tile(Me.sum(axis=1), len(lay)))
    return Ai, Ae, m
