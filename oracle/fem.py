"""Q1 finite elements on a structured box (paper Sec. 3a) and the
anisotropic conductivity tensors (Sec. 2); isoparametric Q1 elements on the
truncated-ellipsoid geometry of Sec. 6.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Nodes are numbered lexicographically, x fastest:
    node(i, j, k) = i + (nx+1) * (j + (ny+1) * k).
Element (ex, ey, ez) owns the 8 nodes (ex+a, ey+b, ez+c), local index
a + 2b + 4c.

On the ellipsoid the same logical grid is mapped to the ellipsoidal
coordinates (phi, theta, r): node i along x sits at phi_min + i (phi_max -
phi_min) / nx, node j along y at theta_min + j (theta_max - theta_min) / ny,
node k along z at r = k / nz (r = 0 the inner surface, r = 1 the outer).
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


# ------------------------------------------------------------ ellipsoid (Sec. 6)
def ellipsoid_axes(g, r):
    """a(r), b(r), c(r): each main axis linear in r from its inner value
    (a_1, b_1, c_1) to its outer value (a_2, b_2, c_2)."""
    a1, a2, b1, b2, c1, c2 = g[:6]
    return a1 + r * (a2 - a1), b1 + r * (b2 - b1), c1 + r * (c2 - c1)


def ellipsoid_point(g, r, theta, phi):
    """The parametric map of the truncated ellipsoid (Sec. 6): x = a cos(theta)
    cos(phi), y = b cos(theta) sin(phi), z = c sin(theta).  The printed
    z-component has sin(phi); read as sin(theta), the form for which the
    surfaces r = const are ellipsoids with axes a(r), b(r), c(r)."""
    a, b, c = ellipsoid_axes(g, r)
    return np.stack([a * np.cos(theta) * np.cos(phi), b * np.cos(theta) * np.sin(phi),
                     c * np.sin(theta)], axis=-1)


def ellipsoid_params(mesh, i, j, k):
    """(r, theta, phi) of the (possibly fractional) grid position (i, j, k)."""
    g = mesh.ellipsoid
    phi = g[8] + (g[9] - g[8]) * np.asarray(i, dtype=float) / mesh.nx
    theta = g[6] + (g[7] - g[6]) * np.asarray(j, dtype=float) / mesh.ny
    r = np.asarray(k, dtype=float) / mesh.nz
    return r, theta, phi


def node_coords(mesh):
    """(N, 3) physical node coordinates of the ellipsoid mesh."""
    k, j, i = np.meshgrid(np.arange(mesh.nz + 1), np.arange(mesh.ny + 1), np.arange(mesh.nx + 1),
                          indexing="ij")
    r, th, ph = ellipsoid_params(mesh, i.ravel(), j.ravel(), k.ravel())
    return ellipsoid_point(mesh.ellipsoid, r, th, ph)


def ellipsoid_frame(g, r, theta, phi):
    """Orthonormal frame (e1, e2, n) at a point: e1 along the circumferential
    tangent dX/dphi, e2 the longitudinal tangent dX/dtheta made orthogonal to
    e1 (Gram-Schmidt), n = e1 x e2 the transmural direction.  On a slab the
    same construction gives (x, y, z)."""
    a, b, c = ellipsoid_axes(g, r)
    xp = np.stack([-a * np.cos(theta) * np.sin(phi), b * np.cos(theta) * np.cos(phi),
                   np.zeros_like(np.asarray(theta, dtype=float))], axis=-1)
    xt = np.stack([-a * np.sin(theta) * np.cos(phi), -b * np.sin(theta) * np.sin(phi),
                   c * np.cos(theta)], axis=-1)
    e1 = xp / np.linalg.norm(xp, axis=-1, keepdims=True)
    t = xt - np.sum(xt * e1, axis=-1, keepdims=True) * e1
    e2 = t / np.linalg.norm(t, axis=-1, keepdims=True)
    return e1, e2, np.cross(e1, e2)


def conductivity_in_frame(sig, alpha, e1, e2, n):
    """D = sum sigma_* a_* a_*^T (Sec. 2) with the fibre a_l at angle alpha
    from e1 in the tangent plane, a_t its in-plane normal and a_n = n; the
    fibres rotate with depth as on the slab (Sec. 6)."""
    al = np.cos(alpha)[..., None] * e1 + np.sin(alpha)[..., None] * e2
    at = -np.sin(alpha)[..., None] * e1 + np.cos(alpha)[..., None] * e2
    outer = lambda u: u[..., :, None] * u[..., None, :]
    return sig[0] * outer(al) + sig[1] * outer(at) + sig[2] * outer(n)


def iso_element_matrices(X, D_list):
    """Isoparametric Q1 elements (Sec. 3a on a mapped hexahedron): for the
    elements' node coordinates X (E, 8, 3) and tensors D (E, 3, 3) per
    medium, the stiffness int_e grad(phi_a)^T D grad(phi_b) and the lumped
    mass int_e phi_a (row sums of the consistent mass, since the basis sums
    to one), both by 2x2x2 Gauss quadrature on the reference cube with the
    Jacobian J = dx/dxi of the trilinear map.  Returns ([A (E, 8, 8) per
    medium], m (E, 8)); raises on a non-positive Jacobian determinant."""
    E = X.shape[0]
    As = [np.zeros((E, 8, 8)) for _ in D_list]
    m = np.zeros((E, 8))
    for s in _GP:
        for t in _GP:
            for u in _GP:
                val, g = _q1_basis(s, t, u)
                J = np.einsum("ead,ar->edr", X, g)
                det = np.linalg.det(J)
                if np.any(det <= 0.0):
                    raise ValueError("isoparametric element with a non-positive Jacobian")
                Jinv = np.linalg.inv(J)
                G = np.einsum("ar,erd->ead", g, Jinv)        # physical gradients
                w = det / 8.0                                # Gauss weights 1/2 per axis
                for A, D in zip(As, D_list):
                    A += w[:, None, None] * np.einsum("ead,edf,ebf->eab", G, D, G)
                m += w[:, None] * val[None, :]
    return As, m


def ellipsoid_elements(mesh, physics, box=None):
    """Per-element stiffness (tau-free) of both media and lumped masses of
    the ellipsoid mesh or of an element box: node coordinates from the
    parametric map, the tensor of each element from the frame at its
    parametric centre and the fibre angle at its centre depth."""
    en, ez = element_node_table(mesh, box)
    Xn = node_coords(mesh)
    X = Xn[en]                                            # (E, 8, 3)
    i0 = en[:, 0] % (mesh.nx + 1)
    j0 = (en[:, 0] // (mesh.nx + 1)) % (mesh.ny + 1)
    r, th, ph = ellipsoid_params(mesh, i0 + 0.5, j0 + 0.5, ez + 0.5)
    e1, e2, n = ellipsoid_frame(mesh.ellipsoid, r, th, ph)
    alpha = physics.theta0 + (physics.theta1 - physics.theta0) * r
    Di = conductivity_in_frame(physics.sigma_i, alpha, e1, e2, n)
    De = conductivity_in_frame(physics.sigma_e, alpha, e1, e2, n)
    (Ai, Ae), m = iso_element_matrices(X, [Di, De])
    return en, Ai, Ae, m


def assemble(mesh, physics, box=None):
    """Global (or box-restricted) stiffness A_i, A_e and lumped mass M.

    A = sum_e P_e^T A^e P_e over the elements; the lumped mass is the row sum
    of the consistent mass ("usual mass lumping", Sec. 3a).  Matrices are
    over all mesh nodes; rows of nodes outside the box are empty."""
    if getattr(mesh, "ellipsoid", ()):
        en, Ai_e, Ae_e, m_e = ellipsoid_elements(mesh, physics, box)
        vi, ve, mv = Ai_e.ravel(), Ae_e.ravel(), m_e.ravel()
    else:
        Ai_l, Ae_l = layer_stiffness(mesh, physics)
        Me = element_mass(mesh.spacing)
        en, lay = element_node_table(mesh, box)
        vi = np.stack(Ai_l)[lay].ravel()
        ve = np.stack(Ae_l)[lay].ravel()
        mv = np.tile(Me.sum(axis=1), len(lay))
    rows = np.repeat(en, 8, axis=1).ravel()          # (e, a, b) -> node a
    cols = np.tile(en, (1, 8)).ravel()               # (e, a, b) -> node b
    n = mesh.nnodes
    Ai = sp.csr_matrix((vi, (rows, cols)), shape=(n, n))
    Ae = sp.csr_matrix((ve, (rows, cols)), shape=(n, n))
    m = np.zeros(n)
    np.add.at(m, en.ravel(), mv)
    return Ai, Ae, m
