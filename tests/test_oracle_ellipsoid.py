"""Pins of the oracle's truncated-ellipsoid geometry and isoparametric Q1
elements (paper Sec. 6 geometry, Sec. 3a elements) against closed forms,
invariances and a library quadrature (no GPU)."""
import math

import numpy as np
from scipy import integrate

from oracle import fem
from workload import ELLIPSOID, Physics, ellipsoid_mesh


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_map_puts_r0_and_r1_on_the_inner_and_outer_ellipsoids():
    """(x/a)^2 + (y/b)^2 + (z/c)^2 = 1 on r = 0 with (a1, b1, c1) and on r = 1
    with (a2, b2, c2), at any (theta, phi)."""
    g = ELLIPSOID
    rng = np.random.default_rng(0)
    th = rng.uniform(g[6], g[7], 50)
    ph = rng.uniform(g[8], g[9], 50)
    for r, (a, b, c) in ((0.0, (g[0], g[2], g[4])), (1.0, (g[1], g[3], g[5]))):
        X = fem.ellipsoid_point(g, np.full(50, r), th, ph)
        q = (X[:, 0] / a) ** 2 + (X[:, 1] / b) ** 2 + (X[:, 2] / c) ** 2
        np.testing.assert_allclose(q, 1.0, rtol=1e-14)


def test_isoparametric_element_on_a_moved_box_is_the_box_element():
    """A box element rotated by R and translated, with the tensor R D R^T,
    has the stiffness of the unrotated box (closed form, pinned against the
    separable integrals elsewhere) and the lumped mass vol / 8 per corner."""
    h = (0.011, 0.017, 0.007)
    D = np.array([[2.0, 0.3, 0.1], [0.3, 1.1, -0.2], [0.1, -0.2, 0.6]])
    R = _rotation(3)
    Xb = np.array([[a * h[0], b * h[1], c * h[2]] for c in (0, 1) for b in (0, 1) for a in (0, 1)])
    X = Xb @ R.T + np.array([0.3, -1.2, 2.5])
    (A,), m = fem.iso_element_matrices(X[None], [(R @ D @ R.T)[None]])
    ref = fem.element_stiffness(D, h)
    np.testing.assert_allclose(A[0], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(m[0], np.full(8, h[0] * h[1] * h[2] / 8.0), rtol=1e-13)


def test_patch_test_on_the_curved_mesh():
    """With one constant tensor on every (curved) element, the assembled
    stiffness maps a field linear in the physical coordinates to zero at
    every interior node: 2x2x2 Gauss integrates int_e grad(phi_a) exactly on
    trilinear elements, and the trilinear space holds the linear fields."""
    m = ellipsoid_mesh(6, 6, 4, 1, 1, 1)
    en, _ = fem.element_node_table(m)
    Xn = fem.node_coords(m)
    D = np.array([[1.7, 0.2, 0.0], [0.2, 0.9, 0.1], [0.0, 0.1, 0.4]])
    (A,), _ = fem.iso_element_matrices(Xn[en], [np.broadcast_to(D, (len(en), 3, 3))])
    K = np.zeros((m.nnodes, m.nnodes))
    for e in range(len(en)):
        K[np.ix_(en[e], en[e])] += A[e]
    u = Xn @ np.array([0.7, -1.3, 2.1]) + 0.4
    y = K @ u
    i, j, k = np.meshgrid(np.arange(1, m.nx), np.arange(1, m.ny), np.arange(1, m.nz), indexing="ij")
    inner = fem.node_id(m, i, j, k).ravel()
    assert np.abs(y[inner]).max() < 1e-12 * np.abs(K).max() * np.abs(u).max()
    # the boundary rows are the outward fluxes and are not zero
    assert np.abs(y).max() > 1e-3 * np.abs(K).max() * np.abs(u).max()


def _exact_volume(g):
    """int |det dX/d(r, theta, phi)| over the parameter box, with the
    determinant written out by hand:
    cos(theta) [a' b c cos^2(theta) cos^2(phi) + a b' c cos^2(theta) sin^2(phi)
    + a b c' sin^2(theta)], integrated by SciPy's adaptive cubature."""
    da, db, dc = g[1] - g[0], g[3] - g[2], g[5] - g[4]

    def f(phi, theta, r):
        a, b, c = fem.ellipsoid_axes(g, r)
        ct, st = math.cos(theta), math.sin(theta)
        return ct * (da * b * c * ct * ct * math.cos(phi) ** 2 + a * db * c * ct * ct * math.sin(phi) ** 2
                     + a * b * dc * st * st)

    v, _ = integrate.tplquad(f, 0.0, 1.0, g[6], g[7], g[8], g[9], epsabs=1e-12, epsrel=1e-12)
    return v


def test_mesh_volume_converges_to_the_parametric_volume():
    """The lumped masses sum to the mesh volume, which tends to the volume of
    the parametric region at second order in the element size."""
    V = _exact_volume(ELLIPSOID)
    errs = []
    for n in ((8, 8, 2), (16, 16, 4), (32, 32, 8)):
        _, _, mass = fem.assemble(ellipsoid_mesh(*n, 1, 1, 1), Physics())
        errs.append(abs(mass.sum() - V) / V)
    assert errs[2] < 3e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_frame_is_orthonormal_and_follows_the_tangents():
    """e1, e2, n are orthonormal, e1 is parallel to the finite-difference
    tangent dX/dphi, and n is normal to both finite-difference tangents."""
    g = ELLIPSOID
    rng = np.random.default_rng(1)
    r, th, ph = rng.uniform(0, 1, 20), rng.uniform(g[6], g[7], 20), rng.uniform(g[8], g[9], 20)
    e1, e2, n = fem.ellipsoid_frame(g, r, th, ph)
    F = np.stack([e1, e2, n], axis=-1)
    np.testing.assert_allclose(np.einsum("eij,eik->ejk", F, F), np.broadcast_to(np.eye(3), F.shape), atol=1e-14)
    d = 1e-6
    tp = (fem.ellipsoid_point(g, r, th, ph + d) - fem.ellipsoid_point(g, r, th, ph - d)) / (2 * d)
    tt = (fem.ellipsoid_point(g, r, th + d, ph) - fem.ellipsoid_point(g, r, th - d, ph)) / (2 * d)
    tp /= np.linalg.norm(tp, axis=1, keepdims=True)
    tt /= np.linalg.norm(tt, axis=1, keepdims=True)
    np.testing.assert_allclose(np.sum(tp * e1, axis=1), 1.0, atol=1e-9)
    assert np.abs(np.sum(n * tp, axis=1)).max() < 1e-9
    assert np.abs(np.sum(n * tt, axis=1)).max() < 1e-9
    # n points outwards (towards growing r)
    tr = fem.ellipsoid_point(g, r + d, th, ph) - fem.ellipsoid_point(g, r - d, th, ph)
    assert np.all(np.sum(n * tr, axis=1) > 0)


def test_frame_tensor_on_the_axes_is_the_slab_tensor():
    """In the frame (x, y, z) the tensor of the ellipsoid is the slab's
    fibre-rotated tensor at the same angle."""
    sig = (3.0, 0.31525, 0.031525)
    e1, e2, n = np.eye(3)
    for alpha in (0.0, 0.4, 2.0 * math.pi / 3.0):
        D = fem.conductivity_in_frame(sig, np.array(alpha), e1, e2, n)
        np.testing.assert_allclose(D, fem.conductivity(sig, alpha), atol=1e-15)


def test_ellipsoid_operators_symmetric_semidefinite_with_constant_kernel():
    """A_i and A_e of the ellipsoid are symmetric positive semidefinite with
    the constants as kernel; the lumped masses are positive."""
    m = ellipsoid_mesh(6, 4, 3, 1, 1, 1)
    Ai, Ae, mass = fem.assemble(m, Physics())
    for A in (Ai, Ae):
        A = A.toarray()
        np.testing.assert_allclose(A, A.T, atol=1e-14 * np.abs(A).max())
        assert np.abs(A.sum(axis=1)).max() < 1e-13 * np.abs(A).max()
        ev = np.linalg.eigvalsh(A)
        assert ev[0] > -1e-12 * ev[-1] and ev[1] > 1e-8 * ev[-1]
    assert mass.min() > 0


def test_ellipsoid_bddc_theory():
    """The theory of Sec. 5 on the curved mesh: the local matrices sum to the
    Jacobian, the BDDC-preconditioned spectrum is >= 1 on the range, and the
    BDDC (interface) and FETI-DP deluxe spectra coincide apart from 0 and 1."""
    from oracle import bddc, bidomain, dd, fetidp
    m = ellipsoid_mesh(8, 8, 4, 2, 2, 2)
    p = bidomain.Problem(m, Physics(), 0.05)
    rng = np.random.default_rng(0)
    v, w = rng.uniform(-10, 40, p.N), rng.uniform(0, 0.2, p.N)
    dec = dd.Decomposition(m)
    B = bddc.BDDC(p, dec, v, w)
    J = p.jacobian(v, w)
    assert abs(sum(B.loc[s].K_full for s in range(dec.nsub)) - J).max() < 1e-12 * abs(J).max()
    n = 2 * p.N
    Minv = np.column_stack([B.apply(e) for e in np.eye(n)])
    ev = np.sort(np.linalg.eigvals(Minv @ J.toarray()).real)
    assert abs(ev[0]) < 1e-9 and ev[1] > 1 - 1e-9
    Sh, gd = B.schur_assembled()
    cols = []
    for i in range(len(gd)):
        e = np.zeros(n)
        e[gd[i]] = 1.0
        cols.append(B.apply_interface(e)[gd])
    evs = np.sort(np.linalg.eigvals(np.column_stack(cols) @ Sh).real)
    F = fetidp.FETIDP(B)
    Fm = np.column_stack([F.F(e) for e in np.eye(F.nlam)])
    Mm = np.column_stack([F.precond(e) for e in np.eye(F.nlam)])
    evf = np.sort(np.linalg.eigvals(Mm @ Fm).real)
    bb, bf = evs[evs > 1 + 1e-8], evf[evf > 1 + 1e-8]
    assert len(bb) == len(bf) and len(bb) > 10
    np.testing.assert_allclose(bb, bf, rtol=1e-9)


def test_ellipsoid_workload_is_the_test2_ellipsoid_mesh():
    """The ellipsoid workload has the element counts and dof count of the
    paper's Test 2 ellipsoid table (128 x 128 x 64 elements, 2,163,330 dofs,
    also in tests/golden/paper_dof_counts.txt), and the paper's 256-process
    partition cuts it into 16^3-element subdomains."""
    from workload import ellipsoid_workload
    wl = ellipsoid_workload((8, 8, 4))
    m = wl.mesh
    assert (m.nx, m.ny, m.nz) == (128, 128, 64) and 2 * m.nnodes == 2163330
    assert m.nsub == 256 and {m.cuts_x[1], m.cuts_y[1], m.cuts_z[1]} == {16}
    assert m.ellipsoid == ELLIPSOID
