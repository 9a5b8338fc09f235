"""Pins of the oracle's mesh, FE operators, ionic model and residual against
what the paper prints and what the mathematics fixes (no GPU)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from conftest import golden, read_remarks
from oracle import bidomain, fem, ionic
from workload import Physics, small_mesh, stimulus_nodal


def test_dof_counts_match_paper_tables():
    """2 * prod(n+1) reproduces every dof count printed in the result tables."""
    with open(golden("paper_dof_counts.txt")) as f:
        rows = [l.split()[:4] for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for nx, ny, nz, dofs in rows:
        m = small_mesh((int(nx), int(ny), int(nz)), (1, 1, 1))
        assert 2 * m.nnodes == int(dofs)
    rem = read_remarks()
    # Test 4: local 24x12x12 elements per subdomain
    m = small_mesh((24, 12, 12), (1, 1, 1))
    assert 2 * m.nnodes == rem["local_dofs_test4"]


def test_q1_laplacian_stencil_closed_form():
    """D = I on cubes of side h: the assembled interior stencil is
    h * (8/3 centre, 0 face, -1/6 edge, -1/12 corner neighbours)."""
    h = 0.01
    m = small_mesh((4, 4, 4), (1, 1, 1), h=h)
    ph = Physics(sigma_i=(1.0, 1.0, 1.0), sigma_e=(1.0, 1.0, 1.0))
    Ai, Ae, _ = fem.assemble(m, ph)
    c = fem.node_id(m, 2, 2, 2)
    row = Ai[c].toarray().ravel()
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                nb = fem.node_id(m, 2 + di, 2 + dj, 2 + dk)
                nz = abs(di) + abs(dj) + abs(dk)
                want = {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}[nz] * h
                assert row[nb] == pytest.approx(want, abs=1e-15)


def test_stiffness_properties():
    m = small_mesh((3, 4, 5), (1, 1, 1))
    Ai, Ae, _ = fem.assemble(m, Physics())
    one = np.ones(m.nnodes)
    for A in (Ai, Ae):
        assert np.abs(A @ one).max() < 1e-15
        assert abs(A - A.T).max() < 1e-16 * abs(A).max()
        ev = np.linalg.eigvalsh(A.toarray())
        assert ev[0] > -1e-15 and ev[1] > 1e-8       # PSD, one-dimensional kernel


def test_fibre_rotation_frame():
    """Zero rotation gives the diagonal tensor diag(sigma_l, sigma_t, sigma_n);
    a 90 degree rotation swaps the l and t conductivities."""
    s = (3.0, 0.5, 0.1)
    assert np.allclose(fem.conductivity(s, 0.0), np.diag(s))
    assert np.allclose(fem.conductivity(s, math.pi / 2), np.diag((0.5, 3.0, 0.1)))
    D = fem.conductivity(s, 0.7)
    assert np.allclose(np.sort(np.linalg.eigvalsh(D)), np.sort(s))


def test_lumped_mass():
    h = 0.01
    m = small_mesh((3, 4, 5), (1, 1, 1), h=h)
    _, _, M = fem.assemble(m, Physics())
    assert M.sum() == pytest.approx(3 * 4 * 5 * h ** 3, rel=1e-14)
    assert M[fem.node_id(m, 1, 1, 1)] == pytest.approx(h ** 3, rel=1e-14)
    assert M[fem.node_id(m, 0, 0, 0)] == pytest.approx(h ** 3 / 8, rel=1e-14)


def test_ionic_zeros_and_coercivity_remark():
    """I_ion vanishes at 0, v_th, v_p; the minimum of dI_ion/dv at w = 0 sits at
    (v_th + v_p)/3 and makes chi C_m + tau dI/dv >= 0 exactly for
    tau <= 0.366 ms, the paper's 0.37 ms remark (Sec. 3c)."""
    ph = Physics()
    for v in (0.0, ph.vth, ph.vp):
        assert ionic.iion(ph, v, 0.0) == pytest.approx(0.0, abs=1e-12)
    vs = np.linspace(-50, 150, 200001)
    d = ionic.diion_dv(ph, vs, 0.0)
    vmin = vs[np.argmin(d)]
    assert vmin == pytest.approx((ph.vth + ph.vp) / 3, abs=2e-3)
    assert d.min() / (ph.chi * ph.G) == pytest.approx(-2.2741, abs=1e-4)
    tau_max = ph.chi * ph.Cm / -d.min()
    assert round(tau_max, 2) == read_remarks()["tau_max_coercive_ms"]
    # derivative against central differences
    rng = np.random.default_rng(1)
    v = rng.uniform(-20, 120, 50)
    w = rng.uniform(0, 1, 50)
    e = 1e-5
    fd = (ionic.iion(ph, v + e, w) - ionic.iion(ph, v - e, w)) / (2 * e)
    assert np.allclose(fd, ionic.diion_dv(ph, v, w), rtol=1e-8, atol=1e-6)


def test_step1_closed_form_is_the_implicit_root():
    ph = Physics()
    rng = np.random.default_rng(2)
    for _ in range(20):
        vn, wn, tau = rng.uniform(-80, 100), rng.uniform(0, 1), rng.uniform(0.01, 0.5)
        f = lambda w: w - tau * ionic.gating_rhs(ph, vn, w) - wn
        ref = brentq(f, -10, 10, xtol=1e-15)
        assert ionic.step1(ph, tau, vn, wn) == pytest.approx(ref, abs=1e-13)


def _problem():
    m = small_mesh((4, 3, 5), (1, 1, 1))
    return bidomain.Problem(m, Physics(), 0.05)


def test_residual_properties():
    p = _problem()
    rng = np.random.default_rng(3)
    v, ue, vn = rng.uniform(-20, 60, (3, p.N))
    w = rng.uniform(0, 0.3, p.N)
    Is = stimulus_nodal(p.mesh, (1, 1, 1), 1e5)
    R = p.residual(v, ue, vn, w, Is)
    # gauge invariance and the compatibility of the second row
    R2 = p.residual(v, ue + 7.5, vn, w, Is)
    assert np.allclose(R, R2, atol=1e-15)
    assert abs(R[p.N:].sum()) < 1e-14
    # hand-written (v, u_e) form: first row is the u_i equation, second the sum
    Ai, Ae, m, tau, c = p.Ai, p.Ae, p.m, p.tau, p.c
    Rv = m * (c * (v - vn) + tau * ionic.iion(p.ph, v, w) - tau * Is) + tau * (Ai @ (v + ue))
    Re = tau * (Ai @ (v + ue)) + tau * (Ae @ ue)
    assert np.allclose(R, np.concatenate([Rv, Re]), rtol=1e-13, atol=1e-18)


def test_jacobian_finite_differences_and_symmetry():
    p = _problem()
    rng = np.random.default_rng(4)
    v, ue = rng.uniform(-20, 60, (2, p.N))
    w = rng.uniform(0, 0.3, p.N)
    Is = np.zeros(p.N)
    J = p.jacobian(v, w)
    assert abs(J - J.T).max() < 1e-18
    d = rng.standard_normal(2 * p.N)
    R = lambda x: p.residual(x[:p.N], x[p.N:], v * 0, w, Is)
    x0 = np.concatenate([v, ue])
    e = 1e-4
    fd = (R(x0 + e * d) - R(x0 - e * d)) / (2 * e)
    assert np.linalg.norm(fd - J @ d) / np.linalg.norm(J @ d) < 1e-9
    # kernel (v = 0, u_e = const)
    k = np.concatenate([np.zeros(p.N), np.ones(p.N)])
    assert np.abs(J @ k).max() < 1e-17
    # reaction diagonal appears on the (v, v) block only
    dg = p.reaction_diag(v, w)
    assert np.allclose((J - J.T).diagonal(), 0)
    assert np.allclose(J.diagonal()[:p.N], dg + p.tau * p.Ai.diagonal(), rtol=1e-13)


def _kron_box_stiffness(D, hs):
    """Q1 box stiffness by separation of variables, an independent route to
    the oracle's Gauss quadrature: with per-axis 1-D matrices
    K1 = int psi_a' psi_b' = [[1, -1], [-1, 1]] / h_d,
    M1 = int psi_a psi_b = h_d [[2, 1], [1, 2]] / 6 and
    C1 = int psi_a' psi_b = [[-1, -1], [1, 1]] / 2 (rows a),
    A = sum_pq D_pq (F_z (x) F_y (x) F_x), F_d = K1 if d = p = q, C1 if
    d = p != q, C1^T if d = q != p, else M1 (local node a + 2b + 4c: x
    fastest, so z is the outer Kronecker factor)."""
    K1 = lambda h: np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M1 = lambda h: h * np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    C1 = np.array([[-1.0, -1.0], [1.0, 1.0]]) / 2.0
    A = np.zeros((8, 8))
    for p in range(3):
        for q in range(3):
            F = []
            for d in range(3):
                if d == p and d == q:
                    F.append(K1(hs[d]))
                elif d == p:
                    F.append(C1)
                elif d == q:
                    F.append(C1.T)
                else:
                    F.append(M1(hs[d]))
            A += D[p, q] * np.kron(F[2], np.kron(F[1], F[0]))
    return A


def test_box_element_stiffness_and_mass_separable_form():
    """Box elements of sizes (0.01, 0.02, 0.02) cm (the Test 4 slab of
    Sec. 6: 1.92 x 1.92 x 0.48 cm on 192 x 96 x 24 elements): the quadrature
    stiffness equals the separable form for a rotated anisotropic tensor,
    kills constants, and the element mass sums to the element volume."""
    hs = (0.01, 0.02, 0.02)
    D = fem.conductivity((3.0, 0.31525, 0.031525), 0.7)
    A = fem.element_stiffness(D, hs)
    assert np.allclose(A, _kron_box_stiffness(D, hs), rtol=1e-13, atol=1e-18)
    assert np.abs(A @ np.ones(8)).max() < 1e-15
    Me = fem.element_mass(hs)
    assert Me.sum() == pytest.approx(0.01 * 0.02 * 0.02, rel=1e-14)
    # the cube case of the same route
    assert np.allclose(fem.element_stiffness(D, 0.01), _kron_box_stiffness(D, (0.01,) * 3), rtol=1e-13)


def test_box_mesh_lumped_mass_and_fibre_heights():
    """On a mesh of box elements the lumped mass sums to the slab volume,
    interior nodes carry hx hy hz, and the fibre angle of the top layer is
    evaluated at its centroid height (nz - 1/2) hz of the slab height nz hz."""
    from workload import Mesh
    m = Mesh(6, 4, 3, 0.01, (0, 3, 6), (0, 2, 4), (0, 1, 3), hy=0.02, hz=0.03)
    assert m.spacing == (0.01, 0.02, 0.03)
    _, _, M = fem.assemble(m, Physics())
    assert M.sum() == pytest.approx(6 * 0.01 * 4 * 0.02 * 3 * 0.03, rel=1e-14)
    assert M[fem.node_id(m, 1, 1, 1)] == pytest.approx(0.01 * 0.02 * 0.03, rel=1e-14)
    Ai, _ = fem.layer_stiffness(m, Physics())
    th = Physics().theta0 + (Physics().theta1 - Physics().theta0) * 2.5 / 3
    assert np.allclose(Ai[2], fem.element_stiffness(fem.conductivity(Physics().sigma_i, th), m.spacing))
