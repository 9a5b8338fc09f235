"""Pins of the oracle's decomposition, Schur complements, deluxe scaling,
BDDC and FETI-DP against the theory of the paper (Sec. 4, 5) and against
direct solves (no GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from conftest import read_remarks
from oracle import bddc, bidomain, dd, fetidp, krylov, newton
from workload import Physics, small_mesh, stimulus_nodal, workload


def _setup(n=(8, 8, 8), parts=(2, 2, 2), seed=0):
    m = small_mesh(n, parts)
    p = bidomain.Problem(m, Physics(), 0.05)
    rng = np.random.default_rng(seed)
    v = rng.uniform(-10, 40, p.N)
    w = rng.uniform(0, 0.2, p.N)
    dec = dd.Decomposition(m)
    return p, dec, v, w


@pytest.fixture(scope="module")
def c0():
    p, dec, v, w = _setup()
    B = bddc.BDDC(p, dec, v, w)
    return p, dec, v, w, B


def test_class_counts():
    """N_x classification: 2x2x2 -> 1 vertex, 6 edges, 12 faces;
    4x4x4 -> 27, 108, 144."""
    dec = dd.Decomposition(small_mesh((8, 8, 8), (2, 2, 2)))
    assert (len(dec.verts), len(dec.edges), len(dec.faces)) == (1, 6, 12)
    dec = dd.Decomposition(small_mesh((16, 16, 16), (4, 4, 4)))
    assert (len(dec.verts), len(dec.edges), len(dec.faces)) == (27, 108, 144)
    # interior subdomain sizes at H/h = 4: 3^3 interior nodes, 6 faces of 3x3
    s = dec.sub[1 + 4 * (1 + 4 * 1)]
    assert s.nI == 2 * 27 and s.nV == 16 and s.nr == 2 * (6 * 9 + 12 * 3)


def test_local_matrices_sum_to_jacobian(c0):
    p, dec, v, w, B = c0
    J = p.jacobian(v, w)
    S = sum(B.loc[s].K_full for s in range(dec.nsub))
    assert abs(S - J).max() < 1e-17


def test_schur_minimum_energy_and_harmonic_constant(c0):
    """s^(j)(u,u) = a^(j)(H u, H u) is the minimum energy over extensions
    (Sec. 4.1); the discrete harmonic extension of a constant is that constant;
    S_Gamma^(j) is PSD with kernel (v = 0, u_e = 1)."""
    p, dec, v, w, B = c0
    rng = np.random.default_rng(5)
    for s in (0, 5):
        lo, info = B.loc[s], dec.sub[s]
        K = lo.K_full[np.concatenate([info.I, info.G])][:, np.concatenate([info.I, info.G])].toarray()
        u = rng.standard_normal(info.nG)
        hI, hG = lo.harmonic_extension(u)
        x = np.concatenate([hI, hG])
        e_h = x @ K @ x
        assert e_h == pytest.approx(u @ lo.SG @ u, rel=1e-10)
        for _ in range(5):
            y = x.copy()
            y[:info.nI] += 1e-2 * rng.standard_normal(info.nI)
            assert y @ K @ y > e_h
        k = np.zeros(info.nG)
        k[1::2] = 1.0
        hI, _ = lo.harmonic_extension(k)
        assert np.allclose(hI[1::2], 1.0, atol=1e-12)    # H(const) = const
        assert np.allclose(hI[0::2], 0.0, atol=1e-12)
        assert np.abs(lo.SG @ k).max() < 1e-15
        ev = np.linalg.eigvalsh(lo.SG)
        assert ev[0] > -1e-14 and ev[1] > 1e-10


def test_deluxe_face_solve_is_two_subdomain_dirichlet(c0):
    """(S_F^j + S_F^k)^{-1} g equals the face values of the Dirichlet problem on
    Omega_j u F u Omega_k with zero interior right-hand side (Sec. 4.2)."""
    p, dec, v, w, B = c0
    J = p.jacobian(v, w)
    rng = np.random.default_rng(6)
    for fid in (0, 7):
        F = dec.faces[fid]
        j, k = F.subs
        Fd = B.obj_dofs(F, p.N)
        dofs = np.concatenate([dec.sub[j].I, dec.sub[k].I, Fd])
        Kjk = (B.loc[j].K_full + B.loc[k].K_full)[dofs][:, dofs].tocsc()
        g = rng.standard_normal(len(Fd))
        rhs = np.zeros(len(dofs))
        rhs[-len(Fd):] = g
        x = spla.spsolve(Kjk, rhs)
        assert np.allclose(x[-len(Fd):], np.linalg.solve(B.Ssum[("F", fid)], g), rtol=1e-10)


def test_deluxe_average_is_projection(c0):
    """E_D is a projection (E_D^2 = E_D) that reproduces continuous interface
    functions (Sec. 4.2)."""
    p, dec, v, w, B = c0
    rng = np.random.default_rng(7)
    N = p.N
    # continuous function: one global interface vector restricted to each subdomain
    u = rng.standard_normal(2 * N)
    wloc = [u[dec.sub[s].G] for s in range(dec.nsub)]
    z = np.zeros(2 * N)
    B.deluxe_values(wloc, z)
    for kind, oid, obj in B._objects():
        d = B.obj_dofs(obj, N)
        assert np.allclose(z[d], u[d], rtol=1e-12)
    # discontinuous: apply twice
    wloc = [rng.standard_normal(dec.sub[s].nG) for s in range(dec.nsub)]
    z1 = np.zeros(2 * N)
    B.deluxe_values(wloc, z1)
    w2 = [z1[dec.sub[s].G] for s in range(dec.nsub)]
    z2 = np.zeros(2 * N)
    B.deluxe_values(w2, z2)
    assert np.allclose(z1, z2, rtol=1e-12, atol=1e-14)


def test_stilde_inverse_equals_partially_assembled_direct_solve(c0):
    """S~^{-1} (local constrained Neumann solves + coarse) equals a direct solve
    of min 1/2 w^T S_Gamma w - <g, w> over the partially assembled space:
    local interface functions whose vertex values and edge averages equal
    global primal unknowns, written as one explicit KKT system (Sec. 4.4)."""
    p, dec, v, w, B = c0
    rng = np.random.default_rng(8)
    nsub, npr = dec.nsub, dec.nprimal
    offs = np.cumsum([0] + [dec.sub[s].nG for s in range(nsub)])
    nW = offs[-1]
    nv2 = 2 * len(dec.verts)
    # load: r-dof residuals per subdomain and assembled vertex residuals, with
    # the component along the kernel (constant u_e) removed
    gloc = [rng.standard_normal(dec.sub[s].nr) for s in range(nsub)]
    gV = np.zeros(npr)
    gV[:nv2] = rng.standard_normal(nv2)
    cnt = sum(len(g[1::2]) for g in gloc) + len(dec.verts)
    tot = (sum(g[1::2].sum() for g in gloc) + gV[1:nv2:2].sum()) / cnt
    for g in gloc:
        g[1::2] -= tot
    gV[1:nv2:2] -= tot
    rows = []
    for s in range(nsub):
        info, C = dec.sub[s], B.C[s]
        for t in range(info.nV):
            r = np.zeros(nW + npr)
            r[offs[s] + info.nr + t] = 1.0
            r[nW + info.primal[t]] = -1.0
            rows.append(r)
        for t in range(C.shape[0]):
            r = np.zeros(nW + npr)
            r[offs[s]:offs[s] + info.nr] = C[t]
            r[nW + info.primal[info.nV + t]] = -1.0
            rows.append(r)
    pin = np.zeros(nW + npr)
    pin[nW + 1] = 1.0                  # removes the constant-u_e kernel
    rows.append(pin)
    Cg = np.array(rows)
    H = np.zeros((nW + npr, nW + npr))
    for s in range(nsub):
        H[offs[s]:offs[s + 1], offs[s]:offs[s + 1]] = B.loc[s].SG
    nc = Cg.shape[0]
    KKT = np.block([[H, Cg.T], [Cg, np.zeros((nc, nc))]])
    rhs = np.zeros(nW + npr + nc)
    for s in range(nsub):
        rhs[offs[s]:offs[s] + dec.sub[s].nr] = gloc[s]
    rhs[nW:nW + npr] = gV
    ref = np.linalg.solve(KKT, rhs)[:nW]
    wloc, _ = B.stilde_inv(gloc, gV)
    diff = np.concatenate(wloc) - ref
    scale = np.abs(ref).max()
    assert np.abs(diff[0::2]).max() < 1e-9 * scale          # v parts agree
    assert np.ptp(diff[1::2]) < 1e-9 * scale                # u_e parts agree up to a constant


def test_bddc_and_fetidp_spectra(c0):
    """lambda_min(M^{-1} J) >= 1 on the range and the non-unit spectra of
    BDDC (interface form) and FETI-DP deluxe coincide (Sec. 5; spectral
    equivalence of the two methods)."""
    p, dec, v, w, B = c0
    J = p.jacobian(v, w).toarray()
    n = 2 * p.N
    Minv = np.column_stack([B.apply(e) for e in np.eye(n)])
    ev = np.sort(np.linalg.eigvals(Minv @ J).real)
    assert abs(ev[0]) < 1e-10 and ev[1] > 1 - 1e-10
    Sh, gd = B.schur_assembled()
    cols = []
    for i in range(len(gd)):
        e = np.zeros(n)
        e[gd[i]] = 1.0
        cols.append(B.apply_interface(e)[gd])
    evs = np.sort(np.linalg.eigvals(np.column_stack(cols) @ Sh).real)
    assert abs(evs[0]) < 1e-10 and evs[1] > 1 - 1e-10
    # full-system spectrum = {1} u interface spectrum
    assert np.allclose(ev[-20:], evs[-20:], rtol=1e-10)
    F = fetidp.FETIDP(B)
    Fm = np.column_stack([F.F(e) for e in np.eye(F.nlam)])
    Mm = np.column_stack([F.precond(e) for e in np.eye(F.nlam)])
    evf = np.sort(np.linalg.eigvals(Mm @ Fm).real)
    bb = evs[evs > 1 + 1e-8]
    bf = evf[evf > 1 + 1e-8]
    assert len(bb) == len(bf) and len(bb) > 10
    assert np.allclose(bb, bf, rtol=1e-10)
    # B_D^T B = P_D = I - E_D on local interface functions
    rng = np.random.default_rng(9)
    wl = [rng.standard_normal(dec.sub[s].nG) for s in range(dec.nsub)]
    for s in range(dec.nsub):
        wl[s][dec.sub[s].nr:] = 0.0
    pd = F.BDT(F.B(wl))
    z = np.zeros(n)
    B.deluxe_values(wl, z)
    for s in range(dec.nsub):
        info = dec.sub[s]
        ed = z[info.G]
        assert np.allclose(pd[s][:info.nr], wl[s][:info.nr] - ed[:info.nr], rtol=1e-10, atol=1e-12)


def test_lanczos_estimate_matches_dense_condition(c0):
    p, dec, v, w, B = c0
    J = p.jacobian(v, w)
    rng = np.random.default_rng(10)
    b = newton.project_range(rng.standard_normal(2 * p.N), p.N)
    res = krylov.pcg(lambda x: J @ x, B.apply, b, rtol=1e-12)
    n = 2 * p.N
    Minv = np.column_stack([B.apply(e) for e in np.eye(n)])
    ev = np.sort(np.linalg.eigvals(Minv @ J.toarray()).real)
    assert res.status == 0
    assert res.cond() == pytest.approx(ev[-1] / 1.0, rel=1e-3)


def test_polylog_condition_growth():
    """cond / (1 + log(H/h))^3 stays bounded and does not increase with H/h for
    the vertex + edge-average deluxe preconditioners (main theorem, Sec. 5)."""
    ratios = []
    for Hh in (2, 3, 4, 6):
        p, dec, v, w = _setup((2 * Hh,) * 3, (2, 2, 2), seed=1)
        B = bddc.BDDC(p, dec, v, w)
        J = p.jacobian(v, w)
        b = newton.project_range(np.random.default_rng(2).standard_normal(2 * p.N), p.N)
        res = krylov.pcg(lambda x: J @ x, B.apply, b, rtol=1e-12)
        ratios.append(res.cond() / (1 + np.log(Hh)) ** 3)
    assert all(r < 3.0 for r in ratios)
    assert all(ratios[i + 1] <= ratios[i] * 1.05 for i in range(len(ratios) - 1))


def test_condition_independent_of_subdomain_count_and_near_paper():
    """At fixed H/h = 4 the condition number does not grow from 2x2x2 to 3x3x3
    subdomains (Sec. 5), and is of the order the paper prints for deluxe
    V+E at H/h = 4 (Sec. 6, Test 3; different slab size and tolerances, so
    only the order is compared)."""
    conds = []
    for parts in ((2, 2, 2), (3, 3, 3)):
        p, dec, v, w = _setup(tuple(4 * q for q in parts), parts, seed=3)
        B = bddc.BDDC(p, dec, v, w)
        J = p.jacobian(v, w)
        b = newton.project_range(np.random.default_rng(4).standard_normal(2 * p.N), p.N)
        res = krylov.pcg(lambda x: J @ x, B.apply, b, rtol=1e-12)
        conds.append(res.cond())
    assert conds[1] < conds[0] * 1.3
    paper = read_remarks()["cond_deluxe_VE_Hh4"]
    assert 0.5 * paper < conds[1] < 2.5 * paper


@pytest.mark.parametrize("method", ["bddc", "fetidp"])
def test_newton_krylov_matches_direct_newton(method):
    """Partition and preconditioner invariance: the Newton solution with
    BDDC-PCG or FETI-DP-PCG equals the direct sparse Newton root."""
    wl = workload("slab8_supra")
    p = bidomain.Problem(wl.mesh, wl.physics, wl.solver.dt)
    dec = dd.Decomposition(wl.mesh)
    v, ue, w = np.zeros(p.N), np.zeros(p.N), np.zeros(p.N)
    Is = stimulus_nodal(wl.mesh, wl.stim_block, wl.stim_amplitude)
    for _ in range(2):
        v1, ue1, w1, st = newton.time_step(p, dec, v, ue, w, Is, method=method)
        vr, uer, wr, _ = bidomain.time_step_direct(p, v, ue, w, Is)
        assert np.linalg.norm(v1 - vr) <= 1e-10 * np.linalg.norm(vr)
        assert np.linalg.norm(ue1 - uer) <= 1e-10 * np.linalg.norm(uer)
        assert 1 <= st.newton_its <= 4 and all(5 <= k <= 40 for k in st.krylov_its)
        v, ue, w = vr, uer, wr
