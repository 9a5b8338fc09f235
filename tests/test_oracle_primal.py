"""Pins of the oracle's primal spaces (V, V+E, V+E+F) and scalings (deluxe,
rho) against the theory of BDDC (Sec. 4.2, 4.4, 5) and the shape of the
paper's optimality test (Sec. 6, Test 3), on the CPU.

  * Both scalings average with matrices D^(m) that sum to the identity on
    every object, so E_D reproduces continuous interface functions and is a
    projection.
  * S~^{-1} equals a direct solve over the partially assembled space of each
    primal space, written as one explicit KKT system.
  * A richer primal space shrinks the partially assembled space, so the
    largest eigenvalue of the preconditioned operator cannot grow:
    cond(V+E+F) <= cond(V+E) <= cond(V), with lambda_min >= 1 throughout.
  * With the same conductivities in every subdomain, rho scaling weighs each
    copy by 1/|N_x|.
  * Shape of Test 3: doubling H/h multiplies cond(V) by about three (the
    paper: 8.4 -> 24.0) and cond(V+E), cond(V+E+F) by far less (1.9 -> 2.6,
    1.7 -> 2.5); rho and deluxe give nearly the same condition numbers.
"""
import numpy as np
import pytest

from conftest import read_test3
from oracle import bddc, bidomain, dd, krylov, newton
from workload import Physics, small_mesh


def _problem(n, parts, seed):
    m = small_mesh(n, parts)
    p = bidomain.Problem(m, Physics(), 0.05)
    rng = np.random.default_rng(seed)
    return m, p, rng.uniform(-10, 40, p.N), rng.uniform(0, 0.2, p.N)


@pytest.fixture(scope="module")
def small():
    m, p, v, w = _problem((8, 8, 8), (2, 2, 2), 0)
    return m, p, v, w


def test_primal_counts():
    """4x4x4 subdomains: 27 vertices, 108 edges, 144 faces; an interior
    subdomain has 8 vertices, 12 edges and 6 faces."""
    m = small_mesh((16, 16, 16), (4, 4, 4))
    for prim, np_ in (("V", 54), ("VE", 54 + 216), ("VEF", 54 + 216 + 288)):
        dec = dd.Decomposition(m, prim)
        assert dec.nprimal == np_
        s = dec.sub[1 + 4 * (1 + 4 * 1)]
        assert len(s.primal) == 16 + {"V": 0, "VE": 24, "VEF": 36}[prim]
        assert len(set(s.primal)) == len(s.primal) and max(s.primal) < dec.nprimal
    with pytest.raises(ValueError):
        dd.Decomposition(m, "EF")


@pytest.mark.parametrize("scaling", ["deluxe", "rho"])
def test_scaling_partition_of_unity_and_projection(small, scaling):
    m, p, v, w = small
    dec = dd.Decomposition(m, "VE")
    B = bddc.BDDC(p, dec, v, w, scaling=scaling)
    N = p.N
    for kind, oid, obj in B._objects():
        Ds = [B.D(kind, oid, s) for s in obj.subs]
        assert np.allclose(sum(Ds), np.eye(Ds[0].shape[0]), atol=1e-12)
        if scaling == "rho":
            for D in Ds:
                assert np.allclose(D, np.eye(D.shape[0]) / len(obj.subs), rtol=0, atol=1e-15)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(2 * N)
    z = np.zeros(2 * N)
    B.deluxe_values([u[dec.sub[s].G] for s in range(dec.nsub)], z)
    for kind, oid, obj in B._objects():
        d = B.obj_dofs(obj, N)
        assert np.allclose(z[d], u[d], rtol=1e-12)
    wl = [rng.standard_normal(dec.sub[s].nG) for s in range(dec.nsub)]
    z1, z2 = np.zeros(2 * N), np.zeros(2 * N)
    B.deluxe_values(wl, z1)
    B.deluxe_values([z1[dec.sub[s].G] for s in range(dec.nsub)], z2)
    assert np.allclose(z1, z2, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("primal", ["V", "VE", "VEF"])
def test_stilde_inverse_equals_partially_assembled_direct_solve(small, primal):
    """S~^{-1} (local constrained Neumann solves + coarse) equals the direct
    minimiser of 1/2 w^T S_Gamma w - <g, w> over local interface functions
    whose vertex values and constrained averages equal global primal
    unknowns (Sec. 4.4)."""
    m, p, v, w = small
    dec = dd.Decomposition(m, primal)
    B = bddc.BDDC(p, dec, v, w)
    rng = np.random.default_rng(8)
    nsub, npr = dec.nsub, dec.nprimal
    offs = np.cumsum([0] + [dec.sub[s].nG for s in range(nsub)])
    nW = offs[-1]
    nv2 = 2 * len(dec.verts)
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
        info = dec.sub[s]
        # constraint rows built here from the object node lists, not from B.C
        for t in range(info.nV):
            r = np.zeros(nW + npr)
            r[offs[s] + info.nr + t] = 1.0
            r[nW + info.primal[t]] = -1.0
            rows.append(r)
        for t, (kind, o) in enumerate(info.cons):
            obj = (dec.edges if kind == "E" else dec.faces)[o]
            off = info.obj_offset[(kind, o)]
            for f in (0, 1):
                r = np.zeros(nW + npr)
                for k in range(len(obj.nodes)):
                    r[offs[s] + off + 2 * k + f] = 1.0 / len(obj.nodes)
                r[nW + info.primal[info.nV + 2 * t + f]] = -1.0
                rows.append(r)
    pin = np.zeros(nW + npr)
    pin[nW + 1] = 1.0
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
    assert np.abs(diff[0::2]).max() < 1e-9 * scale
    assert np.ptp(diff[1::2]) < 1e-9 * scale


def _conds(n, parts, seed, combos):
    m, p, v, w = _problem(n, parts, seed)
    J = p.jacobian(v, w)
    b = newton.project_range(np.random.default_rng(seed + 1).standard_normal(2 * p.N), p.N)
    out = {}
    for prim, sc in combos:
        B = bddc.BDDC(p, dd.Decomposition(m, prim), v, w, scaling=sc)
        res = krylov.pcg(lambda x: J @ x, B.apply, b, rtol=1e-12)
        assert res.status == 0
        out[(prim, sc)] = res.lanczos_extremes()
    return out


def test_richer_primal_space_lowers_condition():
    combos = [(pr, sc) for pr in ("V", "VE", "VEF") for sc in ("deluxe", "rho")]
    ext = _conds((9, 9, 9), (3, 3, 3), 11, combos)
    for sc in ("deluxe", "rho"):
        lo = [ext[(pr, sc)][0] for pr in ("V", "VE", "VEF")]
        hi = [ext[(pr, sc)][1] for pr in ("V", "VE", "VEF")]
        assert min(lo) > 1 - 1e-6, lo
        assert hi[2] <= hi[1] * (1 + 1e-6) and hi[1] <= hi[0] * (1 + 1e-6), hi
        assert hi[0] > 2 * hi[1]


def test_test3_shape():
    """Doubling H/h on 4x4x4 subdomains (H/h 2 -> 4 here, 4 -> 8 in the
    paper's table): cond(V) grows about threefold, cond(V+E) and
    cond(V+E+F) by less than 1.6x, and the two scalings agree within 10%."""
    paper = read_test3()
    combos = [(pr, sc) for pr in ("V", "VE", "VEF") for sc in ("deluxe", "rho")]
    c2 = {k: hi / lo for k, (lo, hi) in _conds((8, 8, 8), (4, 4, 4), 3, combos).items()}
    c4 = {k: hi / lo for k, (lo, hi) in _conds((16, 16, 16), (4, 4, 4), 3, combos).items()}
    for sc in ("deluxe", "rho"):
        pv = paper[(sc, "V", 8)][1] / paper[(sc, "V", 4)][1]
        assert 2.0 < pv < 4.0
        assert 2.0 < c4[("V", sc)] / c2[("V", sc)] < 4.0
        for pr in ("VE", "VEF"):
            pp = paper[(sc, pr, 8)][1] / paper[(sc, pr, 4)][1]
            assert pp < 1.6
            assert c4[(pr, sc)] / c2[(pr, sc)] < 1.6
        for pr in ("V", "VE", "VEF"):
            assert abs(c4[(pr, "rho")] / c4[(pr, "deluxe")] - 1) < 0.1
            assert abs(paper[("rho", pr, 8)][1] / paper[("deluxe", pr, 8)][1] - 1) < 0.1
