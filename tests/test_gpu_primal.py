"""Primal spaces (V, V+E, V+E+F; Sec. 4.4) and scalings (deluxe, rho;
Sec. 4.2) of the HIP path against the FP64 oracle, through the C ABI.

  * One BDDC application, per field (v, u_e) in the relative 2-norm and
    element by element (tests/parity_util.py): FP64 local factors within
    1e-11 relative; FP32 ones within 5e-5 for V+E and V+E+F (FP32 round-off
    times local condition numbers of about 1e3, as for deluxe V+E), and
    within 5e-4 for V alone, whose preconditioned spectrum is more than ten
    times wider (the oracle's condition numbers on 4 x 4 x 4 subdomains at
    H/h = 4: 37 for V against 2.8 for V+E), which amplifies the same local
    round-off in the output by that factor; on a ragged mesh and a 4 x 4 x 2
    grid of uneven subdomains.
  * The FETI-DP operators for the two corner combinations.
  * One time step on 4 x 4 x 4 subdomains (the layout of the optimality test,
    Sec. 6 Test 3): the Newton solution matches the oracle's Newton-Krylov
    solution, PCG from zero takes the same number of iterations, and the
    Lanczos condition estimates agree.
"""
import numpy as np
import pytest

from oracle import bddc, bidomain, dd, fetidp, newton
from parity_util import assert_close
from workload import Mesh, Physics, Solver as SolverOpts, stimulus_nodal, small_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MESHES = {
    "ragged": Mesh(11, 9, 10, 0.01, (0, 3, 7, 11), (0, 5, 9), (0, 4, 10)),
    "uneven442": Mesh(20, 18, 12, 0.01, (0, 4, 9, 13, 20), (0, 5, 9, 14, 18), (0, 5, 12)),
}
PRIMAL = {"V": 1, "VE": 0, "VEF": 2}
SCALING = {"deluxe": 0, "rho": 1}


def _gauge(x, N):
    x = np.array(x, dtype=np.float64).copy()
    x[N:] -= x[N:].mean()
    return x


def _state(N, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-10, 40, N), rng.uniform(0, 0.2, N)


@pytest.mark.parametrize("primal", list(PRIMAL))
@pytest.mark.parametrize("scaling", list(SCALING))
@pytest.mark.parametrize("mname", list(MESHES))
def test_bddc_apply_matches_oracle(mname, scaling, primal):
    import paper_2101_02959_amd as P
    mesh = MESHES[mname]
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    v, w = _state(N, 4)
    B = bddc.BDDC(prob, dd.Decomposition(mesh, primal), v, w, scaling=scaling)
    rs = [newton.project_range(np.random.default_rng(s).standard_normal(2 * N), N) for s in (5, 6)]
    refs = [_gauge(B.apply(r), N) for r in rs]
    for prec, tol in ((0, 1e-11), (1, 5e-4 if primal == "V" else 5e-5)):
        S = P.Solver(mesh, ph, so, precision=prec, scaling=SCALING[scaling], primal=PRIMAL[primal])
        try:
            S.bdm_linearize(v, w)
            for r, zref in zip(rs, refs):
                z = _gauge(S.bdm_bddc_apply(r).cpu().numpy(), N)
                print(mname, scaling, primal, prec, assert_close(z, zref, tol, N, f"bddc prec {prec}"))
        finally:
            S.close()


@pytest.mark.parametrize("scaling,primal", [("rho", "VEF"), ("deluxe", "V"), ("rho", "V")])
def test_fetidp_operators_match_oracle(scaling, primal):
    import paper_2101_02959_amd as P
    mesh = MESHES["uneven442"]
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    v, w = _state(N, 7)
    B = bddc.BDDC(prob, dd.Decomposition(mesh, primal), v, w, scaling=scaling)
    F = fetidp.FETIDP(B)
    S = P.Solver(mesh, ph, so, precision=0, method=P.BDM_SOLVER_FETIDP, scaling=SCALING[scaling],
                 primal=PRIMAL[primal])
    try:
        S.bdm_linearize(v, w)
        assert S.bdm_fetidp_size() == F.nlam
        lam = np.random.default_rng(8).standard_normal(F.nlam)
        for op, ref in ((P.BDM_FETI_F, F.F(lam)), (P.BDM_FETI_PRECOND, F.precond(lam))):
            got = S.bdm_fetidp_apply(op, lam).cpu().numpy()
            assert_close(got, ref, 1e-11, None, f"op {op}")
    finally:
        S.close()


@pytest.mark.parametrize("primal", list(PRIMAL))
@pytest.mark.parametrize("scaling", list(SCALING))
def test_time_step_matches_oracle_on_4x4x4(scaling, primal):
    import paper_2101_02959_amd as P
    mesh = small_mesh((12, 12, 12), (4, 4, 4))
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    Is = stimulus_nodal(mesh, (2, 2, 2), 1e5)
    S = P.Solver(mesh, ph, so, precision=0, scaling=SCALING[scaling], primal=PRIMAL[primal],
                 krylov_reduced=False)
    try:
        S.bdm_set_state(np.zeros(N), np.zeros(N), np.zeros(N))
        S.bdm_set_stimulus(Is, 0, 20)
        st = S.bdm_step(1)
        vg, ueg, _, _ = S.bdm_get_state()
        vg, ueg = vg.cpu().numpy(), ueg.cpu().numpy()
    finally:
        S.close()
    dec = dd.Decomposition(mesh, primal)
    z = np.zeros(N)
    vr, uer, _, ost = newton.time_step(prob, dec, z, z, z, Is, rtol=so.newton_rtol, krtol=so.krylov_rtol,
                                       scaling=scaling)
    assert_close(vg, vr, 1e-8, None, "v")
    assert_close(ueg, uer, 1e-8, None, "u_e")
    assert st.newton_its == ost.newton_its
    for k in range(st.newton_its):
        assert abs(st.krylov_its[k] - ost.krylov_its[k]) <= 1, (k, st.krylov_its[k], ost.krylov_its[k])
        assert st.cond[k] == pytest.approx(ost.conds[k], rel=2e-2)
        assert st.krylov_true_res[k] <= 1e-9


@pytest.mark.parametrize("scaling", list(SCALING))
def test_objects_above_512_dofs(scaling):
    """Faces of more than 512 dofs (289 nodes, boundary rows included, on
    the z-cut of a 34 x 34 x 4 slab in 2 x 2 x 2 subdomains): the deluxe
    factorisation works on the matrix in global memory and the applies stage
    their vectors in LDS sized by the largest object.  One BDDC application
    in FP64 against the oracle."""
    import paper_2101_02959_amd as P
    mesh = Mesh(34, 34, 4, 0.01, (0, 17, 34), (0, 17, 34), (0, 2, 4))
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    dec = dd.Decomposition(mesh)
    assert max(2 * len(o.nodes) for o in dec.faces) > 512
    v, w = _state(N, 4)
    B = bddc.BDDC(prob, dec, v, w, scaling=scaling)
    r = newton.project_range(np.random.default_rng(5).standard_normal(2 * N), N)
    zref = _gauge(B.apply(r), N)
    S = P.Solver(mesh, ph, so, precision=0, scaling=SCALING[scaling])
    try:
        S.bdm_linearize(v, w)
        z = _gauge(S.bdm_bddc_apply(r).cpu().numpy(), N)
        assert_close(z, zref, 1e-11, N, "bddc")
    finally:
        S.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 5e-5)])
def test_blocked_deluxe_sweep_mixed_face_sizes(prec, tol):
    """Faces of 198 dofs (above the 128 of the register sweep, not a
    multiple of the 16- or 8-pivot blocks) beside faces of 36 and 44 dofs in
    one launch: the blocked sweep inverts sum S with partial last blocks.
    One BDDC application with deluxe scaling against the oracle, FP64 and
    FP32 local factors."""
    import paper_2101_02959_amd as P
    mesh = Mesh(22, 18, 4, 0.01, (0, 11, 22), (0, 9, 18), (0, 2, 4))
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    dec = dd.Decomposition(mesh)
    assert sorted({2 * len(o.nodes) for o in dec.faces}) == [36, 44, 198]
    v, w = _state(N, 4)
    B = bddc.BDDC(prob, dec, v, w)
    S = P.Solver(mesh, ph, so, precision=prec)
    try:
        S.bdm_linearize(v, w)
        for seed in (5, 6):
            r = newton.project_range(np.random.default_rng(seed).standard_normal(2 * N), N)
            z = _gauge(S.bdm_bddc_apply(r).cpu().numpy(), N)
            assert_close(z, _gauge(B.apply(r), N), tol, N, f"bddc prec {prec}")
    finally:
        S.close()


def test_objects_above_1024_dofs():
    """Faces of 1058 dofs (529 nodes: the face of an H/h = 24 subdomain,
    above the 1024 of every smaller case) on the z-cut of a 46 x 46 x 4 slab
    in 2 x 2 x 2 subdomains: one BDDC application in FP64 with deluxe
    scaling against the oracle."""
    import paper_2101_02959_amd as P
    mesh = Mesh(46, 46, 4, 0.01, (0, 23, 46), (0, 23, 46), (0, 2, 4))
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    dec = dd.Decomposition(mesh)
    assert max(2 * len(o.nodes) for o in dec.faces) == 1058
    v, w = _state(N, 4)
    B = bddc.BDDC(prob, dec, v, w)
    r = newton.project_range(np.random.default_rng(6).standard_normal(2 * N), N)
    zref = _gauge(B.apply(r), N)
    S = P.Solver(mesh, ph, so, precision=0)
    try:
        S.bdm_linearize(v, w)
        z = _gauge(S.bdm_bddc_apply(r).cpu().numpy(), N)
        assert_close(z, zref, 1e-11, N, "bddc")
    finally:
        S.close()
