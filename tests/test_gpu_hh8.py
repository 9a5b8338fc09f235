"""Parity of the HIP path against the FP64 oracle at the benchmark's
subdomain shape: H/h = 8 (Sec. 6, Test 3 geometry at H/h = 8: a 32^3 slab in
4 x 4 x 4 subdomains), and the same slab cut with per-axis widths drawn from
{6, ..., 10} (the uneven partition of the 2.2M-dof workload at a size the
oracle finishes in seconds: local problems of 686 ... 2662 dofs, interior
factors of up to 10 panels).

Comparisons are per field (v, u_e) and element by element (tests/
parity_util.py):
  * one BDDC application and the four FETI-DP operators, FP64 local factors
    at 1e-11; FP32 local factors at 3e-4 in the relative 2-norm (FP32
    round-off, 6e-8, amplified by the condition numbers of the local
    interior and Neumann problems, about 1e3 at H/h = 8, and by the coarse
    problem; measured up to 1.1e-4) and 2e-3 element by element (measured
    up to 6.2e-4): the FP32 error concentrates on the subdomain vertices
    (printed per node class), the coarse unknowns, where it is 10 to 20
    times the error on interior, face and edge nodes, while a fault in one
    class of objects would put an O(1) error there;
  * time steps of the FP64 path, and of FP32 local factors with the learned
    Newton guess: the Newton solution of each step within 1e-8 of the root of
    R(u) = 0 that the oracle computes from the GPU's u^n (Newton with
    Jacobi-preconditioned CG solves down to round-off, itself pinned against
    the direct bordered solve in tests/test_oracle_newton.py).
"""
import numpy as np
import pytest

from oracle import bddc, bidomain, dd, fetidp, newton
from parity_util import assert_close, error_by_class, gauge
from workload import Mesh, Physics, Solver as SolverOpts, stimulus_nodal, uneven_cuts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MESHES = {
    "hh8": Mesh(32, 32, 32, 0.01, (0, 8, 16, 24, 32), (0, 8, 16, 24, 32), (0, 8, 16, 24, 32)),
    "widths6to10": Mesh(32, 32, 32, 0.01, uneven_cuts(32, 4, range(6, 11), 11),
                        uneven_cuts(32, 4, range(6, 11), 12), uneven_cuts(32, 4, range(6, 11), 13)),
}
TOL64, TOL32, ETOL32 = 1e-11, 3e-4, 2e-3


def _P():
    import paper_2101_02959_amd as P
    return P


@pytest.fixture(scope="module", params=list(MESHES))
def lin(request):
    mesh = MESHES[request.param]
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    rng = np.random.default_rng(4)
    v, w = rng.uniform(-10, 40, N), rng.uniform(0, 0.2, N)
    print(f"oracle BDDC setup on {request.param}", flush=True)
    B = bddc.BDDC(prob, dd.Decomposition(mesh), v, w)
    return request.param, mesh, ph, so, prob, B, v, w


@pytest.mark.parametrize("prec", [0, 1])
def test_bddc_apply_hh8(lin, prec):
    P = _P()
    name, mesh, ph, so, prob, B, v, w = lin
    N = prob.N
    tol, etol = (TOL64, TOL64) if prec == 0 else (TOL32, ETOL32)
    S = P.Solver(mesh, ph, so, precision=prec)
    try:
        S.bdm_linearize(v, w)
        for seed in (5, 6):
            r = newton.project_range(np.random.default_rng(seed).standard_normal(2 * N), N)
            z = gauge(S.bdm_bddc_apply(r).cpu().numpy(), N)
            zref = gauge(B.apply(r), N)
            print(name, prec, seed, error_by_class(z, zref, B.dec, N), flush=True)
            print(name, prec, seed, assert_close(z, zref, tol, N, f"bddc {name} prec {prec}", etol))
    finally:
        S.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_fetidp_operators_hh8(lin, prec):
    P = _P()
    name, mesh, ph, so, prob, B, v, w = lin
    N = prob.N
    tol, etol = (TOL64, TOL64) if prec == 0 else (TOL32, ETOL32)
    F = fetidp.FETIDP(B)
    S = P.Solver(mesh, ph, so, precision=prec, method=P.BDM_SOLVER_FETIDP)
    try:
        S.bdm_linearize(v, w)
        assert S.bdm_fetidp_size() == F.nlam
        rng = np.random.default_rng(7)
        lam = rng.standard_normal(F.nlam)
        assert_close(S.bdm_fetidp_apply(P.BDM_FETI_F, lam).cpu().numpy(), F.F(lam), tol, None, "F", etol)
        assert_close(S.bdm_fetidp_apply(P.BDM_FETI_PRECOND, lam).cpu().numpy(), F.precond(lam), tol, None,
                     "precond", etol)
        r = newton.project_range(rng.standard_normal(2 * N), N)
        g = F.condense(r)
        assert_close(S.bdm_fetidp_apply(P.BDM_FETI_RHS, r).cpu().numpy(), F.rhs(g), tol, None, "rhs", etol)
        z = S.bdm_fetidp_apply(P.BDM_FETI_RECOVER, np.concatenate([r, lam])).cpu().numpy()
        assert_close(gauge(z, N), gauge(F.expand(r, F.recover(g, lam)), N), tol, N, "recover", etol)
    finally:
        S.close()


CASES = [("hh8", 0, "prev", 3), ("hh8", 1, "cnn", 4), ("widths6to10", 1, "extrap", 3)]


@pytest.mark.parametrize("name,prec,guess,steps", CASES)
def test_time_steps_hh8(name, prec, guess, steps):
    """Newton solution per step and per field within 1e-8 of the oracle's
    root from the GPU's u^n.  Corner stimulus of 2 x 2 x 2 elements at the
    paper's amplitude, from rest.  With the learned guess (weights trained
    on this slab's geometry) the judge must pick the network's guess in at
    least one step, so the judged branch is exercised."""
    P = _P()
    from paper_2101_02959_amd import predictor as PR
    mesh = MESHES[name]
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    g = {"prev": P.BDM_GUESS_PREV, "extrap": P.BDM_GUESS_EXTRAP, "cnn": P.BDM_GUESS_CNN}[guess]
    S = P.Solver(mesh, ph, so, precision=prec, guess=g)
    try:
        if guess == "cnn":
            S.bdm_predictor_set(*PR.load())
        Is = stimulus_nodal(mesh, (2, 2, 2), 1e5)
        z = np.zeros(N)
        S.bdm_set_state(z, z, z)
        S.bdm_set_stimulus(Is, 0, 20)
        v, ue, w = z, z, z
        used = []
        for step in range(steps):
            st = S.bdm_step(1)
            vg, ueg, wg, _ = S.bdm_get_state()
            vg, ueg, wg = vg.cpu().numpy(), ueg.cpu().numpy(), wg.cpu().numpy()
            vr, uer, wr, hist = bidomain.time_step_direct(prob, v, ue, w, Is, linear="cg")
            assert hist[-1] <= 1e-12 * hist[0]
            ev = assert_close(vg, vr, 1e-8, None, f"v step {step}")
            ee = assert_close(ueg, uer, 1e-8, None, f"u_e step {step}")
            assert_close(wg, wr, 1e-14, None, f"w step {step}")
            used.append(st.guess_used)
            print(name, prec, guess, step, st.newton_its, list(st.krylov_its)[:st.newton_its], st.guess_used,
                  ev, ee, flush=True)
            assert all(st.krylov_true_res[k] <= 1e-9 for k in range(st.newton_its))
            v, ue, w = vg, ueg, wg
        if guess == "cnn":
            assert 2 in used, used
    finally:
        S.close()
