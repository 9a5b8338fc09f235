"""FETI-DP at scale, by properties that hold at any size (Sec. 4.3).

At the benchmark size (17,040,642 dofs, 32 x 32 x 16 subdomains, FP32 local
factors) the dual operator F = B S~^{-1} B^T and the deluxe Dirichlet
preconditioner are symmetric and positive on the multipliers.  Newton steps
with FETI-DP need FP64 local factors (with FP32 ones F loses definiteness
and PCG breaks down), which are refused with FP32 factors; a step with FP64
factors on the 2.2M-dof uneven slab (16 x 16 x 8 subdomains of 6-10
elements a side) converges, each Newton linear solve within 1e-6 in the FP64
residual of the full system.  (A separate module from the BDDC checks, so
that only one full-size context is alive at a time.)
"""
import numpy as np
import pytest

from workload import initial_state, stimulus_nodal, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

W = workload("slab256")
M = W.mesh
N = (M.nx + 1) * (M.ny + 1) * (M.nz + 1)


@pytest.fixture(scope="module")
def feti():
    import paper_2101_02959_amd as P
    S = P.Solver(M, W.physics, W.solver, precision=P.BDM_PREC_MIXED, method=P.BDM_SOLVER_FETIDP)
    yield P, S
    S.close()


@pytest.mark.parametrize("op", ["F", "PRECOND"])
def test_dual_operators_symmetric_positive(feti, op):
    P, S = feti
    v0, ue0, w0 = initial_state(M, W.physics, 9)
    S.bdm_linearize(v0, w0)
    nl = S.bdm_fetidp_size()
    rng = np.random.default_rng(10)
    l1, l2 = rng.standard_normal(nl), rng.standard_normal(nl)
    code = P.BDM_FETI_F if op == "F" else P.BDM_FETI_PRECOND
    a1 = S.bdm_fetidp_apply(code, l1).cpu().numpy()
    a2 = S.bdm_fetidp_apply(code, l2).cpu().numpy()
    q1, q2 = float(a1 @ l1), float(a2 @ l2)
    assert q1 > 0 and q2 > 0, (q1, q2)
    # FP32 local factors: symmetric to the FP32 round-off of the local solves
    assert abs(float(a1 @ l2) - float(l1 @ a2)) <= 2e-4 * np.sqrt(q1 * q2)


def test_fp32_newton_step_refused(feti):
    P, S = feti
    v0, ue0, w0 = initial_state(M, W.physics, W.perturb_seed)
    S.bdm_set_state(v0, ue0, w0)
    with pytest.raises(P.BidomainError, match="BDM_E_ARG"):
        S.bdm_step(1)


def test_fp64_time_step_converges_uneven_slab():
    import paper_2101_02959_amd as P
    wl = workload("slab128_uneven")
    S = P.Solver(wl.mesh, wl.physics, wl.solver, precision=P.BDM_PREC_FP64, method=P.BDM_SOLVER_FETIDP)
    try:
        v0, ue0, w0 = initial_state(wl.mesh, wl.physics, wl.perturb_seed)
        S.bdm_set_state(v0, ue0, w0)
        S.bdm_set_stimulus(stimulus_nodal(wl.mesh, wl.stim_block, wl.stim_amplitude), 0, wl.stim_steps)
        st = S.bdm_step(1)
        nit = st.newton_its
        assert 1 <= nit <= 5
        res = list(st.res_hist)[:nit + 1]
        assert res[-1] <= wl.solver.newton_rtol * res[0] * 10, res
        for q in range(nit):
            assert 0 < st.krylov_its[q] <= 60
            assert st.cond[q] > 1.0
            assert st.krylov_true_res[q] <= 1e-6, (q, st.krylov_true_res[q])
    finally:
        S.close()
