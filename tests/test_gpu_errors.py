"""Error paths of the linearisation, reached through the public interface.

The coercivity lemma (Sec. 3c) needs a positive lumped reaction diagonal
m_l (chi C_m + tau dI_ion/dv).  At v = v_th and w = 0 the Rogers-McCulloch
current has dI_ion/dv = -G chi (1 - v_th/v_p), so a time step of a few
milliseconds makes the diagonal negative: the linearisation must then fail
with BDM_E_COERCIVITY (checked against the oracle's diagonal), leave the
context usable, and succeed again once the state satisfies the hypothesis.
"""
import dataclasses

import numpy as np
import pytest

from oracle import bidomain
from workload import Mesh, Physics, Solver as SolverOpts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MESH = Mesh(11, 9, 10, 0.01, (0, 3, 7, 11), (0, 5, 9), (0, 4, 10))


@pytest.mark.parametrize("prec", [0, 1])
def test_negative_reaction_diagonal_is_reported(prec):
    import paper_2101_02959_amd as P
    ph = Physics()
    so = dataclasses.replace(SolverOpts(), dt=2.0)
    N = MESH.nnodes
    v_bad, w0 = np.full(N, ph.vth), np.zeros(N)
    prob = bidomain.Problem(MESH, ph, so.dt)
    assert np.all(prob.reaction_diag(v_bad, w0) < 0)
    v_ok = np.zeros(N)
    assert np.all(prob.reaction_diag(v_ok, w0) > 0)
    S = P.Solver(MESH, ph, so, precision=prec)
    try:
        with pytest.raises(P.BidomainError, match="BDM_E_COERCIVITY"):
            S.bdm_linearize(v_bad, w0)
        S.bdm_linearize(v_ok, w0)
        r = np.random.default_rng(3).standard_normal(2 * N)
        z = S.bdm_bddc_apply(r).cpu().numpy()
        assert np.all(np.isfinite(z))
    finally:
        S.close()


def test_interior_too_large_for_the_solve_lds_is_refused():
    """The per-iteration triangular solves keep a subdomain's vector in LDS
    (160 KB per workgroup): the H/h = 24 slab of the optimality test has
    interiors of up to 2 x 24^3 = 27,648 dofs, 221 KB in FP64, so creating
    the context with FP64 local factors fails with BDM_E_ARG and a message
    (before any large allocation), while FP32 local factors (110 KB) are
    accepted by the same check."""
    import paper_2101_02959_amd as P
    from workload import test3
    wl = test3(24, steps=1)
    with pytest.raises(P.BidomainError, match="BDM_E_ARG.*LDS"):
        P.Solver(wl.mesh, wl.physics, wl.solver, precision=P.BDM_PREC_FP64)
