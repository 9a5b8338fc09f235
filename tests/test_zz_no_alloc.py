"""bdm_residual_noalloc (the residual for callers that cannot allocate device
memory) against bdm_residual of a context, through the C ABI: two calls in a
row on one GPU, the second on a smaller mesh, each bitwise equal to the
context's residual (both take every node's 27 products in the same order)
and within 1e-12 per field of the FP64 oracle."""
import numpy as np
import pytest

from oracle import bidomain
from parity_util import assert_close
from workload import Mesh, Physics, Solver as SolverOpts, stimulus_nodal

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MESHES = [Mesh(20, 18, 14, 0.01, (0, 4, 9, 13, 20), (0, 5, 9, 14, 18), (0, 5, 14)),
          Mesh(11, 9, 10, 0.01, (0, 3, 7, 11), (0, 5, 9), (0, 4, 10))]


def test_noalloc_residual_matches_context_residual_twice():
    import paper_2101_02959_amd as P
    ph, so = Physics(), SolverOpts()
    dev = torch.device("cuda", 0)
    for call, mesh in enumerate(MESHES):
        N = mesh.nnodes
        rng = np.random.default_rng(10 + call)
        vn, w = rng.uniform(-10, 40, N), rng.uniform(0, 0.2, N)
        v = vn + rng.uniform(-3, 3, N)
        ue = rng.uniform(-5, 5, N)
        ue -= ue.mean()
        Is = stimulus_nodal(mesh, (2, 2, 2), 1e5)
        print(f"call {call}: mesh {mesh.nx}x{mesh.ny}x{mesh.nz}, N {N}", flush=True)
        t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=dev)
        Rv, Re = P.bdm_residual_noalloc(mesh, ph, so.dt, t(v), t(ue), t(vn), t(w), t(Is))
        S = P.Solver(mesh, ph, so)
        try:
            S.bdm_set_state(vn, np.zeros(N), w)
            S.bdm_set_stimulus(Is, 0, 1)
            R = S.bdm_residual(v, ue).cpu().numpy()
        finally:
            S.close()
        got = np.concatenate([Rv.cpu().numpy(), Re.cpu().numpy()])
        assert np.array_equal(got, R), call
        prob = bidomain.Problem(mesh, ph, so.dt)
        assert_close(got, prob.residual(v, ue, vn, w, Is), 1e-12, N, f"call {call}")
