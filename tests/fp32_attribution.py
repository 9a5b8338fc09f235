"""Which FP32 component of the BDDC preconditioner costs PCG iterations?

An analysis run on the oracle, not a test (pytest does not collect it):

    python3 tests/fp32_attribution.py [--mesh hh8|cube8] [--out FILE]

The library's mixed path keeps the local factors, solves and scaling
matrices in FP32 under the FP64 Krylov and Newton iterations; with them the
Lanczos condition estimate of the preconditioned Newton system grows from
3.68 to 5.74 at 17M dofs and PCG takes 19.2 instead of 17.7 iterations per
Newton step.  Here the oracle's FP64 BDDC (Sec. 4.2, 4.4) is rebuilt with
one component at a time computed in float32 arithmetic (LAPACK single
precision through NumPy/SciPy on float32 arrays), on the H/h = 8 slab of
4 x 4 x 4 subdomains (the benchmark's local size):

  dirichlet  the interior solves K_II^{-1} of the condensation and of the
             harmonic extension (Cholesky of K_II in FP32);
  schur      the local Schur complements S_Gamma, from an FP32 Cholesky of
             K_II (every deluxe block, Neumann problem and coarse basis is
             then built from the rounded S_Gamma);
  neumann    the constrained local Neumann solves (the KKT systems in FP32);
  deluxe     the scaling matrices D^(m) = (sum S)^{-1} S^(m) in FP32;
  coarse     the coarse basis Phi (its KKT solves in FP32; the coarse matrix
             is then assembled and factored in FP64 from it);

and all of them together.  For each variant: PCG (rtol 1e-10, zero start)
on one Newton system, its iteration count and Lanczos condition estimate.
It imports only oracle/ and workload/.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import bddc, bidomain, dd, ionic, krylov, newton  # noqa: E402
from workload import Mesh, initial_state, stimulus_nodal, workload  # noqa: E402

COMPONENTS = ("dirichlet", "schur", "neumann", "deluxe", "coarse")
F32 = np.float32


class _Chol32:
    """K_II^{-1} by a float32 Cholesky factor (solves in float32)."""

    def __init__(self, K):
        self.c = sla.cho_factor(np.asarray(K, dtype=F32), lower=True)

    def solve(self, b):
        return sla.cho_solve(self.c, np.asarray(b, dtype=F32)).astype(np.float64)


class MixedBDDC(bddc.BDDC):
    """The oracle's BDDC with the listed components in float32 arithmetic."""

    def __init__(self, prob, dec, v, w, comps):
        self.comps = set(comps)
        # local blocks first (they feed every other component)
        self.prob, self.dec, self.N, self.scaling = prob, dec, prob.N, "deluxe"
        self.loc = [dd.LocalOps(prob, dec, s, v, w) for s in range(dec.nsub)]
        for lo in self.loc:
            if "schur" in self.comps or "dirichlet" in self.comps:
                c32 = _Chol32(lo.KII.toarray())
            if "schur" in self.comps:
                KIG = lo.KIG.astype(F32)
                SG = lo.KGG.astype(F32) - KIG.T @ sla.cho_solve(c32.c, KIG)
                lo.SG = (0.5 * (SG + SG.T)).astype(np.float64)
            if "dirichlet" in self.comps:
                lo.solve_II = c32.solve
        self._deluxe_setup()
        self._coarse_setup()

    def D(self, kind, oid, m):
        if "deluxe" not in self.comps:
            return super().D(kind, oid, m)
        S = self.Ssum[(kind, oid)].astype(F32)
        return np.linalg.solve(S, self._block(m, kind, oid).astype(F32)).astype(np.float64)

    def _coarse_setup(self):
        if "coarse" not in self.comps:
            return super()._coarse_setup()
        solve = np.linalg.solve
        try:
            np.linalg.solve = lambda A, B: solve(np.asarray(A, F32), np.asarray(B, F32)).astype(np.float64)
            super()._coarse_setup()
        finally:
            np.linalg.solve = solve

    def local_neumann(self, s, g_r):
        if "neumann" not in self.comps:
            return super().local_neumann(s, g_r)
        nc = self.C[s].shape[0]
        rhs = np.concatenate([g_r, np.zeros(nc)]).astype(F32)
        sol = np.linalg.solve(self.KKT[s].astype(F32), rhs)
        return sol[:self.dec.sub[s].nr].astype(np.float64)


def run(mesh_name):
    wl = workload("slab32")
    mesh = wl.mesh if mesh_name == "hh8" else Mesh(8, 8, 8, 0.01, (0, 4, 8), (0, 4, 8), (0, 4, 8))
    prob = bidomain.Problem(mesh, wl.physics, wl.solver.dt)
    dec = dd.Decomposition(mesh)
    N = prob.N
    v, ue, w = initial_state(mesh, wl.physics, wl.perturb_seed)
    Is = stimulus_nodal(mesh, wl.stim_block, wl.stim_amplitude)
    w1 = ionic.step1(prob.ph, prob.tau, v, w)
    R = prob.residual(v, ue, v, w1, Is)
    J = prob.jacobian(v, w1)
    rows = []
    for comps in [()] + [(c,) for c in COMPONENTS] + [COMPONENTS]:
        t0 = time.time()
        B = MixedBDDC(prob, dec, v, w1, comps)
        res = krylov.pcg(lambda x: J @ x, B.apply, -R, rtol=1e-10, maxit=500,
                         project=lambda x: newton.project_range(x, N))
        lo, hi = res.lanczos_extremes()
        row = {"fp32": "+".join(comps) if comps else "none (FP64)", "pcg": res.its,
               "cond": round(hi / lo, 3), "lambda_min": round(lo, 4), "lambda_max": round(hi, 3),
               "seconds": round(time.time() - t0, 1)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mesh", choices=["hh8", "cube8"], default="hh8")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rows = run(a.mesh)
    print("| FP32 component(s) | PCG iterations | Lanczos cond | lambda_min | lambda_max |")
    print("|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['fp32']} | {r['pcg']} | {r['cond']} | {r['lambda_min']} | {r['lambda_max']} |")
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
