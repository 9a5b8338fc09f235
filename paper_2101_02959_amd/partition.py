"""Partition sweep on one GPU, the analogue of the strong-scaling test of
Sec. 6 (Test 2): the 192 x 192 x 32 slab (2,458,434 dofs) cut into more and
more subdomains.  On one GPU every subdomain is a batch entry, so the sweep
trades the dense local work (growing as (H/h)^3 per dof) against the size of
the coarse problem and the preconditioner's iteration count.

    python3 -m paper_2101_02959_amd.partition [--parts 16x16x4 24x24x4 ...]
                                             [--steps 40] [--out FILE]
                                             [--geometry slab|ellipsoid]

With --geometry ellipsoid the mesh is the truncated ellipsoid of the same
test (128 x 128 x 64 elements, 2,163,330 dofs), by default in 8 x 8 x 4,
16 x 16 x 4 and 16 x 16 x 8 subdomains (local meshes of 16^3, 8 x 8 x 16
and 8^3 elements).

For every partition and path (BDDC with FP32 local factors, BDDC in FP64,
FETI-DP in FP64; deluxe V+E) it prints one JSON line: mean Newton iterations
per step (nit), mean PCG iterations per Newton iteration (lit), mean seconds
per step after the first (time), mean Lanczos condition estimate (cond), the
setup and Krylov shares of the step, and the coarse problem size; then a
table.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

PATHS = (("bddc", "mixed"), ("bddc", "f64"), ("fetidp", "f64"))


def run_case(P, wl, method, precision):
    import numpy as np
    from workload import stimulus_nodal
    N = wl.mesh.nnodes
    S = P.Solver(wl.mesh, wl.physics, wl.solver,
                 precision=P.BDM_PREC_MIXED if precision == "mixed" else P.BDM_PREC_FP64,
                 method=P.BDM_SOLVER_FETIDP if method == "fetidp" else P.BDM_SOLVER_BDDC)
    try:
        S.bdm_set_state(np.zeros(N), np.zeros(N), np.zeros(N))
        S.bdm_set_stimulus(stimulus_nodal(wl.mesh, wl.stim_block, wl.stim_amplitude), 0, wl.stim_steps)
        nits, lits, conds, times, tset, tkry = [], [], [], [], [], []
        for k in range(wl.steps):
            st = S.bdm_step(1)
            nit = st.newton_its
            print(f"  step {k}: newton {nit} pcg {list(st.krylov_its)[:nit]} {st.t_step_ms:.1f} ms",
                  file=sys.stderr, flush=True)
            nits.append(nit)
            lits += list(st.krylov_its)[:nit]
            conds += list(st.cond)[:nit]
            if k > 0:
                times.append(st.t_step_ms / 1e3)
                tset.append(st.t_setup_ms / 1e3)
                tkry.append(st.t_krylov_ms / 1e3)
    finally:
        S.close()
    mean = lambda a: float(np.mean(a)) if a else None
    return {"nit": mean(nits), "lit": mean(lits), "time_s": mean(times), "setup_s": mean(tset),
            "krylov_s": mean(tkry), "cond": mean(conds), "steps": wl.steps,
            "subdomains": int(S.nsub), "coarse_dofs": int(S.nprimal)}


ELLIPSOID_PARTS = ((8, 8, 4), (16, 16, 4), (16, 16, 8))


def main(argv=None):
    from workload import TEST2_PARTS, ellipsoid_workload, test2
    ap = argparse.ArgumentParser()
    ap.add_argument("--geometry", choices=("slab", "ellipsoid"), default="slab")
    ap.add_argument("--parts", nargs="+", default=None)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--paths", nargs="+", default=["-".join(p) for p in PATHS],
                    help="method-precision pairs, e.g. bddc-mixed fetidp-f64")
    ap.add_argument("--out", default=None, help="also write the results as JSON")
    args = ap.parse_args(argv)
    import paper_2101_02959_amd as P
    if args.parts is None:
        args.parts = ["x".join(map(str, p)) for p in (ELLIPSOID_PARTS if args.geometry == "ellipsoid"
                                                      else TEST2_PARTS)]
    rows = []
    for ptxt in args.parts:
        parts = tuple(int(v) for v in ptxt.split("x"))
        if args.geometry == "ellipsoid":
            wl = ellipsoid_workload(parts, steps=args.steps)
        else:
            wl = test2(parts, args.steps)
        m = wl.mesh
        for path in args.paths:
            method, precision = path.split("-")
            t0 = time.time()
            rec = {"geometry": args.geometry, "parts": ptxt,
                   "H/h": [m.nx // parts[0], m.ny // parts[1], m.nz // parts[2]], "method": method,
                   "precision": precision, "dofs": 2 * m.nnodes}
            try:
                rec.update(run_case(P, wl, method, precision))
            except P.BidomainError as e:
                rec["error"] = str(e)
            rec["wall_s"] = round(time.time() - t0, 2)
            rows.append(rec)
            print(json.dumps(rec), flush=True)
    print("parts      method precision  nit    lit  time(s) setup(s) krylov(s)  cond  coarse", file=sys.stderr)
    for r in rows:
        if "error" in r:
            print(f"{r['parts']:10s} {r['method']:6s} {r['precision']:6s}  {r['error']}", file=sys.stderr)
        else:
            print(f"{r['parts']:10s} {r['method']:6s} {r['precision']:6s} {r['nit']:5.2f} {r['lit']:6.1f} "
                  f"{r['time_s']:8.3f} {r['setup_s']:8.3f} {r['krylov_s']:8.3f} {r['cond']:6.2f} "
                  f"{r['coarse_dofs']:7d}", file=sys.stderr)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
