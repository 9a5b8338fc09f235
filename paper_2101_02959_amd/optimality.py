"""Optimality sweep of the BDDC preconditioner (Sec. 6, Test 3): a fixed
4 x 4 x 4 grid of subdomains with growing local size H/h, both scalings
(deluxe, rho) and the three primal spaces (V, V+E, V+E+F), each run for 2 ms
of activation on the slab.

    python3 -m paper_2101_02959_amd.optimality [--hh 4 8 12 16] [--steps 40]
                                              [--precision f64|mixed] [--out FILE]
                                              [--scalings rho deluxe] [--primals V VE VEF]

For every (H/h, scaling, primal space) it prints one JSON line with the
columns of the paper's table: mean Newton iterations per time step (nit),
mean PCG iterations per Newton iteration (lit), mean seconds per time step
(time; steps after the first, which carries the one-off autotuning), and the
mean Lanczos condition estimate per Newton solve (cond); then a table.
The mesh is the slab of workload.test3 (a cube of fixed side, so h shrinks
as H/h grows).  PCG runs from zero on the full system (as in the paper), so
that lit counts the same iterations the paper counts.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

SCALINGS = ("rho", "deluxe")
PRIMALS = ("V", "VE", "VEF")


def run_case(P, wl, precision, scaling, primal):
    import numpy as np
    from workload import stimulus_nodal
    code_s = {"deluxe": P.BDM_SCALING_DELUXE, "rho": P.BDM_SCALING_RHO}[scaling]
    code_p = {"V": P.BDM_PRIMAL_V, "VE": P.BDM_PRIMAL_VE, "VEF": P.BDM_PRIMAL_VEF}[primal]
    N = wl.mesh.nnodes
    S = P.Solver(wl.mesh, wl.physics, wl.solver, precision=precision, scaling=code_s, primal=code_p,
                 krylov_reduced=False)
    try:
        S.bdm_set_state(np.zeros(N), np.zeros(N), np.zeros(N))
        S.bdm_set_stimulus(stimulus_nodal(wl.mesh, wl.stim_block, wl.stim_amplitude), 0, wl.stim_steps)
        nits, lits, conds, times = [], [], [], []
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
    finally:
        S.close()
    return {"nit": float(np.mean(nits)), "lit": float(np.mean(lits)) if lits else 0.0,
            "time_s": float(np.mean(times)) if times else None,
            "cond": float(np.mean(conds)) if conds else None, "steps": wl.steps}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--hh", type=int, nargs="+", default=[4, 8, 12, 16])
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--precision", choices=["f64", "mixed"], default="f64")
    ap.add_argument("--out", default=None, help="also write the results as JSON")
    ap.add_argument("--scalings", nargs="+", choices=SCALINGS, default=list(SCALINGS))
    ap.add_argument("--primals", nargs="+", choices=PRIMALS, default=list(PRIMALS))
    args = ap.parse_args(argv)
    import paper_2101_02959_amd as P
    from workload import test3
    prec = P.BDM_PREC_FP64 if args.precision == "f64" else P.BDM_PREC_MIXED
    rows = []
    for Hh in args.hh:
        wl = test3(Hh, args.steps)
        for scaling in args.scalings:
            for primal in args.primals:
                t0 = time.time()
                rec = {"Hh": Hh, "scaling": scaling, "primal": primal, "precision": args.precision,
                       "dofs": 2 * wl.mesh.nnodes, "h_cm": wl.mesh.h}
                try:
                    rec.update(run_case(P, wl, prec, scaling, primal))
                except P.BidomainError as e:
                    rec["error"] = str(e)
                rec["wall_s"] = round(time.time() - t0, 2)
                rows.append(rec)
                print(json.dumps(rec), flush=True)
    print("H/h scaling primal   nit    lit   time(s)   cond", file=sys.stderr)
    for r in rows:
        if "error" in r:
            print(f"{r['Hh']:3d} {r['scaling']:7s} {r['primal']:4s}  {r['error']}", file=sys.stderr)
        else:
            print(f"{r['Hh']:3d} {r['scaling']:7s} {r['primal']:4s} {r['nit']:5.2f} {r['lit']:6.1f} "
                  f"{r['time_s']:8.3f} {r['cond']:7.2f}", file=sys.stderr)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
