"""Whole-beat run on the slab (Sec. 6, Test 4): activation and recovery over
2400 time steps, with the iteration counts tracked along the way.

    python3 -m paper_2101_02959_amd.beat [--parts 24x12x3] [--steps 2400]
        [--method bddc|fetidp] [--precision mixed|f64] [--guess prev|extrap|cnn]
        [--every 100] [--out FILE]

Every --every steps it prints one JSON line for the window just finished:
mean Newton iterations per step (nit), mean PCG iterations per Newton
iteration (lit), mean Lanczos condition estimate, mean seconds per step, the
largest FP64 true residual of a Newton linear solve, the share of steps
whose learned guess won the judge (guess cnn), and the state of the tissue
at the window's end: the fraction of nodes above the threshold v_th
(depolarised) and the largest v.  A summary line closes the run.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--parts", default="24x12x3")
    ap.add_argument("--steps", type=int, default=2400)
    ap.add_argument("--method", choices=["bddc", "fetidp"], default="bddc")
    ap.add_argument("--precision", choices=["mixed", "f64"], default="mixed")
    ap.add_argument("--guess", choices=["prev", "extrap", "cnn"], default="cnn")
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--out", default=None, help="also write the window records as JSON")
    ap.add_argument("--cubic", action="store_true",
                    help="cubic elements of 0.01 cm (1.92 x 0.96 x 0.24 cm) instead of the paper's slab")
    args = ap.parse_args(argv)
    import numpy as np
    import torch

    import paper_2101_02959_amd as P
    from workload import stimulus_nodal, test4
    parts = tuple(int(v) for v in args.parts.split("x"))
    wl = test4(parts, args.steps, paper_geometry=not args.cubic)
    N = wl.mesh.nnodes
    guess = {"prev": P.BDM_GUESS_PREV, "extrap": P.BDM_GUESS_EXTRAP, "cnn": P.BDM_GUESS_CNN}[args.guess]
    S = P.Solver(wl.mesh, wl.physics, wl.solver,
                 precision=P.BDM_PREC_MIXED if args.precision == "mixed" else P.BDM_PREC_FP64,
                 method=P.BDM_SOLVER_FETIDP if args.method == "fetidp" else P.BDM_SOLVER_BDDC, guess=guess)
    if guess == P.BDM_GUESS_CNN:
        from paper_2101_02959_amd import predictor as PR
        S.bdm_predictor_set(*PR.load())
    records = []
    try:
        S.bdm_set_state(np.zeros(N), np.zeros(N), np.zeros(N))
        S.bdm_set_stimulus(stimulus_nodal(wl.mesh, wl.stim_block, wl.stim_amplitude), 0, wl.stim_steps)
        win = {"nit": [], "lit": [], "cond": [], "t": [], "tres": [], "cnn": []}
        t0 = time.time()
        for k in range(wl.steps):
            st = S.bdm_step(1)
            nit = st.newton_its
            win["nit"].append(nit)
            win["lit"] += list(st.krylov_its)[:nit]
            win["cond"] += list(st.cond)[:nit]
            win["tres"] += list(st.krylov_true_res)[:nit]
            win["t"].append(st.t_step_ms / 1e3)
            win["cnn"].append(1.0 if st.guess_used == 2 else 0.0)
            if (k + 1) % args.every == 0 or k + 1 == wl.steps:
                v = S.bdm_get_state()[0]
                rec = {"steps": [k + 1 - len(win["nit"]), k + 1], "t_ms": (k + 1) * wl.solver.dt,
                       "nit": float(np.mean(win["nit"])),
                       "lit": float(np.mean(win["lit"])) if win["lit"] else 0.0,
                       "cond": float(np.mean(win["cond"])) if win["cond"] else None,
                       "s_per_step": float(np.mean(win["t"])),
                       "true_res_max": float(np.max(win["tres"])) if win["tres"] else 0.0,
                       "guess_cnn": float(np.mean(win["cnn"])),
                       "depolarised": float((v > wl.physics.vth).double().mean()),
                       "v_max": float(v.max())}
                records.append(rec)
                print(json.dumps(rec), flush=True)
                win = {key: [] for key in win}
        wall = time.time() - t0
    finally:
        S.close()
    allw = lambda key: [r[key] for r in records]
    summary = {"summary": True, "parts": args.parts, "method": args.method, "precision": args.precision,
               "guess": args.guess, "dofs": 2 * N, "steps": wl.steps, "wall_s": round(wall, 1),
               "nit": float(np.average(allw("nit"), weights=[r["steps"][1] - r["steps"][0] for r in records])),
               "lit_window_range": [min(allw("lit")), max(allw("lit"))],
               "true_res_max": max(allw("true_res_max")), "depolarised_peak": max(allw("depolarised"))}
    print(json.dumps(summary), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"windows": records, "summary": summary}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
