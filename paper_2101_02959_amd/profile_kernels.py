"""Profiling driver for rocprofv3: the hot kernels of one linearised time step,
each launched through bdm_profile_kernel, after a plain device copy of known
size that calibrates the HBM byte counters.

    rocprofv3 --kernel-trace --stats -d OUT -- python3 -m paper_2101_02959_amd.profile_kernels
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT_F -- python3 -m paper_2101_02959_amd.profile_kernels
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT_W -- python3 -m paper_2101_02959_amd.profile_kernels
    python3 -m paper_2101_02959_amd.profile_kernels --summarize OUT_F OUT_W

Options: --workload (default slab256), --precision f32|f64 (default f32).

The copy is an elementwise negation over COPY_MIB of float64 (it reads and
writes COPY_MIB each); its FETCH_SIZE and WRITE_SIZE readings give the factor
by which each counter over- or under-states the bytes moved.  Every dispatch
after it belongs to the profiled kernels: the interior elimination of the first
setup chunk (assembly, panel and rank-k update kernels), one forward and one
backward Dirichlet triangular solve over all subdomains, and one Jacobian
apply.  --summarize reads the two counter runs and prints, per kernel, the
dispatch count and the calibrated HBM bytes read and written per dispatch.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import sys

COPY_MIB = 1024
COPY_TAG = "neg_kernel"


def run(workload_name, precision):
    import numpy as np
    import torch

    import paper_2101_02959_amd as P
    from workload import initial_state, stimulus_nodal, workload

    wl = workload(workload_name)
    prec = P.BDM_PREC_MIXED if precision == "f32" else P.BDM_PREC_FP64
    S = P.Solver(wl.mesh, wl.physics, wl.solver, precision=prec)
    v0, ue0, w0 = initial_state(wl.mesh, wl.physics, wl.perturb_seed)
    S.bdm_set_state(v0, ue0, w0)
    S.bdm_set_stimulus(stimulus_nodal(wl.mesh, wl.stim_block, wl.stim_amplitude), 0, wl.stim_steps)
    S.bdm_linearize(v0, w0)
    torch.cuda.synchronize()
    n = COPY_MIB * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(f"calibration copy: {COPY_MIB} MiB read, {COPY_MIB} MiB written", flush=True)
    del x, y
    for name, kid, reps in (("rank-k update (first setup chunk)", P.BDM_KERNEL_SYRK_UPDATE, 1),
                            ("forward Dirichlet solve", P.BDM_KERNEL_TRSV_DIRICHLET, 1),
                            ("backward Dirichlet solve", P.BDM_KERNEL_TRSV_DIRICHLET_T, 1),
                            ("Jacobian apply", P.BDM_KERNEL_JACOBIAN, 1)):
        ms, work = S.bdm_profile_kernel(kid, reps)
        print(f"{name}: {ms:.4f} ms per launch, {work:.6g} algorithmic units per launch", flush=True)
    S.close()


def _dispatches(d):
    """{dispatch id: (kernel name, summed counter value)} of one --pmc run."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            k = int(r["Dispatch_Id"])
            name, val = out.get(k, (r["Kernel_Name"], 0.0))
            out[k] = (name, val + float(r["Counter_Value"]))
    return out


def _short(name):
    s = name.replace("(anonymous namespace)::", "").split("(")[0]
    return s[5:] if s.startswith("void ") else s


def summarize(dir_fetch, dir_write):
    tables = []
    for d in (dir_fetch, dir_write):
        disp = _dispatches(d)
        ids = sorted(disp)
        cal = [k for k in ids if COPY_TAG in disp[k][0]]
        if not cal:
            raise SystemExit(f"calibration copy ({COPY_TAG}) not found in {d}")
        k0 = cal[-1]
        factor = disp[k0][1] / (COPY_MIB * 1024.0)   # counter KiB per KiB moved
        per = collections.defaultdict(list)
        for k in ids:
            if k > k0:
                per[_short(disp[k][0])].append(disp[k][1])
        tables.append((factor, per))
    (ff, fper), (wf, wper) = tables
    print(f"calibration ({COPY_MIB} MiB copy): FETCH_SIZE reads {ff:.4f} x the bytes read, "
          f"WRITE_SIZE {wf:.4f} x the bytes written")
    print("| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | "
          "calibrated read MB/dispatch | calibrated write MB/dispatch |")
    print("|---|---|---|---|---|---|")
    for name in fper:
        f = sum(fper[name]) / len(fper[name])
        w = sum(wper.get(name, [0.0])) / max(len(wper.get(name, [])), 1)
        print(f"| {name} | {len(fper[name])} | {f:.1f} | {w:.1f} | {f / ff * 1024 / 1e6:.3f} | "
              f"{w / wf * 1024 / 1e6:.3f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="slab256")
    ap.add_argument("--precision", default="f32", choices=("f32", "f64"))
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    a = ap.parse_args()
    if a.summarize:
        summarize(*a.summarize)
    else:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        run(a.workload, a.precision)


if __name__ == "__main__":
    main()
