"""Training and loading of the learned Newton initial guess.

The network, its loss and Adam run in libbidomain's kernels
(``bdm_predictor_*``); this module only records trajectories with the
library's own time stepper, packs them into training samples, fits the input
and output scales and stores the weights.

A sample is six node fields ``[v^n, u_e^n, v^{n-1}, u_e^{n-1}, v^{n+1},
u_e^{n+1}]`` and the network learns the scaled second difference
``(u^{n+1} - 2 u^n + u^{n-1}) / s_y``, i.e. the error of the linear
extrapolation that the guess corrects.

Usage (trains on the 32^3 slab from 50 seeded stimulus sites, writes the
default weights and evaluates on 5 held-out sites):
    python -m paper_2101_02959_amd.predictor
On the 17M-dof slab from 12 sites x 40 steps + 20 steps (500 solver steps),
trained on 33^3-node crops around the sites:
    python -m paper_2101_02959_amd.predictor --from-workload slab256 --sites 12 \
        --site-seed 3000 --extra-steps 20 --out WEIGHTS
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import bidomain as B

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(_HERE, "weights", "predictor.npz")
CHANNELS = (4, 16, 16, 16, 2)


def init_params(seed: int, last_gain: float = 0.1) -> np.ndarray:
    """He-normal weights, zero biases; the last layer scaled by ``last_gain`` so
    that the untrained network stays close to plain extrapolation."""
    rng = np.random.default_rng(seed)
    out = []
    for L, (cin, cout) in enumerate(zip(CHANNELS[:-1], CHANNELS[1:])):
        std = np.sqrt(2.0 / (cin * 27)) * (last_gain if L == 3 else 1.0)
        out.append(rng.normal(0.0, std, size=cout * cin * 27))
        out.append(np.zeros(cout))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == B.Solver.bdm_predictor_size()
    return p


def trajectory(S, steps: int, guess_log=None):
    """Advance the solver ``steps`` times; returns the states (steps + 1, 2, N)
    on the device, starting with the current one, and the per-step stats."""
    import torch
    v, ue, _, _ = S.bdm_get_state()
    states = [torch.stack([v, ue])]
    stats = []
    for _ in range(steps):
        st = S.bdm_step(1)
        stats.append(st)
        v, ue, _, _ = S.bdm_get_state()
        states.append(torch.stack([v, ue]))
        if guess_log is not None:
            guess_log(st)
    return torch.stack(states), stats


def make_samples(states, skip=()):
    """Samples for n = 1 .. len(states) - 2 except those in ``skip``, shape
    (n_samples, 6 N).  A sample whose two steps straddle a switch of the
    stimulus is not predictable from the state history and is best skipped."""
    import torch
    keep = [n for n in range(1, states.shape[0] - 1) if n not in set(skip)]
    idx = torch.tensor(keep, device=states.device)
    cur, prv, nxt = states[idx], states[idx - 1], states[idx + 1]
    return torch.cat([cur, prv, nxt], dim=1).reshape(len(keep), -1).contiguous()


def fit_scales(states) -> np.ndarray:
    """RMS of the states, their first and their second differences, per field
    (v and u_e), over a trajectory (steps + 1, 2, N)."""
    x = states.double()
    d1 = x[1:] - x[:-1]
    d2 = x[2:] - 2 * x[1:-1] + x[:-2]

    def rms(t, c):
        return float(t[:, c].pow(2).mean().sqrt().clamp_min(1e-12))

    return np.array([rms(x, 0), rms(x, 1), rms(d1, 0), rms(d1, 1), rms(d2, 0), rms(d2, 1)])


def train(S, samples, steps: int, lr: float, seed: int, lr_final: float | None = None,
          segments: int = 10):
    """Adam over randomly ordered samples; the learning rate decays
    geometrically from ``lr`` to ``lr_final`` in ``segments`` stages.
    Returns the per-step losses."""
    rng = np.random.default_rng(seed)
    n = samples.shape[0]
    order = rng.integers(0, n, size=steps).astype(np.int32)
    lr_final = lr if lr_final is None else lr_final
    losses = []
    bounds = np.linspace(0, steps, segments + 1).astype(int)
    for k in range(segments):
        a, b = bounds[k], bounds[k + 1]
        if b <= a:
            continue
        lr_k = lr * (lr_final / lr) ** (k / max(segments - 1, 1))
        losses.append(S.bdm_predictor_train(samples, order[a:b], lr_k))
    return np.concatenate(losses) if losses else np.zeros(0)


def save(path: str, params: np.ndarray, scales: np.ndarray, meta: dict):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), scales=np.asarray(scales, dtype=np.float64),
             meta=np.array(repr(sorted(meta.items()))))


def load(path: str = DEFAULT_WEIGHTS):
    """Parameters and scales (no pickled objects are read)."""
    with np.load(path, allow_pickle=False) as z:
        return z["params"].copy(), z["scales"].copy()


def site_solver(mesh, physics, solver_opts, origin, stim_amp=None, stim_block=(2, 2, 2), stim_steps=20,
                precision=B.BDM_PREC_MIXED, guess=B.BDM_GUESS_EXTRAP):
    """A solver at rest with a stimulus on the element block at ``origin``."""
    from workload import PAPER_STIM, initial_state, stimulus_nodal
    S = B.Solver(mesh, physics, solver_opts, precision=precision, guess=guess)
    v0, ue0, w0 = initial_state(mesh, physics, None)
    S.bdm_set_state(v0, ue0, w0)
    amp = PAPER_STIM if stim_amp is None else stim_amp
    S.bdm_set_stimulus(stimulus_nodal(mesh, stim_block, amp, origin), 0, stim_steps)
    return S


def dataset(mesh, physics, opts, origins, steps, stim_steps=20, log=print):
    """Trajectories from every stimulus site, packed as samples (the sample
    that straddles the stimulus switch-off is skipped), and the scales fitted
    on the first trajectory."""
    import torch
    samples, scales = [], None
    for q, o in enumerate(origins):
        S = site_solver(mesh, physics, opts, o, stim_steps=stim_steps)
        t0 = time.time()
        states, stats = trajectory(S, steps)
        S.close()
        if scales is None:
            scales = fit_scales(states)
        samples.append(make_samples(states, skip=(stim_steps,)))
        log(f"  site {q} {o}: {steps} steps in {time.time() - t0:.1f} s, Newton "
            f"{sum(s.newton_its for s in stats)}, setup {sum(s.t_setup_ms for s in stats):.0f} ms, "
            f"Krylov {sum(s.t_krylov_ms for s in stats):.0f} ms")
        del states
    return torch.cat(samples), scales


def crop_nodes(mesh, origin, block, size):
    """Node ids (lexicographic, x fastest) of a size^3 cube of nodes centred
    on the element block at ``origin``, shifted to lie inside the mesh."""
    lo = []
    for o, b, n in zip(origin, block, (mesh.nx, mesh.ny, mesh.nz)):
        lo.append(min(max(o + b // 2 - size // 2, 0), n + 1 - size))
    i = np.arange(lo[0], lo[0] + size)
    j = np.arange(lo[1], lo[1] + size)
    k = np.arange(lo[2], lo[2] + size)
    return (i[None, None, :] + (mesh.nx + 1) * (j[None, :, None] + (mesh.ny + 1) * k[:, None, None])).ravel()


def dataset_crops(mesh, physics, opts, runs, crop, stim_steps=20, log=print):
    """Solver trajectories on a large mesh, one per (origin, steps) in runs,
    each from rest with the stimulus on the 2 x 2 x 2-element block at
    origin; every state is cut to the crop^3 nodes around the site, and the
    crops are packed as samples of a crop^3-node grid (the sample that
    straddles the stimulus switch-off is skipped).  One context serves all
    runs.  Returns the samples (device) and the scales fitted on the first
    run's crops."""
    import torch
    from workload import PAPER_STIM, initial_state, stimulus_nodal
    S = B.Solver(mesh, physics, opts, precision=B.BDM_PREC_MIXED, guess=B.BDM_GUESS_EXTRAP)
    samples, scales = [], None
    try:
        for q, (o, steps) in enumerate(runs):
            v0, ue0, w0 = initial_state(mesh, physics, None)
            S.bdm_set_state(v0, ue0, w0)
            S.bdm_set_stimulus(stimulus_nodal(mesh, (2, 2, 2), PAPER_STIM, o), 0, stim_steps)
            idx = torch.as_tensor(crop_nodes(mesh, o, (2, 2, 2), crop), device=S.device)
            t0 = time.time()
            v, ue, _, _ = S.bdm_get_state()
            states = [torch.stack([v[idx], ue[idx]])]
            nit = 0
            for _ in range(steps):
                st = S.bdm_step(1)
                nit += st.newton_its
                v, ue, _, _ = S.bdm_get_state()
                states.append(torch.stack([v[idx], ue[idx]]))
            states = torch.stack(states)
            if nit == 0:
                raise RuntimeError(f"run {q} at {o}: no Newton iteration in {steps} steps (no stimulus?)")
            if scales is None:
                scales = fit_scales(states)
            samples.append(make_samples(states, skip=(stim_steps,)))
            log(f"  run {q} site {o}: {steps} steps in {time.time() - t0:.1f} s, Newton {nit}")
    finally:
        S.close()
    return torch.cat(samples), scales


def evaluate(mesh, physics, opts, origins, steps, params, scales, stim_steps=20):
    """Held-out comparison of the extrapolated and the learned (judged) guess.
    Per step: Newton and PCG iterations, initial and final residual, the
    guess used and the wall time; and the largest relative difference of the
    final states (the tolerance is unchanged, so they agree to it)."""
    rows, worst = [], 0.0
    for o in origins:
        per = {}
        for name, guess in (("extrap", B.BDM_GUESS_EXTRAP), ("cnn", B.BDM_GUESS_CNN)):
            S = site_solver(mesh, physics, opts, o, stim_steps=stim_steps, guess=guess)
            if guess == B.BDM_GUESS_CNN:
                S.bdm_predictor_set(params, scales)
            out = []
            for k in range(steps):
                st = S.bdm_step(1)
                nit = st.newton_its
                out.append({"newton": nit, "pcg": int(sum(list(st.krylov_its)[:nit])),
                            "r0": st.res_hist[0], "rfinal": st.res_hist[nit], "tol": 1e-8 * st.res_ref,
                            "used": st.guess_used, "ms": st.t_step_ms})
            v, ue, _, _ = S.bdm_get_state()
            per[name] = (out, v.cpu().numpy(), ue.cpu().numpy())
            S.close()
        for f in (1, 2):
            a, b = per["cnn"][f], per["extrap"][f]
            worst = max(worst, float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)))
        for k in range(steps):
            rows.append({"site": o, "step": k, "extrap": per["extrap"][0][k], "cnn": per["cnn"][0][k]})
    return rows, worst


def summarize(rows):
    """Totals and the geometric-mean reduction of the initial residual over
    steps that have a previous step (k >= 1)."""
    e = [r["extrap"] for r in rows]
    c = [r["cnn"] for r in rows]
    g = [np.log(r["extrap"]["r0"] / r["cnn"]["r0"]) for r in rows if r["step"] >= 1]
    return {"steps": len(rows),
            "newton": (sum(x["newton"] for x in e), sum(x["newton"] for x in c)),
            "pcg": (sum(x["pcg"] for x in e), sum(x["pcg"] for x in c)),
            "ms": (sum(x["ms"] for x in e), sum(x["ms"] for x in c)),
            "r0_gain_geomean": float(np.exp(np.mean(g))) if g else 1.0,
            "cnn_used": sum(1 for x in c if x["used"] == 2)}


def main(argv=None):
    import torch
    from workload import Physics, Solver as Opts, small_mesh, stimulus_sites
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--elements", default="32,32,32")
    ap.add_argument("--parts", default="4,4,4")
    ap.add_argument("--sites", type=int, default=50)
    ap.add_argument("--site-seed", type=int, default=7)
    ap.add_argument("--steps-per-site", type=int, default=40)
    ap.add_argument("--heldout-sites", type=int, default=5)
    ap.add_argument("--heldout-seed", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=60000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--from-workload", default=None,
                    help="record the trajectories on this workload's mesh (e.g. slab256) and train on "
                         "crops of --crop^3 nodes around each site, on a crop-sized context")
    ap.add_argument("--crop", type=int, default=33)
    ap.add_argument("--extra-steps", type=int, default=0,
                    help="with --from-workload: one more site (seed site-seed + 1) run this many steps")
    a = ap.parse_args(argv)
    torch.cuda.init()
    log = lambda *x: print(*x, flush=True)  # noqa: E731
    ph, opts = Physics(), Opts()
    if a.from_workload:
        from workload import workload as named
        big = named(a.from_workload).mesh
        sites = stimulus_sites(big, a.sites, a.site_seed)
        runs = [(o, a.steps_per_site) for o in sites]
        if a.extra_steps:
            runs.append((stimulus_sites(big, 1, a.site_seed + 1)[0], a.extra_steps))
        log(f"dataset: {len(runs)} runs, {sum(r[1] for r in runs)} solver steps on {a.from_workload}, "
            f"crops of {a.crop}^3 nodes")
        samples, scales = dataset_crops(big, ph, opts, runs, a.crop, log=log)
        ne, pa = (a.crop - 1,) * 3, (2, 2, 2)
        mesh = small_mesh(ne, pa)
    else:
        ne = tuple(int(x) for x in a.elements.split(","))
        pa = tuple(int(x) for x in a.parts.split(","))
        mesh = small_mesh(ne, pa)
        sites = stimulus_sites(mesh, a.sites, a.site_seed)
        log(f"dataset: {a.sites} sites x {a.steps_per_site} steps on {ne} elements")
        samples, scales = dataset(mesh, ph, opts, sites, a.steps_per_site, log=log)
    log(f"  {samples.shape[0]} samples, scales {np.array2string(scales, precision=4)}")
    S = B.Solver(mesh, ph, opts)
    S.bdm_predictor_set(init_params(a.seed), scales)
    t0 = time.time()
    seg = 20
    rng = np.random.default_rng(a.seed + 1)
    order = rng.integers(0, samples.shape[0], size=a.train_steps).astype(np.int32)
    bounds = np.linspace(0, a.train_steps, seg + 1).astype(int)
    for k in range(seg):
        lr_k = a.lr * (a.lr_final / a.lr) ** (k / (seg - 1))
        L = S.bdm_predictor_train(samples, order[bounds[k]:bounds[k + 1]], lr_k)
        log(f"  train segment {k}: lr {lr_k:.2e} mean loss {L.mean():.4g} ({time.time() - t0:.0f} s)")
    params, sc = S.bdm_predictor_get()
    S.close()
    del samples
    meta = {"elements": ne, "parts": pa, "sites": a.sites, "site_seed": a.site_seed,
            "steps_per_site": a.steps_per_site, "train_steps": a.train_steps, "lr": a.lr,
            "lr_final": a.lr_final, "seed": a.seed, "from_workload": a.from_workload, "crop": a.crop,
            "extra_steps": a.extra_steps}
    save(a.out, params, sc, meta)
    log(f"wrote {a.out}")
    if a.from_workload:
        return
    held = stimulus_sites(mesh, a.heldout_sites, a.heldout_seed)
    rows, worst = evaluate(mesh, ph, opts, held, a.steps_per_site, params, sc)
    s = summarize(rows)
    log(f"held-out {a.heldout_sites} sites x {a.steps_per_site} steps: Newton extrap/cnn {s['newton']}, "
        f"PCG {s['pcg']}, ms {tuple(round(x) for x in s['ms'])}, initial residual reduction "
        f"(geomean) {s['r0_gain_geomean']:.2f}, learned guess used {s['cnn_used']} / {s['steps']}, "
        f"final states differ by {worst:.2e}")


if __name__ == "__main__":
    main()
