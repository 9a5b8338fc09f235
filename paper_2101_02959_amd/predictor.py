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
    a = ap.parse_args(argv)
    torch.cuda.init()
    log = lambda *x: print(*x, flush=True)  # noqa: E731
    ne = tuple(int(x) for x in a.elements.split(","))
    pa = tuple(int(x) for x in a.parts.split(","))
    mesh, ph, opts = small_mesh(ne, pa), Physics(), Opts()
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
            "lr_final": a.lr_final, "seed": a.seed}
    save(a.out, params, sc, meta)
    log(f"wrote {a.out}")
    held = stimulus_sites(mesh, a.heldout_sites, a.heldout_seed)
    rows, worst = evaluate(mesh, ph, opts, held, a.steps_per_site, params, sc)
    s = summarize(rows)
    log(f"held-out {a.heldout_sites} sites x {a.steps_per_site} steps: Newton extrap/cnn {s['newton']}, "
        f"PCG {s['pcg']}, ms {tuple(round(x) for x in s['ms'])}, initial residual reduction "
        f"(geomean) {s['r0_gain_geomean']:.2f}, learned guess used {s['cnn_used']} / {s['steps']}, "
        f"final states differ by {worst:.2e}")


if __name__ == "__main__":
    main()
