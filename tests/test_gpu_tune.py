"""Autotuner: every kernel variant it may choose is checked against the FP64
oracle, and the JSON cache round-trips (a second context reuses the choices
without timing).

The variants are forced through the cache file: each entry names the device,
family and size class that a context reports, and the choice.  In FP64 the
rank-k variants differ only in tiling (every entry accumulates its inner
products in the same order), and the stencil variants (LDS tiles of several
shapes, and the register z-march) take each node's 27 products in the same
order, so all of them must agree bitwise; in FP32 the inner chunk length
changes the two-level accumulation, so those are held to the FP32 bar.
"""
import json

import numpy as np
import pytest
from parity_util import assert_close

from oracle import bddc, bidomain, dd, newton
from workload import Mesh, Physics, Solver as SolverOpts

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MESHES = {
    "ragged": Mesh(11, 9, 10, 0.01, (0, 3, 7, 11), (0, 5, 9), (0, 4, 10)),
    "uneven442": Mesh(20, 18, 12, 0.01, (0, 4, 9, 13, 20), (0, 5, 9, 14, 18), (0, 5, 12)),
}
NSTENCIL, NSYRK = 11, 6


def _gauge(x, N):
    x = np.array(x, dtype=np.float64).copy()
    x[N:] -= x[N:].mean()
    return x


def _state(N, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-10, 40, N), rng.uniform(0, 0.2, N)


def test_cache_roundtrip(tmp_path, monkeypatch):
    import paper_2101_02959_amd as P
    mesh = MESHES["ragged"]
    path = tmp_path / "tune.json"
    monkeypatch.setenv("BDM_TUNE_CACHE", str(path))
    v, w = _state(mesh.nnodes, 4)
    S = P.Solver(mesh, Physics(), SolverOpts(), precision=1)
    S.bdm_linearize(v, w)
    rep = S.bdm_tune_report()
    S.close()
    ent = rep["entries"]
    assert sorted(e["family"] for e in ent) == ["stencil", "syrk", "syrk"]
    for e in ent:
        assert not e["cached"]
        assert len(e["ms"]) == (NSTENCIL if e["family"] == "stencil" else NSYRK)
        ok = [m for m in e["ms"] if m >= 0]
        assert ok and e["ms"][e["choice"]] == min(ok)
    disk = json.loads(path.read_text())
    assert disk["format"] == "bidomain-tune-1" and len(disk["entries"]) == 3
    S2 = P.Solver(mesh, Physics(), SolverOpts(), precision=1)
    S2.bdm_linearize(v, w)
    rep2 = S2.bdm_tune_report()
    S2.close()
    assert all(e["cached"] for e in rep2["entries"])
    key = lambda r: sorted((e["family"], e["class"], e["choice"]) for e in r["entries"])
    assert key(rep2) == key(rep)


def test_unreadable_cache_is_an_error(tmp_path, monkeypatch):
    import paper_2101_02959_amd as P
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    monkeypatch.setenv("BDM_TUNE_CACHE", str(path))
    with pytest.raises(P.BidomainError, match="BDM_E_ARG"):
        P.Solver(MESHES["ragged"], Physics(), SolverOpts())


@pytest.mark.parametrize("mname", list(MESHES))
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 5e-5)])
def test_every_variant_matches_oracle(mname, prec, tol, tmp_path, monkeypatch):
    import paper_2101_02959_amd as P
    mesh = MESHES[mname]
    ph, so = Physics(), SolverOpts()
    prob = bidomain.Problem(mesh, ph, so.dt)
    N = prob.N
    v, w = _state(N, 4)
    B = bddc.BDDC(prob, dd.Decomposition(mesh), v, w)
    rs = [newton.project_range(np.random.default_rng(s).standard_normal(2 * N), N) for s in (5, 6)]
    refs = [_gauge(B.apply(r), N) for r in rs]
    # size classes this mesh reports
    probe = tmp_path / "probe.json"
    monkeypatch.setenv("BDM_TUNE_CACHE", str(probe))
    S = P.Solver(mesh, ph, so, precision=prec)
    S.bdm_linearize(v, w)
    classes = [(e["device"], e["family"], e["class"]) for e in S.bdm_tune_report()["entries"]]
    S.close()
    # every stencil shape and every rank-k variant at least once
    combos = [(v, v) for v in range(NSYRK)] + [(sv, sv % NSYRK) for sv in range(NSYRK, NSTENCIL)]
    first = None
    for sv, yv in combos:
        forced = tmp_path / f"forced_{sv}_{yv}.json"
        forced.write_text(json.dumps({"format": "bidomain-tune-1", "entries": [
            {"device": d, "family": f, "class": c, "choice": sv if f == "stencil" else yv, "ms": []}
            for d, f, c in classes]}))
        monkeypatch.setenv("BDM_TUNE_CACHE", str(forced))
        S = P.Solver(mesh, ph, so, precision=prec)
        S.bdm_linearize(v, w)
        got = {e["family"] + e["class"]: e["choice"] for e in S.bdm_tune_report()["entries"]}
        assert all(ch == (sv if k.startswith("stencil") else yv) for k, ch in got.items()), got
        outs = [S.bdm_bddc_apply(r).cpu().numpy() for r in rs]
        S.close()
        for z, zref in zip(outs, refs):
            assert_close(_gauge(z, N), zref, tol, N, f"stencil {sv} rank-k {yv}")
        if prec == 0:
            if first is None:
                first = outs
            else:
                for a, b in zip(outs, first):
                    assert np.array_equal(a, b), (sv, yv)
