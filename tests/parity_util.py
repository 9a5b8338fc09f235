"""Comparison helpers of the parity tests.

Every comparison is made per field (the v block and the u_e block of a 2N
vector, or the whole vector for multiplier-space results) in two ways:

  * the relative 2-norm  ||a - b|| / ||b|| <= tol, and
  * element by element   max_i |a_i - b_i| <= tol * max_i |b_i|,

so that an error confined to a few entries (one class of interface objects,
one subdomain) cannot hide under a whole-vector norm.
"""
import numpy as np


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elem(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gauge(x, N):
    x = np.array(x, dtype=np.float64).copy()
    x[N:] -= x[N:].mean()
    return x


def fields(x, N):
    """The v and u_e blocks of a 2N vector; other lengths are one field."""
    x = np.asarray(x)
    if N is not None and x.shape[0] == 2 * N:
        return {"v": x[:N], "u_e": x[N:]}
    return {"all": x}


def assert_close(a, b, tol, N=None, what="", etol=None):
    """Per-field relative 2-norm at tol and element-wise bound at etol
    (default tol)."""
    etol = tol if etol is None else etol
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    fa, fb = fields(a, N), fields(b, N)
    out = {}
    for k in fb:
        r, e = rel(fa[k], fb[k]), elem(fa[k], fb[k])
        out[k] = (r, e)
        assert r <= tol and e <= etol, \
            f"{what} field {k}: rel2 {r:.3e} (tol {tol:.1e}) elementwise {e:.3e} (tol {etol:.1e})"
    return out


def error_by_class(a, b, dec, N):
    """Largest |a - b| per node class (interior, face, edge, vertex) and
    field, relative to max |b| of the field: where an error concentrates."""
    cls = {"I": dec.interior_nodes()}
    for kind, objs in (("F", dec.faces), ("E", dec.edges), ("V", dec.verts)):
        cls[kind] = np.concatenate([o.nodes for o in objs]) if objs else np.zeros(0, dtype=np.int64)
    out = {}
    for fname, off in (("v", 0), ("u_e", N)):
        scale = max(np.max(np.abs(b[off:off + N])), 1e-300)
        out[fname] = {k: float(np.max(np.abs(a[off + n] - b[off + n])) / scale) if len(n) else 0.0
                      for k, n in cls.items()}
    return out
