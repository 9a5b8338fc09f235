"""Argument checks of the mesh geometry through the C ABI, without a GPU:
invalid truncated-ellipsoid parameters and unknown geometries are refused by
bdm_create, and mapped meshes by bdm_residual_noalloc, before any device
call is made."""
import ctypes as C
import math
import os

import numpy as np
import pytest

from workload import ELLIPSOID, Physics, Solver as SolverOpts, box_mesh, ellipsoid_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2101_02959_amd", "libbidomain.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")

BDM_E_ARG = -1


def _create(mesh, geometry=None):
    from paper_2101_02959_amd import bidomain as B
    m, ph, op, keep = B.make_structs(mesh, Physics(), SolverOpts())
    if geometry is not None:
        m.geometry = geometry
    out = C.c_void_p(None)
    rc = B.lib().bdm_create(C.byref(m), C.byref(ph), C.byref(op), None, C.byref(out))
    del keep
    return rc, out.value, B.lib().bdm_last_error().decode()


@pytest.mark.parametrize("bad", [
    {6: -math.pi / 2},          # theta_min on the pole
    {7: math.pi / 2},           # theta_max on the pole
    {6: 0.2, 7: 0.1},           # theta_min > theta_max
    {0: 0.0},                   # a1 = 0
    {1: 1.0},                   # a2 < a1
    {4: 5.5},                   # c1 > c2
    {9: 7.0},                   # phi range beyond 2 pi
    {2: float("nan")},          # not finite
])
def test_invalid_ellipsoid_parameters_are_refused(bad):
    g = list(ELLIPSOID)
    for k, x in bad.items():
        g[k] = x
    rc, ctx, msg = _create(ellipsoid_mesh(4, 4, 4, 2, 2, 2, geometry=g))
    assert rc == BDM_E_ARG and ctx is None and "ellipsoid" in msg


def test_unknown_geometry_is_refused():
    rc, ctx, msg = _create(box_mesh(4, 4, 4, 0.01, 2, 2, 2), geometry=5)
    assert rc == BDM_E_ARG and ctx is None and "geometry" in msg


def test_residual_without_allocation_refuses_mapped_meshes():
    """The context-free residual has box coefficient tables only."""
    from paper_2101_02959_amd import bidomain as B
    mesh = ellipsoid_mesh(4, 4, 4, 2, 2, 2)
    m, ph, _, keep = B.make_structs(mesh, Physics(), SolverOpts())
    n = mesh.nnodes
    bufs = [np.zeros(n) for _ in range(6)]
    p = [C.c_void_p(b.ctypes.data) for b in bufs]
    rc = B.lib().bdm_residual_noalloc(C.byref(m), C.byref(ph), 0.05, p[0], p[1], p[2], p[3], None, 0, p[4], p[5],
                                      None)
    del keep
    assert rc == BDM_E_ARG and "box meshes only" in B.lib().bdm_last_error().decode()
