"""Host logic of libbidomain without a GPU: the C++ partition and N_x
classification, built with g++, against the oracle's decomposition; and the
C ABI library exporting every entry point its header declares."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT
import numpy as np

from oracle import bidomain, dd
from workload import Mesh, Physics

EXE = os.path.join(ROOT, "_build", "topo_dump")


@pytest.fixture(scope="module")
def topo_exe():
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    src = [os.path.join(ROOT, "tests", "host", "topo_dump.cpp"),
           os.path.join(ROOT, "paper_2101_02959_amd", "csrc", "topology.cpp")]
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-o", EXE] + src, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    return EXE


PRIMAL_CODE = {"VE": 0, "V": 1, "VEF": 2}


def _dump(exe, mesh, primal="VE"):
    args = [mesh.nx, mesh.ny, mesh.nz, len(mesh.cuts_x) - 1, len(mesh.cuts_y) - 1,
            len(mesh.cuts_z) - 1] + list(mesh.cuts_x) + list(mesh.cuts_y) + list(mesh.cuts_z) \
        + [PRIMAL_CODE[primal]]
    out = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, check=True).stdout
    objs, subs = [], []
    for line in out.splitlines():
        if line.startswith("OBJ"):
            head, nodes = line[4:].split("|")
            h = head.split()
            objs.append((h[0], tuple(int(x) for x in h[1:]), tuple(int(x) for x in nodes.split())))
        elif line.startswith("SUB"):
            parts = line[4:].split("|")
            h = [int(x) for x in parts[0].split()]
            subs.append((h, [int(x) for x in parts[1].split()], [int(x) for x in parts[2].split()],
                         [int(x) for x in parts[3].split()]))
    return objs, subs


MESHES = [
    Mesh(8, 8, 8, 0.01, (0, 4, 8), (0, 4, 8), (0, 4, 8)),
    Mesh(11, 9, 10, 0.01, (0, 3, 7, 11), (0, 5, 9), (0, 4, 10)),
    Mesh(12, 12, 8, 0.01, (0, 4, 8, 12), (0, 3, 6, 12), (0, 4, 8)),
]


@pytest.mark.parametrize("primal", ["VE", "V", "VEF"])
@pytest.mark.parametrize("mesh", MESHES, ids=["cube8", "ragged", "uneven3x3x2"])
def test_partition_matches_oracle(topo_exe, mesh, primal):
    """Same faces / edges / vertices (sharing subdomains and nodes, in the same
    order), same interior node sets and interface node lists per subdomain,
    same primal numbering as the oracle's N_x classification (Sec. 4.1), for
    each primal space (Sec. 4.4).  The library orders the interior nodes for
    its elimination (core first, see the next test); the oracle ascending."""
    objs, subs = _dump(topo_exe, mesh, primal)
    dec = dd.Decomposition(mesh, primal)
    ref = ([("F", o.subs, tuple(o.nodes)) for o in dec.faces]
           + [("E", o.subs, tuple(o.nodes)) for o in dec.edges]
           + [("V", o.subs, tuple(o.nodes)) for o in dec.verts])
    assert objs == ref
    assert len(subs) == dec.nsub
    for s, (h, I, r, prim) in enumerate(subs):
        info = dec.sub[s]
        assert h[0] == s
        assert h[1:6] == [info.nI, info.nr, info.nV, 2 * len(info.cons), info.nV + 2 * len(info.cons)]
        assert sorted(I) == list(info.I_nodes)
        assert r == list(info.r_nodes)
        assert prim == list(info.primal)


@pytest.mark.parametrize("mesh", MESHES, ids=["cube8", "ragged", "uneven3x3x2"])
def test_interior_order_puts_the_core_first(topo_exe, mesh):
    """The interior elimination order: first the core, the interior nodes
    whose rows of K_IGamma (Sec. 4.1) are zero, then the other interior
    nodes, each part ascending; nIc counts the core dofs.  The core is taken
    here from the oracle's assembled local matrix, not from the mesh
    geometry the library uses."""
    _, subs = _dump(topo_exe, mesh)
    dec = dd.Decomposition(mesh, "VE")
    prob = bidomain.Problem(mesh, Physics(), 0.05)
    zero = np.zeros(prob.N)
    for s, (h, I, _, _) in enumerate(subs):
        info = dec.sub[s]
        KIG = dd.LocalOps(prob, dec, s, zero, zero).KIG
        coupled = [bool(np.any(KIG[2 * q:2 * q + 2] != 0.0)) for q in range(len(info.I_nodes))]
        core = [int(n) for n, c in zip(info.I_nodes, coupled) if not c]
        shell = [int(n) for n, c in zip(info.I_nodes, coupled) if c]
        assert h[6] == 2 * len(core)
        assert I == core + shell


def test_partition_rejects_bad_cuts(topo_exe):
    r = subprocess.run([topo_exe, "8", "8", "8", "2", "2", "1", "0", "4", "8", "0", "4", "8", "0", "8"],
                       capture_output=True, text=True)
    assert r.returncode == 1 and "ERROR" in r.stdout


def test_library_exports_every_declared_entry_point():
    """libbidomain.so loads on a machine without a GPU and exports every
    function declared in include/bidomain.h (no compute call is made)."""
    lib_path = os.path.join(ROOT, "paper_2101_02959_amd", "libbidomain.so")
    if not os.path.exists(lib_path):
        pytest.skip("library not built")
    with open(os.path.join(ROOT, "include", "bidomain.h")) as f:
        hdr = f.read()
    names = sorted(set(re.findall(r"\b(bdm_[a-z_]+)\s*\(", hdr)))
    assert "bdm_step" in names and "bdm_bddc_apply" in names and "bdm_fetidp_apply" in names
    lib = ctypes.CDLL(lib_path)
    for n in names:
        assert hasattr(lib, n), n
    from paper_2101_02959_amd import bidomain
    assert set(bidomain.EXPORTS) == set(names)
    lib.bdm_last_error.restype = ctypes.c_char_p
    assert lib.bdm_last_error() is not None


def _header_fields(hdr, name):
    """(field, C type, array length) of `typedef struct name {...} name;`."""
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), hdr, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    out = []
    for decl in filter(None, (d.strip() for d in body.split(";"))):
        m = re.match(r"((?:const\s+)?(?:int|double)\s*\**)\s*(.*)", decl, re.S)
        ctype = m.group(1).replace("const", "").replace(" ", "")
        for item in m.group(2).split(","):
            a = re.match(r"\s*(\w+)\s*(?:\[(\d+)\])?\s*$", item)
            out.append((a.group(1), ctype, int(a.group(2)) if a.group(2) else None))
    return out


@pytest.mark.parametrize("name", ["bdm_mesh", "bdm_physics", "bdm_opts", "bdm_step_stats"])
def test_binding_structs_mirror_header(name):
    """The ctypes structures of the binding declare the header's fields in
    the header's order with the same C types, so that the library reads
    every option where the caller wrote it."""
    with open(os.path.join(ROOT, "include", "bidomain.h")) as f:
        hdr = f.read()
    from paper_2101_02959_amd import bidomain
    cmap = {"int": ctypes.c_int, "double": ctypes.c_double, "int*": ctypes.POINTER(ctypes.c_int)}
    want = _header_fields(hdr, name)
    got = getattr(bidomain, name)._fields_
    assert [f for f, _, _ in want] == [f for f, _ in got]
    for (f, ct, n), (_, t) in zip(want, got):
        if n is None:
            assert t is cmap[ct], f
        else:
            assert t._type_ is cmap[ct] and t._length_ == n, f
