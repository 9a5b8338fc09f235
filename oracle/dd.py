"""Non-overlapping decomposition, N_x equivalence classes and local
operators (paper Sec. 4.1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Subdomains are boxes of elements from a tensor-product set of cuts.  A node
x belongs to the closure of every subdomain in N_x; nodes with |N_x| = 1
(including those on the Neumann boundary) are interior to their subdomain.
Interface nodes are classified by N_x into faces (2 subdomains), edges (4)
and vertices (8).  Objects are ordered by their smallest node id.

Local dofs of subdomain j are ordered [I | r | V]: interior nodes, then the
nodes of j's faces and edges (object by object, nodes ascending), then j's
vertex nodes; every node carries (v, u_e).  Global dof of (node, f) is
f * N + node.

Primal spaces (Sec. 4.4 and the optimality test of Sec. 6): "V" (vertex
values only), "VE" (plus the average of each field over every edge) and
"VEF" (plus the averages over every face).  Vertex values are primal dofs;
edge and face averages are constraints on the r-dofs.  Global primal
numbering: (v, u_e) per vertex, then the two averages per edge, then per face
(only for the objects the primal space includes).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, ionic


def _axis_parts(cuts, i):
    """Parts a with cuts[a] <= i <= cuts[a+1]."""
    return [a for a in range(len(cuts) - 1) if cuts[a] <= i <= cuts[a + 1]]


class Obj:
    def __init__(self, kind, subs, nodes):
        self.kind = kind            # 'F', 'E' or 'V'
        self.subs = tuple(subs)     # sorted subdomain ids (N_x)
        self.nodes = np.array(sorted(nodes), dtype=np.int64)


PRIMAL_SPACES = ("V", "VE", "VEF")


class Decomposition:
    def __init__(self, mesh, primal="VE"):
        if primal not in PRIMAL_SPACES:
            raise ValueError(f"primal space must be one of {PRIMAL_SPACES}")
        self.mesh = mesh
        self.primal_space = primal
        self.cons_edges = "E" in primal
        self.cons_faces = "F" in primal
        ps = (len(mesh.cuts_x) - 1, len(mesh.cuts_y) - 1, len(mesh.cuts_z) - 1)
        if min(ps) < 2:
            raise ValueError("the primal spaces need >= 2 subdomains per axis (interior cross points)")
        self.ps = ps
        self.nsub = ps[0] * ps[1] * ps[2]
        N = mesh.nnodes
        self.N = N
        nx1, ny1 = mesh.nx + 1, mesh.ny + 1
        px = [_axis_parts(mesh.cuts_x, i) for i in range(mesh.nx + 1)]
        py = [_axis_parts(mesh.cuts_y, j) for j in range(mesh.ny + 1)]
        pz = [_axis_parts(mesh.cuts_z, k) for k in range(mesh.nz + 1)]
        self.Nx = [None] * N
        classes = {}
        for k in range(mesh.nz + 1):
            for j in range(mesh.ny + 1):
                for i in range(mesh.nx + 1):
                    n = i + nx1 * (j + ny1 * k)
                    key = tuple(sorted(a + ps[0] * (b + ps[1] * c)
                                       for a, b, c in itertools.product(px[i], py[j], pz[k])))
                    self.Nx[n] = key
                    if len(key) > 1:
                        classes.setdefault(key, []).append(n)
        kinds = {2: "F", 4: "E", 8: "V"}
        objs = [Obj(kinds[len(key)], key, nodes) for key, nodes in classes.items()]
        self.faces = sorted([o for o in objs if o.kind == "F"], key=lambda o: o.nodes[0])
        self.edges = sorted([o for o in objs if o.kind == "E"], key=lambda o: o.nodes[0])
        self.verts = sorted([o for o in objs if o.kind == "V"], key=lambda o: o.nodes[0])
        for o in self.verts:
            assert len(o.nodes) == 1
        # global primal numbering: (vertex v, vertex u_e), ..., then (edge avg v,
        # avg u_e) per edge, then per face, for the constrained object kinds
        self.edge_p0 = 2 * len(self.verts)
        self.face_p0 = self.edge_p0 + (2 * len(self.edges) if self.cons_edges else 0)
        self.nprimal = self.face_p0 + (2 * len(self.faces) if self.cons_faces else 0)
        # per-subdomain boxes and local orderings
        self.sub = []
        for s in range(self.nsub):
            a = s % ps[0]
            b = (s // ps[0]) % ps[1]
            c = s // (ps[0] * ps[1])
            ebox = ((mesh.cuts_x[a], mesh.cuts_x[a + 1]), (mesh.cuts_y[b], mesh.cuts_y[b + 1]),
                    (mesh.cuts_z[c], mesh.cuts_z[c + 1]))
            self.sub.append(_SubInfo(self, s, ebox))

    def gamma_nodes(self):
        return np.array(sorted(n for n in range(self.N) if len(self.Nx[n]) > 1), dtype=np.int64)

    def interior_nodes(self):
        return np.array(sorted(n for n in range(self.N) if len(self.Nx[n]) == 1), dtype=np.int64)


class _SubInfo:
    def __init__(self, dec, s, ebox):
        mesh = dec.mesh
        self.id = s
        self.ebox = ebox
        nx1, ny1 = mesh.nx + 1, mesh.ny + 1
        nodes = [i + nx1 * (j + ny1 * k)
                 for k in range(ebox[2][0], ebox[2][1] + 1)
                 for j in range(ebox[1][0], ebox[1][1] + 1)
                 for i in range(ebox[0][0], ebox[0][1] + 1)]
        self.I_nodes = np.array(sorted(n for n in nodes if len(dec.Nx[n]) == 1), dtype=np.int64)
        self.faces = [f for f, o in enumerate(dec.faces) if s in o.subs]
        self.edges = [e for e, o in enumerate(dec.edges) if s in o.subs]
        self.verts = [v for v, o in enumerate(dec.verts) if s in o.subs]
        r_nodes = []
        self.obj_offset = {}          # ('F'|'E', id) -> offset into the r-dofs
        for f in self.faces:
            self.obj_offset[("F", f)] = 2 * len(r_nodes)
            r_nodes.extend(dec.faces[f].nodes)
        for e in self.edges:
            self.obj_offset[("E", e)] = 2 * len(r_nodes)
            r_nodes.extend(dec.edges[e].nodes)
        self.r_nodes = np.array(r_nodes, dtype=np.int64)
        self.V_nodes = np.array([dec.verts[v].nodes[0] for v in self.verts], dtype=np.int64)
        N = dec.N

        def dofs(nodes):
            return np.array([f * N + n for n in nodes for f in (0, 1)], dtype=np.int64)

        self.I = dofs(self.I_nodes)
        self.r = dofs(self.r_nodes)
        self.V = dofs(self.V_nodes)
        self.G = np.concatenate([self.r, self.V])
        self.nI, self.nr, self.nV = len(self.I), len(self.r), len(self.V)
        self.nG = self.nr + self.nV
        # constrained objects, in the order of their constraint rows and
        # primal dofs: edges, then faces
        self.cons = ([("E", e) for e in self.edges] if dec.cons_edges else []) \
            + ([("F", f) for f in self.faces] if dec.cons_faces else [])
        # local primal -> global primal
        p0 = {"E": dec.edge_p0, "F": dec.face_p0}
        self.primal = np.array([2 * v + f for v in self.verts for f in (0, 1)]
                               + [p0[k] + 2 * o + f for k, o in self.cons for f in (0, 1)],
                               dtype=np.int64)


def local_matrix(prob, dec, s, v_lin, w_lin):
    """K^(j): the Jacobian bilinear form a^(j) restricted to the elements of
    Omega_j (Sec. 4.1), with the local lumped mass in the reaction term, in
    the congruent (v, u_e) form; returned over all 2N global dofs."""
    Ai, Ae, m = fem.assemble(prob.mesh, prob.ph, box=dec.sub[s].ebox)
    d = m * (prob.c + prob.tau * ionic.diion_dv(prob.ph, v_lin, w_lin))
    tAi, tAe = prob.tau * Ai, prob.tau * Ae
    return sp.bmat([[sp.diags(d) + tAi, tAi], [tAi, tAi + tAe]]).tocsr()


class LocalOps:
    """Local blocks K_II, K_IGamma, K_GammaGamma and the local Schur
    complement S_Gamma^(j) = K_GG - K_IG^T K_II^{-1} K_IG (Sec. 4.1)."""

    def __init__(self, prob, dec, s, v_lin, w_lin):
        info = dec.sub[s]
        self.info = info
        K = local_matrix(prob, dec, s, v_lin, w_lin)
        self.K_full = K
        self.KII = K[info.I][:, info.I].tocsc()
        self.KIG = K[info.I][:, info.G].toarray()
        self.KGG = K[info.G][:, info.G].toarray()
        self.KII_lu = spla.splu(self.KII)
        self.SG = self.KGG - self.KIG.T @ self.KII_lu.solve(self.KIG)
        self.SG = 0.5 * (self.SG + self.SG.T)

    def solve_II(self, b):
        return self.KII_lu.solve(b)

    def harmonic_extension(self, wG):
        """H_j w: -K_II^{-1} K_IG w on the interior, w on Gamma (Sec. 4.1)."""
        return -self.KII_lu.solve(self.KIG @ wG), wG
