"""FETI-DP with deluxe or rho scaling (paper Sec. 4.3), on the same local
operators, scaling matrices and coarse space as the BDDC oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Multipliers: one per face dof (pair j < k), and one per dof and per pair
(a < b) of the subdomains sharing an edge (fully redundant).  Ordering: faces
in object order, dofs in node order with (v, u_e) per node; then edges in
object order, pairs in lexicographic order, dofs as for faces.
    (B w)_{ab} = w^(a) - w^(b)
    B_D^T lambda gives subdomain a the value D^(b) lambda_ab and subdomain b
    the value -D^(a) lambda_ab, with D^(m) the scaling matrices of Sec. 4.2
    (deluxe: (sum S)^{-1} S^(m); rho: the diagonal weights),
so that B_D^T B equals the complementary projection P_D = I - E_D.
"""
from __future__ import annotations

import itertools

import numpy as np

from .bddc import BDDC


class FETIDP:
    def __init__(self, bddc: BDDC):
        self.b = bddc
        self.dec = bddc.dec
        self.blocks = []           # (kind, oid, a, b, offset, n)
        off = 0
        for kind, oid, obj in bddc._objects():
            n = 2 * len(obj.nodes)
            for a, b in itertools.combinations(obj.subs, 2):
                self.blocks.append((kind, oid, a, b, off, n))
                off += n
        self.nlam = off

    def _loc_zero(self):
        return [np.zeros(self.dec.sub[s].nG) for s in range(self.dec.nsub)]

    def _seg(self, s, kind, oid, n):
        o = self.dec.sub[s].obj_offset[(kind, oid)]
        return slice(o, o + n)

    def B(self, wloc):
        lam = np.zeros(self.nlam)
        for kind, oid, a, b, off, n in self.blocks:
            lam[off:off + n] = wloc[a][self._seg(a, kind, oid, n)] - wloc[b][self._seg(b, kind, oid, n)]
        return lam

    def BT(self, lam):
        out = self._loc_zero()
        for kind, oid, a, b, off, n in self.blocks:
            out[a][self._seg(a, kind, oid, n)] += lam[off:off + n]
            out[b][self._seg(b, kind, oid, n)] -= lam[off:off + n]
        return out

    def _D(self, kind, oid, m):
        return self.b.D(kind, oid, m)

    def BDT(self, lam):
        out = self._loc_zero()
        for kind, oid, a, b, off, n in self.blocks:
            out[a][self._seg(a, kind, oid, n)] += self._D(kind, oid, b) @ lam[off:off + n]
            out[b][self._seg(b, kind, oid, n)] -= self._D(kind, oid, a) @ lam[off:off + n]
        return out

    def BD(self, wloc):
        lam = np.zeros(self.nlam)
        for kind, oid, a, b, off, n in self.blocks:
            lam[off:off + n] = (self._D(kind, oid, b).T @ wloc[a][self._seg(a, kind, oid, n)]
                                - self._D(kind, oid, a).T @ wloc[b][self._seg(b, kind, oid, n)])
        return lam

    def stilde_inv_loc(self, gloc, gV):
        """S~^{-1} on local interface vectors (r part used; vertex part given
        assembled in gV)."""
        gl = [gloc[s][:self.dec.sub[s].nr] for s in range(self.dec.nsub)]
        wloc, _ = self.b.stilde_inv(gl, gV)
        return wloc

    def F(self, lam):
        """F lambda = B S~^{-1} B^T lambda (Sec. 4.3)."""
        return self.B(self.stilde_inv_loc(self.BT(lam), np.zeros(self.dec.nprimal)))

    def precond(self, lam):
        """M^{-1} lambda = B_D S_Gamma B_D^T lambda (Sec. 4.3)."""
        x = self.BDT(lam)
        y = [self.b.loc[s].SG @ x[s] for s in range(self.dec.nsub)]
        return self.BD(y)

    def split_rhs(self, gG):
        """f~: the condensed interface residual split 1/|N_x| on the dual
        dofs; the vertex (primal) part stays assembled."""
        N = self.b.N
        out = self._loc_zero()
        for s in range(self.dec.nsub):
            info = self.dec.sub[s]
            for kind, oid, obj in self.b._objects():
                if s not in obj.subs:
                    continue
                sl = self._seg(s, kind, oid, 2 * len(obj.nodes))
                out[s][sl] = gG[self.b.obj_dofs(obj, N)] / len(obj.subs)
        return out, self.b.vertex_global(gG)

    def rhs(self, gG):
        """d = B S~^{-1} f~ (Sec. 4.3)."""
        fl, gV = self.split_rhs(gG)
        return self.B(self.stilde_inv_loc(fl, gV))

    def recover(self, gG, lam):
        """w = S~^{-1} (f~ - B^T lambda), continuous on the interface
        (Sec. 4.3); returned as a global interface vector."""
        fl, gV = self.split_rhs(gG)
        bt = self.BT(lam)
        wloc = self.stilde_inv_loc([fl[s] - bt[s] for s in range(self.dec.nsub)], gV)
        N = self.b.N
        z = np.zeros(2 * N)
        for kind, oid, obj in self.b._objects():
            s = obj.subs[0]
            z[self.b.obj_dofs(obj, N)] = wloc[s][self._seg(s, kind, oid, 2 * len(obj.nodes))]
        for v, o in enumerate(self.dec.verts):
            s = o.subs[0]
            info = self.dec.sub[s]
            k = list(info.verts).index(v)
            for f in (0, 1):
                z[f * N + o.nodes[0]] = wloc[s][info.nr + 2 * k + f]
        return z

    def condense(self, r):
        """Interior elimination: t_j = K_II^{-1} r_I, g = r_G - sum K_GI t_j."""
        g = r.copy()
        for s in range(self.dec.nsub):
            info, lo = self.dec.sub[s], self.b.loc[s]
            g[info.G] -= lo.KIG.T @ lo.solve_II(r[info.I])
        return g

    def expand(self, r, zG):
        """z_I = K_II^{-1} (r_I - K_IG z_G) (Sec. 4.1)."""
        z = zG.copy()
        for s in range(self.dec.nsub):
            info, lo = self.dec.sub[s], self.b.loc[s]
            z[info.I] = lo.solve_II(r[info.I] - lo.KIG @ zG[info.G])
        return z
