"""BDDC with deluxe or rho scaling and a vertex, vertex + edge-average or
vertex + edge + face-average primal space (paper Sec. 4.2 and 4.4), applied
to the full Jacobian system.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings taken where the paper is silent or garbled:
  * Edge and face averages are imposed as constraints (Lagrange
    multipliers) in the local Neumann problems; vertex values are eliminated
    as primal dofs.
  * Both scalings act on an object's values through matrices D^(m), one per
    sharing subdomain, with sum_m D^(m) = I:  u_* = sum_m D^(m) u_*^(m), and
    by the transpose on the residual, so M^{-1}_Gamma = E_D S~^{-1} E_D^T.
    Deluxe (Sec. 4.2): D^(m) = (sum_k S_*^(k))^{-1} S_*^(m).
    rho (Sec. 4.2, eq. for the pseudoinverses): D^(m) is diagonal with
    sigma_M^(m) / sum_k sigma_M^(k) on the dofs of each field, sigma_M the
    largest principal conductivity of subdomain m, taken from sigma^i for
    the v dofs and from sigma^e for the u_e dofs.  The tissue here has the
    same conductivities in every subdomain, so every weight is 1/|N_x|.
  * The coarse matrix is singular (kernel: u_e constant, v = 0).  Its
    right-hand side is projected onto the complement of that kernel and the
    u_e value of the first vertex is pinned to zero.
  * On the full system, M^{-1} = L^{-T} diag(K_II^{-1}, M_Gamma) L^{-1} with
    L the block elimination of the interior: an interior Dirichlet correction,
    the interface preconditioner, and the discrete harmonic extension.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .dd import Decomposition, LocalOps


SCALINGS = ("deluxe", "rho")


class BDDC:
    def __init__(self, prob, dec: Decomposition, v_lin, w_lin, scaling="deluxe"):
        if scaling not in SCALINGS:
            raise ValueError(f"scaling must be one of {SCALINGS}")
        self.prob = prob
        self.dec = dec
        self.N = prob.N
        self.scaling = scaling
        self.loc = [LocalOps(prob, dec, s, v_lin, w_lin) for s in range(dec.nsub)]
        self._deluxe_setup()
        self._coarse_setup()

    # ---------------------------------------------------------------- deluxe
    def _block(self, s, kind, oid):
        """Principal minor S_*^(s) of S_Gamma^(s) on the dofs of object (kind, oid)."""
        info = self.dec.sub[s]
        obj = self.dec.faces[oid] if kind == "F" else self.dec.edges[oid]
        off = info.obj_offset[(kind, oid)]
        n = 2 * len(obj.nodes)
        return self.loc[s].SG[off:off + n, off:off + n]

    def _deluxe_setup(self):
        """Per face: S_F^j + S_F^k; per edge: sum_m S_E^{j_m} (Sec. 4.2)."""
        self.Ssum = {}
        for kind, objs in (("F", self.dec.faces), ("E", self.dec.edges)):
            for oid, obj in enumerate(objs):
                self.Ssum[(kind, oid)] = sum(self._block(s, kind, oid) for s in obj.subs)

    def _objects(self):
        for oid, o in enumerate(self.dec.faces):
            yield "F", oid, o
        for oid, o in enumerate(self.dec.edges):
            yield "E", oid, o

    @staticmethod
    def obj_dofs(obj, N):
        return np.array([f * N + n for n in obj.nodes for f in (0, 1)], dtype=np.int64)

    def sigma_max(self, s):
        """(sigma_M^i, sigma_M^e) of subdomain s: the largest principal
        conductivity of each medium (the same in every subdomain here)."""
        ph = self.prob.ph
        return max(ph.sigma_i), max(ph.sigma_e)

    def D(self, kind, oid, m):
        """Scaling matrix D^(m) of subdomain m on object (kind, oid), dofs
        in the object's (node, field) order (Sec. 4.2)."""
        obj = self.dec.faces[oid] if kind == "F" else self.dec.edges[oid]
        if self.scaling == "deluxe":
            return np.linalg.solve(self.Ssum[(kind, oid)], self._block(m, kind, oid))
        num = self.sigma_max(m)
        den = [sum(self.sigma_max(k)[f] for k in obj.subs) for f in (0, 1)]
        w = [num[0] / den[0], num[1] / den[1]]
        return np.diag(np.tile(w, len(obj.nodes)))

    def deluxe_residual(self, gG):
        """E_D^T: split an assembled interface vector (global 2N layout, only
        face and edge dofs read) into local r-vectors g^(j)_* = D^(j)T g_*
        (deluxe: S_*^(j) (sum_m S_*^(m))^{-1} g_*).  Vertex dofs are not
        split; they go to the coarse right-hand side directly."""
        out = [np.zeros(self.dec.sub[s].nr) for s in range(self.dec.nsub)]
        for kind, oid, obj in self._objects():
            gd = gG[self.obj_dofs(obj, self.N)]
            for s in obj.subs:
                off = self.dec.sub[s].obj_offset[(kind, oid)]
                out[s][off:off + len(gd)] = self.D(kind, oid, s).T @ gd
        return out

    def deluxe_values(self, wloc, z):
        """E_D on the values: u_* = sum_m D^(m) u_*^(m) (deluxe:
        (sum_m S_*^(m))^{-1} sum_m S_*^(m) u_*^(m)), written into the global
        vector z at the object's dofs (Sec. 4.2)."""
        for kind, oid, obj in self._objects():
            acc = 0.0
            for s in obj.subs:
                off = self.dec.sub[s].obj_offset[(kind, oid)]
                n = 2 * len(obj.nodes)
                acc = acc + self.D(kind, oid, s) @ wloc[s][off:off + n]
            z[self.obj_dofs(obj, self.N)] = acc

    # ---------------------------------------------------------------- coarse
    def _constraints(self, s):
        """C^(s): two rows per constrained local object (average of v,
        average of u_e over its nodes) on the local r-dofs: edges, then
        faces, as the primal space includes them."""
        info = self.dec.sub[s]
        C = np.zeros((2 * len(info.cons), info.nr))
        for t, (kind, o) in enumerate(info.cons):
            off = info.obj_offset[(kind, o)]
            ne = len((self.dec.edges if kind == "E" else self.dec.faces)[o].nodes)
            for f in (0, 1):
                C[2 * t + f, off + f: off + 2 * ne: 2] = 1.0 / ne
        return C

    def _coarse_setup(self):
        """Coarse basis Phi^(j) (energy-minimising extension of the primal
        values under the average constraints) and
        S_PiPi = sum_j R_Pi^T Phi^T S_Gamma Phi R_Pi (Sec. 4.4)."""
        dec = self.dec
        self.C, self.Phi, self.KKT = [], [], []
        Spp = np.zeros((dec.nprimal, dec.nprimal))
        for s in range(dec.nsub):
            info, SG = dec.sub[s], self.loc[s].SG
            nr, nV = info.nr, info.nV
            C = self._constraints(s)
            nc = C.shape[0]
            Srr, SrV = SG[:nr, :nr], SG[:nr, nr:]
            KKT = np.block([[Srr, C.T], [C, np.zeros((nc, nc))]])
            npi = nV + nc
            rhs = np.zeros((nr + nc, npi))
            rhs[:nr, :nV] = -SrV
            rhs[nr:, nV:] = np.eye(nc)
            sol = np.linalg.solve(KKT, rhs)
            Phi = np.zeros((nr + nV, npi))
            Phi[:nr] = sol[:nr]
            Phi[nr:, :nV] = np.eye(nV)
            Sj = Phi.T @ SG @ Phi
            Spp[np.ix_(info.primal, info.primal)] += Sj
            self.C.append(C)
            self.Phi.append(Phi)
            self.KKT.append(KKT)
        self.Spp = 0.5 * (Spp + Spp.T)
        # kernel of S_PiPi: u_e-primal values 1, v-primal values 0
        self.ker = np.zeros(dec.nprimal)
        self.ker[1::2] = 1.0
        self.pin = 1                    # u_e dof of the first vertex
        keep = np.ones(dec.nprimal, bool)
        keep[self.pin] = False
        self.keep = keep
        self.Spp_chol = sla.cho_factor(self.Spp[np.ix_(keep, keep)])

    def coarse_solve(self, b):
        b = b - self.ker * (self.ker @ b) / (self.ker @ self.ker)
        x = np.zeros_like(b)
        x[self.keep] = sla.cho_solve(self.Spp_chol, b[self.keep])
        return x

    def local_neumann(self, s, g_r):
        """Local constrained problem [[S_rr, C^T], [C, 0]] [zeta; mu] = [g_r; 0]
        with the vertex values fixed at zero (Sec. 4.4, first term of S~^{-1})."""
        nc = self.C[s].shape[0]
        sol = np.linalg.solve(self.KKT[s], np.concatenate([g_r, np.zeros(nc)]))
        return sol[:self.dec.sub[s].nr]

    # ---------------------------------------------------------------- S~^{-1}
    def stilde_inv(self, gloc, gV):
        """S~^{-1} applied to local interface residuals: gloc[s] on the local
        r-dofs, gV the (already assembled) vertex residual in global primal
        numbering.  Returns the local values w^(s) on [r | V] and u_c."""
        dec = self.dec
        b = np.zeros(dec.nprimal)
        b += gV
        for s in range(dec.nsub):
            info = dec.sub[s]
            nr = info.nr
            b[info.primal] += self.Phi[s][:nr].T @ gloc[s]
        uc = self.coarse_solve(b)
        wloc = []
        for s in range(dec.nsub):
            info = dec.sub[s]
            zeta = self.local_neumann(s, gloc[s])
            w = self.Phi[s] @ uc[info.primal]
            w[:info.nr] += zeta
            wloc.append(w)
        return wloc, uc

    def vertex_global(self, gG):
        """Assembled vertex residual in global primal numbering."""
        gV = np.zeros(self.dec.nprimal)
        for v, o in enumerate(self.dec.verts):
            for f in (0, 1):
                gV[2 * v + f] = gG[f * self.N + o.nodes[0]]
        return gV

    # ---------------------------------------------------------------- apply
    def apply_interface(self, gG):
        """M_Gamma g = E_D S~^{-1} E_D^T g for an assembled interface vector g
        (global 2N layout; non-interface entries ignored).  Returns a global
        vector that is nonzero on interface dofs only."""
        gloc = self.deluxe_residual(gG)
        wloc, uc = self.stilde_inv(gloc, self.vertex_global(gG))
        z = np.zeros(2 * self.N)
        self.deluxe_values(wloc, z)
        for v, o in enumerate(self.dec.verts):
            for f in (0, 1):
                z[f * self.N + o.nodes[0]] = uc[2 * v + f]
        return z

    def apply(self, r):
        """Full-system BDDC: z = M^{-1} r (Sec. 4.4 with static condensation,
        Sec. 4.1):
          1. t_j = K_II^{-1} r_I                         (Dirichlet)
          2. g = r_Gamma - sum_j R_j^T K_GI t_j           (condensed residual)
          3. y = E_D S~^{-1} E_D^T g                      (interface BDDC)
          4. z_Gamma = y,  z_I = K_II^{-1} (r_I - K_IG y)  (harmonic extension)"""
        dec = self.dec
        g = r.copy()
        tI = []
        for s in range(dec.nsub):
            info, lo = dec.sub[s], self.loc[s]
            t = lo.solve_II(r[info.I])
            tI.append(t)
            g[info.G] -= lo.KIG.T @ t
        y = self.apply_interface(g)
        z = y.copy()
        for s in range(dec.nsub):
            info, lo = dec.sub[s], self.loc[s]
            z[info.I] = lo.solve_II(r[info.I] - lo.KIG @ y[info.G])
        return z

    # ---------------------------------------------------------------- Schur
    def schur_assembled(self):
        """S^_Gamma = sum_j R_j^T S_Gamma^(j) R_j over the global interface dofs
        (Sec. 4.1); returns (matrix, global dof list)."""
        gam = self.dec.gamma_nodes()
        gd = np.array([f * self.N + n for n in gam for f in (0, 1)], dtype=np.int64)
        pos = {d: i for i, d in enumerate(gd)}
        S = np.zeros((len(gd), len(gd)))
        for s in range(self.dec.nsub):
            idx = np.array([pos[d] for d in self.dec.sub[s].G])
            S[np.ix_(idx, idx)] += self.loc[s].SG
        return S, gd
