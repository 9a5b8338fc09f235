"""ctypes binding of libbidomain (include/bidomain.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Device arrays are torch tensors on the context's GPU (PyTorch is
used for device memory and the stream); the functions named bdm_* mirror the
C entry points one to one.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbidomain.so")

BDM_SOLVER_BDDC, BDM_SOLVER_FETIDP = 0, 1
BDM_PREC_FP64, BDM_PREC_MIXED = 0, 1
BDM_GUESS_PREV, BDM_GUESS_EXTRAP, BDM_GUESS_CNN = 0, 1, 2
BDM_SCHED_QUEUE, BDM_SCHED_GRID = 0, 1
BDM_FETI_F, BDM_FETI_PRECOND, BDM_FETI_RHS, BDM_FETI_RECOVER = 0, 1, 2, 3
BDM_SCALING_DELUXE, BDM_SCALING_RHO = 0, 1
BDM_PRIMAL_VE, BDM_PRIMAL_V, BDM_PRIMAL_VEF = 0, 1, 2
BDM_GEOM_BOX, BDM_GEOM_ELLIPSOID = 0, 1
(BDM_KERNEL_JACOBIAN, BDM_KERNEL_TRSV_DIRICHLET, BDM_KERNEL_POTRF_INTERIOR, BDM_KERNEL_SYRK_UPDATE,
 BDM_KERNEL_TRSV_DIRICHLET_T) = 0, 1, 2, 3, 4

ERRORS = {
    -1: "BDM_E_ARG", -2: "BDM_E_OOM", -3: "BDM_E_HIP", -4: "BDM_E_NOT_SPD",
    -5: "BDM_E_KRYLOV_DIVERGED", -6: "BDM_E_KRYLOV_MAXIT", -7: "BDM_E_NEWTON_MAXIT",
    -8: "BDM_E_COERCIVITY", -9: "BDM_E_STATE", -10: "BDM_E_LINESEARCH",
}

EXPORTS = ("bdm_create", "bdm_destroy", "bdm_set_state", "bdm_get_state", "bdm_set_stimulus",
           "bdm_ionic_update", "bdm_residual", "bdm_linearize", "bdm_jacobian_apply",
           "bdm_bddc_apply", "bdm_fetidp_size", "bdm_fetidp_apply", "bdm_step", "bdm_sizes",
           "bdm_profile_kernel", "bdm_tune_report", "bdm_predictor_size", "bdm_predictor_set", "bdm_predictor_get",
           "bdm_predictor_guess", "bdm_predictor_loss_grad", "bdm_predictor_train", "bdm_residual_noalloc",
           "bdm_last_error")


class BidomainError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class bdm_mesh(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double),
                ("px", C.c_int), ("py", C.c_int), ("pz", C.c_int),
                ("cuts_x", C.POINTER(C.c_int)), ("cuts_y", C.POINTER(C.c_int)),
                ("cuts_z", C.POINTER(C.c_int)), ("hy", C.c_double), ("hz", C.c_double),
                ("geometry", C.c_int), ("ellipsoid", C.c_double * 10)]


class bdm_physics(C.Structure):
    _fields_ = [("sigma_i", C.c_double * 3), ("sigma_e", C.c_double * 3),
                ("theta0", C.c_double), ("theta1", C.c_double), ("chi", C.c_double),
                ("Cm", C.c_double), ("G", C.c_double), ("eta1", C.c_double),
                ("eta2", C.c_double), ("vth", C.c_double), ("vp", C.c_double)]


class bdm_opts(C.Structure):
    _fields_ = [("dt", C.c_double), ("newton_rtol", C.c_double), ("newton_atol", C.c_double),
                ("newton_maxit", C.c_int), ("krylov_rtol", C.c_double), ("krylov_dtol", C.c_double),
                ("krylov_maxit", C.c_int), ("solver", C.c_int), ("precision", C.c_int),
                ("guess", C.c_int), ("krylov_graph", C.c_int), ("schedule", C.c_int),
                ("krylov_reduced", C.c_int), ("scaling", C.c_int), ("primal", C.c_int)]


class bdm_step_stats(C.Structure):
    _fields_ = [("newton_its", C.c_int), ("krylov_its", C.c_int * 32), ("res_hist", C.c_double * 33),
                ("cond", C.c_double * 32), ("t_setup_ms", C.c_double), ("t_krylov_ms", C.c_double),
                ("t_step_ms", C.c_double), ("bad_subdomain", C.c_int), ("guess_used", C.c_int),
                ("guess_res_extrap", C.c_double), ("guess_res_cnn", C.c_double), ("res_ref", C.c_double),
                ("krylov_true_res", C.c_double * 32), ("step_length", C.c_double * 32)]


_lib = None


def lib():
    """Load libbidomain.so; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2101_02959_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, cd, ci = C.c_void_p, C.c_double, C.c_int
    sig = {
        "bdm_create": ([C.POINTER(bdm_mesh), C.POINTER(bdm_physics), C.POINTER(bdm_opts), vp,
                        C.POINTER(vp)], ci),
        "bdm_destroy": ([vp], ci),
        "bdm_tune_report": ([vp, C.c_char_p, C.c_long, C.POINTER(C.c_long)], ci),
        "bdm_set_state": ([vp, vp, vp, vp, cd, ci], ci),
        "bdm_get_state": ([vp, vp, vp, vp, C.POINTER(cd), ci], ci),
        "bdm_set_stimulus": ([vp, vp, ci, ci, ci], ci),
        "bdm_ionic_update": ([vp], ci),
        "bdm_residual": ([vp, vp, vp, vp, vp], ci),
        "bdm_linearize": ([vp, vp, vp], ci),
        "bdm_jacobian_apply": ([vp, vp, vp], ci),
        "bdm_bddc_apply": ([vp, vp, vp], ci),
        "bdm_fetidp_size": ([vp, C.POINTER(C.c_long)], ci),
        "bdm_fetidp_apply": ([vp, ci, vp, vp], ci),
        "bdm_step": ([vp, ci, C.POINTER(bdm_step_stats)], ci),
        "bdm_sizes": ([vp, C.POINTER(C.c_long), C.POINTER(C.c_long), C.POINTER(C.c_long)], ci),
        "bdm_profile_kernel": ([vp, ci, ci, C.POINTER(cd), C.POINTER(cd)], ci),
        "bdm_predictor_size": ([], C.c_long),
        "bdm_predictor_set": ([vp, C.POINTER(C.c_float), C.POINTER(cd)], ci),
        "bdm_predictor_get": ([vp, C.POINTER(C.c_float), C.POINTER(cd)], ci),
        "bdm_predictor_guess": ([vp, vp, vp, vp, vp, vp], ci),
        "bdm_predictor_loss_grad": ([vp, vp, C.POINTER(C.c_float), C.POINTER(cd)], ci),
        "bdm_predictor_train": ([vp, vp, ci, C.POINTER(ci), ci, cd, C.POINTER(cd)], ci),
        "bdm_residual_noalloc": ([C.POINTER(bdm_mesh), C.POINTER(bdm_physics), cd, vp, vp, vp, vp, vp, ci, vp, vp,
                                  vp], ci),
        "bdm_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise BidomainError(rc, lib().bdm_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def make_structs(mesh, physics, solver, precision=BDM_PREC_FP64, method=BDM_SOLVER_BDDC,
                 guess=BDM_GUESS_PREV, krylov_graph=False, schedule=0, krylov_reduced=True,
                 scaling=0, primal=0):
    """Build the C structs from workload descriptions (duck-typed)."""
    cx = (C.c_int * len(mesh.cuts_x))(*mesh.cuts_x)
    cy = (C.c_int * len(mesh.cuts_y))(*mesh.cuts_y)
    cz = (C.c_int * len(mesh.cuts_z))(*mesh.cuts_z)
    ell = tuple(getattr(mesh, "ellipsoid", ()))
    if ell and len(ell) != 10:
        raise ValueError("ellipsoid takes 10 parameters")
    m = bdm_mesh(mesh.nx, mesh.ny, mesh.nz, mesh.h, len(mesh.cuts_x) - 1, len(mesh.cuts_y) - 1,
                 len(mesh.cuts_z) - 1, cx, cy, cz, getattr(mesh, "hy", 0.0), getattr(mesh, "hz", 0.0),
                 BDM_GEOM_ELLIPSOID if ell else BDM_GEOM_BOX, (C.c_double * 10)(*(ell or (0.0,) * 10)))
    ph = bdm_physics((C.c_double * 3)(*physics.sigma_i), (C.c_double * 3)(*physics.sigma_e),
                     physics.theta0, physics.theta1, physics.chi, physics.Cm, physics.G,
                     physics.eta1, physics.eta2, physics.vth, physics.vp)
    op = bdm_opts(solver.dt, solver.newton_rtol, solver.newton_atol, solver.newton_maxit,
                  solver.krylov_rtol, solver.krylov_dtol, solver.krylov_maxit, method, precision,
                  guess, int(bool(krylov_graph)), schedule, int(bool(krylov_reduced)), scaling, primal)
    return m, ph, op, (cx, cy, cz)


class Solver:
    """One libbidomain context on the current torch CUDA device and stream."""

    def __init__(self, mesh, physics, solver, precision=BDM_PREC_FP64, method=BDM_SOLVER_BDDC,
                 guess=BDM_GUESS_PREV, stream=None, krylov_graph=False, schedule=0, krylov_reduced=True,
                 scaling=0, primal=0):
        import torch
        self.torch = torch
        L = lib()
        self.m, self.ph, self.op, self._keep = make_structs(mesh, physics, solver, precision,
                                                            method, guess, krylov_graph, schedule,
                                                            krylov_reduced, scaling, primal)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = C.c_void_p()
        _check(L.bdm_create(C.byref(self.m), C.byref(self.ph), C.byref(self.op), C.c_void_p(stream),
                            C.byref(h)))
        self.h = h
        n, s, p = C.c_long(), C.c_long(), C.c_long()
        _check(L.bdm_sizes(h, C.byref(n), C.byref(s), C.byref(p)))
        self.N, self.nsub, self.nprimal = n.value, s.value, p.value
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "h", None):
            lib().bdm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, x):
        t = self.torch.as_tensor(np.asarray(x) if not hasattr(x, "device") else x,
                                 dtype=self.torch.float64)
        return t.to(self.device).contiguous()

    def vec(self, n=None):
        return self.torch.zeros(2 * self.N if n is None else n, dtype=self.torch.float64,
                                device=self.device)

    # --- entry points (same names as the C ABI)
    def bdm_set_state(self, v, ue, w, t=0.0):
        v, ue, w = self._dev(v), self._dev(ue), self._dev(w)
        _check(lib().bdm_set_state(self.h, _ptr(v), _ptr(ue), _ptr(w), t, 1))

    def bdm_get_state(self):
        v, ue, w = self.vec(self.N), self.vec(self.N), self.vec(self.N)
        t = C.c_double()
        _check(lib().bdm_get_state(self.h, _ptr(v), _ptr(ue), _ptr(w), C.byref(t), 1))
        return v, ue, w, t.value

    def bdm_set_stimulus(self, Is, step_on, step_off):
        Is = self._dev(Is)
        _check(lib().bdm_set_stimulus(self.h, _ptr(Is), step_on, step_off, 1))

    def bdm_ionic_update(self):
        _check(lib().bdm_ionic_update(self.h))

    def bdm_residual(self, v, ue):
        v, ue = self._dev(v), self._dev(ue)
        R = self.vec()
        _check(lib().bdm_residual(self.h, _ptr(v), _ptr(ue), _ptr(R[:self.N]), _ptr(R[self.N:])))
        return R

    def bdm_linearize(self, v, w):
        v, w = self._dev(v), self._dev(w)
        _check(lib().bdm_linearize(self.h, _ptr(v), _ptr(w)))

    def bdm_jacobian_apply(self, x):
        x = self._dev(x)
        y = self.vec()
        _check(lib().bdm_jacobian_apply(self.h, _ptr(x), _ptr(y)))
        return y

    def bdm_bddc_apply(self, r):
        r = self._dev(r)
        z = self.vec()
        _check(lib().bdm_bddc_apply(self.h, _ptr(r), _ptr(z)))
        return z

    def bdm_fetidp_size(self):
        n = C.c_long()
        _check(lib().bdm_fetidp_size(self.h, C.byref(n)))
        return n.value

    def bdm_fetidp_apply(self, op, x):
        x = self._dev(x)
        nl = self.bdm_fetidp_size()
        out = self.vec(2 * self.N if op == BDM_FETI_RECOVER else nl)
        _check(lib().bdm_fetidp_apply(self.h, op, _ptr(x), _ptr(out)))
        return out

    def bdm_profile_kernel(self, kernel, reps=10):
        ms, work = C.c_double(), C.c_double()
        _check(lib().bdm_profile_kernel(self.h, kernel, reps, C.byref(ms), C.byref(work)))
        return ms.value, work.value

    # --- learned initial guess
    @staticmethod
    def bdm_predictor_size():
        return int(lib().bdm_predictor_size())

    def bdm_predictor_set(self, params, scales):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.bdm_predictor_size():
            raise ValueError(f"expected {self.bdm_predictor_size()} parameters, got {p.size}")
        sc = np.ascontiguousarray(scales, dtype=np.float64)
        if sc.size != 6:
            raise ValueError("expected 6 scales (s_v, s_e, s_dv, s_de, s_yv, s_ye)")
        _check(lib().bdm_predictor_set(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                       sc.ctypes.data_as(C.POINTER(C.c_double))))

    def bdm_predictor_get(self):
        p = np.zeros(self.bdm_predictor_size(), dtype=np.float32)
        sc = np.zeros(6)
        _check(lib().bdm_predictor_get(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                       sc.ctypes.data_as(C.POINTER(C.c_double))))
        return p, sc

    def bdm_predictor_guess(self, vn, uen, vprev, ueprev):
        a = [self._dev(x) for x in (vn, uen, vprev, ueprev)]
        out = self.vec()
        _check(lib().bdm_predictor_guess(self.h, *[_ptr(x) for x in a], _ptr(out)))
        return out

    def bdm_predictor_loss_grad(self, sample):
        s6 = self._dev(sample)
        if s6.numel() != 6 * self.N:
            raise ValueError("a sample holds 6 N values")
        g = np.zeros(self.bdm_predictor_size(), dtype=np.float32)
        loss = C.c_double()
        _check(lib().bdm_predictor_loss_grad(self.h, _ptr(s6), g.ctypes.data_as(C.POINTER(C.c_float)),
                                             C.byref(loss)))
        return loss.value, g

    def bdm_predictor_train(self, samples, order, lr):
        S = self._dev(samples)
        if S.numel() % (6 * self.N):
            raise ValueError("samples must hold whole 6 N blocks")
        ns = S.numel() // (6 * self.N)
        o = np.ascontiguousarray(order, dtype=np.int32)
        losses = np.zeros(o.size)
        _check(lib().bdm_predictor_train(self.h, _ptr(S), int(ns), o.ctypes.data_as(C.POINTER(C.c_int)),
                                         int(o.size), float(lr), losses.ctypes.data_as(C.POINTER(C.c_double))))
        return losses

    def bdm_tune_report(self):
        """Autotuner entries this context used, as a dict (JSON from the library)."""
        import json
        n = C.c_long()
        buf = C.create_string_buffer(1 << 14)
        rc = lib().bdm_tune_report(self.h, buf, len(buf), C.byref(n))
        if rc != 0 and n.value >= len(buf):
            buf = C.create_string_buffer(n.value + 1)
            rc = lib().bdm_tune_report(self.h, buf, len(buf), C.byref(n))
        _check(rc)
        return json.loads(buf.value.decode())

    def bdm_step(self, nsteps=1):
        st = bdm_step_stats()
        rc = lib().bdm_step(self.h, nsteps, C.byref(st))
        _check(rc)
        return st


def bdm_residual_noalloc(mesh, physics, dt, v, ue, vn, w, Is=None, stream=None):
    """Residual of bdm_residual without a context or any device allocation
    (C entry point of the same name).  v, ue, vn, w, Is: CUDA float64 tensors
    of N entries (Is optional); returns (Rv, Re) allocated here by torch,
    before the call."""
    import torch
    m, ph, _, keep = make_structs(mesh, physics, _SolverDt(dt))
    dev = v.device
    Rv = torch.empty_like(v)
    Re = torch.empty_like(v)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    _check(lib().bdm_residual_noalloc(C.byref(m), C.byref(ph), float(dt), _ptr(v), _ptr(ue), _ptr(vn), _ptr(w),
                                      _ptr(Is), 1 if Is is not None else 0, _ptr(Rv), _ptr(Re), C.c_void_p(stream)))
    del keep
    return Rv, Re


class _SolverDt:
    """Solver options carrying only dt, for make_structs."""
    def __init__(self, dt):
        self.dt, self.newton_rtol, self.newton_atol, self.newton_maxit = dt, 1e-8, 0.0, 1
        self.krylov_rtol, self.krylov_dtol, self.krylov_maxit = 1e-10, 1e4, 1
