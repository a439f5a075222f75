"""Thin ctypes binding of libfsi.so (C ABI declared in include/fsi.h).

Argument marshalling only: every step of the operator, the V-cycle and the
solver runs in the HIP library.  Torch tensors provide device memory; the
library context is created on torch's current HIP stream so that both sides
are stream-ordered.  There is no CPU fallback: if the library is missing or
no GPU is present, constructing a context raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsi.so")

FSI_OK = 0
FSI_NOT_CONVERGED = 1
FSI_ERR_ARG = -1
FSI_ERR_STATE = -2
FSI_ERR_HIP = -3
FSI_ERR_OOM = -4
FSI_ERR_INVERTED_CELL = -5
FSI_ERR_BREAKDOWN = -6
FSI_ERR_NONFINITE = -7
PREC_FP64 = 0
PREC_MIXED = 1
# cell-kernel launch variants that fsi_set_tuning accepts (0 .. N_LAUNCH_VARIANTS - 1)
N_LAUNCH_VARIANTS = 16
# fsi_set_tuning values of the single atomic launch over all phases (3D levels): one or
# four wavefronts per row, one wavefront over two or four rows along z, four wavefronts
# over two rows along z, one wavefront per half or quarter row
ATOMIC_VARIANTS = (16, 17, 18, 19, 20, 21, 22)
ATOMIC_VARIANTS_2D = (16, 17)   # the same form on 2D levels: one or two wavefronts per workgroup

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_STATE", -3: "ERR_HIP", -4: "ERR_OOM",
                -5: "ERR_INVERTED_CELL", -6: "ERR_BREAKDOWN", -7: "ERR_NONFINITE"}


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_fine", C.c_int * 3), ("extent", C.c_double * 3),
                ("n_coarse", C.c_int * 3), ("dirichlet_faces", C.c_uint32)]


class Sizes(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_vel_nodes", C.c_int64), ("n_vel", C.c_int64), ("n_p", C.c_int64),
                ("n_qp", C.c_int64), ("n_vert", C.c_int64), ("cells", C.c_int * 3), ("vel_nodes", C.c_int * 3),
                ("p_nodes", C.c_int * 3)]


class MGParams(C.Structure):
    _fields_ = [("k_A", C.c_int), ("m", C.c_int), ("n_cycles", C.c_int), ("k_S", C.c_int), ("n_S", C.c_int),
                ("cheb_upper", C.c_double), ("cheb_ratio", C.c_double), ("n_eig", C.c_int),
                ("precision", C.c_int), ("use_graph", C.c_int),
                ("fused", C.c_int), ("tuned", C.c_int), ("vertex_geometry", C.c_int), ("corrector", C.c_int),
                ("atomics", C.c_int)]


class LevelInfo(C.Structure):
    _fields_ = [("lambda_max", C.c_double), ("cheb_lo", C.c_double), ("cheb_hi", C.c_double),
                ("diagA_norm2", C.c_double), ("diagS_norm2", C.c_double), ("coarse_n", C.c_int64)]


class GcsiParams(C.Structure):
    _fields_ = [("k", C.c_int), ("tau", C.c_double), ("rho_f", C.c_double), ("rho_s", C.c_double),
                ("eta_f", C.c_double), ("mu_s", C.c_double), ("eta_V", C.c_double), ("body", C.c_double * 3)]

    @classmethod
    def of(cls, k=2, tau=0.005, rho_f=1e3, rho_s=1e4, eta_f=1.0, mu_s=5e5, eta_V=0.1, body=(0.0, 0.0, 0.0)):
        return cls(k=k, tau=tau, rho_f=rho_f, rho_s=rho_s, eta_f=eta_f, mu_s=mu_s, eta_V=eta_V,
                   body=(C.c_double * 3)(*body))


GCSI_PREDICTOR = 0
GCSI_CORRECTOR = 1


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int), ("restart", C.c_int), ("reorth", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("final_rel_res", C.c_double), ("time_ms", C.c_double), ("n_hist", C.c_int),
                ("res_history", C.POINTER(C.c_double))]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libfsi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2305_08986_amd.build`")
    # torch first: it brings its own HIP runtime, and the library must bind to that same
    # runtime (one per process) so that torch's device pointers and streams are valid in
    # it; loaded the other way round, context creation fails with FSI_ERR_HIP
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    sig = {
        "fsi_create": (i, [C.POINTER(vp), C.POINTER(MeshDesc), vp]),
        "fsi_destroy": (None, [vp]),
        "fsi_last_error": (C.c_char_p, [vp]),
        "fsi_default_mg_params": (None, [C.POINTER(MGParams)]),
        "fsi_get_num_levels": (i, [vp, C.POINTER(i)]),
        "fsi_get_sizes": (i, [vp, i, C.POINTER(Sizes)]),
        "fsi_set_jacobians": (i, [vp, i, vp]),
        "fsi_set_displacement": (i, [vp, vp]),
        "fsi_set_coefficients": (i, [vp, i, vp, vp]),
        "fsi_set_mg_params": (i, [vp, C.POINTER(MGParams)]),
        "fsi_setup": (i, [vp]),
        "fsi_get_level_info": (i, [vp, i, C.POINTER(LevelInfo)]),
        "fsi_apply_A": (i, [vp, i, vp, vp]),
        "fsi_apply_B": (i, [vp, i, vp, vp]),
        "fsi_apply_BT": (i, [vp, i, vp, vp]),
        "fsi_apply_stokes": (i, [vp, i, vp, vp, vp, vp]),
        "fsi_apply_A_f32": (i, [vp, i, vp, vp]),
        "fsi_apply_B_f32": (i, [vp, i, vp, vp]),
        "fsi_apply_BT_f32": (i, [vp, i, vp, vp]),
        "fsi_apply_stokes_f32": (i, [vp, i, vp, vp, vp, vp]),
        "fsi_apply_stokes_f32_noalloc": (i, [vp, i, vp, vp, vp, vp]),
        "fsi_set_convection": (i, [vp, i, vp, vp, C.c_double]),
        "fsi_apply_corrector": (i, [vp, i, vp, vp, vp, vp]),
        "fsi_apply_corrector_f32": (i, [vp, i, vp, vp, vp, vp]),
        "fsi_vcycle": (i, [vp, vp, vp, vp, vp]),
        "fsi_solve": (i, [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
        "fsi_solve_extension": (i, [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
        "fsi_autotune": (i, [vp]),
        "fsi_get_tuning": (i, [vp, i, i, C.POINTER(i), C.POINTER(d)]),
        "fsi_set_tuning": (i, [vp, i, i, i]),
        "fsi_time_operator": (i, [vp, i, i, i, i, C.POINTER(d), C.POINTER(d), C.POINTER(i)]),
        "fsi_set_fixed_cells": (i, [vp, vp]),
        "fsi_lift_dirichlet": (i, [vp, vp, vp, vp]),
        "fsi_fixed_values": (i, [vp, vp, vp]),
        "fsi_gcsi_displacement": (i, [vp, C.POINTER(GcsiParams), vp, vp, vp, vp, vp]),
        "fsi_gcsi_set_coefficients": (i, [vp, C.POINTER(GcsiParams), C.POINTER(vp)]),
        "fsi_gcsi_rhs": (i, [vp, C.POINTER(GcsiParams), i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "fsi_gcsi_set_convection": (i, [vp, C.POINTER(GcsiParams), vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class FSIError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _vp(t):
    """c_void_p of a tensor's data, or NULL for None."""
    return C.c_void_p(None if t is None else _ptr(t))


def _ptr(t) -> int:
    return t.data_ptr()


class Context:
    """One library context (a level hierarchy on one stream)."""

    def __init__(self, dim: int, n_fine, extent, n_coarse, dirichlet_faces: int, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP path has no CPU fallback")
        self.lib = load_library()
        self.torch = torch
        md = MeshDesc()
        md.dim = dim
        for k in range(3):
            md.n_fine[k] = int(n_fine[k]) if k < dim else 1
            md.extent[k] = float(extent[k]) if k < dim else 1.0
            md.n_coarse[k] = int(n_coarse[k]) if k < dim else 1
        md.dirichlet_faces = int(dirichlet_faces)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        st = self.lib.fsi_create(C.byref(h), C.byref(md), C.c_void_p(self.stream.cuda_stream))
        if st != FSI_OK:
            raise FSIError(st, "fsi_create failed")
        self.h = h
        self.dim = dim
        n = C.c_int()
        self.lib.fsi_get_num_levels(self.h, C.byref(n))
        self.n_levels = n.value

    @classmethod
    def from_mesh(cls, mesh, stream=None):
        return cls(mesh.dim, mesh.n_fine, mesh.extent, mesh.n_coarse, mesh.dirichlet_faces, stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.fsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, allow=(FSI_OK,)):
        if st not in allow:
            raise FSIError(st, self.lib.fsi_last_error(self.h).decode())
        return st

    # ---------------------------------------------------------------- queries
    def sizes(self, level: int) -> dict:
        s = Sizes()
        self._check(self.lib.fsi_get_sizes(self.h, level, C.byref(s)))
        return {f: (list(getattr(s, f)) if isinstance(getattr(s, f), C.Array) else getattr(s, f))
                for f, _ in Sizes._fields_}

    def level_info(self, level: int) -> dict:
        li = LevelInfo()
        self._check(self.lib.fsi_get_level_info(self.h, level, C.byref(li)))
        return {f: getattr(li, f) for f, _ in LevelInfo._fields_}

    # ---------------------------------------------------------------- setters
    def _dev64(self, a):
        t = self.torch
        if not isinstance(a, t.Tensor):
            a = t.as_tensor(a)
        return a.to(device="cuda", dtype=t.float64).contiguous()

    def set_jacobians(self, level: int, J):
        J = self._dev64(J)
        self._check(self.lib.fsi_set_jacobians(self.h, level, C.c_void_p(_ptr(J))))
        self.stream.synchronize()

    def set_displacement(self, disp):
        d = self._dev64(disp)
        self._check(self.lib.fsi_set_displacement(self.h, C.c_void_p(_ptr(d))))
        self.stream.synchronize()

    def set_coefficients(self, level: int, c_mass, eta):
        cm = self._dev64(c_mass)
        et = self._dev64(eta)
        self._check(self.lib.fsi_set_coefficients(self.h, level, C.c_void_p(_ptr(cm)), C.c_void_p(_ptr(et))))
        self.stream.synchronize()

    def set_convection(self, level: int, vconv, r, rho: float):
        """Corrector-mode terms on a level (fsi_set_convection): v° [n_cells][Q][3], r [n_cells][Q]."""
        vc = self._dev64(vconv)
        rr = self._dev64(r)
        self._check(self.lib.fsi_set_convection(self.h, level, C.c_void_p(_ptr(vc)), C.c_void_p(_ptr(rr)),
                                                float(rho)))
        self.stream.synchronize()

    def set_mg_params(self, **kw):
        p = MGParams()
        self.lib.fsi_default_mg_params(C.byref(p))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        self._check(self.lib.fsi_set_mg_params(self.h, C.byref(p)))

    def setup(self):
        self._check(self.lib.fsi_setup(self.h))

    def autotune(self):
        self._check(self.lib.fsi_autotune(self.h))

    def tuning(self, level: int, precision: int):
        v = C.c_int()
        us = C.c_double()
        self._check(self.lib.fsi_get_tuning(self.h, level, precision, C.byref(v), C.byref(us)))
        return v.value, us.value


    def set_tuning(self, level: int, precision: int, variant: int):
        """Pin the launch variant (0 .. N_LAUNCH_VARIANTS - 1) of every operator class on a
        level (overrides autotune)."""
        self._check(self.lib.fsi_set_tuning(self.h, level, precision, variant))
    def time_operator(self, level: int, precision: int = 0, mode: int = 1, reps: int = 10):
        """(cell-kernel us, operator us, launches) of one application: medians over `reps`
        timed applications after three warm-ups."""
        k = C.c_double()
        o = C.c_double()
        n = C.c_int()
        self._check(self.lib.fsi_time_operator(self.h, level, precision, mode, reps, C.byref(k), C.byref(o),
                                               C.byref(n)))
        return k.value, o.value, n.value

    # ---------------------------------------------------------------- operators
    def _out(self, n, dtype):
        return self.torch.empty(n, dtype=dtype, device="cuda")

    def apply_A(self, level, u, out=None):
        s = self.sizes(level)
        f32 = u.dtype == self.torch.float32
        v = out if out is not None else self._out(s["n_vel"], u.dtype)
        fn = self.lib.fsi_apply_A_f32 if f32 else self.lib.fsi_apply_A
        self._check(fn(self.h, level, C.c_void_p(_ptr(u)), C.c_void_p(_ptr(v))))
        return v

    def apply_B(self, level, u, out=None):
        s = self.sizes(level)
        f32 = u.dtype == self.torch.float32
        q = out if out is not None else self._out(s["n_p"], u.dtype)
        fn = self.lib.fsi_apply_B_f32 if f32 else self.lib.fsi_apply_B
        self._check(fn(self.h, level, C.c_void_p(_ptr(u)), C.c_void_p(_ptr(q))))
        return q

    def apply_BT(self, level, p, out=None):
        s = self.sizes(level)
        f32 = p.dtype == self.torch.float32
        v = out if out is not None else self._out(s["n_vel"], p.dtype)
        fn = self.lib.fsi_apply_BT_f32 if f32 else self.lib.fsi_apply_BT
        self._check(fn(self.h, level, C.c_void_p(_ptr(p)), C.c_void_p(_ptr(v))))
        return v

    def apply_stokes(self, level, u, p, out_v=None, out_q=None):
        s = self.sizes(level)
        f32 = u.dtype == self.torch.float32
        v = out_v if out_v is not None else self._out(s["n_vel"], u.dtype)
        q = out_q if out_q is not None else self._out(s["n_p"], u.dtype)
        fn = self.lib.fsi_apply_stokes_f32 if f32 else self.lib.fsi_apply_stokes
        self._check(fn(self.h, level, C.c_void_p(_ptr(u)), C.c_void_p(_ptr(p)), C.c_void_p(_ptr(v)),
                       C.c_void_p(_ptr(q))))
        return v, q

    def apply_stokes_f32_noalloc(self, level, u, p, out_v, out_q):
        """FP32 Stokes apply that allocates nothing (fsi_apply_stokes_f32_noalloc); the
        caller provides the outputs."""
        self._check(self.lib.fsi_apply_stokes_f32_noalloc(self.h, level, C.c_void_p(_ptr(u)), C.c_void_p(_ptr(p)),
                                                          C.c_void_p(_ptr(out_v)), C.c_void_p(_ptr(out_q))))
        return out_v, out_q

    def apply_corrector(self, level, u, p, out_v=None, out_q=None):
        """Stokes apply with the corrector-mode terms (fsi_apply_corrector[_f32])."""
        s = self.sizes(level)
        f32 = u.dtype == self.torch.float32
        v = out_v if out_v is not None else self._out(s["n_vel"], u.dtype)
        q = out_q if out_q is not None else self._out(s["n_p"], u.dtype)
        fn = self.lib.fsi_apply_corrector_f32 if f32 else self.lib.fsi_apply_corrector
        self._check(fn(self.h, level, C.c_void_p(_ptr(u)), C.c_void_p(_ptr(p)), C.c_void_p(_ptr(v)),
                       C.c_void_p(_ptr(q))))
        return v, q

    def vcycle(self, r_u, r_p, out_u=None, out_p=None):
        z_u = out_u if out_u is not None else self.torch.empty_like(r_u)
        z_p = out_p if out_p is not None else self.torch.empty_like(r_p)
        self._check(self.lib.fsi_vcycle(self.h, C.c_void_p(_ptr(r_u)), C.c_void_p(_ptr(r_p)),
                                        C.c_void_p(_ptr(z_u)), C.c_void_p(_ptr(z_p))))
        return z_u, z_p

    def solve(self, g_u, g_p, u=None, p=None, rtol: float = 1e-8, max_iter: int = 500, restart: int = 100,
              reorth: int = 0):
        """FGMRES solve; returns (u, p, info).  u/p (if given) are the initial guess, updated in place.
        reorth: 0 one classical Gram-Schmidt pass, 1 second pass when needed, 2 always two."""
        t = self.torch
        u = t.zeros_like(g_u) if u is None else u
        p = t.zeros_like(g_p) if p is None else p
        o = SolveOpts(rtol=rtol, max_iter=max_iter, restart=restart, reorth=reorth)
        hist = (C.c_double * (max_iter + 1))()
        info = SolveInfo()
        info.res_history = C.cast(hist, C.POINTER(C.c_double))
        st = self._check(self.lib.fsi_solve(self.h, C.c_void_p(_ptr(g_u)), C.c_void_p(_ptr(g_p)),
                                            C.c_void_p(_ptr(u)), C.c_void_p(_ptr(p)), C.byref(o), C.byref(info)),
                         allow=(FSI_OK, FSI_NOT_CONVERGED))
        out = dict(status=STATUS_NAMES[st], iters=info.iters, rel_res=info.final_rel_res, time_ms=info.time_ms,
                   history=[hist[k] for k in range(info.n_hist)])
        return u, p, out

    def solve_extension(self, g, u=None, rtol: float = 1e-6, max_iter: int = 200):
        """Extension solve (fsi_solve_extension); returns (u, info).  g holds the wall
        data; u (if given) the interior initial guess, updated in place."""
        t = self.torch
        u = t.zeros_like(g) if u is None else u
        o = SolveOpts(rtol=rtol, max_iter=max_iter, restart=1, reorth=0)
        hist = (C.c_double * (max_iter + 1))()
        info = SolveInfo()
        info.res_history = C.cast(hist, C.POINTER(C.c_double))
        st = self._check(self.lib.fsi_solve_extension(self.h, C.c_void_p(_ptr(g)), C.c_void_p(_ptr(u)), C.byref(o),
                                                      C.byref(info)),
                         allow=(FSI_OK, FSI_NOT_CONVERGED))
        out = dict(status=STATUS_NAMES[st], iters=info.iters, rel_res=info.final_rel_res, time_ms=info.time_ms,
                   history=[hist[k] for k in range(info.n_hist)])
        return u, out

    # ---------------------------------------------------------------- time step (Algorithm 1)
    def set_fixed_cells(self, fixed):
        """Fix every node of the flagged finest-level cells (fsi_set_fixed_cells; host uint8)."""
        import numpy as np
        f = np.ascontiguousarray(np.asarray(fixed, dtype=np.uint8))
        self._check(self.lib.fsi_set_fixed_cells(self.h, f.ctypes.data_as(C.c_void_p)))

    def lift_dirichlet(self, d, g_u, g_p):
        """Nonzero Dirichlet data d into the right-hand side (fsi_lift_dirichlet; in place)."""
        self._check(self.lib.fsi_lift_dirichlet(self.h, C.c_void_p(_ptr(d)), C.c_void_p(_ptr(g_u)),
                                                C.c_void_p(_ptr(g_p))))
        return g_u, g_p

    def fixed_values(self, v, out):
        self._check(self.lib.fsi_fixed_values(self.h, C.c_void_p(_ptr(v)), C.c_void_p(_ptr(out))))
        return out

    def gcsi_displacement(self, prm: GcsiParams, w, u1, u2=None, out=None, disp=None):
        self._check(self.lib.fsi_gcsi_displacement(self.h, C.byref(prm), C.c_void_p(_ptr(w)), C.c_void_p(_ptr(u1)),
                                                   _vp(u2), _vp(out), _vp(disp)))
        return out, disp

    def gcsi_set_coefficients(self, prm: GcsiParams, solid_q):
        """solid_q: per level, a device uint8 tensor [n_cells][3^dim]."""
        arr = (C.c_void_p * len(solid_q))(*[_ptr(x) for x in solid_q])
        self._check(self.lib.fsi_gcsi_set_coefficients(self.h, C.byref(prm), arr))

    def gcsi_rhs(self, prm: GcsiParams, mode: int, solid_q, disp, u_hash, u1, u2, v1, v2, w1, w2, g_u, g_p):
        self._check(self.lib.fsi_gcsi_rhs(self.h, C.byref(prm), mode, C.c_void_p(_ptr(solid_q)),
                                          C.c_void_p(_ptr(disp)), C.c_void_p(_ptr(u_hash)), _vp(u1), _vp(u2),
                                          _vp(v1), _vp(v2), _vp(w1), _vp(w2), C.c_void_p(_ptr(g_u)),
                                          C.c_void_p(_ptr(g_p))))
        return g_u, g_p

    def gcsi_set_convection(self, prm: GcsiParams, v_hash, w_hash):
        self._check(self.lib.fsi_gcsi_set_convection(self.h, C.byref(prm), C.c_void_p(_ptr(v_hash)),
                                                     C.c_void_p(_ptr(w_hash))))

    def raw_status(self, name: str, *args) -> int:
        """Call a C entry point and return its status without raising (error-path tests)."""
        return getattr(self.lib, name)(self.h, *args)


def setup_workload(ctx: Context, wl, levels=None):
    """Hand a generated workload to the library: displacement, coefficients on every level."""
    ctx.set_displacement(wl.disp)
    lv = range(ctx.n_levels) if levels is None else levels
    for j in lv:
        ctx.set_coefficients(j, wl.c_mass[j], wl.eta[j])
