"""ctypes binding of libknp (include/knp.h): argument marshalling only.

Device vectors are torch tensors (float64, contiguous, on the context's HIP
device); host arrays are numpy arrays.  Every call checks the returned status
and raises KnpError with the library's message.  There is no fallback: if the
shared library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libknp.so")

STATUS = {0: "KNP_OK", 1: "KNP_E_ARG", 2: "KNP_E_STATE", 3: "KNP_E_HIP", 4: "KNP_E_NOMEM",
          5: "KNP_E_NOCONV", 6: "KNP_E_NUMERIC"}
KNP_E_NOCONV = 5

EXPORTS = ["knp_create", "knp_destroy", "knp_last_error", "knp_mesh_upload", "knp_get_layout",
           "knp_get_gamma", "knp_set_params", "knp_assemble_step", "knp_assemble_step_noalloc", "knp_amg_setup",
           "knp_mesh_upload_p2", "knp_get_edges",
           "knp_gmres_solve", "knp_adjoint_solve", "knp_step_vjp", "knp_apply",
           "knp_get_scaling", "knp_get_values", "knp_timing", "knp_timing_read", "knp_amg_stats",
           "knp_set_gauge", "knp_extrapolate"]
TIMERS = ["spmv_A", "cheb_L0", "resid_L0", "vcycle", "assembly", "resid_A"]


class KnpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshInfo(C.Structure):
    _fields_ = [("n_vert", C.c_int64), ("n_elem", C.c_int64), ("N_i", C.c_int64), ("N_e", C.c_int64),
                ("N", C.c_int64), ("nnz_A", C.c_int64), ("nnz_P0", C.c_int64), ("n_gamma", C.c_int64),
                ("n_facets", C.c_int64), ("n_cells", C.c_int32), ("dim", C.c_int32), ("pin_dof", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("R", C.c_double), ("T", C.c_double), ("F", C.c_double), ("C_m", C.c_double),
                ("z", C.c_double * 3), ("D", C.c_double * 3), ("g_leak", C.c_double * 3),
                ("gbar_Na", C.c_double), ("gbar_K", C.c_double), ("g_stim_bar", C.c_double),
                ("stim_a", C.c_double), ("stim_tau", C.c_double), ("phi_rest", C.c_double),
                ("rho_pump", C.c_double), ("P_Na", C.c_double), ("P_K", C.c_double),
                ("K_e0", C.c_double), ("K_i0", C.c_double),
                ("n_ode", C.c_int32), ("n_cells", C.c_int32),
                ("cell_model", C.POINTER(C.c_int32)), ("cell_stim", C.POINTER(C.c_int32))]


class AmgOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("strength", C.c_double), ("cheb_degree", C.c_int32),
                ("cheb_ratio", C.c_double), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("coarse_drop", C.c_double), ("cheb_pre_degree", C.c_int32),
                ("coarse_pre_degree", C.c_int32), ("coarse_post_degree", C.c_int32),
                ("operator_step", C.c_int32), ("field_split", C.c_int32),
                ("shared_ion_aggregates", C.c_int32), ("coarse_graph", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_it", C.c_int32),
                ("reorth", C.c_int32), ("precond", C.c_int32)]


class Timer(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("bytes", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("its", C.c_int32), ("restarts", C.c_int32), ("rel_res", C.c_double),
                ("rel_res_est", C.c_double)]


def load_library(path: str = _LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libknp.so not found at {path}; run paper_2403_04491_amd/build.py "
                          "(or __graft_entry__.build()) first")
    # One HIP runtime per process: torch carries its own libamdhip64, and the
    # library's dependency must resolve to that already-loaded runtime.  Loaded
    # before torch, the library would bring in a second runtime whose device
    # state torch's allocations and streams do not belong to.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.knp_create.argtypes = [C.POINTER(P), C.c_int, P]
    lib.knp_destroy.argtypes = [P]
    lib.knp_destroy.restype = None
    lib.knp_last_error.argtypes = [P]
    lib.knp_last_error.restype = C.c_char_p
    lib.knp_mesh_upload.argtypes = [P, C.c_int, I64, P, I64, P, P, I64, C.POINTER(MeshInfo)]
    lib.knp_mesh_upload_p2.argtypes = [P, C.c_int, I64, P, I64, P, P, I64, C.POINTER(MeshInfo)]
    lib.knp_get_edges.argtypes = [P, P, P]
    lib.knp_get_layout.argtypes = [P, P, P, P]
    lib.knp_get_gamma.argtypes = [P, P]
    lib.knp_set_params.argtypes = [P, C.POINTER(Params)]
    lib.knp_assemble_step.argtypes = [P, D, D, P, P, P, P]
    lib.knp_assemble_step_noalloc.argtypes = [P, D, D, P, P, P, P]
    lib.knp_amg_setup.argtypes = [P, C.POINTER(AmgOpts)]
    lib.knp_set_gauge.argtypes = [P, C.c_int32]
    lib.knp_extrapolate.argtypes = [P, P, P, P]
    lib.knp_gmres_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]
    lib.knp_adjoint_solve.argtypes = [P, P, P, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]
    lib.knp_step_vjp.argtypes = [P, P, P, P, P, P]
    lib.knp_apply.argtypes = [P, C.c_int, P, P]
    lib.knp_get_scaling.argtypes = [P, P]
    lib.knp_get_values.argtypes = [P, P]
    lib.knp_timing.argtypes = [P, C.c_int]
    lib.knp_amg_stats.argtypes = [P, P, P, P]
    lib.knp_timing_read.argtypes = [P, P]
    for name in EXPORTS:
        if name not in ("knp_destroy", "knp_last_error"):
            getattr(lib, name).restype = C.c_int
    return lib


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _dptr(t, dtype=None, n=None):
    """Device pointer of a contiguous torch tensor (or None -> NULL)."""
    if t is None:
        return None
    import torch
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    del torch
    return C.c_void_p(t.data_ptr())


def _hptr(a):
    return a.ctypes.data_as(C.c_void_p)


def amg_opts(precision=0, strength=0.6, cheb_degree=5, cheb_ratio=2.5, coarse_max=2000, max_levels=20,
             coarse_drop=0.01, cheb_pre_degree=0, coarse_pre_degree=0, coarse_post_degree=1, operator_step=0,
             field_split=0, shared_ion_aggregates=0, coarse_graph=0):
    return AmgOpts(precision, strength, cheb_degree, cheb_ratio, coarse_max, max_levels, coarse_drop,
                   cheb_pre_degree, coarse_pre_degree, coarse_post_degree, operator_step, field_split,
                   shared_ion_aggregates, coarse_graph)


def solve_opts(rtol=1e-6, restart=30, max_it=2000, reorth=0, precond=1):
    return SolveOpts(rtol, restart, max_it, reorth, precond)


class Context:
    """One libknp context (one device, one stream)."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = lib()
        self._c = C.c_void_p()
        self.device = device
        if device >= 0:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            sp = C.c_void_p(stream.cuda_stream)
        else:
            sp = None
        self._check(self._lib.knp_create(C.byref(self._c), device, sp))
        self.info = None

    def _check(self, st):
        if st != 0:
            msg = self._lib.knp_last_error(self._c if self._c else None).decode()
            raise KnpError(st, msg)

    def close(self):
        if self._c:
            self._lib.knp_destroy(self._c)
            self._c = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ setup
    def mesh_upload(self, dim, xyz, elem, tag, pin_vertex=0, order=1) -> MeshInfo:
        """knp_mesh_upload (order 1) or knp_mesh_upload_p2 (order 2): the vertex mesh."""
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        elem = np.ascontiguousarray(elem, dtype=np.int32)
        tag = np.ascontiguousarray(tag, dtype=np.int32)
        info = MeshInfo()
        fn = {1: self._lib.knp_mesh_upload, 2: self._lib.knp_mesh_upload_p2}[order]
        self._check(fn(self._c, dim, xyz.shape[0], _hptr(xyz), elem.shape[0], _hptr(elem), _hptr(tag),
                       int(pin_vertex), C.byref(info)))
        self.info = info
        return info

    def get_edges(self):
        """[n_edges, 2] vertex pairs of the edge nodes (node n_vert + e) of an order-2 mesh."""
        n = C.c_int64(0)
        self._check(self._lib.knp_get_edges(self._c, C.byref(n), None))
        out = np.empty((n.value, 2), np.int32)
        if n.value:
            self._check(self._lib.knp_get_edges(self._c, None, _hptr(out)))
        return out

    def get_layout(self):
        N, nnz = self.info.N, self.info.nnz_A
        rowptr = np.empty(N + 1, np.int64)
        colidx = np.empty(nnz, np.int32)
        dofv = np.empty(N, np.int32)
        self._check(self._lib.knp_get_layout(self._c, _hptr(rowptr), _hptr(colidx), _hptr(dofv)))
        return rowptr, colidx, dofv

    def get_gamma(self):
        g = np.empty(self.info.n_gamma, np.int32)
        self._check(self._lib.knp_get_gamma(self._c, _hptr(g)))
        return g

    def set_params(self, params: dict, cell_model, cell_stim):
        cm = np.ascontiguousarray(cell_model, dtype=np.int32)
        cs = np.ascontiguousarray(cell_stim, dtype=np.int32)
        p = Params()
        p.R, p.T, p.F, p.C_m = params["R"], params["T"], params["F"], params["C_m"]
        for k in range(3):
            p.z[k] = params["z"][k]
            p.D[k] = params["D"][k]
            p.g_leak[k] = params["g_leak"][k]
        p.gbar_Na, p.gbar_K = params["gbar_Na"], params["gbar_K"]
        p.g_stim_bar, p.stim_a, p.stim_tau = params["g_stim_bar"], params["stim_a"], params["stim_tau"]
        p.phi_rest = params["phi_rest"]
        p.rho_pump, p.P_Na, p.P_K = params["rho_pump"], params["P_Na"], params["P_K"]
        p.K_e0, p.K_i0 = params["conc_e0"][1], params["conc_i0"][1]
        p.n_ode = int(params["n_ode"])
        p.n_cells = len(cm)
        p.cell_model = cm.ctypes.data_as(C.POINTER(C.c_int32))
        p.cell_stim = cs.ctypes.data_as(C.POINTER(C.c_int32))
        self._check(self._lib.knp_set_params(self._c, C.byref(p)))

    # ------------------------------------------------------------------ per step
    def assemble_step(self, t_n, dt, u_prev, gates, theta, f_out):
        import torch
        N = self.info.N
        self._check(self._lib.knp_assemble_step(
            self._c, float(t_n), float(dt), _dptr(u_prev, torch.float64, N),
            _dptr(gates, torch.float64, 3 * self.info.n_gamma) if gates is not None else None,
            _dptr(theta, torch.float64, self.info.n_cells) if theta is not None else None,
            _dptr(f_out, torch.float64, N)))

    def assemble_step_noalloc(self, t_n, dt, u_prev, gates, theta, f_out):
        """knp_assemble_step_noalloc: the same assembly with its scratch in the library's
        static device array (no device allocation)."""
        import torch
        N = self.info.N
        self._check(self._lib.knp_assemble_step_noalloc(
            self._c, float(t_n), float(dt), _dptr(u_prev, torch.float64, N),
            _dptr(gates, torch.float64, 3 * self.info.n_gamma) if gates is not None else None,
            _dptr(theta, torch.float64, self.info.n_cells) if theta is not None else None,
            _dptr(f_out, torch.float64, N)))

    def set_gauge(self, mode: int):
        """knp_set_gauge: 0 = point condition on the reference phi_e DOF in the system;
        1 = system without it, nullspace handled by the forward solve."""
        self._check(self._lib.knp_set_gauge(self._c, int(mode)))

    def extrapolate(self, u1, u2, x0):
        """knp_extrapolate: x0 = 2 u1 - u2 (device float64 [N])."""
        import torch
        N = self.info.N
        self._check(self._lib.knp_extrapolate(self._c, _dptr(u1, torch.float64, N), _dptr(u2, torch.float64, N),
                                              _dptr(x0, torch.float64, N)))

    def amg_setup(self, opts: AmgOpts | None = None):
        self._check(self._lib.knp_amg_setup(self._c, C.byref(opts) if opts is not None else None))

    def _solve(self, fn, b, x, opts, allow_noconv):
        import torch
        info = SolveInfo()
        N = self.info.N
        st = fn(self._c, _dptr(b, torch.float64, N), _dptr(x, torch.float64, N),
                C.byref(opts) if opts is not None else None, C.byref(info))
        if st == KNP_E_NOCONV and allow_noconv:
            return info, False
        self._check(st)
        return info, True

    def gmres_solve(self, b, x, opts: SolveOpts | None = None, allow_noconv=False):
        return self._solve(self._lib.knp_gmres_solve, b, x, opts, allow_noconv)

    def adjoint_solve(self, rhs, lam, opts: SolveOpts | None = None, allow_noconv=False):
        return self._solve(self._lib.knp_adjoint_solve, rhs, lam, opts, allow_noconv)

    def step_vjp(self, u_prev, u_n, lam, u_prev_bar, theta_bar=None):
        import torch
        N = self.info.N
        self._check(self._lib.knp_step_vjp(
            self._c, _dptr(u_prev, torch.float64, N), _dptr(u_n, torch.float64, N),
            _dptr(lam, torch.float64, N), _dptr(u_prev_bar, torch.float64, N),
            _dptr(theta_bar, torch.float64, self.info.n_cells) if theta_bar is not None else None))

    def apply(self, which, x, y):
        import torch
        N = self.info.N
        self._check(self._lib.knp_apply(self._c, int(which), _dptr(x, torch.float64, N),
                                        _dptr(y, torch.float64, N)))

    def get_scaling(self, out):
        import torch
        self._check(self._lib.knp_get_scaling(self._c, _dptr(out, torch.float64, self.info.N)))

    def amg_stats(self):
        nl = C.c_int32()
        rows = np.zeros(32, np.int64)
        nnz = np.zeros(32, np.int64)
        self._check(self._lib.knp_amg_stats(self._c, C.byref(nl), _hptr(rows), _hptr(nnz)))
        return {"rows": rows[:nl.value].tolist(), "nnz": nnz[:nl.value].tolist()}

    def timing(self, enable: bool):
        self._check(self._lib.knp_timing(self._c, 1 if enable else 0))

    def timing_read(self) -> dict:
        arr = (Timer * len(TIMERS))()
        self._check(self._lib.knp_timing_read(self._c, C.cast(arr, C.c_void_p)))
        return {name: {"launches": arr[i].launches, "total_ms": arr[i].total_ms, "bytes": arr[i].bytes}
                for i, name in enumerate(TIMERS)}

    def get_values(self, out):
        import torch
        self._check(self._lib.knp_get_values(self._c, _dptr(out, torch.float64, self.info.nnz_A)))
