"""ctypes binding of libvie.so (the C ABI declared in include/vie.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the operator apply and of the solve runs in the
library's kernels.  There is no CPU fallback: if the library is missing or no
GPU is visible, constructing a Plan raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvie.so")

LAPLACE, HELMHOLTZ, MAXWELL = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
PTR_HOST, STRICT_MEDIUM, NO_GRAPHS = 0x1, 0x2, 0x4
WHOLE_GRID, DENSE_BOX, FULL_LENGTH, GRID_TABLES = 0x8, 0x10, 0x20, 0x40
NOALLOC_SCRATCH_MIB = 128
APPLY_FP64, APPLY_FP32, APPLY_CONV, APPLY_C64 = 0x1, 0x2, 0x4, 0x8
SOLVER_GMRES, SOLVER_BICGSTAB = 0, 1
SOLVE_X0, SOLVE_FP64 = 0x1, 0x2

OK, E_ARG, E_SIZE, E_MEDIUM, E_NOMEM, E_DEVICE, E_STATE, W_NOCONV = 0, -1, -2, -3, -4, -5, -6, 1


class VieError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n", ctypes.c_int), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("omega", ctypes.c_double),
                ("coef", ctypes.c_void_p), ("mu", ctypes.c_void_p), ("precision", ctypes.c_int),
                ("max_rhs", ctypes.c_int), ("flags", ctypes.c_uint)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iters", ctypes.c_int), ("restart", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("solver", ctypes.c_int), ("flags", ctypes.c_uint)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("matvecs_fp32", ctypes.c_int),
                ("matvecs_fp64", ctypes.c_int), ("refinements", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = ["vie_plan_create", "vie_apply", "vie_apply_noalloc", "vie_rhs", "vie_field", "vie_solve", "vie_destroy",
           "vie_plan_info", "vie_copy_tables", "vie_copy_contrast", "vie_status_string",
           "vie_last_error", "vie_supported_n", "vie_profile", "vie_profile_read", "vie_profile_family",
           "vie_footprint_bytes", "vie_potential", "vie_field_h", "vie_fields_at", "vie_far_field",
           "vie_release_cached_memory", "vie_batch_open", "vie_batch_add", "vie_batch_step", "vie_batch_done",
           "vie_batch_take", "vie_batch_close"]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libvie.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1805_04791_amd.build`")
    L = ctypes.CDLL(path)
    vp, ci, cd, cu = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    L.vie_plan_create.argtypes = [ctypes.POINTER(Problem), vp, ctypes.POINTER(vp)]
    L.vie_apply.argtypes = [vp, vp, vp, ci, cu, vp]
    L.vie_apply_noalloc.argtypes = [vp, vp, vp, ci, cu, vp]
    L.vie_rhs.argtypes = [vp, vp, vp, ci, vp]
    L.vie_field.argtypes = [vp, vp, vp, vp, ci, vp]
    L.vie_solve.argtypes = [vp, vp, vp, vp, ci, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), vp]
    L.vie_destroy.argtypes = [vp]
    L.vie_plan_info.argtypes = [vp, ctypes.POINTER(cd), ci]
    L.vie_copy_tables.argtypes = [vp, vp, ctypes.c_long, ctypes.POINTER(ctypes.c_long),
                                  ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.vie_copy_contrast.argtypes = [vp, vp, ctypes.c_long]
    L.vie_status_string.argtypes = [ci]
    L.vie_status_string.restype = ctypes.c_char_p
    L.vie_last_error.argtypes = [vp]
    L.vie_last_error.restype = ctypes.c_char_p
    L.vie_supported_n.argtypes = [ci]
    L.vie_profile.argtypes = [vp, ci]
    L.vie_profile_read.argtypes = [vp, ctypes.POINTER(cd), ctypes.POINTER(ctypes.c_long),
                                   ctypes.POINTER(cd), ctypes.POINTER(cd), ci]
    L.vie_profile_family.argtypes = [ci]
    L.vie_profile_family.restype = ctypes.c_char_p
    L.vie_potential.argtypes = [vp, vp, vp, ci, vp]
    L.vie_field_h.argtypes = [vp, vp, vp, vp, ci, vp]
    L.vie_fields_at.argtypes = [vp, vp, ci, vp, ci, vp, vp]
    L.vie_far_field.argtypes = [vp, vp, ci, vp, ci, vp, vp]
    L.vie_footprint_bytes.argtypes = [ci, ci, ci, ci, ci]
    L.vie_footprint_bytes.restype = ctypes.c_long
    ip = ctypes.POINTER(ci)
    L.vie_batch_open.argtypes = [vp, ci, ctypes.POINTER(SolveOpts), vp]
    L.vie_batch_add.argtypes = [vp, vp, vp, ci, ip, vp]
    L.vie_batch_step.argtypes = [vp, ip, vp]
    L.vie_batch_done.argtypes = [vp, ip, ci, ip, ip]
    L.vie_batch_take.argtypes = [vp, ci, vp, vp, vp, ctypes.POINTER(SolveStats), vp]
    L.vie_batch_close.argtypes = [vp]
    L.vie_release_cached_memory.argtypes = []
    L.vie_release_cached_memory.restype = ctypes.c_long
    for name in ("vie_plan_create", "vie_apply", "vie_apply_noalloc", "vie_rhs", "vie_field", "vie_solve", "vie_destroy",
                 "vie_plan_info", "vie_copy_tables", "vie_copy_contrast", "vie_supported_n",
                 "vie_profile", "vie_profile_read", "vie_potential", "vie_field_h", "vie_fields_at",
                 "vie_far_field", "vie_batch_open", "vie_batch_add", "vie_batch_step", "vie_batch_done",
                 "vie_batch_take", "vie_batch_close"):
        getattr(L, name).restype = ci
    _lib = L
    return L


def release_cached_memory() -> int:
    """Frees the library's cache of device blocks released by destroyed plans
    (and of their pinned host buffers); returns the device bytes it held."""
    return int(load_library().vie_release_cached_memory())


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _device_c128(x, device):
    """A contiguous complex128 tensor on the GPU holding x (numpy or torch)."""
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128))
    if x.dtype != torch.complex128:
        x = x.to(torch.complex128)
    return x.to(device).contiguous()


def supported_n(n: int) -> bool:
    return bool(load_library().vie_supported_n(int(n)))


def footprint_bytes(kind: int, n: int, full: bool, nrhs_batch: int, restart: int) -> int:
    """Peak device bytes of a plan of this size (host-only estimate)."""
    return int(load_library().vie_footprint_bytes(int(kind), int(n), 1 if full else 0, int(nrhs_batch),
                                                  int(restart)))


class Plan:
    """A solver plan: contrast, kernel tables and workspaces on one GPU.

    kind: LAPLACE (coef = eps), HELMHOLTZ (coef = eps^{-1}) or MAXWELL
    (coef = eps, optional mu).  coef / mu: complex arrays [9][n][n][n].
    flags: further vie_problem flags (WHOLE_GRID, DENSE_BOX, FULL_LENGTH, ...).
    """

    def __init__(self, kind: int, coef, omega: float = 0.0, mu=None, h: Optional[float] = None,
                 precision: int = PREC_MIXED, max_rhs: int = 1, strict: bool = False,
                 device: str = "cuda", stream=None, graphs: bool = True, flags: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the volume-integral-equation library runs on MI355X only")
        self.lib = load_library()
        self.device = torch.device(device)
        coef_d = _device_c128(coef, self.device)
        n = int(coef_d.shape[-1])
        if tuple(coef_d.shape) != (9, n, n, n):
            raise ValueError(f"coef must be [9][n][n][n], got {tuple(coef_d.shape)}")
        mu_d = _device_c128(mu, self.device) if mu is not None else None
        self.kind, self.n, self.omega = int(kind), n, float(omega)
        self.h = 2.0 / n if h is None else float(h)
        self.ncomp = 6 if mu is not None else 3
        p = Problem()
        p.kind, p.n, p.h = self.kind, n, self.h
        p.origin = (ctypes.c_double * 3)(-0.5 * n * self.h, -0.5 * n * self.h, -0.5 * n * self.h)
        p.omega = self.omega
        p.coef = coef_d.data_ptr()
        p.mu = mu_d.data_ptr() if mu_d is not None else None
        p.precision = int(precision)
        p.max_rhs = int(max_rhs)
        p.flags = (STRICT_MEDIUM if strict else 0) | (0 if graphs else NO_GRAPHS) | int(flags)
        handle = ctypes.c_void_p()
        rc = self.lib.vie_plan_create(ctypes.byref(p), _stream_ptr(stream), ctypes.byref(handle))
        if rc != OK:
            raise VieError(rc, self.lib.vie_last_error(None).decode())
        self._h = handle
        self.precision = int(precision)

    # -- helpers ---------------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc < 0:
            raise VieError(rc, f"{what}: {self.lib.vie_last_error(self._h).decode()}")
        return rc

    def _vec(self, x, name="x"):
        x = _device_c128(x, self.device)
        if x.dim() == 4:
            x = x.unsqueeze(0)
        if tuple(x.shape[1:]) != (self.ncomp, self.n, self.n, self.n):
            raise ValueError(f"{name} must be [nrhs][{self.ncomp}][n][n][n], got {tuple(x.shape)}")
        return x

    @property
    def handle(self):
        return self._h

    # -- operations --------------------------------------------------------------
    def apply(self, x, flags: int = 0, stream=None):
        """y = A x.  With APPLY_C64 the vectors are complex64 (x is converted)."""
        torch = _torch()
        x = self._vec(x)
        if flags & APPLY_C64:
            x = x.to(torch.complex64)
        y = torch.empty_like(x)
        self._check(self.lib.vie_apply(self._h, x.data_ptr(), y.data_ptr(), x.shape[0], int(flags),
                                       _stream_ptr(stream)), "vie_apply")
        return y

    def apply_noalloc(self, x, y=None, flags: int = 0, stream=None):
        """y = A x through vie_apply_noalloc (the library's static scratch as
        workspace; nothing allocated by the call).  y may be given (reused)."""
        torch = _torch()
        x = self._vec(x)
        if flags & APPLY_C64:
            x = x.to(torch.complex64)
        if y is None:
            y = torch.empty_like(x)
        self._check(self.lib.vie_apply_noalloc(self._h, x.data_ptr(), y.data_ptr(), x.shape[0], int(flags),
                                               _stream_ptr(stream)), "vie_apply_noalloc")
        return y

    def rhs(self, inc, stream=None):
        torch = _torch()
        inc = self._vec(inc, "inc")
        b = torch.empty_like(inc)
        self._check(self.lib.vie_rhs(self._h, inc.data_ptr(), b.data_ptr(), inc.shape[0], _stream_ptr(stream)),
                    "vie_rhs")
        return b

    def field(self, density, inc, stream=None):
        torch = _torch()
        d = self._vec(density, "density")
        inc = self._vec(inc, "inc")
        f = torch.empty_like(inc)
        self._check(self.lib.vie_field(self._h, d.data_ptr(), inc.data_ptr(), f.data_ptr(), d.shape[0],
                                       _stream_ptr(stream)), "vie_field")
        return f

    def potential(self, density, stream=None):
        """phi_scat = div V J on the grid (Laplace, Helmholtz): complex128 [nrhs][n][n][n]."""
        torch = _torch()
        d = self._vec(density, "density")
        phi = torch.empty((d.shape[0], self.n, self.n, self.n), dtype=torch.complex128, device=self.device)
        self._check(self.lib.vie_potential(self._h, d.data_ptr(), phi.data_ptr(), d.shape[0], _stream_ptr(stream)),
                    "vie_potential")
        return phi

    def field_h(self, density, h_inc=None, stream=None):
        """Maxwell with mu = I: H_inc - i omega curl V J on the grid (H_scat if h_inc is None)."""
        torch = _torch()
        d = self._vec(density, "density")
        hi = self._vec(h_inc, "h_inc") if h_inc is not None else None
        out = torch.empty_like(d)
        self._check(self.lib.vie_field_h(self._h, d.data_ptr(), hi.data_ptr() if hi is not None else None,
                                         out.data_ptr(), d.shape[0], _stream_ptr(stream)), "vie_field_h")
        return out

    def fields_at(self, density, points, stream=None):
        """Scattered fields at points away from the support: [nrhs][npts][4] (phi, grad phi) or [nrhs][npts][6] (E, H)."""
        torch = _torch()
        d = self._vec(density, "density")
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
        k = 6 if self.kind == MAXWELL else 4
        out = torch.empty((d.shape[0], pts.shape[0], k), dtype=torch.complex128, device=self.device)
        self._check(self.lib.vie_fields_at(self._h, d.data_ptr(), d.shape[0], pts.ctypes.data, pts.shape[0],
                                           out.data_ptr(), _stream_ptr(stream)), "vie_fields_at")
        return out

    def far_field(self, density, dirs, stream=None):
        """Far-field patterns in unit directions: [nrhs][ndirs][1] (Helmholtz) or [nrhs][ndirs][6] (Maxwell)."""
        torch = _torch()
        d = self._vec(density, "density")
        dd = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 3))
        k = 6 if self.kind == MAXWELL else 1
        out = torch.empty((d.shape[0], dd.shape[0], k), dtype=torch.complex128, device=self.device)
        self._check(self.lib.vie_far_field(self._h, d.data_ptr(), d.shape[0], dd.ctypes.data, dd.shape[0],
                                           out.data_ptr(), _stream_ptr(stream)), "vie_far_field")
        return out

    def solve(self, inc, tol: float = 1e-10, max_iters: int = 2000, restart: int = 40,
              inner_tol: float = 0.0, solver: int = SOLVER_GMRES, fp64: bool = False, x0=None,
              want_field: bool = True, stream=None):
        """Returns (density, field or None, list of stats dicts, status)."""
        torch = _torch()
        inc = self._vec(inc, "inc")
        nrhs = inc.shape[0]
        if x0 is not None:
            dens = self._vec(x0, "x0").clone()
        else:
            dens = torch.empty_like(inc)
        fld = torch.empty_like(inc) if want_field else None
        o = SolveOpts(float(tol), int(max_iters), int(restart), float(inner_tol), int(solver),
                      (SOLVE_X0 if x0 is not None else 0) | (SOLVE_FP64 if fp64 else 0))
        st = (SolveStats * nrhs)()
        rc = self.lib.vie_solve(self._h, inc.data_ptr(), dens.data_ptr(),
                                fld.data_ptr() if fld is not None else None, nrhs, ctypes.byref(o), st,
                                _stream_ptr(stream))
        self._check(rc, "vie_solve")
        return dens, fld, [s.as_dict() for s in st], rc

    # -- continuous batching (one open batch per plan) ------------------------------
    def batch_open(self, capacity: int, tol: float = 1e-10, max_iters: int = 2000, restart: int = 40,
                   inner_tol: float = 0.0, solver: int = SOLVER_GMRES, fp64: bool = False, stream=None):
        """Open a batch of `capacity` solver slots on this plan (vie_batch_open)."""
        o = SolveOpts(float(tol), int(max_iters), int(restart), float(inner_tol), int(solver),
                      SOLVE_FP64 if fp64 else 0)
        self._check(self.lib.vie_batch_open(self._h, int(capacity), ctypes.byref(o), _stream_ptr(stream)),
                    "vie_batch_open")

    def batch_add(self, inc, x0=None, stream=None) -> list:
        """Right-hand sides [k][c][n][n][n] join free slots at the next cycle; returns the slots."""
        inc = self._vec(inc, "inc")
        x = self._vec(x0, "x0") if x0 is not None else None
        k = inc.shape[0]
        slots = (ctypes.c_int * k)()
        self._check(self.lib.vie_batch_add(self._h, inc.data_ptr(), x.data_ptr() if x is not None else None, k,
                                           slots, _stream_ptr(stream)), "vie_batch_add")
        return list(slots)

    def batch_step(self, stream=None) -> int:
        """One outer cycle of every slot still iterating; returns how many still iterate."""
        n = ctypes.c_int()
        self._check(self.lib.vie_batch_step(self._h, ctypes.byref(n), _stream_ptr(stream)), "vie_batch_step")
        return n.value

    def batch_done(self):
        """(finished slots not yet taken, free slots)."""
        cap = 256
        slots = (ctypes.c_int * cap)()
        nd, nf = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.vie_batch_done(self._h, slots, cap, ctypes.byref(nd), ctypes.byref(nf)), "vie_batch_done")
        return list(slots[:min(nd.value, cap)]), nf.value

    def batch_take(self, slot: int, inc=None, want_field: bool = False, stream=None):
        """Density (and total field) of a finished slot, which is freed: (density, field, stats, status)."""
        torch = _torch()
        d = torch.empty((self.ncomp, self.n, self.n, self.n), dtype=torch.complex128, device=self.device)
        f = torch.empty_like(d) if want_field else None
        i = self._vec(inc, "inc") if want_field else None
        st = SolveStats()
        rc = self.lib.vie_batch_take(self._h, int(slot), d.data_ptr(), f.data_ptr() if f is not None else None,
                                     i.data_ptr() if i is not None else None, ctypes.byref(st), _stream_ptr(stream))
        self._check(rc, "vie_batch_take")
        return d, f, st.as_dict(), rc

    def batch_close(self):
        self._check(self.lib.vie_batch_close(self._h), "vie_batch_close")

    def info(self) -> dict:
        out = (ctypes.c_double * 20)()
        self._check(self.lib.vie_plan_info(self._h, out, 20), "vie_plan_info")
        keys = ["n", "ncomp", "P", "M", "max_contrast_norm", "table_entries", "device_bytes", "graph_launches",
                "box_x0", "box_y0", "box_z0", "box_nx", "box_ny", "box_nz", "unknown_points", "box_P",
                "workspace_rhs_fp32", "workspace_rhs_fp64", "krylov_slots", "box_Pz"]
        d = dict(zip(keys, list(out)))
        d["box"] = tuple(int(d.pop(k)) for k in keys[8:14])
        for k in ("unknown_points", "box_P", "workspace_rhs_fp32", "workspace_rhs_fp64", "krylov_slots", "box_Pz"):
            d[k] = int(d[k])
        return d

    def tables(self) -> np.ndarray:
        """FP64 octant tables as complex128 [n+1][n+1][ne][nxp] (a transposed
        view of the library's [n+1][n+1][nxp][ne])."""
        need = ctypes.c_long()
        nxp = ctypes.c_int()
        ne = ctypes.c_int()
        self._check(self.lib.vie_copy_tables(self._h, None, 0, ctypes.byref(need), ctypes.byref(nxp),
                                             ctypes.byref(ne)), "vie_copy_tables")
        arr = np.empty(need.value // 16, dtype=np.complex128)
        self._check(self.lib.vie_copy_tables(self._h, arr.ctypes.data, need.value, None, None, None),
                    "vie_copy_tables")
        n1 = self.n + 1
        return arr.reshape(n1, n1, nxp.value, ne.value).transpose(0, 1, 3, 2)

    def contrast(self) -> np.ndarray:
        k = 2 if self.ncomp == 6 else 1
        arr = np.empty(k * 9 * self.n ** 3, dtype=np.complex128)
        self._check(self.lib.vie_copy_contrast(self._h, arr.ctypes.data, arr.nbytes), "vie_copy_contrast")
        return arr.reshape(k, 9, self.n, self.n, self.n)

    def profile(self, enable: bool = True):
        """Start (and reset) or stop per-kernel HIP-event timing."""
        self._check(self.lib.vie_profile(self._h, 1 if enable else 0), "vie_profile")

    def profile_read(self) -> dict:
        """{family: (total ms, launches, algorithmic bytes, nominal flops)} since profile(True)."""
        ms = (ctypes.c_double * 16)()
        cnt = (ctypes.c_long * 16)()
        by = (ctypes.c_double * 16)()
        fl = (ctypes.c_double * 16)()
        nf = self._check(self.lib.vie_profile_read(self._h, ms, cnt, by, fl, 16), "vie_profile_read")
        out = {}
        for i in range(nf):
            if cnt[i]:
                out[self.lib.vie_profile_family(i).decode()] = (ms[i], cnt[i], by[i], fl[i])
        return out

    def close(self):
        if getattr(self, "_h", None):
            self.lib.vie_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
