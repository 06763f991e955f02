"""ctypes binding of libfelbm.so (include/felbm.h).  Argument marshalling
only: every step of the time step runs in the library's HIP kernels.  There
is no fallback: if the library is missing, loading raises."""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libfelbm.so")

FP64, FP32 = 0, 1
FIELDS = {"C": 0, "RHO": 1, "P": 2, "UX": 3, "UY": 4, "MU": 5, "LAPC": 6, "LAPMU": 7, "UZ": 8}
ERRORS = {-1: "EINVAL", -2: "EMESH", -3: "ESTATE", -4: "ENONFINITE", -5: "ESOLVER", -6: "EDEVICE", -7: "ENOMEM"}


class FelbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Params(ct.Structure):
    _fields_ = [("sigma", ct.c_double), ("xi", ct.c_double), ("mobility", ct.c_double),
                ("rho_l", ct.c_double), ("rho_v", ct.c_double), ("nu_l", ct.c_double), ("nu_v", ct.c_double),
                ("dt", ct.c_double), ("precision", ct.c_int32), ("solver_sweeps", ct.c_int32),
                ("lambda_min", ct.c_double), ("lambda_max", ct.c_double), ("kernels", ct.c_int32),
                ("force_scheme", ct.c_int32)]


class Diag(ct.Structure):
    _fields_ = [("step", ct.c_int64), ("mass", ct.c_double), ("mean_ke", ct.c_double), ("max_u", ct.c_double),
                ("band_ke", ct.c_double), ("band_nodes", ct.c_int64), ("nonfinite", ct.c_int32),
                ("solver_sweeps", ct.c_int32), ("solver_residual", ct.c_double), ("residual_step", ct.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KStat(ct.Structure):
    _fields_ = [("name", ct.c_char * 32), ("launches", ct.c_int64), ("total_ms", ct.c_double),
                ("bytes_per_launch", ct.c_double)]


_lib = None
_P = ct.c_void_p
_D = ct.POINTER(ct.c_double)
_I = ct.POINTER(ct.c_int32)

_SIGNATURES = {
    "felbm_create": ([ct.POINTER(Params), ct.POINTER(_P)], ct.c_int),
    "felbm_last_error": ([_P], ct.c_char_p),
    "felbm_upload_mesh": ([_P, ct.c_int64, _D, ct.c_int64, _I, ct.c_int64, _I, ct.c_double], ct.c_int),
    "felbm_set_wetting": ([_P, _D], ct.c_int),
    "felbm_set_wetting_device": ([_P, _P], ct.c_int),
    "felbm_init": ([_P, _D, _D, _D], ct.c_int),
    "felbm_step": ([_P, ct.c_int64], ct.c_int),
    "felbm_step_async": ([_P, ct.c_int64], ct.c_int),
    "felbm_read": ([_P, ct.c_int32, _D], ct.c_int),
    "felbm_read_device": ([_P, ct.c_int32, _P], ct.c_int),
    "felbm_read_populations": ([_P, _D], ct.c_int),
    "felbm_step_debug": ([_P, _D, _D, _D], ct.c_int),
    "felbm_set_band": ([_P, ct.c_double, ct.c_double, ct.c_double, ct.c_double], ct.c_int),
    "felbm_diagnostics": ([_P, ct.POINTER(Diag)], ct.c_int),
    "felbm_diagnostics_noalloc": ([_P, ct.POINTER(Diag)], ct.c_int),
    "felbm_history": ([_P, ct.POINTER(Diag), ct.c_int64, ct.POINTER(ct.c_int64)], ct.c_int),
    "felbm_state_bytes": ([_P], ct.c_int64),
    "felbm_save_state": ([_P, ct.c_void_p, ct.c_int64], ct.c_int),
    "felbm_load_state": ([_P, ct.c_void_p, ct.c_int64], ct.c_int),
    "felbm_bind_stream": ([_P, ct.c_void_p], ct.c_int),
    "felbm_kernel_timing": ([_P, ct.c_int32], ct.c_int),
    "felbm_kernel_stats": ([_P, ct.POINTER(KStat), ct.c_int32, ct.POINTER(ct.c_int32)], ct.c_int),
    "felbm_mesh_info": ([_P, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64),
                         ct.POINTER(ct.c_int64)], ct.c_int),
    "felbm_validate_mesh": ([ct.c_int64, _D, ct.c_int64, _I, ct.c_int64, _I, ct.c_double, ct.c_char_p, ct.c_int32],
                            ct.c_int),
    "felbm_forward_ckpt": ([_P, ct.c_int64, ct.c_int64], ct.c_int),
    "felbm_adjoint_run": ([_P, ct.POINTER(ct.c_int64)], ct.c_int),
    "felbm_set_residual_sampling": ([_P, ct.c_int64], ct.c_int),
    "felbm_backward": ([_P, ct.c_void_p, ct.c_void_p], ct.c_int),
    "felbm_backward_host": ([_P, _D, _D], ct.c_int),
    "felbm_lumped_mass": ([_P, _D], ct.c_int),
    "felbm_backward_full": ([_P, _D, _D, _D, _D], ct.c_int),
    "felbm_destroy": ([_P], None),
    # 3-D (include/felbm3d.h)
    "felbm3d_create": ([ct.POINTER(Params), ct.POINTER(_P)], ct.c_int),
    "felbm3d_last_error": ([_P], ct.c_char_p),
    "felbm3d_upload_mesh": ([_P, ct.c_int64, _D, ct.c_int64, _I, ct.c_int64, _I, ct.c_double, ct.c_double], ct.c_int),
    "felbm3d_set_wetting": ([_P, _D], ct.c_int),
    "felbm3d_init": ([_P, _D, _D, _D], ct.c_int),
    "felbm3d_step": ([_P, ct.c_int64], ct.c_int),
    "felbm3d_step_async": ([_P, ct.c_int64], ct.c_int),
    "felbm3d_read": ([_P, ct.c_int32, _D], ct.c_int),
    "felbm3d_read_populations": ([_P, _D], ct.c_int),
    "felbm3d_diagnostics": ([_P, ct.POINTER(Diag)], ct.c_int),
    "felbm3d_bind_stream": ([_P, ct.c_void_p], ct.c_int),
    "felbm3d_kernel_timing": ([_P, ct.c_int32], ct.c_int),
    "felbm3d_kernel_stats": ([_P, ct.POINTER(KStat), ct.c_int32, ct.POINTER(ct.c_int32)], ct.c_int),
    "felbm3d_mesh_info": ([_P, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64),
                           ct.POINTER(ct.c_int64)], ct.c_int),
    "felbm3d_destroy": ([_P], None),
}


def library_path() -> str:
    return _LIB_PATH


def load_library() -> ct.CDLL:
    """Load libfelbm.so from the package tree; raises if it was not built."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch ships its own copy of the HIP
        # runtime under the same soname, and whichever is loaded first serves
        # both.  Loading torch's first keeps torch usable and makes torch
        # streams valid handles for felbm_bind_stream.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_1708_04678_amd.build)")
        lib = ct.CDLL(_LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def validate_mesh(xy, tri, wall_edges, period_x=0.0):
    """Host-side mesh validation (no device needed); returns (code, message)."""
    lib = load_library()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    we = np.ascontiguousarray(wall_edges, dtype=np.int32).reshape(-1, 2)
    msg = ct.create_string_buffer(256)
    rc = lib.felbm_validate_mesh(xy.shape[0], xy.ctypes.data_as(_D), tri.shape[0], tri.ctypes.data_as(_I),
                                 we.shape[0], we.ctypes.data_as(_I), float(period_x), msg, 256)
    return rc, msg.value.decode()


def _dptr(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


class Context:
    """One FE-LBM simulation on the current HIP device (see include/felbm.h)."""

    def __init__(self, *, sigma, xi, mobility, rho_l, rho_v, nu_l, nu_v, dt, precision="fp64",
                 solver_sweeps=28, lambda_min=0.0, lambda_max=0.0, kernels="auto", force_scheme="mixed"):
        lib = load_library()
        prec = {"fp64": FP64, "fp32": FP32}[precision] if isinstance(precision, str) else int(precision)
        kern = {"auto": 0, "global": 1}[kernels] if isinstance(kernels, str) else int(kernels)
        forces = ({"mixed": 0, "nodal": 1, "nodal_collide": 2}[force_scheme] if isinstance(force_scheme, str)
                  else int(force_scheme))
        self.params = Params(sigma, xi, mobility, rho_l, rho_v, nu_l, nu_v, dt, prec, int(solver_sweeps),
                             lambda_min, lambda_max, kern, forces)
        h = _P()
        rc = lib.felbm_create(ct.byref(self.params), ct.byref(h))
        if rc != 0:
            raise FelbmError(rc, lib.felbm_last_error(None).decode())
        self._lib, self._h = lib, h
        self.n_nodes = self.n_tris = 0

    def _check(self, rc):
        if rc != 0:
            raise FelbmError(rc, self._lib.felbm_last_error(self._h).decode())

    # -- setup -------------------------------------------------------------
    def upload_mesh(self, xy, tri, wall_edges, period_x=0.0):
        xy = _f64(xy)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        we = np.ascontiguousarray(wall_edges, dtype=np.int32).reshape(-1, 2)
        self._check(self._lib.felbm_upload_mesh(self._h, xy.shape[0], _dptr(xy), tri.shape[0], tri.ctypes.data_as(_I),
                                                we.shape[0], we.ctypes.data_as(_I), float(period_x)))
        self.n_nodes, self.n_tris = xy.shape[0], tri.shape[0]

    def set_wetting(self, omega_c):
        om = _f64(omega_c, (self.n_nodes,))
        self._check(self._lib.felbm_set_wetting(self._h, _dptr(om)))

    def set_wetting_device(self, omega_dev_ptr):
        """Device pointer (int) to N doubles, caller node order."""
        self._check(self._lib.felbm_set_wetting_device(self._h, ct.c_void_p(omega_dev_ptr)))

    def init(self, C, u=None, p=None):
        C = _f64(C, (self.n_nodes,))
        u = None if u is None else _f64(u, (self.n_nodes, 2))
        p = None if p is None else _f64(p, (self.n_nodes,))
        self._check(self._lib.felbm_init(self._h, _dptr(C), None if u is None else _dptr(u),
                                         None if p is None else _dptr(p)))

    # -- stepping ----------------------------------------------------------
    def step(self, n=1):
        self._check(self._lib.felbm_step(self._h, int(n)))

    def step_async(self, n=1):
        self._check(self._lib.felbm_step_async(self._h, int(n)))

    def step_debug(self):
        N = self.n_nodes
        hat, rhs, d = (np.empty((18, N)) for _ in range(3))
        self._check(self._lib.felbm_step_debug(self._h, _dptr(hat), _dptr(rhs), _dptr(d)))
        return hat, rhs, d

    # -- read back ---------------------------------------------------------
    def read(self, field):
        fid = FIELDS[field] if isinstance(field, str) else int(field)
        out = np.empty(self.n_tris if fid == FIELDS["LAPMU"] else self.n_nodes)
        self._check(self._lib.felbm_read(self._h, fid, _dptr(out)))
        return out

    def read_device(self, field, out_dev_ptr):
        """A nodal field into a device buffer of N doubles (caller order), queued on the bound stream."""
        fid = FIELDS[field] if isinstance(field, str) else int(field)
        self._check(self._lib.felbm_read_device(self._h, fid, ct.c_void_p(out_dev_ptr)))

    def read_populations(self):
        out = np.empty((18, self.n_nodes))
        self._check(self._lib.felbm_read_populations(self._h, _dptr(out)))
        return out

    def set_band(self, xc, yc, R, w):
        self._check(self._lib.felbm_set_band(self._h, xc, yc, R, w))

    def diagnostics(self):
        d = Diag()
        self._check(self._lib.felbm_diagnostics(self._h, ct.byref(d)))
        return d.as_dict()

    def diagnostics_noalloc(self):
        """felbm_diagnostics without device allocation (fixed per-device scratch)."""
        d = Diag()
        self._check(self._lib.felbm_diagnostics_noalloc(self._h, ct.byref(d)))
        return d.as_dict()

    def set_residual_sampling(self, every):
        """Sample the solve's relative residual every `every` steps (0 = off)."""
        self._check(self._lib.felbm_set_residual_sampling(self._h, int(every)))

    def history(self, max_entries=16384):
        buf = (Diag * max_entries)()
        n = ct.c_int64()
        self._check(self._lib.felbm_history(self._h, buf, max_entries, ct.byref(n)))
        return [buf[k].as_dict() for k in range(n.value)]

    def save_state(self) -> bytes:
        nb = self._lib.felbm_state_bytes(self._h)
        buf = ct.create_string_buffer(nb)
        self._check(self._lib.felbm_save_state(self._h, buf, nb))
        return buf.raw

    def load_state(self, data: bytes):
        buf = ct.create_string_buffer(data, len(data))
        self._check(self._lib.felbm_load_state(self._h, buf, len(data)))

    def bind_stream(self, stream_handle):
        """stream_handle: a hipStream_t as an int (e.g. torch.cuda.current_stream().cuda_stream) or None."""
        self._check(self._lib.felbm_bind_stream(self._h, None if stream_handle is None else ct.c_void_p(stream_handle)))

    def kernel_timing(self, enable=True):
        self._check(self._lib.felbm_kernel_timing(self._h, 1 if enable else 0))

    def kernel_stats(self):
        buf = (KStat * 32)()
        n = ct.c_int32()
        self._check(self._lib.felbm_kernel_stats(self._h, buf, 32, ct.byref(n)))
        return [{"name": buf[k].name.decode(), "launches": buf[k].launches, "total_ms": buf[k].total_ms,
                 "bytes_per_launch": buf[k].bytes_per_launch} for k in range(n.value)]

    # -- adjoint ---------------------------------------------------------------
    def forward_ckpt(self, n_steps, every):
        self._check(self._lib.felbm_forward_ckpt(self._h, int(n_steps), int(every)))

    def adjoint_run(self):
        """Identifier of the forward_ckpt run that backward would reverse (0 = none)."""
        v = ct.c_int64()
        self._check(self._lib.felbm_adjoint_run(self._h, ct.byref(v)))
        return v.value

    def backward(self, dL_dC_dev_ptr, dL_domega_dev_ptr):
        """Device pointers (ints) to N doubles each, caller node order."""
        self._check(self._lib.felbm_backward(self._h, ct.c_void_p(dL_dC_dev_ptr), ct.c_void_p(dL_domega_dev_ptr)))

    def backward_host(self, dL_dC):
        g = _f64(dL_dC, (self.n_nodes,))
        out = np.empty(self.n_nodes)
        self._check(self._lib.felbm_backward_host(self._h, _dptr(g), _dptr(out)))
        return out

    def backward_full(self, dL_dpsi=None, dL_dC=None, want_dpsi0=True):
        N = self.n_nodes
        dpsi = None if dL_dpsi is None else _f64(dL_dpsi, (18, N))
        dC = None if dL_dC is None else _f64(dL_dC, (N,))
        gom = np.empty(N)
        d0 = np.empty((18, N)) if want_dpsi0 else None
        self._check(self._lib.felbm_backward_full(self._h, None if dpsi is None else _dptr(dpsi),
                                                  None if dC is None else _dptr(dC), _dptr(gom),
                                                  None if d0 is None else _dptr(d0)))
        return gom, d0

    def lumped_mass(self):
        out = np.empty(self.n_nodes)
        self._check(self._lib.felbm_lumped_mass(self._h, _dptr(out)))
        return out

    def mesh_info(self):
        v = [ct.c_int64() for _ in range(4)]
        self._check(self._lib.felbm_mesh_info(self._h, *[ct.byref(x) for x in v]))
        return dict(zip(["n_nodes", "n_tris", "n_wall_edges", "mass_offdiag_nnz"], [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.felbm_destroy(self._h)
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


class Context3D:
    """One 3-D FE-LBM simulation (D3Q19 on linear tetrahedra) on the current
    HIP device (see include/felbm3d.h).  Marshalling only."""

    def __init__(self, *, sigma, xi, mobility, rho_l, rho_v, nu_l, nu_v, dt, precision="fp64", solver_sweeps=28,
                 lambda_min=0.0, lambda_max=0.0):
        lib = load_library()
        prec = {"fp64": FP64, "fp32": FP32}[precision] if isinstance(precision, str) else int(precision)
        self.params = Params(sigma, xi, mobility, rho_l, rho_v, nu_l, nu_v, dt, prec, int(solver_sweeps),
                             lambda_min, lambda_max, 0, 0)
        h = _P()
        rc = lib.felbm3d_create(ct.byref(self.params), ct.byref(h))
        if rc != 0:
            raise FelbmError(rc, lib.felbm3d_last_error(None).decode())
        self._lib, self._h = lib, h
        self.n_nodes = self.n_tets = 0

    def _check(self, rc):
        if rc != 0:
            raise FelbmError(rc, self._lib.felbm3d_last_error(self._h).decode())

    def upload_mesh(self, xyz, tet, wall_faces, period=(0.0, 0.0)):
        xyz = _f64(xyz)
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        wf = np.ascontiguousarray(wall_faces, dtype=np.int32).reshape(-1, 3)
        self._check(self._lib.felbm3d_upload_mesh(self._h, xyz.shape[0], _dptr(xyz), tet.shape[0],
                                                  tet.ctypes.data_as(_I), wf.shape[0], wf.ctypes.data_as(_I),
                                                  float(period[0]), float(period[1])))
        self.n_nodes, self.n_tets = xyz.shape[0], tet.shape[0]

    def set_wetting(self, omega_c):
        om = _f64(omega_c, (self.n_nodes,))
        self._check(self._lib.felbm3d_set_wetting(self._h, _dptr(om)))

    def init(self, C, u=None, p=None):
        C = _f64(C, (self.n_nodes,))
        u = None if u is None else _f64(u, (self.n_nodes, 3))
        p = None if p is None else _f64(p, (self.n_nodes,))
        self._check(self._lib.felbm3d_init(self._h, _dptr(C), None if u is None else _dptr(u),
                                           None if p is None else _dptr(p)))

    def step(self, n=1):
        self._check(self._lib.felbm3d_step(self._h, int(n)))

    def step_async(self, n=1):
        self._check(self._lib.felbm3d_step_async(self._h, int(n)))

    def read(self, field):
        fid = FIELDS[field] if isinstance(field, str) else int(field)
        out = np.empty(self.n_tets if fid == FIELDS["LAPMU"] else self.n_nodes)
        self._check(self._lib.felbm3d_read(self._h, fid, _dptr(out)))
        return out

    def read_populations(self):
        out = np.empty((38, self.n_nodes))
        self._check(self._lib.felbm3d_read_populations(self._h, _dptr(out)))
        return out

    def diagnostics(self):
        d = Diag()
        self._check(self._lib.felbm3d_diagnostics(self._h, ct.byref(d)))
        return d.as_dict()

    def bind_stream(self, stream_handle):
        self._check(self._lib.felbm3d_bind_stream(self._h, None if stream_handle is None else ct.c_void_p(stream_handle)))

    def kernel_timing(self, enable=True):
        self._check(self._lib.felbm3d_kernel_timing(self._h, 1 if enable else 0))

    def kernel_stats(self):
        buf = (KStat * 32)()
        n = ct.c_int32()
        self._check(self._lib.felbm3d_kernel_stats(self._h, buf, 32, ct.byref(n)))
        return [{"name": buf[k].name.decode(), "launches": buf[k].launches, "total_ms": buf[k].total_ms,
                 "bytes_per_launch": buf[k].bytes_per_launch} for k in range(n.value)]

    def mesh_info(self):
        v = [ct.c_int64() for _ in range(4)]
        self._check(self._lib.felbm3d_mesh_info(self._h, *[ct.byref(x) for x in v]))
        return dict(zip(["n_nodes", "n_tets", "n_wall_faces", "mass_offdiag_nnz"], [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.felbm3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
