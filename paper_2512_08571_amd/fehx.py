"""Python binding of libfehx (argument marshalling only).

Every numerical step runs in the HIP library; this module converts Python /
NumPy / torch arguments to the C-ABI of include/fe_hx.h and raises on any
non-zero status.  torch is used only for device memory and streams.  If the
library has not been built, loading fails with a RuntimeError: there is no
fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfehx.so")

FE_F64, FE_F32, FE_BF16 = 0, 1, 2
FE_MASS_LUMPED, FE_MASS_CONSISTENT = 0, 1
TILE_CANDIDATES = 8       # FE_TILE_CANDIDATES: entries of the autotuner's candidate arrays
PREC = {"f64": FE_F64, "f32": FE_F32, "bf16": FE_BF16}

EXPORTS = ["fe_abi_version", "fe_last_error", "fe_mesh_create", "fe_mesh_destroy", "fe_mesh_query",
           "fe_mesh_cell_dofs", "fe_mesh_quad_points", "fe_mesh_lumped_mass", "fe_set_potential",
           "fe_set_projectors", "fe_projector_entries", "fe_apply_H", "fe_cheb_filter", "fe_lanczos",
           "fe_rayleigh_ritz", "fe_chfsi", "fe_batch_apply", "fe_set_tile", "fe_get_tile", "fe_autotune",
           "fe_filter_graph_create", "fe_filter_graph_launch", "fe_filter_graph_destroy",
           "fe_server_create", "fe_server_submit", "fe_server_progress", "fe_server_drain", "fe_server_status",
           "fe_server_stats", "fe_server_destroy", "fe_apply_M", "fe_set_mass", "fe_apply_H_noalloc",
           "fe_mesh_set_geometry", "fe_server_pool_stats", "fe_server_set_work_cap"]


class MeshDesc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_double * 9), ("ncell", ctypes.c_int32 * 3),
                ("degree", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("periodic", ctypes.c_int32 * 3), ("kpoint", ctypes.c_double * 3),
                ("is_complex", ctypes.c_int32), ("device", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("mesh", ctypes.c_void_p), ("kind", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("nvec", ctypes.c_int64),
                ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int64), ("lam", ctypes.c_void_p),
                ("degree", ctypes.c_int32), ("lam_min", ctypes.c_double), ("lam_T", ctypes.c_double),
                ("lam_max", ctypes.c_double)]


class Projector(ctypes.Structure):
    _fields_ = [("atom", ctypes.c_int32), ("l", ctypes.c_int32), ("m", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("rc", ctypes.c_double), ("h", ctypes.c_double)]


_lib = None
c_p = ctypes.c_void_p
i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


def lib():
    """Load libfehx.so (once); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (python -m paper_2512_08571_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        L.fe_abi_version.restype = i32
        L.fe_last_error.restype = ctypes.c_char_p
        sig = {
            "fe_mesh_create": [ctypes.POINTER(MeshDesc), ctypes.POINTER(c_p)],
            "fe_mesh_destroy": [c_p],
            "fe_mesh_query": [c_p, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
            "fe_mesh_cell_dofs": [c_p, i64, i64, c_p],
            "fe_mesh_quad_points": [c_p, c_p],
            "fe_mesh_lumped_mass": [c_p, c_p],
            "fe_set_potential": [c_p, c_p, c_p],
            "fe_mesh_set_geometry": [c_p, c_p],
            "fe_set_projectors": [c_p, i32, c_p, i32, c_p],
            "fe_projector_entries": [c_p, ctypes.POINTER(i64), c_p, c_p, c_p],
            "fe_apply_H": [c_p, c_p, i64, c_p, i64, i64, i32, c_p],
            "fe_apply_H_noalloc": [c_p, c_p, i64, c_p, i64, i64, i32, c_p],
            "fe_cheb_filter": [c_p, c_p, i64, c_p, i64, i32, dbl, dbl, dbl, i32, c_p],
            "fe_lanczos": [c_p, c_p, i32, c_p, c_p],
            "fe_rayleigh_ritz": [c_p, c_p, i64, i64, c_p, c_p],
            "fe_chfsi": [c_p, c_p, i64, i64, c_p, i32, i32, i32, i32, c_p, c_p, c_p],
            "fe_batch_apply": [i32, c_p, c_p, c_p, c_p, c_p, c_p, i32, c_p],
            "fe_set_tile": [c_p, i32, i32, i32],
            "fe_filter_graph_create": [c_p, c_p, i64, c_p, i64, i32, dbl, dbl, dbl, i32, ctypes.POINTER(c_p)],
            "fe_filter_graph_launch": [c_p, c_p],
            "fe_filter_graph_destroy": [c_p],
            "fe_server_create": [i32, i64, i32, ctypes.POINTER(c_p)],
            "fe_server_submit": [c_p, ctypes.POINTER(Request), ctypes.POINTER(i64)],
            "fe_server_progress": [c_p, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
            "fe_server_drain": [c_p],
            "fe_server_status": [c_p, i64, ctypes.POINTER(i32), c_p, ctypes.POINTER(i32)],
            "fe_server_stats": [c_p, ctypes.POINTER(i64), ctypes.POINTER(i64)],
            "fe_server_pool_stats": [c_p, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
            "fe_server_set_work_cap": [c_p, i64],
            "fe_server_destroy": [c_p],
            "fe_apply_M": [c_p, c_p, i64, c_p, i64, i64, i32, c_p],
            "fe_set_mass": [c_p, i32],
            "fe_get_tile": [c_p, i32, i32, ctypes.POINTER(i32)],
            "fe_autotune": [c_p, i32, i32, i64, i32, ctypes.POINTER(i32), c_p, c_p, ctypes.POINTER(i32)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        _lib = L
    return _lib


class FeError(RuntimeError):
    def __init__(self, fn, code):
        msg = lib().fe_last_error().decode(errors="replace")
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


def _check(fn, code):
    if code != 0:
        raise FeError(fn, code)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dtypes(prec, cplx):
    """torch element type(s) a block of this precision has (real / complex mesh)."""
    import torch
    if prec == "f64":
        return torch.complex128 if cplx else torch.float64
    if prec == "f32":
        return torch.complex64 if cplx else torch.float32
    return torch.bfloat16


def _check_block(mesh, t, prec, name):
    """Validate a vector block for 'mesh' before any library call: element type
    of the precision (complex bf16 as [m, ld, 2] pairs), one row per DoF,
    row-major with unit vector stride, on the mesh's device."""
    if prec not in PREC:
        raise ValueError(f"unknown precision {prec!r}")
    want = _dtypes(prec, mesh.is_complex)
    if t.dtype != want:
        raise ValueError(f"{name}: dtype {t.dtype} does not match precision {prec!r} on a "
                         f"{'complex' if mesh.is_complex else 'real'} mesh (expected {want})")
    two = prec == "bf16" and mesh.is_complex
    if t.dim() != (3 if two else 2) or (two and t.shape[2] != 2):
        raise ValueError(f"{name}: expected a [ndofs, ld{', 2' if two else ''}] block, got shape {tuple(t.shape)}")
    if t.shape[0] != mesh.ndofs:
        raise ValueError(f"{name}: {t.shape[0]} rows, the mesh has {mesh.ndofs} DoFs")
    if t.device.type != "cuda" or t.device.index != mesh.device:
        raise ValueError(f"{name}: block on {t.device}, the mesh is on cuda:{mesh.device}")


def _check_nvec(n, nx, name="X"):
    if n is None:
        return nx
    n = int(n)
    if n < 0 or n > nx:
        raise ValueError(f"{name}: nvec {n} outside 0..{nx}")
    return n


def _check_vec(mesh, t, n, name, complex_ok=True):
    """A device FP64 vector (complex128 on complex meshes when complex_ok) with at least n entries."""
    import torch
    want = torch.complex128 if (mesh.is_complex and complex_ok) else torch.float64
    if t.dtype != want:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {want}")
    if not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{name}: needs a contiguous vector of at least {n} entries")
    if t.device.type != "cuda" or t.device.index != mesh.device:
        raise ValueError(f"{name}: vector on {t.device}, the mesh is on cuda:{mesh.device}")


def _block(t, cplx):
    """(pointer, ld in elements of the block's type, nvec) of a torch block [m, ld(,2)]."""
    if t.dim() == 3:                     # complex bf16 stored as [m, ld, 2]
        if t.shape[2] != 2 or t.stride(2) != 1 or t.stride(1) != 2:
            raise ValueError("complex bf16 blocks must be contiguous [m, ld, 2]")
        return t.data_ptr(), t.stride(0) // 2, t.shape[1]
    if t.stride(1) != 1:
        raise ValueError("vector blocks must be row-major with unit vector stride")
    return t.data_ptr(), t.stride(0), t.shape[1]


class Mesh:
    """A periodic FE mesh on one GPU with its operator data (libfehx handle)."""

    def __init__(self, lattice, ncell, degree, nq=None, kpoint=(0.0, 0.0, 0.0), is_complex=None, device=0,
                 periodic=(True, True, True)):
        L = lib()
        d = MeshDesc()
        A = np.asarray(lattice, float).reshape(9)
        d.lattice[:] = list(A)
        d.ncell[:] = [int(n) for n in ncell]
        d.degree = int(degree)
        d.nq = int(degree + 1 if nq is None else nq)
        d.periodic[:] = [int(bool(v)) for v in periodic]
        d.kpoint[:] = [float(v) for v in kpoint]
        k2 = float(np.dot(kpoint, kpoint))
        d.is_complex = int(bool(is_complex) or k2 > 0) if is_complex is not None else int(k2 > 0)
        d.device = int(device)
        h = c_p()
        _check("fe_mesh_create", L.fe_mesh_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.is_complex = bool(d.is_complex)
        self.degree, self.nq = d.degree, d.nq
        self.ncell = tuple(d.ncell)
        self.periodic = tuple(bool(v) for v in periodic)
        self.device = device
        q = [i64() for _ in range(4)]
        _check("fe_mesh_query", L.fe_mesh_query(h, *[ctypes.byref(v) for v in q]))
        self.ndofs, self.ncells, self.nq3 = q[0].value, q[1].value, q[2].value

    def close(self):
        if getattr(self, "_h", None):
            lib().fe_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def footprint(self):
        v = i64()
        _check("fe_mesh_query", lib().fe_mesh_query(self._h, None, None, None, ctypes.byref(v)))
        return v.value

    def cell_dofs(self, first=0, count=None):
        count = self.ncells - first if count is None else count
        out = np.empty((count, (self.degree + 1) ** 3), np.int32)
        _check("fe_mesh_cell_dofs", lib().fe_mesh_cell_dofs(self._h, first, count, out.ctypes.data))
        return out

    def quad_points(self):
        out = np.empty((self.ncells * self.nq3, 3))
        _check("fe_mesh_quad_points", lib().fe_mesh_quad_points(self._h, out.ctypes.data))
        return out

    def lumped_mass(self):
        out = np.empty(self.ndofs)
        _check("fe_mesh_lumped_mass", lib().fe_mesh_lumped_mass(self._h, out.ctypes.data))
        return out

    def set_geometry(self, vdisp=None):
        """Displace the periodic vertex grid ([N0 N1 N2, 3], vertex i + N0 (j + N1 k)):
        trilinear (distorted) cells; None restores the affine cells.  Clears the
        potential and the projectors."""
        if vdisp is None:
            _check("fe_mesh_set_geometry", lib().fe_mesh_set_geometry(self._h, None))
            return
        v = np.ascontiguousarray(vdisp, dtype=np.float64)
        if v.size != 3 * self.ncells:
            raise ValueError("vdisp must hold one 3-vector per vertex of the periodic grid")
        _check("fe_mesh_set_geometry", lib().fe_mesh_set_geometry(self._h, v.ctypes.data))

    def set_potential(self, vloc, vgga=None):
        v = np.ascontiguousarray(vloc, dtype=np.float64)
        g = None if vgga is None else np.ascontiguousarray(vgga, dtype=np.float64)
        if v.size != self.ncells * self.nq3 or (g is not None and g.size != 3 * v.size):
            raise ValueError("potential arrays must hold one value (three for V^G) per quadrature point")
        _check("fe_set_potential", lib().fe_set_potential(self._h, v.ctypes.data, None if g is None else g.ctypes.data))

    def set_projectors(self, positions, projectors):
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        arr = (Projector * max(len(projectors), 1))()
        for i, p in enumerate(projectors):
            arr[i] = Projector(int(p["atom"]), int(p["l"]), int(p["m"]), float(p["sigma"]), float(p["rc"]), float(p["h"]))
        _check("fe_set_projectors", lib().fe_set_projectors(self._h, len(pos), pos.ctypes.data, len(projectors),
                                                          ctypes.cast(arr, c_p)))

    def projector_entries(self):
        """(rows, cols, values) of the assembled projector matrix (host)."""
        n = i64()
        _check("fe_projector_entries", lib().fe_projector_entries(self._h, ctypes.byref(n), None, None, None))
        rows = np.empty(n.value, np.int32)
        cols = np.empty(n.value, np.int32)
        vals = np.empty(n.value * (2 if self.is_complex else 1))
        _check("fe_projector_entries", lib().fe_projector_entries(self._h, ctypes.byref(n), rows.ctypes.data,
                                                                cols.ctypes.data, vals.ctypes.data))
        if self.is_complex:
            vals = vals[0::2] + 1j * vals[1::2]
        return rows, cols, vals

    def apply(self, X, Y, prec="f64", stream=None, nvec=None):
        _check_block(self, X, prec, "X")
        _check_block(self, Y, prec, "Y")
        px, ldx, nx = _block(X, self.is_complex)
        py, ldy, ny = _block(Y, self.is_complex)
        n = _check_nvec(nvec, min(nx, ny))
        _check("fe_apply_H", lib().fe_apply_H(self._h, px, ldx, py, ldy, n, PREC[prec], _stream_ptr(stream)))

    def apply_noalloc(self, X, Y, prec="f64", stream=None, nvec=None):
        """Y = H X through fe_apply_H_noalloc (no device allocation; static scratch)."""
        _check_block(self, X, prec, "X")
        _check_block(self, Y, prec, "Y")
        px, ldx, nx = _block(X, self.is_complex)
        py, ldy, ny = _block(Y, self.is_complex)
        n = _check_nvec(nvec, min(nx, ny))
        _check("fe_apply_H_noalloc", lib().fe_apply_H_noalloc(self._h, px, ldx, py, ldy, n, PREC[prec],
                                                              _stream_ptr(stream)))

    def apply_mass(self, X, Y, prec="f64", stream=None, nvec=None):
        """Y = M X with the consistent mass matrix."""
        _check_block(self, X, prec, "X")
        _check_block(self, Y, prec, "Y")
        px, ldx, nx = _block(X, self.is_complex)
        py, ldy, ny = _block(Y, self.is_complex)
        n = _check_nvec(nvec, min(nx, ny))
        _check("fe_apply_M", lib().fe_apply_M(self._h, px, ldx, py, ldy, n, PREC[prec], _stream_ptr(stream)))

    def set_mass(self, kind):
        """'lumped' (M = D) or 'consistent' for the filter residual and Rayleigh-Ritz."""
        _check("fe_set_mass", lib().fe_set_mass(self._h, {"lumped": 0, "consistent": 1}[kind]))

    def cheb_filter(self, X, lam, degree, lmin, lT, lmax, inner="f32", stream=None):
        if inner not in PREC:
            raise ValueError(f"unknown inner precision {inner!r}")
        _check_block(self, X, "f64", "X")
        px, ldx, nx = _block(X, self.is_complex)
        _check_vec(self, lam, nx, "lam", complex_ok=False)
        _check("fe_cheb_filter", lib().fe_cheb_filter(self._h, px, ldx, lam.data_ptr(), nx, int(degree),
                                                      float(lmin), float(lT), float(lmax), PREC[inner],
                                                      _stream_ptr(stream)))

    def lanczos(self, v0, steps=10):
        _check_vec(self, v0, self.ndofs, "v0")
        theta = np.empty(steps)
        beta = dbl()
        _check("fe_lanczos", lib().fe_lanczos(self._h, v0.data_ptr(), int(steps), theta.ctypes.data, ctypes.byref(beta)))
        return theta, beta.value

    def rayleigh_ritz(self, X, ritz, stream=None):
        _check_block(self, X, "f64", "X")
        px, ldx, nx = _block(X, self.is_complex)
        _check_vec(self, ritz, nx, "ritz", complex_ok=False)
        _check("fe_rayleigh_ritz", lib().fe_rayleigh_ritz(self._h, px, ldx, nx, ritz.data_ptr(), _stream_ptr(stream)))

    def chfsi(self, X, v0, outer=3, degree=40, lanczos_steps=10, inner="f64", stream=None):
        """Lanczos bounds, then 'outer' filter + Rayleigh-Ritz passes; returns (ritz, bounds)."""
        if inner not in PREC:
            raise ValueError(f"unknown inner precision {inner!r}")
        _check_block(self, X, "f64", "X")
        _check_vec(self, v0, self.ndofs, "v0")
        px, ldx, nx = _block(X, self.is_complex)
        ritz = np.empty(nx)
        bounds = np.empty((max(outer, 1), 3))
        _check("fe_chfsi", lib().fe_chfsi(self._h, px, ldx, nx, v0.data_ptr(), int(outer), int(degree),
                                          int(lanczos_steps), PREC[inner], ritz.ctypes.data, bounds.ctypes.data,
                                          _stream_ptr(stream)))
        return ritz, bounds[:outer]

    def set_tile(self, prec, vt, kind=0):
        _check("fe_set_tile", lib().fe_set_tile(self._h, PREC[prec], int(kind), int(vt)))

    def get_tile(self, prec, kind=0):
        v = i32()
        _check("fe_get_tile", lib().fe_get_tile(self._h, PREC[prec], int(kind), ctypes.byref(v)))
        return v.value

    def autotune(self, prec, nvec, kind=0, reps=3):
        """Time every vector tile; keep the fastest.  Returns (best, {vt: ms})."""
        best, nc = i32(), i32()
        vts = np.zeros(TILE_CANDIDATES, np.int32)
        ms = np.zeros(TILE_CANDIDATES)
        _check("fe_autotune", lib().fe_autotune(self._h, PREC[prec], int(kind), int(nvec), int(reps),
                                                ctypes.byref(best), vts.ctypes.data, ms.ctypes.data,
                                                ctypes.byref(nc)))
        return best.value, {int(vts[i]): float(ms[i]) for i in range(nc.value)}

    def filter_graph(self, X, lam, degree, lmin, lT, lmax, inner="f32"):
        """Capture one filter pass on (X, lam) as a replayable graph."""
        return FilterGraph(self, X, lam, degree, lmin, lT, lmax, inner)


class FilterGraph:
    """A captured fe_cheb_filter pass; launch() replays it on a stream."""

    def __init__(self, mesh, X, lam, degree, lmin, lT, lmax, inner):
        if inner not in PREC:
            raise ValueError(f"unknown inner precision {inner!r}")
        _check_block(mesh, X, "f64", "X")
        px, ldx, nx = _block(X, mesh.is_complex)
        _check_vec(mesh, lam, nx, "lam", complex_ok=False)
        h = c_p()
        _check("fe_filter_graph_create", lib().fe_filter_graph_create(mesh._h, px, ldx, lam.data_ptr(), nx, int(degree),
                                                                      float(lmin), float(lT), float(lmax),
                                                                      PREC[inner], ctypes.byref(h)))
        self._h, self.mesh = h, mesh

    def launch(self, stream=None):
        _check("fe_filter_graph_launch", lib().fe_filter_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().fe_filter_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over resident meshes (fe_server_*)."""

    QUEUED, ACTIVE, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, hbm_budget, max_active=16, device=0):
        h = c_p()
        _check("fe_server_create", lib().fe_server_create(int(device), int(hbm_budget), int(max_active),
                                                          ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self._meshes = []          # the server counts their bytes until it is destroyed

    def _submit(self, req, keep):
        rid = i64()
        _check("fe_server_submit", lib().fe_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._keep[rid.value] = keep
        if not any(m is keep[0] for m in self._meshes):
            self._meshes.append(keep[0])
        return rid.value

    def submit_apply(self, mesh, X, Y, prec="f64"):
        _check_block(mesh, X, prec, "X")
        _check_block(mesh, Y, prec, "Y")
        px, ldx, nx = _block(X, mesh.is_complex)
        py, ldy, _ = _block(Y, mesh.is_complex)
        r = Request(mesh._h.value, 0, PREC[prec], px, ldx, nx, py, ldy, None, 0, 0.0, 0.0, 0.0)
        return self._submit(r, (mesh, X, Y))

    def submit_filter(self, mesh, X, lam, degree, lmin, lT, lmax, inner="f32"):
        if inner not in PREC:
            raise ValueError(f"unknown inner precision {inner!r}")
        _check_block(mesh, X, "f64", "X")
        px, ldx, nx = _block(X, mesh.is_complex)
        _check_vec(mesh, lam, nx, "lam", complex_ok=False)
        r = Request(mesh._h.value, 1, PREC[inner], px, ldx, nx, None, 0, lam.data_ptr(), int(degree),
                    float(lmin), float(lT), float(lmax))
        return self._submit(r, (mesh, X, lam))

    def progress(self, block=False):
        a, q = i32(), i32()
        _check("fe_server_progress", lib().fe_server_progress(self._h, int(bool(block)), ctypes.byref(a),
                                                              ctypes.byref(q)))
        return a.value, q.value

    def drain(self):
        _check("fe_server_drain", lib().fe_server_drain(self._h))

    def status(self, rid):
        """(state, (t_submit, t_admit, t_done), status code)."""
        st, err = i32(), i32()
        t = np.zeros(3)
        _check("fe_server_status", lib().fe_server_status(self._h, int(rid), ctypes.byref(st), t.ctypes.data,
                                                          ctypes.byref(err)))
        return st.value, tuple(t), err.value

    def stats(self):
        t, b = i64(), i64()
        _check("fe_server_stats", lib().fe_server_stats(self._h, ctypes.byref(t), ctypes.byref(b)))
        return t.value, b.value

    def set_work_cap(self, cap):
        """Stop admitting into a non-empty batch past 'cap' DoF x real lanes per step (0: no cap)."""
        _check("fe_server_set_work_cap", lib().fe_server_set_work_cap(self._h, int(cap)))

    def pool_stats(self):
        """(allocations, frees, idle bytes) of the request workspace pool."""
        a, f, b = i64(), i64(), i64()
        _check("fe_server_pool_stats", lib().fe_server_pool_stats(self._h, ctypes.byref(a), ctypes.byref(f),
                                                                  ctypes.byref(b)))
        return a.value, f.value, b.value

    def release(self, rid):
        """Drop the Python references kept for a finished request."""
        self._keep.pop(rid, None)

    def close(self):
        if getattr(self, "_h", None):
            lib().fe_server_destroy(self._h)
            self._h = None
            self._keep.clear()
            self._meshes = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_apply(meshes, Xs, Ys, prec="f64", stream=None, nvecs=None):
    """Y_i = H_i X_i for several meshes in batched persistent launches."""
    n = len(meshes)
    hs = (c_p * n)(*[m._h for m in meshes])
    px, lx, py, ly, nv = [], [], [], [], []
    if not (len(Xs) == n and len(Ys) == n):
        raise ValueError("one X and one Y block per mesh")
    for i, (m, X, Y) in enumerate(zip(meshes, Xs, Ys)):
        _check_block(m, X, prec, f"X[{i}]")
        _check_block(m, Y, prec, f"Y[{i}]")
        a, l1, n1 = _block(X, m.is_complex)
        b, l2, n2 = _block(Y, m.is_complex)
        px.append(a); lx.append(l1); py.append(b); ly.append(l2)
        nv.append(_check_nvec(None if nvecs is None else nvecs[i], min(n1, n2), f"X[{i}]"))
    arr = lambda t, v: (t * n)(*v)
    _check("fe_batch_apply", lib().fe_batch_apply(n, hs, arr(c_p, px), arr(i64, lx), arr(c_p, py), arr(i64, ly),
                                                  arr(i64, nv), PREC[prec], _stream_ptr(stream)))


def abi_version():
    return lib().fe_abi_version()
