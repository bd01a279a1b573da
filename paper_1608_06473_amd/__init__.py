"""MI355X (gfx950) two-scale surrogate-stencil library: Python binding.

Thin ctypes binding of ``libtwoscale.so`` (C ABI declared in
``include/twoscale.h``).  The functions keep the C names and only marshal
arguments: device vectors are torch tensors on ``cuda`` (their data pointers
are passed), streams are torch streams.  Every computation runs in the HIP
library; importing this module fails loudly if the library is missing.

Method: Bauer et al., "A two-scale approach for efficient on-the-fly operator
assembly in massively parallel high performance multigrid codes" (arXiv
1608.06473): P1 finite elements on refined macro tetrahedra of a spherical
shell, volume stencils from surrogate polynomials (Sec. 3), multigrid
(Sec. 4 introduction).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtwoscale.so")

TS_OK, TS_EINVAL, TS_ENOMEM, TS_EHIP, TS_ENOCONV, TS_ENONFINITE = range(6)
TS_GEOM_SHELL, TS_GEOM_AFFINE = 0, 1
TS_IFEM, TS_LSQP, TS_IPOLY, TS_LSQP_SYM, TS_CONS = 0, 1, 2, 3, 4
TS_CENTER_POLY, TS_CENTER_ROWSUM = 0, 1
TS_F64, TS_F32, TS_F16W = 0, 1, 2
TS_RHS_MANUFACTURED, TS_RHS_BUMPS, TS_RHS_ONE = 0, 1, 2
TS_MAX_HIST = 256

ERROR_NAMES = {1: "TS_EINVAL", 2: "TS_ENOMEM", 3: "TS_EHIP", 4: "TS_ENOCONV", 5: "TS_ENONFINITE"}


class TSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, str(code)), msg))
        self.code = code


class ts_layout_info(C.Structure):
    _fields_ = [("level", C.c_int), ("N", C.c_int), ("n_macros", C.c_int64),
                ("block_size", C.c_int64), ("vec_len", C.c_int64), ("n_unique", C.c_int64),
                ("n_free", C.c_int64), ("n_volume", C.c_int64)]


class ts_op_params(C.Structure):
    _fields_ = [("method", C.c_int), ("q", C.c_int), ("sample_j", C.c_int), ("center", C.c_int),
                ("fallback_tol", C.c_double), ("face_surrogate", C.c_int),
                ("coarse_from_finest", C.c_int)]


class ts_solve_params(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("max_cycles", C.c_int),
                ("precision", C.c_int), ("rtol", C.c_double), ("diverge_window", C.c_int),
                ("dd", C.c_int)]


class ts_solve_info(C.Structure):
    _fields_ = [("cycles", C.c_int), ("status", C.c_int), ("rel_residual", C.c_double),
                ("n_hist", C.c_int), ("hist", C.c_double * TS_MAX_HIST)]


_SIGS = {
    "ts_last_error": (C.c_char_p, []),
    "ts_mesh_create": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int, C.c_void_p]),
    "ts_mesh_destroy": (C.c_int, [C.c_void_p]),
    "ts_mesh_check_shell": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double]),
    "ts_mesh_set_vertices": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ts_solver_set_vertices": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_mesh_create_like": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_layout": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "ts_canon_to_block": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_block_to_canon": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_node_coords": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ts_rhs": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ts_op_create": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_op_destroy": (C.c_int, [C.c_void_p]),
    "ts_op_coeffs_export": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    "ts_op_coeffs_import": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    "ts_op_macro_flags": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    "ts_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_apply_volume": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_residual": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p]),
    "ts_smooth": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                            C.c_void_p]),
    "ts_restrict": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_prolongate_add": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "ts_norm2": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_norm2_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "ts_solver_create": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ts_solver_destroy": (C.c_int, [C.c_void_p]),
    "ts_vcycle": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_solve_begin": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_solve_step": (C.c_int, [C.c_void_p]),
    "ts_solve_query": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ts_solve_batch_step": (C.c_int, [C.c_void_p, C.c_int]),
    "ts_device_bytes": (C.c_int, [C.c_void_p]),
}

EXPORTED = sorted(_SIGS)
_lib = None


def lib():
    """Load libtwoscale.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtwoscale.so is not built: run __graft_entry__.build() or "
                              "python paper_1608_06473_amd/build.py")
        # PyTorch supplies the device memory and streams; its HIP runtime must
        # be initialised before the library makes the first HIP call
        import torch
        torch.cuda.is_available()
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def ts_last_error():
    return lib().ts_last_error().decode()


def _check(rc):
    if rc != TS_OK:
        raise TSError(rc, ts_last_error())
    return rc


def _ptr(t):
    """Device (or host numpy) data pointer of a tensor/array; None passes NULL."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


def _stream(s):
    """A torch stream, a raw hipStream_t value (int) or None (torch's current)."""
    if isinstance(s, int):
        return C.c_void_p(s)
    if s is None:
        import torch
        s = torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ----------------------------------------------------------------- C names

def ts_mesh_create(vtx, tet, geom=TS_GEOM_SHELL):
    vtx = np.ascontiguousarray(vtx, dtype=np.float64)
    tet = np.ascontiguousarray(tet, dtype=np.int64)
    h = C.c_void_p()
    _check(lib().ts_mesh_create(_ptr(vtx), vtx.shape[0], _ptr(tet), tet.shape[0], geom,
                                C.byref(h)))
    return h


def ts_mesh_destroy(h):
    return _check(lib().ts_mesh_destroy(h))


def ts_mesh_check_shell(h, r_in, r_out, tol=1e-12):
    return _check(lib().ts_mesh_check_shell(h, r_in, r_out, tol))


def ts_mesh_create_like(like, vtx):
    v = np.ascontiguousarray(vtx, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().ts_mesh_create_like(like, v.ctypes.data_as(C.c_void_p), C.byref(h)))
    return h


def ts_mesh_set_vertices(h, vtx):
    v = np.ascontiguousarray(vtx, dtype=np.float64)
    return _check(lib().ts_mesh_set_vertices(h, v.ctypes.data_as(C.c_void_p)))


def ts_solver_set_vertices(sv, vtx, stream=None):
    v = np.ascontiguousarray(vtx, dtype=np.float64)
    return _check(lib().ts_solver_set_vertices(sv, v.ctypes.data_as(C.c_void_p), _stream(stream)))


def ts_layout(mesh, level):
    info = ts_layout_info()
    _check(lib().ts_layout(mesh, level, C.byref(info)))
    return info


def ts_canon_to_block(mesh, level, canon, block, stream=None):
    return _check(lib().ts_canon_to_block(mesh, level, _ptr(canon), _ptr(block), _stream(stream)))


def ts_block_to_canon(mesh, level, block, canon, stream=None):
    return _check(lib().ts_block_to_canon(mesh, level, _ptr(block), _ptr(canon), _stream(stream)))


def ts_node_coords(mesh, level, xyz, stream=None):
    return _check(lib().ts_node_coords(mesh, level, _ptr(xyz), _stream(stream)))


def ts_rhs(mesh, level, kind, params, f, stream=None):
    par = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    return _check(lib().ts_rhs(mesh, level, kind, _ptr(par) if par.size else None, par.size,
                               _ptr(f), _stream(stream)))


def ts_op_create(mesh, max_level, method=TS_LSQP, q=2, sample_j=2, center=TS_CENTER_POLY,
                 fallback_tol=0.0, stream=None, face_surrogate=False, coarse_from_finest=False):
    p = ts_op_params(method, q, sample_j, center, fallback_tol, 1 if face_surrogate else 0,
                     1 if coarse_from_finest else 0)
    h = C.c_void_p()
    _check(lib().ts_op_create(mesh, max_level, C.byref(p), _stream(stream), C.byref(h)))
    return h


def ts_op_destroy(h):
    return _check(lib().ts_op_destroy(h))


def ts_op_coeffs_export(op, level, out):
    out = np.ascontiguousarray(out, dtype=np.float64)
    _check(lib().ts_op_coeffs_export(op, level, _ptr(out), out.size))
    return out


def ts_op_coeffs_import(op, level, coeffs):
    c = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(-1)
    return _check(lib().ts_op_coeffs_import(op, level, _ptr(c), c.size))


def ts_op_macro_flags(op, level, out):
    out = np.ascontiguousarray(out, dtype=np.uint8)
    _check(lib().ts_op_macro_flags(op, level, _ptr(out), out.size))
    return out


def ts_apply(op, level, dtype, x, y, stream=None):
    return _check(lib().ts_apply(op, level, dtype, _ptr(x), _ptr(y), _stream(stream)))


def ts_apply_volume(op, level, dtype, x, y, stream=None):
    return _check(lib().ts_apply_volume(op, level, dtype, _ptr(x), _ptr(y), _stream(stream)))


def ts_residual(op, level, dtype, f, u, r, stream=None):
    return _check(lib().ts_residual(op, level, dtype, _ptr(f), _ptr(u), _ptr(r), _stream(stream)))


def ts_smooth(op, level, dtype, f, u, sweeps=1, stream=None):
    return _check(lib().ts_smooth(op, level, dtype, _ptr(f), _ptr(u), sweeps, _stream(stream)))


def ts_restrict(op, level, dtype, rf, rc, stream=None):
    return _check(lib().ts_restrict(op, level, dtype, _ptr(rf), _ptr(rc), _stream(stream)))


def ts_prolongate_add(op, level, dtype, uc, uf, stream=None):
    return _check(lib().ts_prolongate_add(op, level, dtype, _ptr(uc), _ptr(uf), _stream(stream)))


def ts_norm2(mesh, level, dtype, x, stream=None):
    out = C.c_double()
    _check(lib().ts_norm2(mesh, level, dtype, _ptr(x), C.byref(out), _stream(stream)))
    return out.value


def ts_norm2_noalloc(mesh, level, dtype, x, out, stream=None):
    """The norm into the device tensor out (one float64), no allocation."""
    return _check(lib().ts_norm2_noalloc(mesh, level, dtype, _ptr(x), _ptr(out),
                                         _stream(stream)))


def ts_solver_create(op, level, nu1=3, nu2=3, max_cycles=60, precision=TS_F64, rtol=1e-10,
                     diverge_window=3, dd=False):
    p = ts_solve_params(nu1, nu2, max_cycles, precision, rtol, diverge_window, 1 if dd else 0)
    h = C.c_void_p()
    _check(lib().ts_solver_create(op, level, C.byref(p), C.byref(h)))
    return h


def ts_solver_destroy(h):
    return _check(lib().ts_solver_destroy(h))


def ts_vcycle(sv, dtype, f, u, stream=None):
    return _check(lib().ts_vcycle(sv, dtype, _ptr(f), _ptr(u), _stream(stream)))


def ts_solve(sv, f, u, stream=None, raise_on_fail=True):
    """Returns (status, info); raises TSError on failure if raise_on_fail."""
    info = ts_solve_info()
    rc = lib().ts_solve(sv, _ptr(f), _ptr(u), C.byref(info), _stream(stream))
    if rc != TS_OK and (raise_on_fail or rc not in (TS_ENOCONV, TS_ENONFINITE)):
        raise TSError(rc, ts_last_error())
    return rc, info


TS_SOLVE_RUNNING, TS_SOLVE_READY, TS_SOLVE_DONE = 1, 2, 3


def ts_solve_begin(sv, f, u, stream=None):
    return _check(lib().ts_solve_begin(sv, _ptr(f), _ptr(u), _stream(stream)))


def ts_solve_step(sv):
    return _check(lib().ts_solve_step(sv))


def ts_solve_query(sv, info=None):
    """Non-blocking: TS_SOLVE_RUNNING / READY / DONE (info filled if given)."""
    st = C.c_int(0)
    _check(lib().ts_solve_query(sv, C.byref(st), C.byref(info) if info is not None else None))
    return st.value


def ts_solve_batch_step(solvers):
    """One outer iteration on each solver (handles or Solver objects), in
    the order given; all must be ready, else nothing is enqueued."""
    hs = [getattr(v, "h", v) for v in solvers]
    arr = (C.c_void_p * max(len(hs), 1))(*hs)
    return _check(lib().ts_solve_batch_step(arr, len(hs)))


def ts_device_bytes():
    b = C.c_int64(0)
    _check(lib().ts_device_bytes(C.byref(b)))
    return b.value


# ----------------------------------------------------------------- helpers

def dtype_torch(dt):
    import torch
    return torch.float64 if dt == TS_F64 else torch.float32


def check_vector(t, n, dt, what="vector"):
    """Reject a tensor the library cannot take as a block vector of n entries
    of dtype dt: wrong element type, not contiguous, wrong length, or not in
    device memory (the kernels would read or write past the buffer).  Raises
    TSError(TS_EINVAL) before any library call."""
    want = dtype_torch(dt)
    if getattr(t, "dtype", None) != want:
        raise TSError(TS_EINVAL, "%s: dtype %s, expected %s" % (what, getattr(t, "dtype", type(t)),
                                                                want))
    if not t.is_contiguous():
        raise TSError(TS_EINVAL, "%s: not contiguous" % what)
    if t.numel() != n:
        raise TSError(TS_EINVAL, "%s: %d entries, the level's block vector has %d"
                      % (what, t.numel(), n))
    if not t.is_cuda:
        raise TSError(TS_EINVAL, "%s: not a device tensor" % what)
    return t


class Mesh:
    """Owning wrapper of a ts_mesh handle."""

    def __init__(self, vtx, tet, geom=TS_GEOM_SHELL, like=None):
        """like: a Mesh with the same connectivity whose built levels are
        shared (ts_mesh_create_like); tet and geom are then its own."""
        self.vtx = np.ascontiguousarray(vtx, dtype=np.float64)
        if like is not None:
            if self.vtx.shape != like.vtx.shape:
                raise ValueError("vertex array of a different shape")
            self.tet = like.tet
            self.h = ts_mesh_create_like(like.h, self.vtx)
        else:
            self.tet = np.ascontiguousarray(tet, dtype=np.int64)
            self.h = ts_mesh_create(self.vtx, self.tet, geom)

    def check_shell(self, r_in, r_out, tol=1e-12):
        """Raise TSError unless the mesh is a shell r_in <= |x| <= r_out whose
        boundary faces lie on the two spheres."""
        ts_mesh_check_shell(self.h, r_in, r_out, tol)

    def layout(self, level):
        return ts_layout(self.h, level)

    def set_vertices(self, vtx):
        """New vertex coordinates, same connectivity; the levels built so far
        are kept (no operator on this mesh may be alive)."""
        v = np.ascontiguousarray(vtx, dtype=np.float64)
        if v.shape != self.vtx.shape:
            raise ValueError("vertex array of a different shape")
        ts_mesh_set_vertices(self.h, v)
        self.vtx = v

    def zeros(self, level, dt=TS_F64):
        import torch
        return torch.zeros(self.layout(level).vec_len, dtype=dtype_torch(dt), device="cuda")

    def to_block(self, level, canon):
        import torch
        c = torch.as_tensor(np.ascontiguousarray(canon, dtype=np.float64), device="cuda")
        b = self.zeros(level)
        ts_canon_to_block(self.h, level, c, b)
        return b

    def to_canon(self, level, block):
        import torch
        c = torch.zeros(self.layout(level).n_unique, dtype=torch.float64, device="cuda")
        ts_block_to_canon(self.h, level, block, c)
        return c

    def coords(self, level):
        import torch
        x = torch.zeros(3 * self.layout(level).vec_len, dtype=torch.float64, device="cuda")
        ts_node_coords(self.h, level, x)
        return x.view(-1, 3)

    def rhs(self, level, kind, params=(), stream=None):
        f = self.zeros(level)
        ts_rhs(self.h, level, kind, params, f, stream)
        return f

    def norm(self, level, x, dt=TS_F64):
        return ts_norm2(self.h, level, dt, x)

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.ts_mesh_destroy(self.h)
            self.h = None


class Operator:
    """Owning wrapper of a ts_op handle (keeps its mesh alive)."""

    def __init__(self, mesh, max_level, method=TS_LSQP, q=2, sample_j=2, center=TS_CENTER_POLY,
                 fallback_tol=0.0, stream=None, face_surrogate=False, coarse_from_finest=False):
        self.mesh = mesh
        if method == TS_CONS:
            q = 0  # one constant stencil per macro: degree-0 coefficients
        self.method, self.q = method, q
        self.max_level = max_level
        self.h = ts_op_create(mesh.h, max_level, method, q, sample_j, center, fallback_tol,
                              stream, face_surrogate, coarse_from_finest)

    def macro_flags(self, level):
        """1 for macros whose volume rows stay IFEM on this level."""
        return ts_op_macro_flags(self.h, level, np.zeros(self.mesh.tet.shape[0], np.uint8))

    def coeffs(self, level):
        nt = self.mesh.tet.shape[0]
        mq = (self.q + 1) * (self.q + 2) * (self.q + 3) // 6
        out = np.zeros(nt * 15 * mq)
        ts_op_coeffs_export(self.h, level, out)
        return out.reshape(nt, 15, mq)

    def set_coeffs(self, level, c):
        ts_op_coeffs_import(self.h, level, c)

    def _n(self, level):
        return self.mesh.layout(level).vec_len

    def apply(self, level, x, y=None, dt=TS_F64):
        n = self._n(level)
        check_vector(x, n, dt, "x")
        if y is None:
            y = self.mesh.zeros(level, dt)
        check_vector(y, n, dt, "y")
        ts_apply(self.h, level, dt, x, y)
        return y

    def residual(self, level, f, u, r=None, dt=TS_F64):
        n = self._n(level)
        check_vector(f, n, dt, "f")
        check_vector(u, n, dt, "u")
        if r is None:
            r = self.mesh.zeros(level, dt)
        check_vector(r, n, dt, "r")
        ts_residual(self.h, level, dt, f, u, r)
        return r

    def smooth(self, level, f, u, sweeps=1, dt=TS_F64):
        n = self._n(level)
        check_vector(f, n, dt, "f")
        check_vector(u, n, dt, "u")
        ts_smooth(self.h, level, dt, f, u, sweeps)
        return u

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.ts_op_destroy(self.h)
            self.h = None


class Solver:
    def __init__(self, op, level, **kw):
        self.op = op
        self.level = level
        self.h = ts_solver_create(op.h, level, **kw)

    def _n(self):
        return self.op.mesh.layout(self.level).vec_len

    def vcycle(self, f, u, dt=TS_F64):
        n = self._n()
        check_vector(f, n, dt, "f")
        check_vector(u, n, dt, "u")
        ts_vcycle(self.h, dt, f, u)
        return u

    def solve(self, f, u=None, raise_on_fail=True, stream=None):
        n = self._n()
        check_vector(f, n, TS_F64, "f")
        if u is None:
            u = self.op.mesh.zeros(self.level)
        check_vector(u, n, TS_F64, "u")
        rc, info = ts_solve(self.h, f, u, stream=stream, raise_on_fail=raise_on_fail)
        return u, rc, info

    def begin(self, f, u, stream=None):
        n = self._n()
        check_vector(f, n, TS_F64, "f")
        check_vector(u, n, TS_F64, "u")
        ts_solve_begin(self.h, f, u, stream)

    def step(self):
        ts_solve_step(self.h)

    def set_vertices(self, vtx, stream=None):
        """Move the solver, its operator and its mesh to new vertex
        coordinates of the same connectivity, rebuilding every
        geometry-dependent part in place (no solve may be in progress; the
        mesh must carry this operator only)."""
        v = np.ascontiguousarray(vtx, dtype=np.float64)
        mesh = self.op.mesh
        if v.shape != mesh.vtx.shape:
            raise ValueError("vertex array of a different shape")
        ts_solver_set_vertices(self.h, v, stream)
        mesh.vtx = v

    def query(self, info=None):
        return ts_solve_query(self.h, info)

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.ts_solver_destroy(self.h)
            self.h = None
