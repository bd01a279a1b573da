"""FP64 CPU oracle of the two-scale surrogate-stencil method (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``ts_oracle.c`` (plain C,
written from the paper, sharing no code with the HIP library) through ctypes,
and ``brute.py`` adds an independent global-assembly check in NumPy/SciPy.

Every function takes N, the number of fine intervals per macro edge (the
paper's level l has N = 2^(l+2)).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ts_oracle.c")
_LIB = os.path.join(_HERE, "libtsoracle.so")

NW = 15
DIRS = np.array(
    [[0, 0, 0], [-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [1, -1, 0], [-1, 1, 0],
     [0, 0, -1], [1, 0, -1], [0, 1, -1], [-1, 1, -1], [0, 0, 1], [-1, 0, 1], [0, -1, 1],
     [1, -1, 1]], dtype=np.int64)
NAMES = ["mc", "mw", "me", "ms", "mn", "mse", "mnw", "bc", "be", "bn", "bnw", "tc", "tw",
         "ts", "tse"]

IFEM, LSQP, IPOLY, SYM, CONS = 0, 1, 2, 3, 4


def _opkind(kind):
    """operator kind of the C oracle: 0 element-wise, 1 surrogate (15
    polynomials per macro), 2 symmetric surrogate (7 edge polynomials), 3
    constant stencils of the unmapped macros on the volume"""
    return {IFEM: 0, SYM: 2, CONS: 3}.get(kind, 1)


def build(force=False):
    """Compile the oracle with gcc (plain C, OpenMP over rows).

    With TS_ORACLE_NATIVE=1 in the environment (the benchmark's CPU leg) a
    second copy is built for the host it runs on (-O3 -march=native) in the
    temporary directory and used instead; the tests use the portable -O2
    build."""
    if os.environ.get("TS_ORACLE_NATIVE") == "1":
        import tempfile
        lib_path = os.path.join(tempfile.gettempdir(), "libtsoracle_native_%d.so" % os.getpid())
        cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-o", lib_path,
               _SRC, "-lm"]
        subprocess.check_call(cmd)
        return lib_path
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P, I64, I, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
        sig = {
            "or_mesh_new": (P, [P, I64, P, I64, I]),
            "or_mesh_free": (None, [P]),
            "or_mesh_counts": (I64, [P, P]),
            "or_num_unique": (I64, [P, I]),
            "or_canon": (I64, [P, I, I64, I, I, I]),
            "or_is_dirichlet": (I, [P, I, I64]),
            "or_copies": (I, [P, I, I64, P, P, I]),
            "or_node_xyz": (None, [P, I, I64, I, I, I, P]),
            "or_coords": (None, [P, I, P]),
            "or_ifem_stencil": (None, [P, I, I64, I, I, I, P]),
            "or_tets_at_count": (I, [I, I, I, I]),
            "or_macro_fine_volume": (D, [P, I, I64]),
            "or_num_coeffs": (I, [I]),
            "or_poly_eval": (D, [I, I, P, I, I, I]),
            "or_sample_points": (I64, [I, I, I, P]),
            "or_fit": (I, [P, I, I, I, I, P]),
            "or_apply": (None, [P, I, I, I, I, P, P, P]),
            "or_apply_rows": (None, [P, I, I, I, I, P, P, P, I64, P]),
            "or_residual": (None, [P, I, I, I, I, P, P, P, P]),
            "or_gs_phase": (I, [P, I, I64]),
            "or_gs_sweep": (None, [P, I, I, I, I, P, P, P]),
            "or_prolongate": (None, [P, I, P, P]),
            "or_restrict": (None, [P, I, P, P]),
            "or_coarse_new": (P, [P, I]),
            "or_coarse_free": (None, [P]),
            "or_coarse_size": (I64, [P]),
            "or_coarse_solve": (None, [P, P, P, P]),
            "or_mg_new": (P, [P, I, I, I, I, I, I, I, P]),
            "or_mg_free": (None, [P]),
            "or_vcycle": (None, [P, P, P]),
            "or_norm_free": (D, [P, I, P]),
            "or_solve": (I, [P, P, P, D, I, P]),
            "or_rhs": (None, [P, I, I, P, I, P]),
            "or_exact_manufactured": (D, [D, D, P]),
            "or_node_volumes": (None, [P, I, P]),
            "or_block_size": (I64, [I]),
            "or_block_index": (I64, [I, I, I, I]),
            "or_canon_to_block": (None, [P, I, P, P]),
            "or_block_to_canon": (D, [P, I, P, P]),
            "or_block_canon_ids": (None, [P, I, P]),
            "or_dirichlet_mask": (None, [P, I, P]),
            "or_fit_values": (I, [I, I, I, I, P, P]),
            "or_tets_at_list": (I, [I, I, I, I, P]),
            "or_set_ifem_flags": (None, [P]),
            "or_fallback_flags": (None, [P, I, I, P, D, P]),
            "or_mg_set_flags": (None, [P, I, P]),
            "or_mg_set_dd": (None, [P, I]),
            "or_mg_set_face_coeffs": (None, [P, I, P]),
            "or_set_face_coeffs": (None, [P]),
            "or_num_coeffs2": (I, [I]),
            "or_face_sample_points": (I64, [I, I, P]),
            "or_face_fit": (I, [P, I, I, I, P]),
            "or_face_row_exact": (I, [P, I, I64, P, P]),
            "or_face_fit_values": (I, [I, I, I, P, P]),
            "or_face_poly_eval": (D, [I, I, P, I, I]),
            "or_fit_sym": (I, [P, I, I, I, P]),
            "or_fit_sym_values": (I, [I, I, I, P, P]),
            "or_poly_eval_mid": (D, [I, I, P, I, I, I, I]),
            "or_solve_dd": (I, [P, P, P, D, I, P]),
            "or_gs_rows": (None, [P, I, I, I, I, P, P, P, P, I64, P]),
            "or_row_neighbours": (I, [P, I, I64, P, I]),
            "or_set_gs_order": (None, [I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Mesh:
    """Macro mesh handle of the oracle (vertex order of each macro = frame)."""

    def __init__(self, vtx, tet, affine=False):
        self.vtx = _f64(vtx)
        self.tet = np.ascontiguousarray(tet, dtype=np.int64)
        self.h = lib().or_mesh_new(_p(self.vtx), self.vtx.shape[0], _p(self.tet),
                                   self.tet.shape[0], 1 if affine else 0)
        c = np.zeros(4, dtype=np.int64)
        lib().or_mesh_counts(self.h, _p(c))
        self.nv, self.ne, self.nf, self.nt = (int(v) for v in c)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_mesh_free(self.h)
            self.h = None

    # --- counting and numbering -------------------------------------------
    def num_unique(self, N):
        return int(lib().or_num_unique(self.h, N))

    def dirichlet_mask(self, N):
        m = np.zeros(self.num_unique(N), dtype=np.uint8)
        lib().or_dirichlet_mask(self.h, N, _p(m))
        return m.astype(bool)

    def num_free(self, N):
        return int((~self.dirichlet_mask(N)).sum())

    def canon(self, N, t, i, j, k):
        return int(lib().or_canon(self.h, N, t, i, j, k))

    def copies(self, N, u, maxc=256):
        ct = np.zeros(maxc, dtype=np.int64)
        ijk = np.zeros((maxc, 3), dtype=np.int32)
        n = lib().or_copies(self.h, N, u, _p(ct), _p(ijk), maxc)
        return [(int(ct[c]), tuple(int(v) for v in ijk[c])) for c in range(n)]

    def coords(self, N):
        x = np.zeros((self.num_unique(N), 3))
        lib().or_coords(self.h, N, _p(x))
        return x

    def node_xyz(self, N, t, i, j, k):
        x = np.zeros(3)
        lib().or_node_xyz(self.h, N, t, i, j, k, _p(x))
        return x

    def gs_phase(self, N, u):
        return int(lib().or_gs_phase(self.h, N, u))

    # --- stencils and fits ------------------------------------------------
    def ifem_stencil(self, N, t, i, j, k):
        s = np.zeros(NW)
        lib().or_ifem_stencil(self.h, N, t, i, j, k, _p(s))
        return s

    def fallback_flags(self, N, q, coeffs, tol):
        """Macros that keep IFEM rows on this level (selective surrogate)."""
        f = np.zeros(self.nt, dtype=np.uint8)
        lib().or_fallback_flags(self.h, N, q, _p(_f64(coeffs)), tol, _p(f))
        return f

    def macro_fine_volume(self, N, t):
        return float(lib().or_macro_fine_volume(self.h, N, t))

    def fit(self, N, method=LSQP, q=2, jsamp=2):
        mq = num_coeffs(q)
        c = np.zeros((self.nt, NW, mq))
        err = lib().or_fit(self.h, N, method, q, jsamp, _p(c))
        if err:
            raise ValueError("oracle fit failed (method %d, q %d)" % (method, q))
        return c

    def fit_sym(self, N, q=2, jsamp=2):
        """Pair polynomials of the symmetric surrogate: nt x 7 x m_q."""
        c = np.zeros((self.nt, 7, num_coeffs(q)))
        if lib().or_fit_sym(self.h, N, q, jsamp, _p(c)):
            raise ValueError("oracle symmetric fit failed (q %d)" % q)
        return c

    def face_fit(self, N, q=2, jsamp=2):
        """Per-face fits of the rows of interior-face nodes: nf x 15 x m2 in
        the face frame (zero for faces that are not fitted)."""
        c = np.zeros((self.nf, NW, num_coeffs2(q)))
        err = lib().or_face_fit(self.h, N, q, jsamp, _p(c))
        if err:
            raise ValueError("oracle face fit failed (q %d)" % q)
        return c

    def face_row_exact(self, N, u):
        """Exact 15 entries of the face node u and their unique ids."""
        s = np.zeros(NW)
        nb = np.zeros(NW, dtype=np.int64)
        lib().or_face_row_exact(self.h, N, int(u), _p(s), _p(nb))
        return s, nb

    # --- operator ---------------------------------------------------------
    def apply(self, N, x, kind=IFEM, q=2, center=0, coeffs=None, flags=None, fcoeffs=None):
        _set_flags(flags, fcoeffs)
        x = _f64(x)
        y = np.zeros_like(x)
        cf = _f64(coeffs) if coeffs is not None else np.zeros(1)
        lib().or_apply(self.h, N, _opkind(kind), q, center, _p(cf), _p(x), _p(y))
        return y

    def apply_rows(self, N, x, rows, kind=IFEM, q=2, center=0, coeffs=None, flags=None,
                   fcoeffs=None):
        _set_flags(flags, fcoeffs)
        x = _f64(x)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        y = np.zeros(rows.shape[0])
        cf = _f64(coeffs) if coeffs is not None else np.zeros(1)
        lib().or_apply_rows(self.h, N, _opkind(kind), q, center, _p(cf), _p(x), _p(rows),
                            rows.shape[0], _p(y))
        return y

    def residual(self, N, f, u, kind=IFEM, q=2, center=0, coeffs=None, flags=None,
                 fcoeffs=None):
        _set_flags(flags, fcoeffs)
        f, u = _f64(f), _f64(u)
        r = np.zeros_like(u)
        cf = _f64(coeffs) if coeffs is not None else np.zeros(1)
        lib().or_residual(self.h, N, _opkind(kind), q, center, _p(cf), _p(f), _p(u), _p(r))
        return r

    def gs_sweep(self, N, f, u, kind=IFEM, q=2, center=0, coeffs=None, flags=None,
                 fcoeffs=None):
        _set_flags(flags, fcoeffs)
        f = _f64(f)
        u = np.array(u, dtype=np.float64, copy=True)
        cf = _f64(coeffs) if coeffs is not None else np.zeros(1)
        lib().or_gs_sweep(self.h, N, _opkind(kind), q, center, _p(cf), _p(f), _p(u))
        return u

    def gs_rows(self, N, f, x, rows, kind=IFEM, q=2, center=0, coeffs=None):
        """Gauss-Seidel values (f_u - off_u(x)) / diag_u of the listed rows."""
        _set_flags(None)
        f, x = _f64(f), _f64(x)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(rows.shape[0])
        cf = _f64(coeffs) if coeffs is not None else np.zeros(1)
        lib().or_gs_rows(self.h, N, _opkind(kind), q, center, _p(cf), _p(f), _p(x), _p(rows),
                         rows.shape[0], _p(out))
        return out

    def row_neighbours(self, N, u):
        """Free unique nodes sharing a fine edge with node u."""
        out = np.zeros(256, dtype=np.int64)
        n = lib().or_row_neighbours(self.h, N, int(u), _p(out), 256)
        return out[:n]

    def prolongate(self, N, uc):
        uc = _f64(uc)
        uf = np.zeros(self.num_unique(N))
        lib().or_prolongate(self.h, N, _p(uc), _p(uf))
        return uf

    def restrict(self, N, rf):
        rf = _f64(rf)
        rc = np.zeros(self.num_unique(N // 2))
        lib().or_restrict(self.h, N, _p(rf), _p(rc))
        return rc

    def rhs(self, N, kind, params=()):
        par = _f64(np.asarray(params, dtype=np.float64).reshape(-1) if len(params) else np.zeros(1))
        f = np.zeros(self.num_unique(N))
        lib().or_rhs(self.h, N, kind, _p(par), len(params), _p(f))
        return f

    def node_volumes(self, N):
        v = np.zeros(self.num_unique(N))
        lib().or_node_volumes(self.h, N, _p(v))
        return v

    def norm_free(self, N, r):
        return float(lib().or_norm_free(self.h, N, _p(_f64(r))))

    # --- block layout -----------------------------------------------------
    def canon_to_block(self, N, c):
        c = _f64(c)
        b = np.zeros(self.nt * block_size(N))
        lib().or_canon_to_block(self.h, N, _p(c), _p(b))
        return b

    def block_to_canon(self, N, b):
        b = _f64(b)
        c = np.zeros(self.num_unique(N))
        worst = lib().or_block_to_canon(self.h, N, _p(b), _p(c))
        return c, float(worst)

    def block_canon_ids(self, N):
        ids = np.zeros(self.nt * block_size(N), dtype=np.int64)
        lib().or_block_canon_ids(self.h, N, _p(ids))
        return ids


class Multigrid:
    """V(nu1, nu2) cycle of the oracle on levels N = 2^lam, lam0..lamL."""

    def __init__(self, mesh, lam0, lamL, kind=IFEM, q=2, center=0, coeffs=None, nu1=3, nu2=3,
                 flags=None, dd=False, fcoeffs=None):
        self.mesh = mesh
        self.lam0, self.lamL = lam0, lamL
        nl = lamL - lam0 + 1
        self._keep = []
        arr = (C.c_void_p * nl)()
        for l in range(nl):
            if coeffs is not None and coeffs[l] is not None:
                a = _f64(coeffs[l])
                self._keep.append(a)
                arr[l] = a.ctypes.data
            else:
                arr[l] = None
        self._arr = arr
        self.h = lib().or_mg_new(mesh.h, lam0, lamL, _opkind(kind), q, center, nu1, nu2,
                                 C.cast(arr, C.c_void_p))
        if flags is not None:
            for l in range(nl):
                if flags[l] is not None:
                    a = np.ascontiguousarray(flags[l], dtype=np.uint8)
                    self._keep.append(a)
                    lib().or_mg_set_flags(self.h, lam0 + l, _p(a))
        if dd:
            lib().or_mg_set_dd(self.h, 1)
        if fcoeffs is not None:
            for l in range(nl):
                if fcoeffs[l] is not None:
                    a = _f64(fcoeffs[l])
                    self._keep.append(a)
                    lib().or_mg_set_face_coeffs(self.h, lam0 + l, _p(a))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_mg_free(self.h)
            self.h = None

    def vcycle(self, f, u):
        f = _f64(f)
        u = np.array(u, dtype=np.float64, copy=True)
        lib().or_vcycle(self.h, _p(f), _p(u))
        return u

    def solve(self, f, u0=None, rtol=1e-10, max_cycles=50):
        f = _f64(f)
        u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
        hist = np.zeros(max_cycles + 1)
        c = lib().or_solve(self.h, _p(f), _p(u), rtol, max_cycles, _p(hist))
        n = c if c >= 0 else max_cycles
        return u, int(c), hist[: n + 1]

    def solve_dd(self, f, u0=None, rtol=1e-10, max_cycles=50):
        """Cycles until the relative update ||u_c - u_(c-1)|| / ||u_c|| <= rtol
        (the stop test of double discretisation, Sec. 4 introduction)."""
        f = _f64(f)
        u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
        hist = np.zeros(max_cycles)
        c = lib().or_solve_dd(self.h, _p(f), _p(u), rtol, max_cycles, _p(hist))
        n = c if c >= 0 else max_cycles
        return u, int(c), hist[:n]


_flag_keep = [None, None]


def _set_flags(flags, fcoeffs=None):
    """Per-macro IFEM fallback flags and per-face fits for the next operator
    call (None: none)."""
    if flags is None:
        _flag_keep[0] = None
        lib().or_set_ifem_flags(None)
    else:
        a = np.ascontiguousarray(flags, dtype=np.uint8)
        _flag_keep[0] = a
        lib().or_set_ifem_flags(_p(a))
    if fcoeffs is None:
        _flag_keep[1] = None
        lib().or_set_face_coeffs(None)
    else:
        a = _f64(fcoeffs)
        _flag_keep[1] = a
        lib().or_set_face_coeffs(_p(a))


def set_gs_order(mode):
    """Ordering of every following Gauss-Seidel sweep of the oracle: 0 the
    multicolour phases (default), 1 the interface nodes one after the other
    in canonical order, 2 every node one after the other (lexicographic)."""
    lib().or_set_gs_order(int(mode))


def num_coeffs2(q):
    return (q + 1) * (q + 2) // 2


def face_sample_points(N, jsamp=2):
    n = lib().or_face_sample_points(N, jsamp, None)
    p = np.zeros((n, 2), dtype=np.int32)
    lib().or_face_sample_points(N, jsamp, _p(p))
    return p


def fit_sym_values(N, vals, q=2, jsamp=2):
    """Pair polynomials (7 x m_q) fitted to values (ns x 15) at the LSQP
    sampling points."""
    c = np.zeros((7, num_coeffs(q)))
    if lib().or_fit_sym_values(N, q, jsamp, _p(_f64(vals)), _p(c)):
        raise ValueError("symmetric fit failed")
    return c


def poly_eval_mid(q, N, c, i, j, k, w):
    return float(lib().or_poly_eval_mid(q, N, _p(_f64(c)), int(i), int(j), int(k), int(w)))


def face_poly_eval(q, N, c, a, b):
    return float(lib().or_face_poly_eval(q, N, _p(_f64(c)), int(a), int(b)))


def face_fit_values(N, vals, q=2, jsamp=2):
    """Least-squares fit (15 x m2) of values (ns x 15) at the face sampling
    points."""
    c = np.zeros((NW, num_coeffs2(q)))
    if lib().or_face_fit_values(N, q, jsamp, _p(_f64(vals)), _p(c)):
        raise ValueError("face fit failed")
    return c


def num_coeffs(q):
    return (q + 1) * (q + 2) * (q + 3) // 6


def block_size(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def block_index(N, i, j, k):
    return int(lib().or_block_index(N, i, j, k))


def sample_points(N, method=LSQP, jsamp=2):
    n = int(lib().or_sample_points(N, method, jsamp, None))
    pts = np.zeros((n, 3), dtype=np.int32)
    lib().or_sample_points(N, method, jsamp, _p(pts))
    return pts


def poly_eval(q, N, a, i, j, k):
    return float(lib().or_poly_eval(q, N, _p(_f64(a)), i, j, k))


def fit_values(N, vals, method=LSQP, q=2, jsamp=2):
    """Fit 15 polynomials to given values (ns x 15) at the sampling points."""
    vals = _f64(vals)
    c = np.zeros((NW, num_coeffs(q)))
    if lib().or_fit_values(N, method, q, jsamp, _p(vals), _p(c)):
        raise ValueError("fit failed")
    return c


def tets_at_list(N, i, j, k):
    out = np.zeros((32, 4, 3), dtype=np.int32)
    n = lib().or_tets_at_list(N, i, j, k, _p(out))
    return out[:n].astype(np.int64)


def tets_at_count(N, i, j, k):
    return int(lib().or_tets_at_count(N, i, j, k))


def exact_manufactured(r1, r2, xyz):
    xyz = np.atleast_2d(_f64(xyz))
    out = np.zeros(xyz.shape[0])
    for n in range(xyz.shape[0]):
        row = np.ascontiguousarray(xyz[n])
        out[n] = lib().or_exact_manufactured(r1, r2, _p(row))
    return out
