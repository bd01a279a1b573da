"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module holds no arithmetic of the two-scale method: it only builds macro
meshes (vertex coordinates plus tetrahedron connectivity), draws seeded random
numbers and draws the parameters of right-hand sides.  Both the HIP path and
the CPU oracle consume what it produces.

Meshes
------
* ``single_macro()``: one macro tetrahedron cut from the shell r in [0.55, 1]
  with vertices (1,0,0), (0,1,0), (0,0,1) and 0.55*(1,1,1)/sqrt(3).
* ``cubed_shell(n_split, radii)``: a spherical shell built from the cube
  surface.  Each cube face is cut into n_split x n_split quads on the cube
  (plain normalised cube grid, not equiangular), every quad is projected to the
  sphere, and every (quad, radial layer) hexahedron is cut into 6 tetrahedra.
  The cut follows the minimum-global-vertex-id rule on every quadrilateral
  face, so the tetrahedra of neighbouring hexahedra share faces exactly
  (conforming).  Vertex ids are layer-major (id = layer * n_surface + s), so a
  hexahedron's inner and outer quads take parallel diagonals.  Every
  tetrahedron lists its vertex ids in ascending order; that order is the
  macro's (i, j, k) frame.

  n_split=1 with radii (0.55, 1.0) gives the 36-macro shell; n_split=2 with
  radii (0.55, 0.775, 1.0) gives the 288-macro shell (the middle radius is the
  arithmetic mean, a choice made here because the workload does not fix it).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "single_macro",
    "reference_tet",
    "cubed_shell",
    "shell36",
    "shell288",
    "uniform",
    "gaussian_bumps",
    "scaled_shell36",
]


def single_macro():
    """One macro of the shell r in [0.55, 1]; vertex order is the frame."""
    v3 = 0.55 / math.sqrt(3.0)
    vtx = np.array(
        [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [v3, v3, v3]],
        dtype=np.float64,
    )
    tet = np.array([[0, 1, 2, 3]], dtype=np.int64)
    return vtx, tet


def reference_tet(scale=1.0):
    """The reference tetrahedron (0,0,0), (1,0,0), (0,1,0), (0,0,1)."""
    vtx = scale * np.array(
        [[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]],
        dtype=np.float64,
    )
    tet = np.array([[0, 1, 2, 3]], dtype=np.int64)
    return vtx, tet


def _cube_surface(n):
    """Vertices (unit vectors) and quads of a cube surface split n x n per face."""
    keys = {}
    pts = []

    def vid(c):
        c = tuple(int(v) for v in c)
        if c not in keys:
            keys[c] = len(pts)
            pts.append(c)
        return keys[c]

    quads = []
    # face: fixed axis a with sign s; free axes (b, c) chosen so that the
    # quad orientation is irrelevant (orientation is not used anywhere).
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        for s in (-1, 1):
            for u in range(n):
                for v in range(n):
                    corners = []
                    for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0, 0, 0]
                        p[a] = s * n
                        p[b] = -n + 2 * (u + du)
                        p[c] = -n + 2 * (v + dv)
                        corners.append(vid(p))
                    quads.append(corners)
    # renumber vertices in sorted integer-coordinate order (deterministic)
    order = sorted(range(len(pts)), key=lambda i: pts[i])
    newid = {old: new for new, old in enumerate(order)}
    unit = np.zeros((len(pts), 3))
    for old, new in newid.items():
        p = np.array(pts[old], dtype=np.float64)
        unit[new] = p / np.linalg.norm(p)
    quads = [[newid[q] for q in quad] for quad in quads]
    return unit, quads


def _prism_to_tets(a, b):
    """Cut the prism with bottom a[0..2] and top b[0..2] (a[i]-b[i] vertical
    edges) into 3 tetrahedra using the minimum-id diagonal on each quad face."""
    a = list(a)
    b = list(b)
    six = a + b
    m = min(six)
    if m in b:
        a, b = b, a
    r = a.index(m)
    a = a[r:] + a[:r]
    b = b[r:] + b[:r]
    a0, a1, a2 = a
    b0, b1, b2 = b
    if min(a1, b2) < min(a2, b1):
        return [[a0, a1, a2, b2], [a0, a1, b2, b1], [a0, b1, b2, b0]]
    return [[a0, a1, a2, b1], [a0, b1, a2, b2], [a0, b1, b2, b0]]


def cubed_shell(n_split, radii):
    """Conforming tetrahedral macro mesh of the shell radii[0] < r < radii[-1]."""
    unit, quads = _cube_surface(n_split)
    ns = unit.shape[0]
    radii = [float(r) for r in radii]
    vtx = np.concatenate([r * unit for r in radii], axis=0)
    tets = []
    for layer in range(len(radii) - 1):
        lo = layer * ns
        hi = (layer + 1) * ns
        for q in quads:
            p = q.index(min(q))
            q = q[p:] + q[:p]
            for tri in ((q[0], q[1], q[2]), (q[0], q[2], q[3])):
                bottom = [lo + t for t in tri]
                top = [hi + t for t in tri]
                for t in _prism_to_tets(bottom, top):
                    tets.append(sorted(t))
    return vtx.astype(np.float64), np.array(tets, dtype=np.int64)


def shell36(r_in=0.55, r_out=1.0):
    return cubed_shell(1, (r_in, r_out))


def scaled_shell36(r_in, r_out=1.0):
    """The 36-macro shell topology with the given radii (serving requests)."""
    return cubed_shell(1, (r_in, r_out))


def shell288(r_in=0.55, r_out=1.0):
    return cubed_shell(2, (r_in, 0.5 * (r_in + r_out), r_out))


def shell2304(r_in=0.55, r_out=1.0):
    """The 288-macro shell refined once in every direction: each cube face
    split 4 x 4 and four radial layers at equal spacing (2,304 macros)."""
    return cubed_shell(4, tuple(r_in + (r_out - r_in) * q / 4.0 for q in range(5)))


def uniform(n, seed, lo=-1.0, hi=1.0):
    """n values ~ U[lo, hi) from NumPy's PCG64 generator with the given seed."""
    return np.random.default_rng(seed).uniform(lo, hi, size=int(n))


def gaussian_bumps(seed, r_in, r_out=1.0, n_bumps=8):
    """Parameters of a sum of isotropic Gaussian bumps inside the shell.

    Returns a flat float64 array of n_bumps records (cx, cy, cz, sigma, amp):
    centre = random direction times a radius ~ U[r_in, r_out], sigma ~
    U[0.05, 0.15], amplitude ~ U[-1, 1].
    """
    rng = np.random.default_rng(seed)
    out = np.zeros((n_bumps, 5))
    for b in range(n_bumps):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(r_in, r_out)
        out[b, :3] = r * d
        out[b, 3] = rng.uniform(0.05, 0.15)
        out[b, 4] = rng.uniform(-1.0, 1.0)
    return out.reshape(-1)


def serving_trace(n, rate=50.0, seed=0, levels=(4, 5, 6, 7), r_in=(0.4, 0.7)):
    """Request trace of shell solves: Poisson arrivals (exponential gaps with
    mean 1/rate, PCG64 seed `seed`), level uniform on `levels` and inner radius
    ~ U[r_in] (PCG64 seed `seed` + 1).  The right-hand side of request i is
    gaussian_bumps(i, r_inner) on the shell r_inner < r < 1."""
    ra = np.random.default_rng(seed)
    rb = np.random.default_rng(seed + 1)
    t = np.cumsum(ra.exponential(1.0 / rate, size=int(n)))
    lv = rb.choice(np.asarray(levels), size=int(n))
    ri = rb.uniform(r_in[0], r_in[1], size=int(n))
    return [{"id": i, "t": float(t[i]), "level": int(lv[i]), "r_in": float(ri[i])}
            for i in range(int(n))]
