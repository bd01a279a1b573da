"""Brute-force global assembly of the P1 stiffness matrix (test infrastructure).

An independent second implementation used to pin the matrix-free C oracle on
small meshes.  It shares nothing with ``ts_oracle.c``: node identity comes from
exact integer keys {(global vertex id, barycentric weight * N)}, the fine
tetrahedra are enumerated per lattice cell with vectorised NumPy, and the
global matrix is assembled by scipy.sparse from 4x4 element matrices
K_T = |T| G G^T (Sec. 2.2 of the paper, eq. (algebraic)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# the six fine tetrahedra of a lattice cell (offsets from the cell base):
# up, the octahedron cut around its (0,1,0)-(1,0,1) diagonal, down
CELL = np.array([
    [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]],
    [[0, 1, 0], [1, 0, 1], [1, 0, 0], [0, 0, 1]],
    [[0, 1, 0], [1, 0, 1], [0, 0, 1], [0, 1, 1]],
    [[0, 1, 0], [1, 0, 1], [0, 1, 1], [1, 1, 0]],
    [[0, 1, 0], [1, 0, 1], [1, 1, 0], [1, 0, 0]],
    [[1, 1, 0], [1, 0, 1], [0, 1, 1], [1, 1, 1]],
])


def local_nodes(N):
    """All (i, j, k) >= 0 with i+j+k <= N in block order (k, j, i)."""
    out = []
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - k - j):
                out.append((i, j, k))
    return np.array(out, dtype=np.int64)


class Brute:
    def __init__(self, vtx, tet, N, affine=False):
        vtx = np.asarray(vtx, dtype=np.float64)
        tet = np.asarray(tet, dtype=np.int64)
        self.N = N
        loc = local_nodes(N)
        nloc = loc.shape[0]
        self.nloc = nloc
        lut = {tuple(p): n for n, p in enumerate(loc)}
        keys = {}
        slot_node = np.zeros(tet.shape[0] * nloc, dtype=np.int64)
        node_xyz = []
        node_verts = []
        radii = np.linalg.norm(vtx, axis=1)
        for t in range(tet.shape[0]):
            g = tet[t]
            for n, (i, j, k) in enumerate(loc):
                mu = (N - i - j - k, i, j, k)
                key = tuple(sorted((int(g[a]), int(mu[a])) for a in range(4) if mu[a] > 0))
                if key not in keys:
                    keys[key] = len(node_xyz)
                    y = sum(m / N * vtx[gid] for gid, m in key)
                    if affine:
                        x = y
                    else:
                        rho = sum(m / N * radii[gid] for gid, m in key)
                        x = rho * y / np.linalg.norm(y)
                    node_xyz.append(x)
                    node_verts.append(frozenset(gid for gid, _ in key))
                slot_node[t * nloc + n] = keys[key]
        self.xyz = np.array(node_xyz)
        self.slot_node = slot_node
        self.n = len(node_xyz)

        # boundary faces: faces of exactly one macro
        fc = {}
        for t in range(tet.shape[0]):
            for o in range(4):
                f = frozenset(int(v) for a, v in enumerate(tet[t]) if a != o)
                fc[f] = fc.get(f, 0) + 1
        bfaces = [f for f, c in fc.items() if c == 1]
        self.dirichlet = np.array(
            [any(s <= f for f in bfaces) for s in node_verts], dtype=bool)

        # fine tetrahedra -> element matrices -> COO
        rows, cols, vals = [], [], []
        vol_total = np.zeros(tet.shape[0])
        for t in range(tet.shape[0]):
            tets = []
            for c in loc:
                for ty in range(6):
                    v = c[None, :] + CELL[ty]
                    if (v.min() >= 0) and (v.sum(axis=1).max() <= N):
                        tets.append([t * nloc + lut[tuple(p)] for p in v])
            tets = np.array(tets, dtype=np.int64)
            ids = slot_node[tets]
            X = self.xyz[ids]                      # (m, 4, 3)
            E = X[:, 1:, :] - X[:, :1, :]          # (m, 3, 3) rows a, b, c
            det = np.linalg.det(E)
            inv = np.linalg.inv(E)                 # columns: grad(lambda_1..3)
            G = np.zeros((ids.shape[0], 4, 3))
            G[:, 1:, :] = np.transpose(inv, (0, 2, 1))
            G[:, 0, :] = -G[:, 1:, :].sum(axis=1)
            vol = np.abs(det) / 6.0
            vol_total[t] = vol.sum()
            K = vol[:, None, None] * np.einsum("mad,mbd->mab", G, G)
            rows.append(np.repeat(ids, 4, axis=1).reshape(-1))
            cols.append(np.tile(ids, (1, 4)).reshape(-1))
            vals.append(K.reshape(-1))
        self.macro_volume = vol_total
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n, self.n)).tocsr()
        self.A = A
        free = ~self.dirichlet
        self.free = free

    def node_values_from_block(self, b):
        """Node values from a consistent block vector (first copy)."""
        out = np.zeros(self.n)
        seen = np.zeros(self.n, dtype=bool)
        for s, n in enumerate(self.slot_node):
            if not seen[n]:
                out[n] = b[s]
                seen[n] = True
        return out

    def apply_block(self, xb):
        """y = L x with Dirichlet rows and columns removed, block layout."""
        x = self.node_values_from_block(xb)
        x[self.dirichlet] = 0.0
        y = self.A @ x
        y[self.dirichlet] = 0.0
        return y[self.slot_node]

    def solve_block(self, fb):
        """Exact discrete solution of L u = f on the free nodes."""
        import scipy.sparse.linalg as spla
        f = self.node_values_from_block(fb)
        free = self.free
        Aff = self.A[free][:, free].tocsc()
        u = np.zeros(self.n)
        u[free] = spla.spsolve(Aff, f[free])
        return u[self.slot_node]
