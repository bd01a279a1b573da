"""One multicolour Gauss-Seidel sweep evaluated by the oracle at sampled
nodes only (for levels whose full oracle sweep would take minutes).

A sweep visits the phases 0..9 in order (vertices, edges, faces, volume
colours) and updates every node of a phase from the values at the start of
that phase (eq. iteration-scheme in multicolour order).  The value a node ends
with therefore depends on the new values of its neighbours in earlier phases,
and theirs on their earlier-phase neighbours: a cone of at most ten phases.
sweep_at_samples collects that cone for every sample and replays the phases
over it with the oracle's row-wise update (or_gs_rows).
"""
import numpy as np


def sweep_at_samples(O, N, f, x0, samples, **kw):
    """Returns (ids, values): every node of the samples' cones (the samples
    included) and its value after one sweep started from x0."""
    phase = {}

    def ph(u):
        p = phase.get(u)
        if p is None:
            p = phase[u] = O.gs_phase(N, u)
        return p

    need = set(int(u) for u in samples)
    stack = list(need)
    while stack:
        u = stack.pop()
        pu = ph(u)
        for v in O.row_neighbours(N, u):
            v = int(v)
            if v not in need and ph(v) < pu:
                need.add(v)
                stack.append(v)
    x = np.array(x0, dtype=np.float64, copy=True)
    ids = np.array(sorted(need), dtype=np.int64)
    ph_of = np.array([ph(int(u)) for u in ids])
    for p in range(10):
        rows = ids[ph_of == p]
        if rows.size:
            x[rows] = O.gs_rows(N, f, x, rows, **kw)
    return ids, x[ids]


def sample_free_nodes(O, N, rng, n_vol, n_lower, deep=0):
    """Random free nodes: n_vol interior nodes of random macros (at least
    `deep` steps inside), n_lower free face / edge / vertex nodes, and every
    free macro vertex (too few to be drawn at random)."""
    out = []
    while len(out) < n_vol:
        t = int(rng.integers(0, O.nt))
        i, j, k = (int(v) for v in rng.integers(1 + deep, N - 2 - deep, 3))
        if i + j + k > N - 1 - deep:
            continue
        out.append(O.canon(N, t, i, j, k))
    n_vol_base = O.nv + O.ne * (N - 1) + O.nf * (N - 1) * (N - 2) // 2
    dmask = O.dirichlet_mask(N)[:n_vol_base]
    free_lower = np.flatnonzero(~dmask)
    if free_lower.size and n_lower:
        out += [int(u) for u in rng.choice(free_lower, size=min(n_lower, free_lower.size),
                                           replace=False)]
    out += [int(u) for u in np.flatnonzero(~dmask[:O.nv])]
    return np.unique(np.array(out, dtype=np.int64))
