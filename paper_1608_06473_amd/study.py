"""Discretisation error over levels, macro meshes and stencil schemes on the
GPU: an analogue of the paper's study of the refinement level, the macro mesh
size H and the polynomial degree q (Sec. 4.1, Tab. hHstudy), on the
cubed-sphere shells of 36, 288 and 2,304 macros (the paper's meshes are not
available).

For each (mesh, level, scheme) the manufactured problem
u = sin(pi (r - r1) / (r2 - r1)) x y z, f = -Laplace u, on the shell
r1 = 0.55 <= |x| <= r2 = 1 with zero Dirichlet data is solved by V(3,3)
cycles in FP64 to a relative residual of 1e-10 (relative update for double
discretisation), and the error to the exact solution is measured as
e = (sum_I V_I (u(x_I) - u_I)^2)^(1/2) over the unique nodes, V_I a quarter
of the volume of the node's fine tetrahedra (the consistent mass matrix
applied to the constant 1).  Schemes: the exact element-wise operator
(IFEM), LSQP of degree 1..4 with sampling j = 2, IPOLY (q = 2), and double
discretisation with LSQP q = 2 (Sec. 4 introduction).

    python -m paper_1608_06473_amd.study [--meshes 36,288,2304] [--levels 3-6]
"""
from __future__ import annotations

import argparse
import json
import math
import time

from . import (TS_F64, TS_IFEM, TS_IPOLY, TS_LSQP, TS_OK, TS_RHS_MANUFACTURED, TS_RHS_ONE, Mesh,
               Operator, Solver, inputs)

R1, R2 = 0.55, 1.0

MESHES = {36: inputs.shell36, 288: inputs.shell288, 2304: inputs.shell2304}

SCHEMES = [
    ("IFEM", dict(method=TS_IFEM), False),
    ("LSQP q=1", dict(method=TS_LSQP, q=1), False),
    ("LSQP q=2", dict(method=TS_LSQP, q=2), False),
    ("LSQP q=3", dict(method=TS_LSQP, q=3), False),
    ("LSQP q=4", dict(method=TS_LSQP, q=4), False),
    ("IPOLY q=2", dict(method=TS_IPOLY, q=2), False),
    ("LSQP q=2 DD", dict(method=TS_LSQP, q=2), True),
]


def exact_solution(X):
    """The manufactured solution at points X (n x 3, torch)."""
    r = X.norm(dim=1)
    return (math.pi * (r - R1) / (R2 - R1)).sin() * X[:, 0] * X[:, 1] * X[:, 2]


def error_norm(mesh, lam, u):
    """(sum_I V_I (u(x_I) - u_I)^2)^(1/2) over the unique nodes."""
    import torch
    V = mesh.to_canon(lam, mesh.rhs(lam, TS_RHS_ONE))
    X = mesh.coords(lam)
    Xc = torch.stack([mesh.to_canon(lam, X[:, d].contiguous()) for d in range(3)], dim=1)
    d = exact_solution(Xc) - mesh.to_canon(lam, u)
    return float((V * d * d).sum().sqrt())


def run_case(mesh, lam, kw, dd, rtol=1e-10, max_cycles=100):
    """Solve on one level with one scheme; returns (status, cycles, error,
    seconds)."""
    import torch
    t0 = time.perf_counter()
    op = Operator(mesh, lam, sample_j=2, **kw)
    sv = Solver(op, lam, rtol=rtol, max_cycles=max_cycles, precision=TS_F64, dd=dd)
    f = mesh.rhs(lam, TS_RHS_MANUFACTURED, [R1, R2])
    u, rc, info = sv.solve(f, raise_on_fail=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err = error_norm(mesh, lam, u) if rc == TS_OK else float("nan")
    del sv, op
    return rc, info.cycles, err, dt


def study(meshes=(36, 288, 2304), levels=(3, 4, 5, 6), max_dof=1.2e8, log=print):
    """Run every scheme on every (mesh, level) with at most max_dof unknowns;
    returns a list of records."""
    out = []
    for nm in meshes:
        v, t = MESHES[nm](R1, R2)
        mesh = Mesh(v, t)
        for lam in levels:
            info = mesh.layout(lam)
            if info.n_free > max_dof:
                continue
            for name, kw, dd in SCHEMES:
                rc, cyc, err, dt = run_case(mesh, lam, kw, dd)
                rec = {"macros": nm, "level": lam, "dof": int(info.n_free), "scheme": name,
                       "status": int(rc), "cycles": int(cyc), "error": err, "s": round(dt, 3)}
                out.append(rec)
                log(json.dumps(rec))
    return out


def table(records):
    """Markdown table: error per scheme (columns) and (mesh, level) (rows),
    with the ratio to the next coarser level in parentheses."""
    names = [n for n, _, _ in SCHEMES]
    by = {(r["macros"], r["level"], r["scheme"]): r for r in records}
    rows = sorted({(r["macros"], r["level"]) for r in records})
    lines = ["| macros | level | DoF | " + " | ".join(names) + " |",
             "|---" * (3 + len(names)) + "|"]
    for nm, lam in rows:
        cells = []
        for n in names:
            r = by.get((nm, lam, n))
            if r is None:
                cells.append("")
                continue
            if r["status"] != TS_OK:
                cells.append("no conv.")
                continue
            c = "%.3e" % r["error"]
            p = by.get((nm, lam - 1, n))
            if p is not None and p["status"] == TS_OK and r["error"] > 0:
                c += " (%.2f)" % (p["error"] / r["error"])
            cells.append(c)
        lines.append("| %d | %d | %d | " % (nm, lam, by[(nm, lam, names[0])]["dof"])
                     + " | ".join(cells) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--meshes", default="36,288,2304")
    ap.add_argument("--levels", default="3-6")
    ap.add_argument("--max-dof", type=float, default=1.2e8)
    args = ap.parse_args()
    a, b = (int(x) for x in args.levels.split("-"))
    recs = study(tuple(int(m) for m in args.meshes.split(",")), tuple(range(a, b + 1)),
                 args.max_dof, log=lambda s: print(s, flush=True))
    print(table(recs), flush=True)


if __name__ == "__main__":
    main()
