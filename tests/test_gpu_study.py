"""The discretisation-error study (Sec. 4.1, Tab. hHstudy analogue) on the
288-macro shell at levels 4 and 5: the trends the paper reports.

- the exact operator converges like h^2 (error ratio about 4 per level);
- degree 1 surrogates stagnate, the surrogate error falls with the degree,
  and LSQP beats IPOLY at q = 2;
- double discretisation keeps the exact operator's error.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def recs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_06473_amd import study
    out = study.study(meshes=(288,), levels=(4, 5), log=lambda s: None)
    return {(r["level"], r["scheme"]): r for r in out}


def test_all_converge(recs):
    from paper_1608_06473_amd import TS_OK
    assert all(r["status"] == TS_OK for r in recs.values())


def test_trends(recs):
    e = {k: r["error"] for k, r in recs.items()}
    assert 3.5 < e[4, "IFEM"] / e[5, "IFEM"] < 4.5
    assert e[5, "LSQP q=1"] > 3 * e[5, "IFEM"]                # q = 1 stagnates
    assert e[5, "LSQP q=1"] > e[5, "LSQP q=2"]
    assert abs(e[5, "LSQP q=4"] - e[5, "IFEM"]) < 0.05 * e[5, "IFEM"]
    assert e[5, "IPOLY q=2"] > e[5, "LSQP q=2"]               # LSQP fits better
    assert abs(e[5, "LSQP q=2 DD"] - e[5, "IFEM"]) < 0.01 * e[5, "IFEM"]


@pytest.mark.parametrize("nm,lam", [(36, 3), (36, 4), (288, 3)])
def test_errors_match_oracle_solves(nm, lam):
    """Every entry of the study at small sizes against the oracle's own
    solve: its fits, its V(3,3) cycles to the same tolerance (the update for
    double discretisation), its node volumes and coordinates.  Both solves
    stop within 1e-10 of the discrete solution, so the errors agree to about
    1e-10 / (e / |u|); the bound is 1e-6 relative."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import numpy as np

    import oracle
    from paper_1608_06473_amd import TS_IFEM, TS_IPOLY, TS_OK, Mesh, study
    v, t = study.MESHES[nm](study.R1, study.R2)
    G, O = Mesh(v, t), oracle.Mesh(v, t)
    N = 2 ** lam
    f = O.rhs(N, 0, [study.R1, study.R2])
    X = O.coords(N)
    r = np.linalg.norm(X, axis=1)
    ue = np.sin(np.pi * (r - study.R1) / (study.R2 - study.R1)) * X[:, 0] * X[:, 1] * X[:, 2]
    V = O.node_volumes(N)
    for name, kw, dd in study.SCHEMES:
        rc, _, eg, _ = study.run_case(G, lam, kw, dd)
        assert rc == TS_OK, name
        meth = kw["method"]
        q = kw.get("q", 2)
        kind = {TS_IFEM: oracle.IFEM, TS_IPOLY: oracle.IPOLY}.get(meth, oracle.LSQP)
        coeffs = None
        if meth != TS_IFEM:
            coeffs = [None] + [O.fit(2 ** l, kind, q, 2) for l in range(3, lam + 1)]
        mg = oracle.Multigrid(O, 2, lam, kind=kind, q=q, coeffs=coeffs, dd=dd)
        if dd:
            u, c, _ = mg.solve_dd(f, rtol=1e-10, max_cycles=100)
        else:
            u, c, _ = mg.solve(f, rtol=1e-10, max_cycles=100)
        assert c > 0, name
        eo = float(np.sqrt(np.sum(V * (ue - u) ** 2)))
        assert abs(eg - eo) <= 1e-6 * eo, (name, eg, eo)
