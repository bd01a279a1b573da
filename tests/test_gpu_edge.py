"""Degenerate and malformed inputs through the C ABI: meshes the library must
refuse, a zero right-hand side, and a solver moved to a degenerate shell."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


def test_malformed_meshes_are_refused(ts):
    v, t = inputs.single_macro()
    # four coplanar vertices: a macro of zero volume
    flat = v.copy()
    flat[3] = (flat[0] + flat[1] + flat[2]) / 3.0
    with pytest.raises(ts.TSError) as e:
        ts.Mesh(flat, t)
    assert e.value.code == ts.TS_EINVAL
    # a vertex id out of range
    with pytest.raises(ts.TSError) as e:
        ts.Mesh(v, np.array([[0, 1, 2, 4]], dtype=np.int64))
    assert e.value.code == ts.TS_EINVAL
    # one face shared by three macros
    v3 = np.vstack([v, [[0.9, 0.9, 0.9]], [[-0.3, -0.2, -0.1]]])
    t3 = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], dtype=np.int64)
    with pytest.raises(ts.TSError) as e:
        ts.Mesh(v3, t3, geom=ts.TS_GEOM_AFFINE)
    assert e.value.code == ts.TS_EINVAL


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_rhs_gives_zero_without_a_cycle(ts, prec):
    # f = 0: the solution is 0 whatever the initial guess; the solve ends
    # before its first cycle, blocking and asynchronous alike
    lam = 4
    v, t = inputs.shell288(0.5, 1.0)
    G = ts.Mesh(v, t)
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    sv = ts.Solver(op, lam, precision=prec, rtol=1e-8)
    f = G.zeros(lam)
    u = G.to_block(lam, inputs.uniform(G.layout(lam).n_unique, 5))
    u, rc, info = sv.solve(f, u)
    assert rc == ts.TS_OK and info.cycles == 0 and info.rel_residual == 0.0
    assert int(torch.count_nonzero(u)) == 0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        u2 = torch.ones_like(f)
    sv.begin(f, u2, s)
    info2 = ts.ts_solve_info()
    while sv.query(info2) != ts.TS_SOLVE_DONE:
        pass
    torch.cuda.synchronize()
    assert info2.status == ts.TS_OK and info2.cycles == 0
    assert int(torch.count_nonzero(u2)) == 0


def test_solver_moved_to_a_degenerate_shell_is_unchanged(ts):
    lam = 4
    v, t = inputs.shell288(0.5, 1.0)
    G = ts.Mesh(v, t)
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    sv = ts.Solver(op, lam, precision=ts.TS_F32, rtol=1e-8)
    f = G.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(2, 0.5))
    u0, rc, _ = sv.solve(f)
    assert rc == ts.TS_OK
    bad = v.copy()
    a, b, c, d = t[0]
    bad[d] = (bad[a] + bad[b] + bad[c]) / 3.0  # flattens macro 0
    with pytest.raises(ts.TSError) as e:
        sv.set_vertices(bad)
    assert e.value.code == ts.TS_EINVAL
    u1, rc1, _ = sv.solve(f)
    assert rc1 == ts.TS_OK and torch.equal(u0, u1)
