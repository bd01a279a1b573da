"""Double discretisation (Sec. 4 introduction) through the C ABI vs the oracle.

The cycle smooths with the surrogate and computes every residual with the
exact element-wise rows; the solve stops on the relative update.  The oracle's
fit is imported, so both sides run the same two operators.  A V-cycle composes
several FP64 operations of 1e-12 relative each (the same bound as the plain
V-cycle test); the stopped solves are compared on the iterate, whose distance
to the fixed point is of the order of the last update.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402

from test_gpu_parity import block_of, pair, rel, share_fits  # noqa: E402


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("name,lam", [("shell36", 4), ("shell288", 4)])
def test_dd_vcycle(ts, name, lam):
    import oracle
    G, O = pair(name)
    N = 2 ** lam
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    coeffs = share_fits(op, O, lam)
    mg = oracle.Multigrid(O, 2, lam, kind=oracle.LSQP, q=2, coeffs=coeffs, dd=True)
    f = O.rhs(N, 0, [0.55, 1.0])
    u0 = inputs.uniform(O.num_unique(N), 14) * 1e-3
    uo = mg.vcycle(f, mg.vcycle(f, u0))
    sv = ts.Solver(op, lam, dd=True)
    ub = G.to_block(lam, u0)
    fb = G.to_block(lam, f)
    sv.vcycle(fb, ub)
    sv.vcycle(fb, ub)
    assert rel(ub.cpu().numpy(), block_of(O, N, uo)) < 1e-10


def test_dd_solve_matches_oracle(ts):
    import oracle
    G, O = pair("shell36")
    lam, N = 4, 16
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    coeffs = share_fits(op, O, lam)
    mg = oracle.Multigrid(O, 2, lam, kind=oracle.LSQP, q=2, coeffs=coeffs, dd=True)
    f = O.rhs(N, 0, [0.55, 1.0])
    uo, cyc, hist = mg.solve_dd(f, rtol=1e-10, max_cycles=60)
    assert cyc > 0
    sv = ts.Solver(op, lam, rtol=1e-10, dd=True)
    ub, rc, info = sv.solve(G.to_block(lam, f))
    assert rc == ts.TS_OK
    assert abs(info.cycles - cyc) <= 1
    k = min(info.cycles, cyc)
    gh = np.array(info.hist[: info.n_hist])
    assert info.n_hist == info.cycles and info.rel_residual == gh[-1] <= 1e-10
    assert rel(gh[: k - 1], hist[: k - 1]) < 1e-6
    ug = G.to_canon(lam, ub).cpu().numpy()
    assert rel(ug, uo) < 1e-8
    # the answer is the mixed scheme's fixed point, not the solution of
    # either operator: both residuals stay well above the update size
    nf = O.norm_free(N, f)
    rL = O.norm_free(N, O.residual(N, f, ug, kind=oracle.IFEM)) / nf
    rS = O.norm_free(N, O.residual(N, f, ug, kind=oracle.LSQP, q=2, coeffs=coeffs[-1])) / nf
    assert rL > 1e-3 and rS > 1e-3


def test_dd_async_steps_match_blocking_solve(ts):
    G, O = pair("shell288")
    lam, N = 4, 16
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    share_fits(op, O, lam)
    fb = G.to_block(lam, O.rhs(N, 0, [0.55, 1.0]))
    sv = ts.Solver(op, lam, rtol=1e-9, dd=True)
    ua, rc, info = sv.solve(fb)
    assert rc == ts.TS_OK
    sv2 = ts.Solver(op, lam, rtol=1e-9, dd=True)
    ub = G.zeros(lam)
    sv2.begin(fb, ub)
    inf = ts.ts_solve_info()
    while True:
        st = sv2.query(inf)
        if st == ts.TS_SOLVE_DONE:
            break
        if st == ts.TS_SOLVE_READY:
            sv2.step()
    torch.cuda.synchronize()
    assert inf.status == ts.TS_OK and inf.cycles == info.cycles
    assert torch.equal(ua, ub)


def test_dd_requires_fp64(ts):
    G, _ = pair("shell288")
    op = ts.Operator(G, 3, method=ts.TS_LSQP, q=2)
    for prec in (ts.TS_F32, ts.TS_F16W):
        with pytest.raises(ts.TSError) as e:
            ts.Solver(op, 3, precision=prec, dd=True)
        assert e.value.code == ts.TS_EINVAL


def test_dd_keeps_the_fem_error_order(ts):
    # Sec. 4.1 (the study of the error over refinement levels): on the
    # 288-macro shell the pure surrogate's error to the manufactured solution
    # stops decaying like h^2, while the mixed scheme stays on the Galerkin
    # solution's error.  Error: sum over nodes of V_I (u_exact - u_I)^2, V_I a
    # quarter of the volume of the node's fine tetrahedra.
    import oracle
    G, O = pair("shell288")
    err = {}
    for lam in (5, 6):
        N = 2 ** lam
        ue = oracle.exact_manufactured(0.55, 1.0, O.coords(N))
        V = O.node_volumes(N)
        fb = G.rhs(lam, ts.TS_RHS_MANUFACTURED, [0.55, 1.0])
        for name, meth, dd in (("ifem", ts.TS_IFEM, False), ("lsqp", ts.TS_LSQP, False),
                               ("dd", ts.TS_LSQP, True)):
            op = ts.Operator(G, lam, method=meth, q=2)
            u, rc, _ = ts.Solver(op, lam, rtol=1e-10, max_cycles=100, dd=dd).solve(fb)
            assert rc == ts.TS_OK
            uc = G.to_canon(lam, u).cpu().numpy()
            err[name, lam] = np.sqrt((V * (uc - ue) ** 2).sum())
    assert err["dd", 6] < 1.01 * err["ifem", 6]
    assert err["lsqp", 6] > 2.0 * err["ifem", 6]
    assert err["dd", 5] / err["dd", 6] > 3.5
    assert err["lsqp", 5] / err["lsqp", 6] < 2.0
