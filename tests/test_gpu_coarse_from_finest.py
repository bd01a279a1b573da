"""The finest level's surrogate polynomials on the coarser levels (the remark
in Sec. 3.4 on using the fine-level polynomial on the coarser meshes;
ts_op_params.coarse_from_finest) through the C ABI against the oracle: the
coarse coefficients are the finest ones scaled by the mesh-size ratio
(exactly, a power of two), and the oracle's V-cycle with those coefficients
matches the library's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402

from test_gpu_parity import block_of, pair, rel  # noqa: E402


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


def test_coarse_coefficients_are_the_scaled_finest(ts):
    G, _ = pair("shell288")
    lam = 5
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2, coarse_from_finest=True)
    ref = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    fine = op.coeffs(lam)
    # the finest level is fitted as without the option
    assert np.array_equal(fine, ref.coeffs(lam))
    for lev in range(3, lam):
        assert np.array_equal(op.coeffs(lev), fine * 2.0 ** (lam - lev))
        # and differs from that level's own fit (by a fraction of a percent)
        own = ref.coeffs(lev)
        d = np.abs(op.coeffs(lev) - own).max() / np.abs(own).max()
        assert 0.0 < d < 0.05


def test_vcycle_and_solve_against_the_oracle(ts):
    import oracle
    G, O = pair("shell288")
    lam, N = 5, 32
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2, coarse_from_finest=True)
    coeffs = [None] + [op.coeffs(lev) for lev in range(3, lam + 1)]
    mg = oracle.Multigrid(O, 2, lam, kind=oracle.LSQP, q=2, coeffs=coeffs)
    f = O.rhs(N, 0, [0.55, 1.0])
    u0 = inputs.uniform(O.num_unique(N), 12) * 1e-3
    uo = mg.vcycle(f, u0)
    ub = G.to_block(lam, u0)
    ts.Solver(op, lam).vcycle(G.to_block(lam, f), ub)
    assert rel(ub.cpu().numpy(), block_of(O, N, uo)) < 1e-10
    # a solve to 1e-10, as with one fit per level; the oracle measures the
    # answer's residual
    ub, rc, info = ts.Solver(op, lam, rtol=1e-10).solve(G.to_block(lam, f))
    assert rc == ts.TS_OK and info.rel_residual <= 1e-10
    ug = G.to_canon(lam, ub).cpu().numpy()
    r = O.residual(N, f, ug, kind=oracle.LSQP, q=2, coeffs=coeffs[-1])
    assert O.norm_free(N, r) / O.norm_free(N, f) <= 1.05e-10
    _, rc2, info2 = ts.Solver(ts.Operator(G, lam, method=ts.TS_LSQP, q=2), lam,
                              rtol=1e-10).solve(G.to_block(lam, f))
    print("cycles to 1e-10: coarse from finest %d, one fit per level %d"
          % (info.cycles, info2.cycles))
    assert rc2 == ts.TS_OK and abs(info.cycles - info2.cycles) <= 3


def test_refused_for_the_symmetric_surrogate(ts):
    G, _ = pair("shell288")
    with pytest.raises(ts.TSError) as e:
        ts.Operator(G, 4, method=ts.TS_LSQP_SYM, q=2, coarse_from_finest=True)
    assert e.value.code == ts.TS_EINVAL
