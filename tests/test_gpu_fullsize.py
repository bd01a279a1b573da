"""Large levels through the C ABI vs the oracle.

Level 6 is compared on every entry.  Level 7 of the 288-macro shell (the
benchmark workload, in the launch configuration the benchmark times, with the
lower-primitive rows running beside the volume kernel) is compared on sampled
rows the oracle evaluates one by one: random volume and face rows and every
edge and vertex row.  The oracle's own fit is imported, so both sides apply the
same operator; tolerance 1e-12 relative in the max norm.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402

from test_gpu_parity import TOL, block_of, pair, rel  # noqa: E402


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("name", ["shell36", "shell288"])
def test_level6_apply_and_residual_every_entry(ts, name):
    import oracle
    G, O = pair(name)
    lam, N = 6, 64
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    c = O.fit(N, oracle.LSQP, 2, 2)
    op.set_coeffs(lam, c)
    nu = O.num_unique(N)
    x, f = inputs.uniform(nu, 31), inputs.uniform(nu, 32)
    yo = O.apply(N, x, kind=oracle.LSQP, q=2, coeffs=c)
    yb = op.apply(lam, G.to_block(lam, x)).cpu().numpy()
    assert rel(yb, block_of(O, N, yo)) < TOL
    ro = O.residual(N, f, x, kind=oracle.LSQP, q=2, coeffs=c)
    rb = op.residual(lam, G.to_block(lam, f), G.to_block(lam, x)).cpu().numpy()
    assert rel(rb, block_of(O, N, ro)) < TOL


def _sample_rows(O, N, rng, n_vol=6000, n_face=6000):
    """Canonical row ids: all vertices and edge nodes, random face and volume
    nodes, all free."""
    nv, ne, nf = O.nv, O.ne, O.nf
    n_edge = nv + ne * (N - 1)
    n_low = n_edge + nf * (N - 1) * (N - 2) // 2
    nu = O.num_unique(N)
    rows = np.concatenate([np.arange(n_edge),
                           rng.integers(n_edge, n_low, n_face),
                           rng.integers(n_low, nu, n_vol)])
    rows = np.unique(rows)
    mask = O.dirichlet_mask(N)
    return rows[~mask[rows]]


def test_level7_shell288_sampled_rows(ts):
    import oracle
    G, O = pair("shell288")
    lam, N = 7, 128
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2, sample_j=2)
    c = O.fit(N, oracle.LSQP, 2, 2)
    op.set_coeffs(lam, c)
    nu = O.num_unique(N)
    x = inputs.uniform(nu, 0)
    f = inputs.uniform(nu, 1)
    xb = G.to_block(lam, x)
    yb = op.apply(lam, xb)
    yc = G.to_canon(lam, yb).cpu().numpy()
    rows = _sample_rows(O, N, np.random.default_rng(5))
    yo = O.apply_rows(N, x, rows, kind=oracle.LSQP, q=2, coeffs=c)
    assert rel(yc[rows], yo) < TOL
    # every copy of every node holds the same value: the canonical vector
    # read back from the first copies reproduces the block vector exactly
    back = G.to_block(lam, yc)
    assert torch.equal(back, yb)
    # residual in the same configuration
    rb = op.residual(lam, G.to_block(lam, f), xb)
    rc = G.to_canon(lam, rb).cpu().numpy()
    assert rel(rc[rows], f[rows] - yo) < TOL
    # the Dirichlet rows are zero
    mask = O.dirichlet_mask(N)
    assert not np.any(yc[mask])
