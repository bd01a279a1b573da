"""The largest levels through the C ABI vs the oracle: the wider staging of
the surrogate volume kernel (4 entries per lane from level 8 on, 8 at level
9), the largest blocks, and the transfers and load vector (32-bit block
indices) at those sizes.

One macro at levels 8 and 9 (N = 512: 22.6 M nodes) and the 36-macro shell
at level 8 (36 macros, not a multiple of the 8 XCDs: a ragged launch), with
the oracle's fit imported:
- apply and residual on sampled rows the oracle evaluates one by one, 1e-12
  relative in the max norm (FP64), and the FP32 apply at 2e-5 (FP32
  rounding of 15-term sums, as for the smaller levels);
- one Gauss-Seidel sweep, checked on sampled volume nodes of colour 0 at
  least two steps inside their macro: their neighbours are all volume nodes
  of the other three colours, so the sweep updates them from the initial
  values, u_I + (f_I - (L~u)_I) / s_mc(I), which the oracle evaluates per
  node.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402

from test_gpu_fullsize import _sample_rows  # noqa: E402
from test_gpu_parity import TOL, block_of, pair, rel  # noqa: E402


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


def _colour0_deep(O, N, rng, n):
    """n random (t, i, j, k) with i, j, k >= 2, i + j + k <= N - 2 and
    (i + 2j + 3k) mod 4 = 0, with their canonical row ids."""
    out, rows = [], []
    while len(out) < n:
        t = int(rng.integers(0, O.nt))
        i, j, k = (int(v) for v in rng.integers(2, N - 3, 3))
        if i + j + k > N - 2 or (i + 2 * j + 3 * k) % 4:
            continue
        out.append((t, i, j, k))
        rows.append(O.canon(N, t, i, j, k))
    return out, np.array(rows, dtype=np.int64)


@pytest.mark.parametrize("name,lam", [("single", 8), ("single", 9), ("shell36", 8)])
def test_largest_levels_sampled(ts, name, lam):
    import oracle
    G, O = pair(name)
    N = 2 ** lam
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    c = O.fit(N, oracle.LSQP, 2, 2)
    op.set_coeffs(lam, c)
    nu = O.num_unique(N)
    rng = np.random.default_rng(lam)
    rows = _sample_rows(O, N, rng, n_vol=4000, n_face=2000)
    x = inputs.uniform(nu, 40)
    f = inputs.uniform(nu, 41)
    xb, fb = G.to_block(lam, x), G.to_block(lam, f)
    yo = O.apply_rows(N, x, rows, kind=oracle.LSQP, q=2, coeffs=c)

    yc = G.to_canon(lam, op.apply(lam, xb)).cpu().numpy()
    assert rel(yc[rows], yo) < TOL
    rc = G.to_canon(lam, op.residual(lam, fb, xb)).cpu().numpy()
    assert rel(rc[rows], f[rows] - yo) < TOL
    del yc, rc

    y32 = op.apply(lam, xb.float(), dt=ts.TS_F32).double()
    y32c = G.to_canon(lam, y32).cpu().numpy()
    assert rel(y32c[rows], yo) < 2e-5
    del y32, y32c

    nodes, grow = _colour0_deep(O, N, rng, 1500)
    ub = xb.clone()
    op.smooth(lam, fb, ub, sweeps=1)
    uc = G.to_canon(lam, ub).cpu().numpy()
    lo = O.apply_rows(N, x, grow, kind=oracle.LSQP, q=2, coeffs=c)
    diag = np.array([oracle.poly_eval(2, N, c[t][0], i, j, k) for t, i, j, k in nodes])
    expect = x[grow] + (f[grow] - lo) / diag
    assert rel(uc[grow], expect) < TOL


@pytest.mark.parametrize("name,lam", [("single", 8), ("single", 9), ("shell36", 7)])
def test_transfers_largest_levels(ts, name, lam):
    """R = P^T and u_f += P u_c against the oracle on every entry (FP64);
    the 36-macro shell adds the face and edge rows of the restriction."""
    G, O = pair(name)
    Nf, Nc = 2 ** lam, 2 ** (lam - 1)
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    rf = inputs.uniform(O.num_unique(Nf), 50)
    rf[O.dirichlet_mask(Nf)] = 0
    rco = O.restrict(Nf, rf)
    rcb = G.zeros(lam - 1)
    ts.ts_restrict(op.h, lam, ts.TS_F64, G.to_block(lam, rf), rcb)
    assert rel(rcb.cpu().numpy(), block_of(O, Nc, rco)) < TOL
    del rf, rco, rcb
    uc = inputs.uniform(O.num_unique(Nc), 51)
    ufo = O.prolongate(Nf, uc)
    base = inputs.uniform(O.num_unique(Nf), 52)
    ufb = G.to_block(lam, base)
    ts.ts_prolongate_add(op.h, lam, ts.TS_F64, G.to_block(lam - 1, uc), ufb)
    base[O.dirichlet_mask(Nf)] = 0
    assert rel(ufb.cpu().numpy(), block_of(O, Nf, base + ufo)) < TOL


@pytest.mark.parametrize("kind", [0, 1])
def test_load_vector_level8(ts, kind):
    """The two-pass load vector (f once per slot, then the mass rows) against
    the oracle's on every entry, one macro at level 8."""
    G, O = pair("single")
    lam, N = 8, 256
    params = [0.55, 1.0] if kind == 0 else list(inputs.gaussian_bumps(3, 0.55))
    fo = O.rhs(N, kind, params)
    fb = G.rhs(lam, kind, params).cpu().numpy()
    assert rel(fb, block_of(O, N, fo)) < TOL
