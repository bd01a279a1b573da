"""The constant-stencil operator (TS_CONS: one stencil per macro, the exact
stencil of its unmapped fine tetrahedra; the paper's 29-FLOP lower bound,
Sec. 4.2.1 Tab. flops and Sec. 5 introduction) against the oracle's CONS
kind, through the C ABI.  The library computes the stencils on the device
and the oracle assembles every row from the affine coordinates, so nothing
is shared: FP64 applies and residuals at 1e-12, two sweeps at 1e-11, a
V-cycle at 1e-10, the FP32 apply at 2e-5, sampled rows at level 7 on the
288-macro shell (the benchmark's launch)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402

from gs_sampled import sample_free_nodes, sweep_at_samples  # noqa: E402
from test_gpu_fullsize import _sample_rows  # noqa: E402
from test_gpu_parity import TOL, block_of, pair, rel  # noqa: E402


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


def test_stencils_are_the_affine_macro_stencils(ts, orc):
    G, _ = pair("shell288")
    v, t = inputs.shell288()
    A = orc.Mesh(v, t, affine=True)
    for lam in (3, 5, 7):
        N = 2 ** lam
        op = ts.Operator(G, lam, method=ts.TS_CONS)
        c = op.coeffs(lam)[:, :, 0]
        ref = np.array([A.ifem_stencil(N, m, 2, 1, 1) for m in range(A.nt)])
        assert np.abs(c - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("name,lam", [("single", 5), ("shell36", 4), ("shell288", 4)])
def test_apply_residual_every_entry(ts, name, lam):
    import oracle
    G, O = pair(name)
    N = 2 ** lam
    op = ts.Operator(G, lam, method=ts.TS_CONS)
    nu = O.num_unique(N)
    x, f = inputs.uniform(nu, 70), inputs.uniform(nu, 71)
    yo = O.apply(N, x, kind=oracle.CONS)
    yb = op.apply(lam, G.to_block(lam, x)).cpu().numpy()
    assert rel(yb, block_of(O, N, yo)) < TOL
    ro = O.residual(N, f, x, kind=oracle.CONS)
    rb = op.residual(lam, G.to_block(lam, f), G.to_block(lam, x)).cpu().numpy()
    assert rel(rb, block_of(O, N, ro)) < TOL
    y32 = op.apply(lam, G.to_block(lam, x).float(), dt=ts.TS_F32).double().cpu().numpy()
    assert rel(y32, block_of(O, N, yo)) < 2e-5


def test_affine_mesh_gives_the_exact_operator(ts):
    import oracle
    G, O = pair("shell288", affine=True)
    lam, N = 4, 16
    op = ts.Operator(G, lam, method=ts.TS_CONS)
    x = inputs.uniform(O.num_unique(N), 72)
    yo = O.apply(N, x, kind=oracle.IFEM)
    yb = op.apply(lam, G.to_block(lam, x)).cpu().numpy()
    assert rel(yb, block_of(O, N, yo)) < TOL


def test_gauss_seidel_and_vcycle(ts):
    import oracle
    G, O = pair("shell288")
    lam, N = 4, 16
    op = ts.Operator(G, lam, method=ts.TS_CONS)
    nu = O.num_unique(N)
    u, f = inputs.uniform(nu, 73), inputs.uniform(nu, 74)
    uo = O.gs_sweep(N, f, u, kind=oracle.CONS)
    uo = O.gs_sweep(N, f, uo, kind=oracle.CONS)
    ub = G.to_block(lam, u)
    op.smooth(lam, G.to_block(lam, f), ub, sweeps=2)
    assert rel(ub.cpu().numpy(), block_of(O, N, uo)) < 1e-11
    mg = oracle.Multigrid(O, 2, lam, kind=oracle.CONS)
    f[O.dirichlet_mask(N)] = 0
    u0 = inputs.uniform(nu, 75) * 1e-3
    vo = mg.vcycle(f, u0)
    sv = ts.Solver(op, lam)
    vb = G.to_block(lam, u0)
    sv.vcycle(G.to_block(lam, f), vb)
    assert rel(vb.cpu().numpy(), block_of(O, N, vo)) < 1e-10


def test_level7_shell288_sampled(ts):
    import oracle
    G, O = pair("shell288")
    lam, N = 7, 128
    op = ts.Operator(G, lam, method=ts.TS_CONS)
    nu = O.num_unique(N)
    rng = np.random.default_rng(7)
    rows = _sample_rows(O, N, rng, n_vol=3000, n_face=1500)
    x, f = inputs.uniform(nu, 76), inputs.uniform(nu, 77)
    x[O.dirichlet_mask(N)] = 0
    xb, fb = G.to_block(lam, x), G.to_block(lam, f)
    yo = O.apply_rows(N, x, rows, kind=oracle.CONS)
    yc = G.to_canon(lam, op.apply(lam, xb)).cpu().numpy()
    assert rel(yc[rows], yo) < TOL
    s = sample_free_nodes(O, N, rng, 400, 200)
    ids, expect = sweep_at_samples(O, N, f, x, s, kind=oracle.CONS)
    op.smooth(lam, fb, xb, sweeps=1)
    got = G.to_canon(lam, xb).cpu().numpy()[ids]
    assert rel(got, expect) < TOL
