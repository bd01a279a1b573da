"""Gauss-Seidel sweeps and the V-cycle at the sizes the benchmark runs,
against the oracle, through the C ABI (oracle fits imported on every level):

- two sweeps on the 288-macro shell at level 6, every entry (the interface
  phases and all four volume colours; 1e-11, the 1e-12 bound per operation
  composed over two sweeps);
- one sweep at sampled nodes of every phase: the 288-macro shell at level 7
  (the benchmark's configuration, two-plane staging) and one macro at levels
  8 and 9 (4- and 8-wide staging).  The oracle replays the sweep over each
  sample's dependency cone (tests/gs_sampled.py), and every node of the
  cones is compared (1e-12: one sweep);
- one V(3,3) cycle on the 288-macro shell at level 6 (1e-10).

The first test is CPU only: the sampled replay equals the oracle's full
sweep bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402

from gs_sampled import sample_free_nodes, sweep_at_samples  # noqa: E402
from test_gpu_parity import TOL, block_of, pair, rel, share_fits  # noqa: E402


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("name,lam", [("shell288", 4), ("shell36", 4), ("single", 5)])
def test_sampled_sweep_equals_full_oracle_sweep(orc, name, lam):
    v, t = {"single": inputs.single_macro, "shell36": inputs.shell36,
            "shell288": inputs.shell288}[name]()
    O = orc.Mesh(v, t)
    N = 2 ** lam
    c = O.fit(N, orc.LSQP, 2, 2)
    nu = O.num_unique(N)
    u, f = inputs.uniform(nu, 4), inputs.uniform(nu, 5)
    u[O.dirichlet_mask(N)] = 0
    full = O.gs_sweep(N, f, u, kind=orc.LSQP, q=2, coeffs=c)
    s = sample_free_nodes(O, N, np.random.default_rng(lam), 200, 100)
    ids, vals = sweep_at_samples(O, N, f, u, s, kind=orc.LSQP, q=2, coeffs=c)
    assert set(s.tolist()) <= set(ids.tolist())
    assert np.array_equal(vals, full[ids])


@pytest.mark.gpu
def test_two_sweeps_shell288_level6_every_entry(ts):
    import oracle
    G, O = pair("shell288")
    lam, N = 6, 64
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    c = share_fits(op, O, lam)[-1]
    nu = O.num_unique(N)
    u, f = inputs.uniform(nu, 14), inputs.uniform(nu, 15)
    uo = O.gs_sweep(N, f, u, kind=oracle.LSQP, q=2, coeffs=c)
    uo = O.gs_sweep(N, f, uo, kind=oracle.LSQP, q=2, coeffs=c)
    ub = G.to_block(lam, u)
    op.smooth(lam, G.to_block(lam, f), ub, sweeps=2)
    assert rel(ub.cpu().numpy(), block_of(O, N, uo)) < 1e-11


@pytest.mark.gpu
@pytest.mark.parametrize("name,lam", [("shell288", 7), ("single", 8), ("single", 9)])
def test_one_sweep_sampled_every_phase(ts, name, lam):
    import oracle
    G, O = pair(name)
    N = 2 ** lam
    print("gs sampled sweep: %s level %d" % (name, lam), flush=True)
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    c = O.fit(N, oracle.LSQP, 2, 2)
    op.set_coeffs(lam, c)
    nu = O.num_unique(N)
    u, f = inputs.uniform(nu, 60), inputs.uniform(nu, 61)
    u[O.dirichlet_mask(N)] = 0
    rng = np.random.default_rng(100 + lam)
    s = sample_free_nodes(O, N, rng, 600, 300)
    ids, expect = sweep_at_samples(O, N, f, u, s, kind=oracle.LSQP, q=2, coeffs=c)
    phases = {O.gs_phase(N, int(v)) for v in ids}
    # every volume colour, and the interface phases where the mesh has free
    # interface nodes
    assert {6, 7, 8, 9} <= phases
    if name != "single":
        assert {0, 1, 2, 3, 4, 5} <= phases
    ub = G.to_block(lam, u)
    op.smooth(lam, G.to_block(lam, f), ub, sweeps=1)
    got = G.to_canon(lam, ub).cpu().numpy()[ids]
    assert rel(got, expect) < TOL


@pytest.mark.gpu
def test_vcycle_shell288_level6(ts):
    import oracle
    G, O = pair("shell288")
    lam, N = 6, 64
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    coeffs = share_fits(op, O, lam)
    mg = oracle.Multigrid(O, 2, lam, kind=oracle.LSQP, q=2, coeffs=coeffs)
    nu = O.num_unique(N)
    f = inputs.uniform(nu, 16)
    f[O.dirichlet_mask(N)] = 0
    u0 = inputs.uniform(nu, 17) * 1e-3
    uo = mg.vcycle(f, u0)
    sv = ts.Solver(op, lam)
    ub = G.to_block(lam, u0)
    sv.vcycle(G.to_block(lam, f), ub)
    assert rel(ub.cpu().numpy(), block_of(O, N, uo)) < 1e-10
