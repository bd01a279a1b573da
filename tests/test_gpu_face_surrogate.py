"""Surrogate rows on interior faces through the C ABI vs the oracle.

The volume coefficients are the oracle's (imported), so the volume rows are
the same operator on both sides; each side fits its own face polynomials
(GPU: FP64 normal equations in the first macro's face coordinates with one
step of iterative refinement on the FP64 residual, oracle: Householder QR in
the face frame), the same least-squares function up to rounding, so the
operators meet the 1e-12 bound of the applies (measured on MI355X:
1.1e-15 .. 1.6e-14, q = 2 and q = 4).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1608_06473_amd import inputs  # noqa: E402

from test_gpu_parity import block_of, pair, rel, share_fits  # noqa: E402

OWN = {2: 1e-12, 4: 1e-12}
GS2 = 1e-11  # two Gauss-Seidel sweeps: the apply bound per operation, composed


@pytest.fixture(scope="module")
def ts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1608_06473_amd as m
    m.lib()
    return m


def _ops(ts, O, G, lam, q=2):
    """Library operator with face fits and the oracle's volume fits; the
    oracle's (volume, face) coefficients of the finest level."""
    import oracle
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=q, face_surrogate=True)
    cf = share_fits(op, O, lam, q=q)
    fc = [None] + [O.face_fit(2 ** l, q=q) for l in range(3, lam + 1)]
    assert oracle.num_coeffs2(q) == fc[-1].shape[2]
    return op, cf, fc


@pytest.mark.parametrize("name,lam,q", [("shell36", 4, 2), ("shell288", 4, 2), ("shell288", 5, 2),
                                        ("shell288", 4, 4), ("shell36", 3, 2)])
def test_apply_and_residual(ts, name, lam, q):
    import oracle
    G, O = pair(name)
    N = 2 ** lam
    op, cf, fc = _ops(ts, O, G, lam, q)
    nu = O.num_unique(N)
    x, f = inputs.uniform(nu, 21), inputs.uniform(nu, 22)
    yo = O.apply(N, x, kind=oracle.LSQP, q=q, coeffs=cf[-1], fcoeffs=fc[-1])
    yb = op.apply(lam, G.to_block(lam, x)).cpu().numpy()
    assert rel(yb, block_of(O, N, yo)) < OWN[q]
    ro = O.residual(N, f, x, kind=oracle.LSQP, q=q, coeffs=cf[-1], fcoeffs=fc[-1])
    rb = op.residual(lam, G.to_block(lam, f), G.to_block(lam, x)).cpu().numpy()
    assert rel(rb, block_of(O, N, ro)) < OWN[q]
    # the face fits change the face rows only: without them the operator is
    # the one with exact face rows
    ye = O.apply(N, x, kind=oracle.LSQP, q=q, coeffs=cf[-1])
    lo = O.nv + O.ne * (N - 1)
    hi = lo + O.nf * (N - 1) * (N - 2) // 2
    d = np.abs(yo - ye)
    assert d[:lo].max() == 0 and d[hi:].max() == 0 and d[lo:hi].max() > 0


@pytest.mark.parametrize("dt", [0, 1])
def test_gauss_seidel_sweep(ts, dt):
    import oracle
    G, O = pair("shell288")
    lam, N = 4, 16
    op, cf, fc = _ops(ts, O, G, lam)
    nu = O.num_unique(N)
    u, f = inputs.uniform(nu, 4), inputs.uniform(nu, 5)
    uo = O.gs_sweep(N, f, u, kind=oracle.LSQP, q=2, coeffs=cf[-1], fcoeffs=fc[-1])
    uo = O.gs_sweep(N, f, uo, kind=oracle.LSQP, q=2, coeffs=cf[-1], fcoeffs=fc[-1])
    ub = G.to_block(lam, u)
    fb = G.to_block(lam, f)
    if dt == 0:
        op.smooth(lam, fb, ub, sweeps=2)
        assert rel(ub.cpu().numpy(), block_of(O, N, uo)) < GS2
    else:  # FP32 vectors, FP64 face-row evaluation
        u32 = ub.float()
        op.smooth(lam, fb.float(), u32, sweeps=2, dt=ts.TS_F32)
        assert rel(u32.double().cpu().numpy(), block_of(O, N, uo)) < 1e-5


def test_vcycle_and_dd_vcycle(ts):
    import oracle
    G, O = pair("shell288")
    lam, N = 4, 16
    op, cf, fc = _ops(ts, O, G, lam)
    f = O.rhs(N, 0, [0.55, 1.0])
    u0 = inputs.uniform(O.num_unique(N), 12) * 1e-3
    for dd in (False, True):
        mg = oracle.Multigrid(O, 2, lam, kind=oracle.LSQP, q=2, coeffs=cf, fcoeffs=fc, dd=dd)
        uo = mg.vcycle(f, u0)
        sv = ts.Solver(op, lam, dd=dd)
        ub = G.to_block(lam, u0)
        sv.vcycle(G.to_block(lam, f), ub)
        assert rel(ub.cpu().numpy(), block_of(O, N, uo)) < 1e-10


def test_level6_every_entry_and_level7_sampled_rows(ts):
    import oracle
    from test_gpu_fullsize import _sample_rows
    G, O = pair("shell288")
    for lam in (6, 7):
        N = 2 ** lam
        op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2, face_surrogate=True)
        c = O.fit(N, oracle.LSQP, 2, 2)
        op.set_coeffs(lam, c)
        fc = O.face_fit(N, q=2)
        nu = O.num_unique(N)
        x = inputs.uniform(nu, 0)
        yb = op.apply(lam, G.to_block(lam, x))
        yc = G.to_canon(lam, yb).cpu().numpy()
        if lam == 6:
            yo = O.apply(N, x, kind=oracle.LSQP, q=2, coeffs=c, fcoeffs=fc)
            assert rel(yc, yo) < OWN[2]
        else:
            rows = _sample_rows(O, N, np.random.default_rng(6), n_vol=2000, n_face=20000)
            yo = O.apply_rows(N, x, rows, kind=oracle.LSQP, q=2, coeffs=c, fcoeffs=fc)
            assert rel(yc[rows], yo) < OWN[2]
        del op


def test_flagged_level_keeps_exact_face_rows(ts):
    # where the selective surrogate keeps IFEM volume rows on some macro, the
    # level keeps the exact face rows: the operator equals the one built
    # without face fits, bit for bit
    G, O = pair("shell36")
    lam = 4
    a = ts.Operator(G, lam, method=ts.TS_LSQP, q=2, fallback_tol=0.01, face_surrogate=True)
    b = ts.Operator(G, lam, method=ts.TS_LSQP, q=2, fallback_tol=0.01)
    assert a.macro_flags(lam).any()
    xb = G.to_block(lam, inputs.uniform(O.num_unique(2 ** lam), 3))
    assert torch.equal(a.apply(lam, xb), b.apply(lam, xb))
