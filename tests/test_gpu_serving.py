"""Asynchronous solves and the continuous-batching request loop.

- the non-blocking begin / step / query sequence, and the batched step over
  several solvers, reproduce the blocking solves bitwise;
- requests solved alone and inside a mix of concurrent requests give bitwise
  identical solutions (tolerance 0: no atomics, fixed reduction order);
- the oracle's operator measures the residual of a served solution.
"""
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


@pytest.mark.parametrize("prec", [0, 1])
def test_async_steps_match_blocking_solve(ts, prec):
    v, t = inputs.shell288(0.5, 1.0)
    G = ts.Mesh(v, t)
    lam = 5
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
    sv = ts.Solver(op, lam, precision=prec, rtol=1e-8)
    f = G.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(4, 0.5))
    u1, rc, info1 = sv.solve(f)
    assert rc == ts.TS_OK
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        u2 = G.zeros(lam)
    sv.begin(f, u2, s)
    info2 = ts.ts_solve_info()
    steps = 0
    while True:
        st = sv.query(info2)
        if st == ts.TS_SOLVE_DONE:
            break
        if st == ts.TS_SOLVE_READY:
            sv.step()
            steps += 1
    torch.cuda.synchronize()
    assert info2.status == ts.TS_OK and steps == info1.cycles == info2.cycles
    assert info2.rel_residual == info1.rel_residual
    assert torch.equal(u1, u2)


def test_batched_steps_match_blocking_solves(ts):
    # three solves (two meshes, two levels, two precisions) on streams of
    # their own, advanced only through the batched step: each ends bitwise
    # where its blocking solve ends
    cases = []
    for r_in, lam, prec, seed in ((0.5, 5, 1, 3), (0.6, 4, 0, 4), (0.5, 4, 1, 5)):
        v, t = inputs.shell288(r_in, 1.0)
        G = ts.Mesh(v, t)
        op = ts.Operator(G, lam, method=ts.TS_LSQP, q=2)
        sv = ts.Solver(op, lam, precision=prec, rtol=1e-8)
        f = G.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(seed, r_in))
        u1, rc, info1 = sv.solve(f)
        assert rc == ts.TS_OK
        cases.append((G, op, sv, f, u1, info1))
    ts.ts_solve_batch_step([])  # empty batch: nothing to do
    run = []
    for G, op, sv, f, u1, info1 in cases:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            u2 = G.zeros(sv.level)
        sv.begin(f, u2, s)
        run.append((sv, u2, ts.ts_solve_info()))
    # a batch holding a solver that is still running, or one solver twice,
    # is refused whole
    torch.cuda.synchronize()
    assert all(sv.query() == ts.TS_SOLVE_READY for sv, _, _ in run)
    ts.ts_solve_batch_step([run[0][0]])
    for bad in ([run[1][0], run[0][0]], [run[1][0], run[1][0]]):
        with pytest.raises(ts.TSError) as e:
            ts.ts_solve_batch_step(bad)
        assert e.value.code == ts.TS_EINVAL
    torch.cuda.synchronize()
    assert run[1][0].query() == ts.TS_SOLVE_READY  # not stepped by the refused calls
    while True:
        ready, live = [], 0
        for sv, _, info in run:
            st = sv.query(info)
            if st != ts.TS_SOLVE_DONE:
                live += 1
            if st == ts.TS_SOLVE_READY:
                ready.append(sv)
        if not live:
            break
        ts.ts_solve_batch_step(ready)
    torch.cuda.synchronize()
    for (G, op, sv, f, u1, info1), (_, u2, info2) in zip(cases, run):
        assert info2.status == ts.TS_OK and info2.cycles == info1.cycles
        assert info2.rel_residual == info1.rel_residual
        assert torch.equal(u1, u2)


def test_mesh_with_new_vertices_matches_a_fresh_mesh(ts):
    # the levels built on a mesh are kept when its vertices change, or shared
    # by a mesh created like it; stored interface stencils, coordinates, fits
    # and the coarse inverse follow each mesh's geometry: every result equals
    # the one on a freshly built mesh
    lam = 5
    va, t = inputs.shell288(0.5, 1.0)
    vb, _ = inputs.shell288(0.62, 1.0)
    A = ts.Mesh(va, t)
    op = ts.Operator(A, lam, method=ts.TS_LSQP, q=2, face_surrogate=True)
    xa = A.to_block(lam, inputs.uniform(A.layout(lam).n_unique, 2))
    op.apply(lam, xa)
    ts.Operator(A, lam, method=ts.TS_IFEM).apply(lam, xa)  # stored coordinates, old geometry
    with pytest.raises(ts.TSError) as e:  # an operator is still alive
        A.set_vertices(vb)
    assert e.value.code == ts.TS_EINVAL
    del op
    A.set_vertices(vb)
    B = ts.Mesh(vb, t)
    # a third mesh sharing B's built levels, with its own vertices
    C = ts.Mesh(vb, None, like=B)
    x = inputs.uniform(B.layout(lam).n_unique, 2)
    f = B.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(3, 0.62))
    assert torch.equal(A.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(3, 0.62)), f)
    for kw in ({"method": ts.TS_LSQP}, {"method": ts.TS_LSQP, "face_surrogate": True},
               {"method": ts.TS_IFEM}):
        ob = ts.Operator(B, lam, q=2, **kw)
        yb = ob.apply(lam, B.to_block(lam, x))
        ub, rcb, ib = ts.Solver(ob, lam, rtol=1e-9, precision=ts.TS_F32).solve(f)
        assert rcb == ts.TS_OK
        for M in (A, C):
            om = ts.Operator(M, lam, q=2, **kw)
            assert torch.equal(om.apply(lam, M.to_block(lam, x)), yb)
            um, rcm, im = ts.Solver(om, lam, rtol=1e-9, precision=ts.TS_F32).solve(f)
            assert rcm == ts.TS_OK and im.cycles == ib.cycles and torch.equal(um, ub)
            del om
        del ob


@pytest.mark.parametrize("topo,kw,prec", [
    ("shell288", {"method": 1, "q": 2, "fallback_tol": 0.25}, 1),
    ("shell288", {"method": 1, "q": 2, "face_surrogate": True}, 0),
    ("shell36", {"method": 1, "q": 2, "fallback_tol": 0.25}, 1),
    ("shell288", {"method": 0}, 1),
    ("shell288", {"method": 2, "q": 2}, 0),
    ("shell288", {"method": 3}, 1),
])
def test_solver_with_new_vertices_matches_a_fresh_solver(ts, topo, kw, prec):
    # a resident solver moved to another shell (ts_solver_set_vertices: mesh,
    # fits, fallback flags, face fits, stored rows, coarse inverse rebuilt in
    # place) gives bitwise what a solver built afresh on that shell gives
    lam = 5
    shell = getattr(inputs, topo)
    va, t = shell(0.5, 1.0)
    vb, _ = shell(0.62, 1.0)
    kw = dict(kw, method={0: ts.TS_IFEM, 1: ts.TS_LSQP, 2: ts.TS_LSQP_SYM,
                          3: ts.TS_CONS}[kw["method"]])
    A = ts.Mesh(va, t)
    oa = ts.Operator(A, lam, **kw)
    sa = ts.Solver(oa, lam, rtol=1e-9, precision=prec)
    fa = A.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(2, 0.5))
    _, rc, _ = sa.solve(fa)
    assert rc == ts.TS_OK
    sa.set_vertices(vb)
    B = ts.Mesh(vb, t)
    ob = ts.Operator(B, lam, **kw)
    sb = ts.Solver(ob, lam, rtol=1e-9, precision=prec)
    if kw["method"] != ts.TS_IFEM:
        # every surrogate kind rebuilds its coefficients for the new shell
        for l in range(3, lam + 1):
            assert np.array_equal(oa.coeffs(l), ob.coeffs(l))
            assert np.array_equal(oa.macro_flags(l), ob.macro_flags(l))
    x = B.to_block(lam, inputs.uniform(B.layout(lam).n_unique, 2))
    assert torch.equal(oa.apply(lam, x), ob.apply(lam, x))
    f = B.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(3, 0.62))
    assert torch.equal(A.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(3, 0.62)), f)
    ub, rcb, ib = sb.solve(f)
    ua, rca, ia = sa.solve(f)
    assert rca == rcb == ts.TS_OK and ia.cycles == ib.cycles
    assert ia.rel_residual == ib.rel_residual and torch.equal(ua, ub)


def test_solver_set_vertices_refusals(ts):
    lam = 4
    va, t = inputs.shell288(0.5, 1.0)
    vb, _ = inputs.shell288(0.6, 1.0)
    A = ts.Mesh(va, t)
    op = ts.Operator(A, lam, method=ts.TS_LSQP, q=2)
    sv = ts.Solver(op, lam, rtol=1e-8, precision=ts.TS_F32)
    f = A.rhs(lam, ts.TS_RHS_BUMPS, inputs.gaussian_bumps(1, 0.5))
    u0, rc, _ = sv.solve(f)
    c0 = op.coeffs(4)
    # a second operator on the mesh
    other = ts.Operator(A, lam, method=ts.TS_IFEM)
    with pytest.raises(ts.TSError) as e:
        sv.set_vertices(vb)
    assert e.value.code == ts.TS_EINVAL
    del other
    # a solve in progress
    u = A.zeros(lam)
    sv.begin(f, u)
    with pytest.raises(ts.TSError) as e:
        sv.set_vertices(vb)
    assert e.value.code == ts.TS_EINVAL
    while sv.query() != ts.TS_SOLVE_DONE:
        if sv.query() == ts.TS_SOLVE_READY:
            sv.step()
    torch.cuda.synchronize()
    assert torch.equal(u, u0)
    # non-finite coordinates: refused, nothing changed
    bad = vb.copy()
    bad[3, 1] = np.nan
    with pytest.raises(ts.TSError) as e:
        sv.set_vertices(bad)
    assert e.value.code == ts.TS_ENONFINITE
    assert np.array_equal(op.coeffs(4), c0)
    u1, rc1, _ = sv.solve(f)
    assert rc1 == ts.TS_OK and torch.equal(u1, u0)


def _trace(n, rate, levels, seed=3):
    return inputs.serving_trace(n, rate=rate, seed=seed, levels=levels)


def test_served_alone_and_in_mix_are_bitwise_equal(ts):
    from paper_1608_06473_amd.serve import Server
    trace = _trace(36, 500.0, (4, 5))
    keep = list(range(12))
    # alone: one slot, the kept requests one after another
    alone = Server(max_active=1, keep=keep)
    ra, sa = alone.run([rec for rec in trace if rec["id"] in keep])
    alone.close()
    assert sa["levels_shared"] > 0  # later requests shared the built levels
    # mix: every request of the trace, many in flight
    mix = Server(max_active=24, keep=keep)
    rm, sm = mix.run(trace)
    mix.close()
    bad = [(r.id, r.status, r.error) for r in ra + rm if r.status != ts.TS_OK]
    assert not bad, bad
    assert sa["completed_ok"] == len(keep) and sm["completed_ok"] == len(trace)
    assert sm["mean_active"] > 2.0  # the mix really overlapped
    A = {r.id: r for r in ra}
    for r in rm:
        if r.id in A:
            assert r.cycles == A[r.id].cycles
            assert np.array_equal(r.u_host, A[r.id].u_host), r.id
        assert r.rel <= 1e-8


def test_served_solution_residual_by_oracle(ts):
    import oracle
    from paper_1608_06473_amd.serve import Server
    rec = {"id": 7, "t": 0.0, "level": 4, "r_in": 0.45}
    srv = Server(keep=[7])
    (r,), summ = srv.run([rec])
    srv.close()
    assert r.status == ts.TS_OK
    v, t = inputs.shell288(0.45, 1.0)
    O = oracle.Mesh(v, t)
    lam, N = 4, 16
    c = O.fit(N, oracle.LSQP, 2, 2)
    fl = O.fallback_flags(N, 2, c, 0.25)
    f = O.rhs(N, 1, inputs.gaussian_bumps(7, 0.45))
    u = r.u_host.reshape(-1)
    ids = O.block_canon_ids(N)
    ucan = np.zeros(O.num_unique(N))
    ucan[ids] = u
    res = O.residual(N, f, ucan, kind=oracle.LSQP, q=2, coeffs=c, flags=fl)
    assert O.norm_free(N, res) / O.norm_free(N, f) <= 1.05e-8


def test_failed_setup_ends_its_request_only(ts):
    # a request whose shell is invalid (inner radius above the outer one:
    # the mesh check refuses it) fails alone; the requests around it, on
    # new and on resident solvers, are served
    from paper_1608_06473_amd.serve import Server
    trace = _trace(8, 200.0, (4,), seed=11)
    trace[3] = dict(trace[3], r_in=1.2)
    srv = Server(max_active=3)
    reqs, summ = srv.run(trace)
    srv.close()
    by = {r.id: r for r in reqs}
    assert by[trace[3]["id"]].status == ts.TS_EINVAL
    assert all(by[rec["id"]].status == ts.TS_OK for i, rec in enumerate(trace) if i != 3)
    assert summ["failed"] == 1 and summ["completed_ok"] == 7
