"""Host logic of the request loop (no GPU): the request trace and the
admission estimate."""
import numpy as np

from paper_1608_06473_amd import inputs


def test_serving_trace_is_seeded_and_shaped():
    a = inputs.serving_trace(2000, rate=50.0, seed=3)
    b = inputs.serving_trace(2000, rate=50.0, seed=3)
    assert a == b
    t = np.array([r["t"] for r in a])
    assert np.all(np.diff(t) > 0) and t[0] > 0
    # exponential gaps of mean 1/rate: the sample mean of 2000 gaps lies
    # within 4 standard errors (each gap has standard deviation 1/rate)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.02) < 4 * 0.02 / np.sqrt(gaps.size)
    assert {r["level"] for r in a} == {4, 5, 6, 7}
    ri = np.array([r["r_in"] for r in a])
    assert ri.min() >= 0.4 and ri.max() <= 0.7
    assert [r["id"] for r in a] == list(range(2000))
    assert inputs.serving_trace(5, seed=4) != inputs.serving_trace(5, seed=3)


def test_admission_estimate_covers_the_vectors():
    # the serve module imports the binding (ctypes only; no GPU call here)
    from paper_1608_06473_amd import TS_F32, TS_F64
    from paper_1608_06473_amd.serve import request_bytes

    def slots(n_macros, lam):
        N = 2 ** lam
        return n_macros * (N + 1) * (N + 2) * (N + 3) // 6

    for lam in (4, 5, 6, 7):
        b32 = request_bytes(288, lam, TS_F32)
        b64 = request_bytes(288, lam, TS_F64)
        # at least f and u in FP64 and the outer residual at the finest level
        assert b32 >= 24 * slots(288, lam) and b64 >= 24 * slots(288, lam)
        if lam > 4:
            assert request_bytes(288, lam, TS_F32) > request_bytes(288, lam - 1, TS_F32)
    # a level-7 request of the 288-macro shell is a few GB, far below one
    # GPU's 288 GB
    assert 2e9 < request_bytes(288, 7, TS_F32) < 2e10


def test_request_over_the_budget_is_rejected_alone():
    # a request that can never fit the HBM budget retires with TS_ENOMEM at
    # admission; the loop goes on and ends normally (no set-up is started, so
    # this runs without a GPU)
    from paper_1608_06473_amd import TS_ENOMEM
    from paper_1608_06473_amd.serve import Server, request_bytes
    trace = [{"id": 0, "t": 0.0, "level": 7, "r_in": 0.55},
             {"id": 1, "t": 0.001, "level": 6, "r_in": 0.5}]
    srv = Server(hbm_budget=request_bytes(288, 4), max_active=4)
    try:
        reqs, summ = srv.run(trace)
    finally:
        srv.close()
    assert [r.status for r in reqs] == [TS_ENOMEM, TS_ENOMEM]
    assert all(r.t_admit is None and r.t_done is not None for r in reqs)
    assert "HBM budget" in reqs[0].error
    assert summ["failed"] == 2 and summ["completed_ok"] == 0
    assert summ["failed_by_status"] == {str(TS_ENOMEM): 2}


class _Fut:
    def __init__(self):
        self.ok = False

    def done(self):
        return self.ok

    def result(self):
        return None


def test_memory_is_held_until_its_release_completes():
    # a retired request's estimate stays held while the releasing thread
    # works (freeing device memory waits for the device); only a completed
    # release makes room for new admissions
    from paper_1608_06473_amd.serve import Ledger
    L = Ledger(budget=100, reserve=0)
    L.admit(60)
    L.set_up(60)
    assert not L.fits(50)
    fut = _Fut()
    L.release(fut, 60, now=1.0)
    L.poll(now=2.0)
    assert L.held == 60 and not L.fits(50) and not L.idle()
    fut.ok = True
    L.poll(now=3.5)
    assert L.held == 0 and L.fits(50) and L.idle()
    assert L.release_s == [2.5] and L.peak == 60


def test_admission_counts_requests_not_yet_set_up():
    # a free-memory snapshot does not show requests admitted but not set up
    # yet: a burst of admissions from one snapshot must not exceed it
    from paper_1608_06473_amd.serve import Ledger
    L = Ledger(budget=1000, reserve=10)
    free = 100
    assert L.fits(40, free)
    L.admit(40)
    assert L.fits(40, free)        # 40 + 40 + 10 <= 100
    L.admit(40)
    assert not L.fits(40, free)    # the third would overrun the snapshot
    L.set_up(40)                   # set-up done: now part of the snapshot
    L.set_up(40)
    assert L.fits(40, free - 80 + 80)
    assert not L.fits(40, free - 80)
