"""The C-ABI library loads and exports every symbol include/twoscale.h declares
(no compute: this runs on machines without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "twoscale.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ts_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["ts_mesh_create", "ts_op_create", "ts_apply", "ts_residual", "ts_smooth",
              "ts_vcycle", "ts_solve", "ts_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1608_06473_amd as ts
    if not os.path.exists(ts.LIB_PATH):
        pytest.fail("libtwoscale.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ts.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared entry points
    assert sorted(ts.EXPORTED) == _declared()


def test_last_error_callable_without_gpu():
    import paper_1608_06473_amd as ts
    assert isinstance(ts.ts_last_error(), str)


def test_invalid_arguments_are_rejected_without_gpu():
    import paper_1608_06473_amd as ts
    with pytest.raises(ts.TSError) as e:
        ts.ts_op_create(ctypes.c_void_p(), 5, stream=0)
    assert e.value.code == ts.TS_EINVAL


def test_batched_step_rejects_bad_batches_without_gpu():
    # argument checks come before any device work: a negative count, a
    # null array with a positive count, a null solver and a repeated solver
    # are refused with TS_EINVAL; an empty batch is a no-op
    import paper_1608_06473_amd as ts
    L = ts.lib()
    assert L.ts_solve_batch_step(None, 0) == ts.TS_OK
    assert L.ts_solve_batch_step(None, -1) == ts.TS_EINVAL
    assert L.ts_solve_batch_step(None, 2) == ts.TS_EINVAL
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.ts_solve_batch_step(arr, 2) == ts.TS_EINVAL
    assert "twice" in ts.ts_last_error()
    arr1 = (ctypes.c_void_p * 1)(None)
    assert L.ts_solve_batch_step(arr1, 1) == ts.TS_EINVAL
    assert "null solver" in ts.ts_last_error()


def test_vector_checks_reject_before_the_library():
    # the binding refuses vectors the kernels would overrun (wrong element
    # type, strided, short or long, host memory) with TS_EINVAL before any
    # library call; the device check comes last so that the others can be
    # exercised with host tensors
    import torch

    import paper_1608_06473_amd as ts
    n = 100
    cases = [(torch.zeros(n, dtype=torch.float32), ts.TS_F64, "dtype"),
             (torch.zeros(n, dtype=torch.float64), ts.TS_F32, "dtype"),
             (torch.zeros(2 * n, dtype=torch.float64)[::2], ts.TS_F64, "contiguous"),
             (torch.zeros(n - 1, dtype=torch.float64), ts.TS_F64, "entries"),
             (torch.zeros(n + 1, dtype=torch.float32), ts.TS_F16W, "entries"),
             (torch.zeros(n, dtype=torch.float64), ts.TS_F64, "device"),
             (np.zeros(n), ts.TS_F64, "dtype")]
    for t, dt, what in cases:
        with pytest.raises(ts.TSError) as e:
            ts.check_vector(t, n, dt, "x")
        assert e.value.code == ts.TS_EINVAL
        assert what in str(e.value), (what, str(e.value))
