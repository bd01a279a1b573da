"""ts_norm2_noalloc (partial sums in the library's fixed device array, the
norm written to device memory, nothing allocated) against ts_norm2 (the
same kernels with a stream-ordered temporary), through the C ABI: two calls
in a row on the same GPU, the second on a smaller input, each equal bit for
bit to ts_norm2 of the same vector (same kernels, same reduction order)."""
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


def test_noalloc_norm_matches_norm2_on_two_calls(ts):
    v, t = inputs.shell288()
    G = ts.Mesh(v, t)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for lam, seed, dt in ((7, 80, ts.TS_F64), (4, 81, ts.TS_F64), (6, 82, ts.TS_F32)):
        info = G.layout(lam)
        x = torch.empty(info.vec_len, dtype=torch.float64, device="cuda").uniform_(
            -1.0, 1.0, generator=torch.Generator(device="cuda").manual_seed(seed))
        x = ts.check_vector(x if dt == ts.TS_F64 else x.float(), info.vec_len, dt, "x")
        ref = ts.ts_norm2(G.h, lam, dt, x)
        out.fill_(-1.0)
        ts.ts_norm2_noalloc(G.h, lam, dt, x, out)
        torch.cuda.synchronize()
        got = float(out.cpu()[0])
        assert got == ref, (lam, got, ref)
        assert np.isfinite(got) and got > 0


def test_noalloc_norm_refuses_an_unbuilt_level(ts):
    v, t = inputs.shell36()
    G = ts.Mesh(v, t)
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(ts.TSError) as e:
        ts.ts_norm2_noalloc(G.h, 5, ts.TS_F64, x, out)
    assert e.value.code == ts.TS_EINVAL and "not built" in str(e.value)
