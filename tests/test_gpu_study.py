"""The discretisation-error study (Sec. 4.1, Tab. hHstudy analogue) on the
288-macro shell at levels 4 and 5: the trends the paper reports.

- the exact operator converges like h^2 (error ratio about 4 per level);
- degree 1 surrogates stagnate, the surrogate error falls with the degree,
  and LSQP beats IPOLY at q = 2;
- double discretisation keeps the exact operator's error.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def recs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_06473_amd import study
    out = study.study(meshes=(288,), levels=(4, 5), log=lambda s: None)
    return {(r["level"], r["scheme"]): r for r in out}


def test_all_converge(recs):
    from paper_1608_06473_amd import TS_OK
    assert all(r["status"] == TS_OK for r in recs.values())


def test_trends(recs):
    e = {k: r["error"] for k, r in recs.items()}
    assert 3.5 < e[4, "IFEM"] / e[5, "IFEM"] < 4.5
    assert e[5, "LSQP q=1"] > 3 * e[5, "IFEM"]                # q = 1 stagnates
    assert e[5, "LSQP q=1"] > e[5, "LSQP q=2"]
    assert abs(e[5, "LSQP q=4"] - e[5, "IFEM"]) < 0.05 * e[5, "IFEM"]
    assert e[5, "IPOLY q=2"] > e[5, "LSQP q=2"]               # LSQP fits better
    assert abs(e[5, "LSQP q=2 DD"] - e[5, "IFEM"]) < 0.01 * e[5, "IFEM"]
