"""The paper's table protocols (Sec. 5.2-5.4) at the smallest size: they run end to end on the
HIP path and show the qualitative behaviour the paper reports for its iteration table."""
import pytest

from gpu_util import torch_gpu

pytestmark = pytest.mark.gpu


def test_tables_small():
    torch_gpu()
    from paper_2407_06834_amd import tables
    op = tables.operator_table([64])
    assert op[0]["windows"] == 17 and op[0]["product_ms"] > 0
    sol = tables.solution_table([64])
    assert sol[0]["status"] == "OK" and sol[0]["iters"] <= 200
    it = tables.iterations_table([64])[0]
    assert it["windows"] == 41
    for lam in tables.LAMBDAS:
        none, pa, pb, none_u, pa_u, pb_u = it[f"lambda={lam:g}"]
        # deflated (U basis) Jacobi and l2 columns converge for every lambda
        assert pa_u != "x" and pb_u != "x"
        # the two diagonal preconditioners are nearly equivalent (P_a <= P_b <= sqrt(2) P_a)
        if pa != "x" and pb != "x":
            assert abs(pa - pb) <= 2
        if pa != "x":
            assert pa_u <= pa
    # without a preconditioner CG stalls once lambda is small
    assert it["lambda=1e-09"][0] == "x"
