"""The learned warm start on a reduced workload: the network is trained on the GPU on solves the
method generates, and PCG from its output reaches the same solution as plain PCG from f in
fewer iterations on held-out images."""
import pytest

from gpu_util import torch_gpu

pytestmark = pytest.mark.gpu


def test_warm_start_reaches_the_same_solution_in_fewer_iterations():
    torch_gpu()
    from paper_2407_06834_amd import warmstart as WS
    from paper_2407_06834_amd.cnn import WarmStartNet
    data = WS.generate(range(20000, 20064), sides=(256, 384))
    assert len(data) == 64
    net = WarmStartNet(n_cond=10, seed=0)
    losses = WS.train(net, data, steps=1500, crop=128)
    assert sum(losses[-100:]) < 0.5 * sum(losses[:100])
    res = WS.evaluate(net, range(20100, 20104), side=512)
    net.close()
    # both solutions satisfy ||u - u*|| <= 1e-6 ||f_perp||, so they differ by at most twice that
    assert res["max_diff_rel"] <= 3e-6
    assert res["iters_warm"] < res["iters_plain"], res
