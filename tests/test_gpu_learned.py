"""The learned correction, trained on the GPU by the library's own kernels,
lowers the mean relative error of the plain estimator over the true super
points of the small configuration's traffic (window exact counts >= theta)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01527_amd import binding
    binding.load()
    return torch


def test_committed_weights_beat_plain(torch_cuda):
    from paper_1807_01527_amd import learned
    from paper_1807_01527_amd.binding import Mlp
    w = learned.load_weights("small")
    assert w is not None, "paper_1807_01527_amd/weights/small.npy missing"
    res = learned.evaluate("small", Mlp(w), seeds=range(10, 16))
    print(res)
    assert res["hosts"] > 300
    assert res["learned"] < 0.8 * res["plain"]


def test_training_from_scratch_reproduces_committed_weights(torch_cuda):
    """The committed small-configuration weights come from this exact recipe:
    1M GPU-generated samples (seed 1), 40 epochs of at_mlp_train_step.  Every
    step is deterministic (counter-based inputs, fixed-order reductions), so
    training again reproduces them and their gain over the plain estimator."""
    from paper_1807_01527_amd import learned
    from paper_1807_01527_amd.binding import Mlp
    X, T = learned.build_dataset("small", 1_000_000, seed=1, log=lambda m: None)
    net = Mlp(learned.init_params(1))
    losses = learned.train(net, X, T, epochs=40, log=lambda m: None)
    assert losses[-1] < 0.5 * losses[0]
    w = learned.load_weights("small")
    p = net.get_params()
    assert np.max(np.abs(p - w)) <= 1e-6 * (1 + np.max(np.abs(w)))
    res = learned.evaluate("small", net, seeds=range(0, 4))
    print(res)
    assert res["learned"] < 0.8 * res["plain"]


def test_large_weights_beat_plain(torch_cuda):
    """The large configuration's network (k = 60, 2^28-AT pool, load about
    3) on held-out links of that traffic (seeds 4 and 5; training traces
    start at seed 1100, the benchmark's links are seeds 0-3)."""
    from paper_1807_01527_amd import learned
    from paper_1807_01527_amd.binding import Mlp
    w = learned.load_weights("large")
    assert w is not None, "paper_1807_01527_amd/weights/large.npy missing"
    res = learned.evaluate_stream("large", Mlp(w), seeds=(4, 5))
    print(res)
    assert res["hosts"] > 5000
    assert res["learned"] < 0.8 * res["plain"]


def test_large_training_reproduces_committed_weights(torch_cuda):
    """weights/large.npy comes from this recipe: 500k samples of whole
    large-configuration traces (seed 1; each trace's true super points and as
    many hosts with 16 to 1023 distinct bips), 40 epochs of at_mlp_train_step."""
    from paper_1807_01527_amd import learned
    from paper_1807_01527_amd.binding import Mlp
    X, T = learned.build_dataset_stream("large", 500_000, seed=1, log=lambda m: None)
    net = Mlp(learned.init_params(1))
    losses = learned.train(net, X, T, epochs=40, log=lambda m: None)
    assert losses[-1] < 0.5 * losses[0]
    w = learned.load_weights("large")
    p = net.get_params()
    assert np.max(np.abs(p - w)) <= 1e-6 * (1 + np.max(np.abs(w)))
