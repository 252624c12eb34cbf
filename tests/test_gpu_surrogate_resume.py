"""Surrogate training resumed from a checkpoint of the optimiser state
reproduces an uninterrupted run (the minibatches are a function of the seed
and the step, the kernels' reductions run in a fixed order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _data(torch):
    rng = np.random.default_rng(11)
    X = rng.normal(size=(20000, 12))
    A = rng.normal(size=(12, 10)) / np.sqrt(12)
    T = np.tanh(X @ A) + 0.1 * X[:, :10] ** 2
    return (torch.as_tensor(X, dtype=torch.float32, device="cuda"),
            torch.as_tensor(T, dtype=torch.float32, device="cuda"))


def test_resume_reproduces_uninterrupted_training(tmp_path):
    import torch
    from paper_2510_23993_amd import surrogate
    X, T = _data(torch)
    quiet = lambda *a: None   # noqa: E731
    kw = dict(steps=60, batch=1024, seed=3, log=quiet)
    p_full, norm_full, _ = surrogate.train(X.clone(), T.clone(), **kw)
    ck = str(tmp_path / "state.npz")
    p_half, _, _ = surrogate.train(X.clone(), T.clone(), checkpoint=ck, stop_after=25, **kw)
    with np.load(ck, allow_pickle=False) as f:
        assert list(f["schedule"]) == [25, 60, 1024, 3]
        assert np.array_equal(f["params"], p_half)
    p_res, norm_res, _ = surrogate.train(X.clone(), T.clone(), resume=ck, **kw)
    assert not np.allclose(p_half, p_full)          # the first half alone is not the answer
    np.testing.assert_allclose(p_res, p_full, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(norm_res["mean_x"], norm_full["mean_x"], rtol=1e-6)
    # a checkpoint of another schedule is refused
    with pytest.raises(ValueError, match="schedule"):
        surrogate.train(X.clone(), T.clone(), resume=ck, steps=61, batch=1024, seed=3, log=quiet)
