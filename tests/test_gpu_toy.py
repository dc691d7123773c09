"""Prop. 4.1 toy on the GPU (mqo_toy_reset through the C-ABI) against the
oracle: every trial's first hit and final point bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import toy  # noqa: E402


@pytest.fixture(scope="module")
def mqo():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_06921_amd import mqo as m
    return m


@pytest.mark.parametrize("n,trials,attempts", [(1, 70, 20), (7, 300, 150), (32, 257, 500), (64, 128, 700)])
def test_global_reset_bit_exact(mqo, n, trials, attempts):
    first, x = mqo.toy_reset(17, n, trials, attempts, mode="global", device="cuda:0")
    rf, rx = toy.global_reset(17, n, trials, attempts)
    assert np.array_equal(first.cpu().numpy(), rf)
    assert np.array_equal(x.cpu().numpy(), rx)


def test_global_reset_unconverged_descent(mqo):
    """Few descent steps leave interior values; the comparison of phi then
    decides on non-binary points, still bit for bit."""
    first, x = mqo.toy_reset(18, 9, 200, 60, mode="global", steps=3, alpha=0.3, beta=0.7, device="cuda:0")
    rf, rx = toy.global_reset(18, 9, 200, 60, alpha=0.3, beta=0.7, steps=3)
    assert np.array_equal(first.cpu().numpy(), rf)
    assert np.array_equal(x.cpu().numpy(), rx)
    assert np.any(np.abs(rx) < 1)


@pytest.mark.parametrize("n", [1, 5, 9])
def test_full_restart_bit_exact(mqo, n):
    first, _ = mqo.toy_reset(19, n, 500, 80, mode="restart", device="cuda:0")
    rf, _ = toy.full_restart(19, n, 500, 80)
    assert np.array_equal(first.cpu().numpy(), rf)


def test_toy_rejects_bad_arguments(mqo):
    with pytest.raises(mqo.MqoError):
        mqo.toy_reset(1, 65, 4, 4, device="cuda:0")
    with pytest.raises(mqo.MqoError):
        mqo.toy_reset(1, 8, 4, 4, beta=1.0, device="cuda:0")
