"""Host logic of the assimilation's gradient descent (no GPU): the step rule
on stand-in least-squares losses of very different scales."""
import pytest

torch = pytest.importorskip("torch")

from paper_2508_18202_amd.assimilation import Assimilation


def _descent(scale, truth=(1.08, 0.22), curv=(1.0, 0.3)):
    da = Assimilation.__new__(Assimilation)
    t = torch.tensor(truth, dtype=torch.float64)
    c = torch.tensor(curv, dtype=torch.float64)

    def loss(p):
        return scale * (c * (p - t) ** 2).sum()

    da.loss = loss
    return da


@pytest.mark.parametrize("scale", [1e-6, 1.0, 1e6, 1e10])
def test_first_step_is_taken_at_any_loss_scale(scale):
    """A sum-of-squares loss scaled by 1e-6 .. 1e10 (observations of any
    magnitude): the first iteration from (1.0, 0.15) is accepted within the
    backtracking budget and lowers the loss."""
    da = _descent(scale)
    hist = da.run((1.0, 0.15), iters=1)
    assert hist[0]["accepted"], hist
    start = da.loss(torch.tensor((1.0, 0.15), dtype=torch.float64))
    end = da.loss(torch.tensor((hist[0]["mu"], hist[0]["s"]), dtype=torch.float64))
    assert float(end) < float(start)


@pytest.mark.parametrize("scale", [1.0, 1e8])
def test_descent_converges_to_the_minimum(scale):
    da = _descent(scale)
    hist = da.run((1.0, 0.15), iters=80)
    losses = [h["loss"] for h in hist]
    assert all(b <= a for a, b in zip(losses, losses[1:]))
    last = hist[-1]
    assert abs(last["mu"] - 1.08) < 1e-6 and abs(last["s"] - 0.22) < 1e-6, last


def test_spread_stays_positive():
    """Trials with a non-positive spread are never evaluated."""
    da = _descent(1.0, truth=(1.0, 0.001))
    hist = da.run((1.0, 0.15), iters=30)
    assert all(h["s"] > 0 for h in hist)
