"""The least-squares fit of the paper's device runtime model T = a n + T0
(device-level load balancing, Fig. 3(b)), on the CPU through the C ABI:
exact recovery of a line, residuals of noisy data orthogonal to the
regressors (the normal equations) and equal to numpy's fit, and argument
checks before any GPU call."""
import numpy as np
import pytest

from paper_1711_03244_amd import mcx


def test_exact_lines_are_recovered():
    for a, b in [(5.96e-6, 9.3), (1.0, 0.0), (-2.5, 1e3)]:
        x = np.array([1e6, 5e6, 2e7, 1e8])
        ga, gb = mcx.mcx_fit_linear(x, a * x + b)
        assert ga == pytest.approx(a, rel=1e-12) and gb == pytest.approx(b, rel=1e-9, abs=1e-9)
    # two points: the line through them (the paper's two-pilot estimate)
    ga, gb = mcx.mcx_fit_linear([1e6, 5e6], [15.1, 38.9])
    assert ga == pytest.approx((38.9 - 15.1) / 4e6, rel=1e-12)
    assert gb == pytest.approx(15.1 - ga * 1e6, rel=1e-12)


def test_residuals_of_noisy_lines():
    rng = np.random.default_rng(3)
    x = rng.uniform(1e5, 1e8, 40)
    y = 6e-6 * x + 9.0 + rng.normal(0, 2.0, x.size)
    a, b = mcx.mcx_fit_linear(x, y)
    r = y - (a * x + b)
    # the normal equations: residuals sum to zero and are orthogonal to x
    assert abs(r.sum()) < 1e-9 * np.abs(y).sum()
    assert abs((r * (x - x.mean())).sum()) < 1e-9 * np.abs(y * x).sum()
    pa, pb = np.polyfit(x, y, 1)
    assert a == pytest.approx(pa, rel=1e-9) and b == pytest.approx(pb, rel=1e-6)


@pytest.mark.parametrize("x,y", [([1.0], [2.0]), ([3.0, 3.0], [1.0, 2.0]),
                                 ([1.0, float("nan")], [1.0, 2.0])])
def test_degenerate_fits_are_refused(x, y):
    with pytest.raises(mcx.McxError) as e:
        mcx.mcx_fit_linear(x, y)
    assert e.value.status == mcx.MCX_EINVAL


def test_balance_and_pilot_arguments_checked():
    L = mcx.lib()
    assert L.mcx_set_balance(None, None) == mcx.MCX_EINVAL
    assert L.mcx_fit_runtime(None, None, None, None, None, None) == mcx.MCX_EINVAL
