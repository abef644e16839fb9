"""Pins of the oracle's Vegas map adaptation of one dimension (Lepage's rule, damping exponent alpha of Appendix C).

The rule: bin averages d_j = h_j / c_j; smoothing (7 d_0 + d_1)/8, (d_{j-1} + 6 d_j + d_{j+1})/8, (d_{n-2} + 7 d_{n-1})/8;
normalisation to unit sum; damping w_j = ((1 - d_j) / ln(1/d_j))^alpha (0 for d_j = 0); new interior edges where
the running sum of w reaches k sum(w) / n, placed linearly inside the old bin; outer edges fixed.

The expected edges below are closed forms worked out by hand from that rule for small bin counts (the derivation is
in each docstring); none re-runs the rule step by step.  Mistakes each case catches: smoothing weights other than
(7,1)/(1,6,1)/(1,7) over 8 (nb = 3 delta, nb = 4 corner), the damping exponent applied wrongly or the logarithm
inverted (nb = 2 with alpha = 1, nb = 3 with alpha = 1/2), a zero-weight bin given weight (nb = 4), an edge placed
in the wrong old bin or from the wrong end of it (all cases), the outer edges moved (all cases).
"""
import math

import numpy as np
import pytest

from oracle import binding as ob


def test_two_bins_alpha_one():
    """h = (3, 1), c = (1, 1): d = (3, 1); smoothed (22/8, 10/8), sum 4, so d_hat = (11/16, 5/16).
    alpha = 1: w_0 = (5/16) / ln(16/11), w_1 = (11/16) / ln(16/5); w_0 > (w_0 + w_1)/2, so the one interior edge
    lies in old bin 0 = [0, 1] at the fraction (w_0 + w_1) / (2 w_0)."""
    w0 = (5 / 16) / math.log(16 / 11)
    w1 = (11 / 16) / math.log(16 / 5)
    assert w0 > 0.5 * (w0 + w1)
    e = ob.adapt_dim([0.0, 1.0, 2.0], [3.0, 1.0], [1.0, 1.0], 1.0)
    assert e[0] == 0.0 and e[2] == 2.0
    assert e[1] == pytest.approx((w0 + w1) / (2 * w0), rel=1e-14)


def test_three_bins_delta_alpha_half():
    """d = (0, 1, 0) (h = (0, 5, 0), c = (3, 5, 2)): smoothed (1/8, 6/8, 1/8), already normalised.
    alpha = 1/2: w_0 = w_2 = sqrt((7/8) / ln 8), w_1 = sqrt((1/4) / ln(4/3)), and w_0 < w_1, so both interior
    edges lie in old bin 1 = [1, 2]: edge 1 = 1 + (W/3 - w_0)/w_1 = 4/3 - w_0/(3 w_1) and
    edge 2 = 1 + (2W/3 - w_0)/w_1 = 5/3 + w_0/(3 w_1), with W = 2 w_0 + w_1."""
    w0 = math.sqrt((7 / 8) / math.log(8))
    w1 = math.sqrt((1 / 4) / math.log(4 / 3))
    assert w0 < w1
    e = ob.adapt_dim([0.0, 1.0, 2.0, 3.0], [0.0, 5.0, 0.0], [3.0, 5.0, 2.0], 0.5)
    assert e[0] == 0.0 and e[3] == 3.0
    assert e[1] == pytest.approx(4 / 3 - w0 / (3 * w1), rel=1e-14)
    assert e[2] == pytest.approx(5 / 3 + w0 / (3 * w1), rel=1e-14)


def test_four_bins_corner_with_empty_bins():
    """d = (1, 0, 0, 0): smoothed (7/8, 1/8, 0, 0), normalised as is; w_0 = sqrt((1/8) / ln(8/7)),
    w_1 = sqrt((7/8) / ln 8), w_2 = w_3 = 0, W = w_0 + w_1.  Targets W/4 and W/2 fall in old bin 0 = [0, 1]
    (both below w_0), 3W/4 in old bin 1 = [1, 2]: edges W/(4 w_0), W/(2 w_0), 1 + (3W/4 - w_0)/w_1; the empty bins
    2 and 3 collapse into the last new bin."""
    w0 = math.sqrt((1 / 8) / math.log(8 / 7))
    w1 = math.sqrt((7 / 8) / math.log(8))
    W = w0 + w1
    assert W / 2 < w0 < 3 * W / 4
    e = ob.adapt_dim([0.0, 1.0, 2.0, 3.0, 4.0], [2.0, 0.0, 0.0, 0.0], [2.0, 1.0, 1.0, 1.0], 0.5)
    assert e[0] == 0.0 and e[4] == 4.0
    np.testing.assert_allclose(e[1:4], [W / (4 * w0), W / (2 * w0), 1 + (0.75 * W - w0) / w1], rtol=1e-14)


@pytest.mark.parametrize("nb", [2, 3, 7, 50])
def test_uniform_averages_keep_edges(nb):
    """Equal averages in every bin smooth to equal values (the end weights (7+1)/8 and the interior (1+6+1)/8 both
    sum to 1), so every damped weight is equal and the edges stay where they are, to the rounding of the running
    sums (a few ulps of the range)."""
    rng = np.random.default_rng(nb)
    edges = np.concatenate([[0.0], np.cumsum(rng.uniform(0.5, 2.0, nb))])
    cnt = rng.integers(1, 50, nb).astype(float)
    e = ob.adapt_dim(edges, 2.5 * cnt, cnt, 0.5)
    np.testing.assert_allclose(e, edges, rtol=0, atol=8 * nb * 2.2e-16 * edges[-1])


def test_alpha_zero_keeps_edges():
    """alpha = 0 damps every nonzero bin to weight 1, whatever the averages."""
    edges = np.array([0.0, 0.3, 0.45, 1.7, 2.0, 3.1])
    e = ob.adapt_dim(edges, [1.0, 9.0, 0.2, 4.0, 0.5], [1.0, 1.0, 1.0, 1.0, 1.0], 0.0)
    np.testing.assert_allclose(e, edges, rtol=0, atol=4e-16 * edges[-1])


def test_scale_invariance_and_empty_histogram():
    """Multiplying every h_j by 4 (or h and c together by 2) leaves the normalised averages, and so the edges,
    bitwise unchanged; an all-zero histogram leaves the edges as they are."""
    edges = np.linspace(0.0, 1.0, 11)
    h = np.array([0.1, 0.5, 2.0, 7.0, 3.0, 1.0, 0.4, 0.1, 0.0, 0.2])
    c = np.array([5, 6, 7, 5, 4, 6, 5, 5, 3, 4], dtype=float)
    e1 = ob.adapt_dim(edges, h, c, 0.5)
    assert not np.array_equal(e1, edges)
    assert np.array_equal(ob.adapt_dim(edges, 4 * h, c, 0.5), e1)
    assert np.array_equal(ob.adapt_dim(edges, 2 * h, 2 * c, 0.5), e1)
    assert np.array_equal(ob.adapt_dim(edges, 0 * h, c, 0.5), edges)


def test_edges_stay_monotone_and_concentrate_weight():
    """Bins of large weight shrink: after one step the new bins around the peak are narrower than before."""
    edges = np.linspace(0.0, 1.0, 51)
    x = 0.5 * (edges[1:] + edges[:-1])
    h = np.exp(-((x - 0.3) / 0.05) ** 2)
    e = ob.adapt_dim(edges, h, np.ones(50), 0.5)
    assert np.all(np.diff(e) > 0)
    k = np.searchsorted(e, 0.3) - 1
    assert e[k + 1] - e[k] < 0.02
