"""Pins of the exact-GEV bias (Lemma 3.2) and its approximation (Lemma 3.4):
Monte-Carlo expectation of the maximum of Gaussians, the single-element
cases of the lemma, and the convergence of Eq. 5 to the exact gap."""
import math

import numpy as np
import pytest

from oracle import gev


def test_probit_known_values():
    assert gev.probit_upper(40.0) == pytest.approx(1.959963984540054, rel=1e-12)  # Phi^-1(0.975)
    assert gev.probit_upper(2.0) == pytest.approx(0.0, abs=1e-15)


def test_single_element_has_no_bias():
    assert gev.Bn(1) == 0.0
    # d = 1: B_o = 0 (one leaf in pi_o's sub-tree); A = 2, d = 1: B_e = 0 too
    assert gev.exact_gap(0.0, 5.0, 7, 1) == 0.0
    assert gev.exact_gap(3.0, 5.0, 2, 1) == 0.0


@pytest.mark.parametrize("n", [50, 400, 3000])
def test_bias_matches_monte_carlo_max(n):
    """E[max of n iid N(0,1)] ~ Bn(n) (the GEV limit; a few % at these n)."""
    rng = np.random.default_rng(n)
    m = rng.standard_normal((4000, n)).max(axis=1).mean()
    assert gev.Bn(n) == pytest.approx(m, rel=0.03)


def test_bias_monotone_and_gap_positive():
    vals = [gev.Bn(n) for n in (1, 2, 5, 20, 100, 1000)]
    assert all(b > a for a, b in zip(vals, vals[1:]))
    for A in (3, 4, 18):
        for d in (1, 2, 3, 4):
            assert gev.exact_gap(4.0, 1.0, A, d) > 0.0


def test_approx_close_to_exact_for_deep_trees():
    """Appendix A.7's setting: A = 3, sigma_o = 1, sigma_e = 4.  Eq. 5 is
    meant for A^(d-1) >> 1: within 10% of the exact gap from d = 4 on, and
    loose at d = 1 (where A^(d-1) = 1)."""
    for d in (4, 8, 16, 32, 64):
        ex = gev.exact_gap(4.0, 1.0, 3, d)
        ap = gev.approx_gap(4.0, 1.0, 3, d)
        assert abs(ap - ex) / ex < 0.10, d
    assert abs(gev.approx_gap(4.0, 1.0, 3, 1) / gev.exact_gap(4.0, 1.0, 3, 1) - 1) > 0.5


def test_probit_approximation():
    """Phi^-1(1 - 1/n) ~ sqrt(2 log n) - 0.5, the approximation behind Eq. 5."""
    for n in (1e3, 1e6, 1e12):
        assert gev.probit_upper(n) == pytest.approx(math.sqrt(2 * math.log(n)) - 0.5, rel=0.06)
