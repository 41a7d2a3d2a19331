"""Pins of the oracle's parameter rules against numbers the paper prints
(tests/golden/appendixF_dynamic_range.txt, appendix F): with alpha the peak
estimate, the rescaled noise level sigma = tau / (alpha sqrt(2L)) (eq. C3) is
the inverse of the target dynamic range the paper states for each band, and the
denoiser's training level is the inverse of its dynamic range."""
import math
import os

import pytest

from oracle import fb as OF

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    for line in open(os.path.join(HERE, "golden", "appendixF_dynamic_range.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            vals[k] = float(v)
    return vals


@pytest.mark.parametrize("band,digits", [("low", 1), ("high", 2)])
def test_sigma_rule_reproduces_printed_dynamic_ranges(band, digits):
    g = _golden()
    L = 7.0e9                                           # any L: the rule only uses tau / sqrt(2L)
    noise_jy = g[f"noise_{band}_mJy"] * 1e-3
    tau = noise_jy * math.sqrt(2.0 * L)
    assert OF.threshold(tau, L) == pytest.approx(noise_jy, rel=1e-15)      # eq. B2 noise level
    sigma = OF.sigma_from(tau, g[f"peak_{band}_Jy"], L)                    # eq. C3 with alpha = peak
    dr = 1.0 / sigma
    # the paper rounds to `digits` significant figures
    assert float(f"{dr:.{digits - 1}e}") == pytest.approx(g[f"target_dr_{band}"], rel=1e-12)


def test_denoiser_level_is_inverse_dynamic_range_and_alpha_matches_it():
    g = _golden()
    assert 1.0 / g["denoiser_dr"] == pytest.approx(g["sigma_train"], rel=1e-12)
    # at the high band the data point to a lower dynamic range than the denoiser's, so
    # alpha is raised above the peak estimate until tau / (alpha sqrt(2L)) = sigma_train (eq. C3)
    L = 7.0e9
    tau = g["noise_high_mJy"] * 1e-3 * math.sqrt(2.0 * L)
    alpha = OF.alpha_rescale(g["peak_high_Jy"], 1.0, tau, L, g["sigma_train"])
    assert alpha > g["peak_high_Jy"]
    assert OF.sigma_from(tau, alpha, L) == pytest.approx(g["sigma_train"], rel=1e-12)
