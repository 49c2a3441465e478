"""Extrapolation and phase-diagram post-processing (CPU only).

Checked against mathematics, not against a retyped formula: polynomials of
degree <= d are reproduced exactly by the degree-d fit; the fitted values
agree with numpy.polyfit (an independent SVD-based least-squares routine);
nested least squares cannot increase the residual with the degree; the zero
crossing of a line is its root; the classification separates a plateau from
a decay and from a steady drift.
"""
import numpy as np
import pytest

from paper_1910_11359_amd import analysis as an


def _series(n=31, t1=3.0):
    return np.linspace(0.0, t1, n)


def test_exact_polynomials_are_reproduced():
    t = _series()
    y = 0.9 - 0.4 * t + 0.07 * t ** 2 - 0.01 * t ** 4
    fits = an.imbalance_fits(t, y)
    assert set(fits) == {1, 2, 4, 5}
    for d in (4, 5):
        assert fits[d]["rms"] < 1e-13
        np.testing.assert_allclose(an.extrapolate(fits[d], [4.0, 5.0]),
                                   0.9 - 0.4 * np.array([4, 5.]) + 0.07 * np.array([4, 5.]) ** 2
                                   - 0.01 * np.array([4, 5.]) ** 4, atol=1e-9)
    assert fits[1]["rms"] > 1e-3


def test_fits_agree_with_numpy_polyfit():
    rng = np.random.default_rng(3)
    t = _series(40)
    y = np.exp(-0.5 * t) * np.cos(2 * t) + 0.01 * rng.normal(size=t.size)
    fits = an.imbalance_fits(t, y)
    for d, f in fits.items():
        ref = np.polyval(np.polyfit(t, y, d), np.concatenate([t, [3.5, 4.0]]))
        got = an.extrapolate(f, np.concatenate([t, [3.5, 4.0]]))
        np.testing.assert_allclose(got, ref, atol=1e-9)


def test_residuals_do_not_grow_with_degree():
    rng = np.random.default_rng(4)
    t = _series(25)
    y = 1.0 / (1.0 + t ** 2) + 0.02 * rng.normal(size=t.size)
    fits = an.imbalance_fits(t, y)
    rms = [fits[d]["rms"] for d in (1, 2, 4, 5)]
    assert all(a >= b - 1e-15 for a, b in zip(rms, rms[1:]))
    np.testing.assert_allclose(np.sqrt(np.mean(fits[2]["residuals"] ** 2)), fits[2]["rms"], rtol=1e-14)


def test_zero_crossing_of_a_line():
    t = _series(11, 1.0)
    f = an.imbalance_fits(t, 1.0 - 0.5 * t, degrees=(1,))[1]
    assert abs(an.zero_crossing(f, 0.0, 10.0) - 2.0) < 1e-12
    assert an.zero_crossing(f, 0.0, 1.5) is None


def test_too_few_points_skip_high_degrees():
    fits = an.imbalance_fits(_series(4), np.ones(4))
    assert set(fits) == {1, 2}
    with pytest.raises(ValueError):
        an.imbalance_fits(np.zeros(3), np.zeros(4))


def test_classification_and_phase_diagram():
    t = _series(31, 3.0)
    plateau = 0.6 + 0.05 * np.cos(3 * t) * np.exp(-t)
    plateau[0] = 1.0
    decay = np.exp(-1.2 * t)
    drift = 0.9 - 0.2 * t          # far from zero at the end, but still falling
    assert an.classify(t, plateau) == "localized"
    assert an.classify(t, decay) == "ergodic"
    assert an.classify(t, drift) == "ergodic"
    pd = an.phase_diagram({(5, 6.0): (t, plateau), (2, 6.0): (t, decay)})
    assert pd == {(5, 6.0): "localized", (2, 6.0): "ergodic"}


def test_classification_details_report_free_parameters_and_fit_crossings():
    t = _series(31, 3.0)
    drift = 0.9 - 0.2 * t
    d = an.classify(t, drift, details=True)
    assert d["label"] == "ergodic"
    assert d["free_parameters"]["plateau"] == 0.3 and d["free_parameters"]["drift"] == 0.1
    # a line is its own fit of every degree: each continuation reaches zero at 4.5
    for deg in (1, 2, 4, 5):
        assert abs(d["fit_zero_crossing"][deg] - 4.5) < 1e-9
    assert abs(d["tail_fall_per_time"] - 0.2 / 0.9) < 1e-12
    pd = an.phase_diagram({(2, 6.0): (t, drift)}, details=True)
    assert pd[(2, 6.0)]["label"] == "ergodic"
