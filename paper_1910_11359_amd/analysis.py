"""Extrapolation of the imbalance and the dynamical phase diagram (the
imbalance figure with its polynomial fits and the dynamical phase diagram of
the Results section).

Host post-processing of imbalance series I(t) that the device path returns
(one per parameter point (d_A, h)); nothing here touches the GPU.

* `imbalance_fits`: least-squares polynomials of degree 1, 2, 4 and 5 (the
  degrees the paper uses) with their residuals; `extrapolate` evaluates a fit
  beyond the simulated window and `zero_crossing` finds where an
  extrapolation first reaches I = 0.
* `classify` labels a series "localized" or "ergodic".  The paper's
  criterion is qualitative (whether the simulated imbalance, or its
  polynomial continuation, localizes in time) and names no threshold.  The
  reading taken: a series is localized when the imbalance over the last
  third of the simulated window stays at or above `plateau` (0.3 of the
  initial imbalance by default) and the degree-1 fit over that third falls
  by less than `drift` (0.1 of the initial imbalance) per unit of simulated
  time, i.e. slow dynamics far from zero; ergodic otherwise.  Both
  thresholds are free parameters of this reading, reported as such with
  each label (details=True), next to the zero crossings of the paper's own
  polynomial continuations.  Those continuations alone do not decide: on a
  pure exponential decay the degree-2 and degree-4 fits curve upwards and
  never reach zero, so a vote over the degrees calls it localized.
* `phase_diagram` applies `classify` to a set of parameter points.
"""
import numpy as np

FIT_DEGREES = (1, 2, 4, 5)


def _design(t, degree, t_scale):
    """Vandermonde matrix in the scaled time s = t / t_scale (columns s^0..s^d)."""
    s = np.asarray(t, dtype=np.float64) / t_scale
    return s[:, None] ** np.arange(degree + 1)[None, :]


def imbalance_fits(t, imbalance, degrees=FIT_DEGREES):
    """Least-squares fits of I(t) for each degree: a dict degree -> fit, a fit
    being {"coef": coefficients of 1, s, s^2, ... in s = t / t_max,
    "t_scale": t_max, "rms": root-mean-square residual, "residuals": I - fit}.
    The problem is solved by a QR factorisation of the scaled Vandermonde
    matrix (no normal equations).  A degree needs more points than
    coefficients; larger degrees are skipped."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(imbalance, dtype=np.float64)
    if t.shape != y.shape or t.ndim != 1:
        raise ValueError("t and imbalance must be 1-d arrays of the same length")
    t_scale = float(np.max(np.abs(t))) or 1.0
    fits = {}
    for d in degrees:
        if len(t) <= d:
            continue
        A = _design(t, d, t_scale)
        Q, R = np.linalg.qr(A)
        coef = np.linalg.solve(R, Q.T @ y)
        res = y - A @ coef
        fits[d] = {"coef": coef, "t_scale": t_scale, "rms": float(np.sqrt(np.mean(res ** 2))),
                   "residuals": res}
    return fits


def extrapolate(fit, t):
    """The fitted polynomial at times t (any, also beyond the fitted window)."""
    t = np.asarray(t, dtype=np.float64)
    return _design(np.atleast_1d(t), len(fit["coef"]) - 1, fit["t_scale"]) @ fit["coef"]


def zero_crossing(fit, t_from, t_to, n_grid=4001):
    """First time in [t_from, t_to] where the extrapolated imbalance reaches 0
    (bisection on the first sign change of a grid), or None."""
    grid = np.linspace(t_from, t_to, n_grid)
    v = extrapolate(fit, grid)
    if v[0] == 0.0:
        return float(grid[0])
    idx = np.flatnonzero(np.sign(v[1:]) != np.sign(v[:-1]))
    if len(idx) == 0:
        return None
    a, b = grid[idx[0]], grid[idx[0] + 1]
    fa = extrapolate(fit, a)[0]
    for _ in range(60):
        m = 0.5 * (a + b)
        fm = extrapolate(fit, m)[0]
        if (fm > 0) == (fa > 0):
            a, fa = m, fm
        else:
            b = m
    return float(0.5 * (a + b))


def classify(t, imbalance, plateau=0.3, drift=0.1, horizon=2.0, details=False):
    """'localized' or 'ergodic' for one series (reading in the module notes).
    The imbalance is taken relative to its value at the first time.

    plateau and drift are free parameters of this reading: the paper states
    its criterion only qualitatively and fixes no threshold.  details=True
    returns a dict with the label, the two thresholds (marked as free
    parameters), the quantities they are compared with (the smallest
    relative imbalance over the last third of the window and the fall per
    unit time of its degree-1 fit), and, for the paper's fits of degree 1, 2,
    4 and 5 over the whole window, the first time their extrapolation
    reaches zero before horizon * t_max (None: not before), the continuation
    the imbalance figure draws."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(imbalance, dtype=np.float64)
    if len(t) < 3:
        raise ValueError("need at least 3 observations")
    y0 = y[0] if y[0] != 0 else 1.0
    yr = y / y0
    tail = t >= t[0] + (2.0 / 3.0) * (t[-1] - t[0])
    if tail.sum() < 2:
        tail[-2:] = True
    slope = np.polyfit(t[tail], yr[tail], 1)[0] if tail.sum() >= 2 else 0.0
    tail_min = float(np.min(yr[tail]))
    localized = tail_min >= plateau and -slope < drift
    label = "localized" if localized else "ergodic"
    if not details:
        return label
    fits = imbalance_fits(t, y)
    return {"label": label, "tail_min_relative": tail_min, "tail_fall_per_time": float(-slope),
            "free_parameters": {"plateau": plateau, "drift": drift, "horizon": horizon,
                                "note": "thresholds of this reading; the paper fixes none"},
            "fit_zero_crossing": {d: zero_crossing(f, t[0], horizon * t[-1]) for d, f in fits.items()}}


def phase_diagram(series, details=False, **kw):
    """series: {(d_A, h): (t, imbalance)} -> {(d_A, h): 'localized' | 'ergodic'}
    (details=True: the per-point dicts of classify, free parameters included)."""
    return {key: classify(t, y, details=details, **kw) for key, (t, y) in series.items()}
