"""Interpolation stencils and the error-bounded quantizer (oracle).

Eq. interp-linear: y_i = (x_{i-1} + x_{i+1}) / 2.
Eq. interp-cubic:  y_i = -x_{i-3}/16 + 9 x_{i-1}/16 + 9 x_{i+1}/16 - x_{i+3}/16.
Sec. 4.2.2: the residual y_l = x_l - P_l x^_{l+1} is quantized, and the
reconstruction x^_l = P_l x^_{l+1} + y^_l overwrites the data that later levels
predict from, so |x - x^| <= eb holds at every point (Eq.
error-prediction-interp).

Readings used (the paper is silent on them):

* Near the boundary, with b, c the neighbours at -+1 and a, e at -+3 (level
  units): no c -> copy b; cubic with a missing -> the quadratic through
  (-1, +1, +3): (3b + 6c - e) / 8; e missing -> (3c + 6b - a) / 8; both missing
  -> linear.  Every stencil has sum |coef| <= p (1 linear, 1.25 cubic), which
  keeps Thm. 1's amplification factor valid.
* Fixed evaluation order, one rounding per operation in the field's dtype:
    linear   ((b + c) * 0.5)
    cubic    (((b + c) * 9) - (a + e)) * 0.0625
    quad-lo  (((b * 3) + (c * 6)) - e) * 0.125
    quad-hi  (((c * 3) + (b * 6)) - a) * 0.125
* Quantizer bin 2*eb, round half to even, then an explicit check in float64;
  a value that fails the check, is not finite, or whose code exceeds QMAX is an
  outlier: code 0 and the exact input value is kept.
"""

from __future__ import annotations

import numpy as np

LINEAR, CUBIC = 0, 1

QMAX = {np.dtype(np.float32): 1 << 24, np.dtype(np.float64): 1 << 30}


def amplification(interp: int) -> float:
    """Infinity norm of the stencils (Thm. 1: p = 1 linear, 1.25 cubic)."""
    return 1.0 if interp == LINEAR else 1.25


def quant_constants(dtype, eb: float):
    """two_eb = T(2 eb) and inv = T(1 / (2 eb)), both formed in float64 first."""
    t = np.dtype(dtype).type
    return t(2.0 * eb), t(1.0 / (2.0 * eb))


def stencil_1d(interp: int, b, c, a, e, has_c, has_a, has_e, dtype):
    """Prediction for one target from its neighbours (scalar version).

    b, c: values at -+1; a, e: values at -+3 (level units).  has_*: whether the
    neighbour exists inside the grid (b always exists).
    """
    t = np.dtype(dtype).type
    if not has_c:
        return t(b)
    b, c = t(b), t(c)
    if interp == LINEAR or (not has_a and not has_e):
        return t(t(b + c) * t(0.5))
    if has_a and has_e:
        a, e = t(a), t(e)
        return t(t(t(t(b + c) * t(9.0)) - t(a + e)) * t(0.0625))
    if has_e:  # a missing
        e = t(e)
        return t(t(t(t(b * t(3.0)) + t(c * t(6.0))) - e) * t(0.125))
    a = t(a)   # e missing
    return t(t(t(t(c * t(3.0)) + t(b * t(6.0))) - a) * t(0.125))


def predict_along(G: np.ndarray, axis: int, interp: int) -> np.ndarray:
    """Predictions for all odd positions of ``G`` along ``axis``.

    ``G`` holds the current reconstruction of the level grid restricted to the
    pass's lattice in every other dimension; along ``axis`` it holds every
    level coordinate.  Returns an array with the odd positions along ``axis``.
    """
    dt = G.dtype.type
    n = G.shape[axis]
    n_odd = n // 2
    evens = np.take(G, np.arange(0, n, 2), axis=axis)
    n_even = evens.shape[axis]
    out_shape = list(G.shape)
    out_shape[axis] = n_odd
    out = np.empty(out_shape, dtype=G.dtype)
    if n_odd == 0:
        return out

    def ev(idx):
        return np.take(evens, idx, axis=axis)

    def put(idx, val):
        sl = [slice(None)] * G.ndim
        sl[axis] = idx
        out[tuple(sl)] = val

    m = np.arange(n_odd)
    has_c = m + 1 < n_even
    has_a = m >= 1
    has_e = m + 2 < n_even
    with np.errstate(all="ignore"):
        # copy
        sel = np.nonzero(~has_c)[0]
        if sel.size:
            put(sel, ev(sel))
        if interp == LINEAR:
            sel = np.nonzero(has_c)[0]
            if sel.size:
                put(sel, (ev(sel) + ev(sel + 1)) * dt(0.5))
            return out
        # cubic family
        sel = np.nonzero(has_c & has_a & has_e)[0]
        if sel.size:
            b, c, a, e = ev(sel), ev(sel + 1), ev(sel - 1), ev(sel + 2)
            put(sel, (((b + c) * dt(9.0)) - (a + e)) * dt(0.0625))
        sel = np.nonzero(has_c & ~has_a & has_e)[0]
        if sel.size:
            b, c, e = ev(sel), ev(sel + 1), ev(sel + 2)
            put(sel, (((b * dt(3.0)) + (c * dt(6.0))) - e) * dt(0.125))
        sel = np.nonzero(has_c & has_a & ~has_e)[0]
        if sel.size:
            b, c, a = ev(sel), ev(sel + 1), ev(sel - 1)
            put(sel, (((c * dt(3.0)) + (b * dt(6.0))) - a) * dt(0.125))
        sel = np.nonzero(has_c & ~has_a & ~has_e)[0]
        if sel.size:
            put(sel, (ev(sel) + ev(sel + 1)) * dt(0.5))
    return out


def quantize(x: np.ndarray, pred: np.ndarray, eb: float):
    """Error-bounded quantization of x against pred.

    Returns (q int64, xhat T, outlier bool), elementwise.
    """
    dt = x.dtype
    t = dt.type
    two_eb, inv = quant_constants(dt, eb)
    qmax = QMAX[dt]
    with np.errstate(all="ignore"):
        diff = x - pred
        qf = np.rint(diff * inv)
        out = ~(np.abs(qf) <= t(qmax))
        q = np.where(out, t(0), qf).astype(np.int64)
        xr = pred + q.astype(dt) * two_eb
        out |= ~(np.abs(xr.astype(np.float64) - x.astype(np.float64)) <= eb)
    q[out] = 0
    xhat = np.where(out, x, xr)
    return q, xhat, out


def quantize_scalar(x, pred, eb: float, dtype):
    """Scalar version of :func:`quantize` (used by the brute-force reference)."""
    t = np.dtype(dtype).type
    two_eb, inv = quant_constants(dtype, eb)
    qmax = QMAX[np.dtype(dtype)]
    x, pred = t(x), t(pred)
    with np.errstate(all="ignore"):
        diff = t(x - pred)
        qf = t(np.rint(t(diff * inv)))
        if not (abs(qf) <= t(qmax)):
            return 0, x, True
        q = int(qf)
        xr = t(pred + t(t(q) * two_eb))
        if not (abs(float(xr) - float(x)) <= eb):
            return 0, x, True
    return q, xr, False
