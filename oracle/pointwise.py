"""Single outputs of large fields, one point at a time (oracle; test
infrastructure only).

The value a point takes after compression (x^, Sec. 4.2.2) or after a
retrieval with a plan (x~, Alg. 1) depends only on its dependency cone: the
neighbours its one-dimensional stencil reads (at -+h and -+3h along the pass's
dimension, Sec. 4.1), theirs in turn, down to the anchors.  Every neighbour
lies in an earlier pass -- same level with an earlier dimension, or a coarser
level -- so the cone is finite and a memoised recursion over it evaluates one
output without touching the rest of the field.  For a 512^3 field a cone holds
a few thousand points, so sampled outputs of a full-size field can be checked
against the definitions in seconds.

Written from the definitions, independently of the vectorized codec:

* the pass of a point comes from its coordinates (``brute.pass_of_point``);
* the stencil and the quantizer are the scalar forms of ``predict``;
* a retrieval keeps the negabinary digits b_s..31 of each code of pass s
  (Thm. 1 with b_s discarded planes), digits found by repeated division by -2;
* outliers take their stored value whatever the plan (Sec. 4.2.2).

The arithmetic is the field's dtype, one IEEE operation per step, as in the
rest of the oracle.
"""

from __future__ import annotations

import sys

import numpy as np

from . import predict
from .brute import levels, negabinary_digits, pass_of_point


def truncated_code(q: int, b: int) -> int:
    """q with its b lowest negabinary digits set to zero."""
    if b <= 0:
        return int(q)
    d = negabinary_digits(int(q))
    return sum(d[k] * (-2) ** k for k in range(b, 32))


class Cone:
    """Memoised evaluation of single points of one field.

    x: the original field (any array supporting x[i] for index tuples);
    eb: absolute error bound; interp: ``predict.LINEAR`` or ``predict.CUBIC``.
    """

    def __init__(self, x, eb: float, interp: int = predict.CUBIC):
        self.x = x
        self.dims = tuple(int(d) for d in x.shape)
        self.D = len(self.dims)
        self.K = levels(self.dims)
        self.dt = np.dtype(x.dtype)
        self.t = self.dt.type
        self.eb = float(eb)
        self.interp = interp
        self.two_eb, _ = predict.quant_constants(self.dt, self.eb)
        self._c = {}      # point -> (q, x^, outlier)
        self._r = {}      # (plan key, point) -> x~
        # a cone is at most 3 passes deep per level
        sys.setrecursionlimit(max(sys.getrecursionlimit(), 200 + 8 * self.D * (self.K + 1)))

    def pass_of(self, i):
        """(pass index, level, dimension) of point i."""
        return pass_of_point(i, self.dims, self.K)

    def _neighbours(self, i, lev, k):
        """Stencil inputs of point i of a pass along k at level lev: the
        neighbour points at -1, +1, -3, +3 (level units) or None if absent."""
        h = 1 << (lev - 1)
        t = i[k]
        out = []
        for off in (-1, 1, -3, 3):
            c = t + off * h
            if 0 <= c < self.dims[k]:
                j = list(i)
                j[k] = c
                out.append(tuple(j))
            else:
                out.append(None)
        return out

    def _predict(self, i, value_of):
        s, lev, k = self.pass_of(i)
        if s == 0:
            return self.t(0.0)
        b, c, a, e = self._neighbours(i, lev, k)
        return predict.stencil_1d(self.interp, value_of(b),
                                  value_of(c) if c is not None else 0.0,
                                  value_of(a) if a is not None else 0.0,
                                  value_of(e) if e is not None else 0.0,
                                  c is not None, a is not None, e is not None, self.dt)

    def compressed(self, i):
        """(code q, reconstruction x^, outlier flag) of point i at compression."""
        i = tuple(int(v) for v in i)
        r = self._c.get(i)
        if r is None:
            pred = self._predict(i, self.xhat)
            r = predict.quantize_scalar(self.x[i], pred, self.eb, self.dt)
            self._c[i] = r
        return r

    def xhat(self, i):
        return self.compressed(i)[1]

    def code(self, i) -> int:
        return int(self.compressed(i)[0])

    def retrieved(self, i, plan):
        """x~ of point i for a retrieval that discards plan[s] planes of pass s."""
        key = tuple(int(b) for b in plan)
        return self._retrieved(tuple(int(v) for v in i), key)

    def _retrieved(self, i, key):
        r = self._r.get((key, i))
        if r is not None:
            return r
        q, _, out = self.compressed(i)
        if out:
            r = self.t(self.x[i])
        else:
            s = self.pass_of(i)[0]
            qb = truncated_code(q, key[s])
            pred = self._predict(i, lambda j: self._retrieved(j, key))
            r = self.t(pred + self.t(self.t(qb) * self.two_eb))
        self._r[(key, i)] = r
        return r

    def cone_size(self) -> int:
        """Distinct points evaluated so far (compression side)."""
        return len(self._c)
