"""Plain CPU oracle for the IPComp hot path (test infrastructure only).

This package is the slow, obviously-correct reference that the HIP path is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product library never
does, and it shares no code, tables or helpers with the HIP path.

What it computes (IPComp, arXiv 2502.04093):

* ``schedule``  -- the multilevel interpolation hierarchy: strides 2^(l-1), one
  one-dimensional pass per dimension inside every level (Sec. 4.1, Fig.
  "interp-design"); the grouping of each pass's codes into chunks.
* ``predict``   -- the linear and cubic interpolation stencils (Eq. interp-linear,
  Eq. interp-cubic) and the error-bounded quantizer of the prediction model
  (Sec. 4.2.2, Eq. error-prediction-interp).
* ``coding``    -- negabinary (Sec. 4.4.2), the two-prefix-bit XOR predictive
  bitplane code (Sec. 4.4.1), bitplane packing (Sec. 4.3, Fig. "overwrite") and
  the truncation-loss table delta-y (Thm. 1).
* ``stream``    -- the serialized container of independently loadable blocks,
  raw or with every block entropy coded.
* ``entropy``   -- the entropy stage that stands in for the paper's lossless
  compressor (zstd, Sec. 6 setup): an adaptive binary range coder per block.
* ``planner``   -- the Thm. 1 bound (per-pass reading) and the two knapsack
  dynamic programs of Sec. 5.2 (error-bound mode) and Sec. 5.3 (bitrate mode).
* ``codec``     -- compress, retrieve (Alg. 1) and refine (Alg. 2, recompute
  form).
* ``brute``     -- scalar per-point versions for tiny grids.
* ``pointwise`` -- single outputs of full-size fields through their dependency
  cones (memoised recursion), for sampled checks at sizes the codec would take
  minutes on.

Arithmetic runs in the field's own dtype (float32 or float64) with one IEEE
operation per step and no fused multiply-add, because the GPU path must agree
with it bit for bit; NumPy never contracts.

Parity pins (what ties this oracle to something other than itself) live in
``tests/test_oracle_*.py``.  Every function here has at least one pin; none is
"parity unpinned".  Compression ratio and bitrate-mode plans versus the paper's
own numbers are unpinned (the paper's zstd stage and datasets are absent).
"""

from . import schedule, predict, coding, entropy, stream, planner, codec, pointwise  # noqa: F401
