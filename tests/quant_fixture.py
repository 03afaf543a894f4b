"""Exact rounding-tie fixture for the gradient quantisation.

The quantised gradient is rint(mag * Q / max(mag)) with ties to even (the
reading taken for the pre-processing, which the paper leaves open; its inputs
are raw integer images). This module builds a float image whose unnormalised
Sobel magnitudes are known exactly, so that mag * Q / max lands exactly on
k + 1/2 for most pixels: a truncating, flooring or round-half-up quantiser
gives a different byte there.

Construction (3 identical rows, nx = 2K + 2 columns, no blur):
  * identical rows make the y derivative 0 and the [1, 2, 1] smoothing across
    rows a factor 4, so mag(x) = 4 |f(x+1) - f(x-1)| with the mirrored border
    f(-1) = f(0), f(nx) = f(nx - 1);
  * columns 2j and 2j + 1 hold the same value e_j / 8 with e_0 = 0 and
    e_{j+1} = e_j + 2 m_j, so mag is 0 at both ends and m_j at columns
    2j + 1 and 2j + 2;
  * the m_j are odd integers plus one largest value 2 Q, so max(mag) = 2 Q and
    every odd m_j scales to exactly m_j / 2 = (m_j - 1) / 2 + 1/2.
All values are dyadic and below 2^24, so float32 and float64 evaluate the
magnitudes without rounding.
"""
from __future__ import annotations

import numpy as np


def tie_values(Q: int):
    """The m_j: odd magnitudes (several .5 ties) and the maximum 2 Q."""
    if Q == 255:
        odd = list(range(1, 2 * Q, 2))                # every tie 0.5 .. 254.5
    else:
        odd = list(range(1, 64, 2)) + [101, 1001, 65535, 65537, 131067, 131069]
    return odd + [2 * Q]


def tie_image(Q: int):
    """(float32 image (3, nx), exact magnitudes (3, nx), expected bytes (3, nx))."""
    m = np.array(tie_values(Q), dtype=np.int64)
    e = np.concatenate([[0], np.cumsum(2 * m)])        # e_0 .. e_K
    f = np.repeat(e, 2).astype(np.float64) / 8.0        # columns 2j, 2j + 1
    nx = f.size
    mag = np.zeros(nx, dtype=np.float64)
    mag[1:-1] = np.repeat(m, 2)                         # columns 1 .. nx - 2
    assert f.max() < 2 ** 21 and (f * 8 == np.round(f * 8)).all()
    img = np.tile(f.astype(np.float32), (3, 1))
    # the expected bytes from the definition: round half to even of mag / 2
    half = mag / 2.0
    q = np.floor(half)
    frac = half - q
    q = q + np.where(frac > 0.5, 1, np.where(frac < 0.5, 0, q % 2))
    expect = np.tile(q.astype(np.int64), (3, 1))
    return img, np.tile(mag, (3, 1)), expect
