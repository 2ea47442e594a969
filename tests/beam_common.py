"""Set-up and measurement of the free-streaming beam of Sect. 3.2, shared by
the oracle pin and the GPU measurement (no arithmetic of the method here).

Reading of the set-up: the rectangle x in [0.5, 0.6], y in [0.3, 0.44] keeps
the beam state (E = 1e12, F_x = F_y = E / sqrt 2) for the whole run, so that
it emits a steady oblique beam; the paper places the beam inside the domain
in place of the oblique boundary injection of earlier work, and its two cuts
(x = 1 and x = 4.35) are taken on one snapshot of the steady beam, each
centred on its maximum.  The beam reaches x = 4.35 at t = 3.75 sqrt 2 = 5.3;
the snapshot is taken at t = 5.9."""
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PAPER = json.load(open(os.path.join(GOLDEN, "paper_printed.json")))["beam"]
T_END = 5.9
CUTS = (1.0, 4.35)
# bands around the printed changes (-8 %, +7 %): +-4 percentage points, which
# PLM (-16 %, +17 % at this resolution) and a once-released packet (-50 % and
# more) fall outside
PEAK_BAND = (PAPER["peak_change"] - 0.04, PAPER["peak_change"] + 0.04)
FWHM_BAND = (PAPER["fwhm_change"] - 0.04, PAPER["fwhm_change"] + 0.04)


def emitter_mask(N):
    """Cells (j, i) of an N x N grid on [0, 5]^2 whose centres lie in the beam rectangle."""
    L = PAPER["box"]
    c = (np.arange(N) + 0.5) * L / N
    Y, X = np.meshgrid(c, c, indexing="ij")
    x0, x1 = PAPER["beam_x"]
    y0, y1 = PAPER["beam_y"]
    return (X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1)


def emitter_state():
    E = PAPER["beam_E"]
    return E, E / math.sqrt(2.0), E / math.sqrt(2.0)


def cut(E, x):
    """Peak (above the background), full width at half maximum and centre of
    the vertical cut of E (indexed [j, i], N x N on [0, 5]^2) at x, linear
    in x between the two cell columns around it and in y at the half-maximum
    crossings."""
    N = E.shape[0]
    L = PAPER["box"]
    y = (np.arange(N) + 0.5) * L / N
    g = x / (L / N) - 0.5
    i = int(math.floor(g))
    w = g - i
    prof = (1 - w) * E[:, i] + w * E[:, i + 1] - PAPER["background_E"]
    j = int(np.argmax(prof))
    half = 0.5 * prof[j]
    lo = j
    while lo > 0 and prof[lo - 1] > half:
        lo -= 1
    hi = j
    while hi < N - 1 and prof[hi + 1] > half:
        hi += 1
    yl = y[lo - 1] + (half - prof[lo - 1]) / (prof[lo] - prof[lo - 1]) * (y[lo] - y[lo - 1])
    yr = y[hi] + (half - prof[hi]) / (prof[hi + 1] - prof[hi]) * (y[hi + 1] - y[hi])
    return prof[j], yr - yl, y[j]


def changes(E):
    """(peak change, FWHM change, centre shift in y) between the two cuts."""
    (p1, w1, y1), (p2, w2, y2) = (cut(E, x) for x in CUTS)
    return p2 / p1 - 1.0, w2 / w1 - 1.0, y2 - y1
