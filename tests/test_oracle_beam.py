"""The oracle reproduces the free-streaming beam numbers the paper prints
(Sect. 3.2): at 300 x 300, Courant number 0.4, HLL, LimO3 with the
f-preserving face fix and second-order steps, the beam maximum falls by
8 % and its full width at half maximum grows by 7 % between the cuts at
x = 1 and x = 4.35.  The emitter reading and the cut measurement are those
of beam_common.  PLM at the same resolution diffuses about twice as much,
outside the band; the beam stays on the diagonal."""
import math

import numpy as np

from paper_2606_26268_amd import inputs as I
from tests import beam_common as B


def _run(orc, N, limiter):
    p = I.make_beam(N=N)
    p.limiter = limiter
    o = orc.Oracle(p)
    f = {k: np.array(v) for k, v in p.fields.items()}
    m = B.emitter_mask(N)
    Eb, Fxb, Fyb = B.emitter_state()
    for _ in range(int(B.T_END / p.dt)):
        f, _ = o.run(f, p.dt, 1, rk2=True)
        f = {k: np.array(v) for k, v in f.items()}
        f["E"][0][m], f["Fx"][0][m], f["Fy"][0][m] = Eb, Fxb, Fyb
    return f["E"][0]


def test_limo3_beam_matches_the_printed_peak_and_width(orc):
    dp, dw, dy = B.changes(_run(orc, B.PAPER["resolution"], 1))
    print(f"oracle beam, LimO3 300^2: peak {100 * dp:+.1f} %, FWHM {100 * dw:+.1f} % (paper -8 %, +7 %)")
    assert B.PEAK_BAND[0] < dp < B.PEAK_BAND[1], dp
    assert B.FWHM_BAND[0] < dw < B.FWHM_BAND[1], dw
    # the centre moves along the diagonal: by 3.35 in y, within a cell
    assert abs(dy - (B.CUTS[1] - B.CUTS[0])) < 5.0 / 300


def test_plm_beam_at_a_third_of_the_resolution_diffuses_more(orc):
    """PLM at a third of the resolution (a 2-cell-wide beam) loses much more
    of its peak than the band allows: the band tells coarse from fine."""
    dp, dw, _ = B.changes(_run(orc, 100, 0))
    assert dp < B.PEAK_BAND[0] and dw > B.FWHM_BAND[1], (dp, dw)
