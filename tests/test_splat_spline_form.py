"""The form in which the GPU splat evaluates the M4 spline (Eq. 12's kernel).

The gather kernel sums m t^3 and m s^3 with t = max(1 - q/2, 0) and
s = max(1 - q, 0), q = r / h, and takes sigma (2 A - B) as sum m W.  This
checks, in float64 on the host, that sigma (2 t^3 - s^3) is the oracle's
kernel W(r, h) for every r, including the knots q = 1 and q = 2 and beyond
the support (the clamps then give exact zeros).
"""
import numpy as np

import oracle


def test_clamped_form_is_the_m4_spline():
    h = 0.04
    sigma = 1.0 / (np.pi * h ** 3)
    r = np.concatenate([np.linspace(0.0, 3.0 * h, 30001), [h, 2.0 * h, 2.0 * h * (1 + 1e-12)]])
    q = r / h
    t = np.maximum(1.0 - q / 2.0, 0.0)
    s = np.maximum(1.0 - q, 0.0)
    w_form = sigma * (2.0 * t ** 3 - s ** 3)
    w_ref = oracle.kernel(r, h)
    assert np.allclose(w_form, w_ref, rtol=1e-12, atol=1e-12 * sigma)
    assert (w_form[q >= 2.0] == 0.0).all()
    # the inner sum only matters inside q < 1, where s > 0
    assert (s[q >= 1.0] == 0.0).all() and (s[q < 1.0] > 0.0).all()
