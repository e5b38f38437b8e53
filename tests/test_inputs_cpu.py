"""CPU: the seeded input builders and the paper-value fixtures under
tests/golden (their transcription, not the method)."""
import json
import math
import os

import numpy as np
from scipy import ndimage

from paper_2606_04347_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_convergence_tables_rates_are_log2_error_ratios():
    """Tables 1-2 (Section 4.1) print each rate as log2 of consecutive error
    ratios for halved tau; the transcription must reproduce every printed
    rate to its three decimals."""
    d = json.load(open(os.path.join(GOLDEN, "convergence_tables.json")))
    assert all(abs(d["tau"][k] - d["tau"][k - 1] / 2) <= 1e-20 for k in range(1, len(d["tau"])))
    for name, rows in d["tables"].items():
        for eps, v in rows.items():
            for k in range(1, len(v["err"])):
                r = math.log2(v["err"][k - 1] / v["err"][k])
                assert abs(r - v["rate"][k]) <= 1.5e-3, (name, eps, k, r, v["rate"][k])


def test_fixed_patch_study_geometry():
    """The convergence-study circle (Section 4.1): g = 18 (phi^2 - phi)^2 of the
    tanh profile, positive everywhere; U^0 the indicator of one connected
    patch of {g >= 1e-3} holding 35 % of its g-mass (to one point's share)."""
    fi = inputs.fixed_patch_study(n=128, eps_u_in_h=10.0)
    h = 2.0 / 128
    X = inputs.mesh(fi.shape, fi.half_len)
    r = np.sqrt(X[0] ** 2 + X[1] ** 2)
    phi = 0.5 + 0.5 * np.tanh(3.0 * (0.4 - r) / (10.0 * h))
    g_def = 18.0 * (phi * phi - phi) ** 2
    assert (fi.g > 0).all()
    assert np.abs(fi.g - g_def).max() <= 1e-14
    mem = fi.g >= 1e-3
    assert set(np.unique(fi.u0)) == {0.0, 1.0}
    assert (fi.u0[~mem] == 0).all()
    frac = (fi.g * fi.u0).sum() / fi.g[mem].sum()
    assert 0.35 - fi.g.max() / fi.g[mem].sum() <= frac <= 0.35
    _, ncomp = ndimage.label(fi.u0 > 0)
    assert ncomp == 1
    assert abs(fi.eps_u - 10.0 * h) <= 1e-15 and fi.gamma == 100.0 and fi.ubar == 0.3
