"""Narrow band, recovery and the optional mass projection.

TEST INFRASTRUCTURE ONLY (see the package header).

  * band list: ascending C-order linear indices of the points with
    |2 phi - 1| < threshold, decided in FP64.  In the [0,1] convention this is
    the +-1 condition |phi_pm| < threshold, an instance of the paper's
    Omega_band = {g(phi) >= delta} (Section 3.2).
  * recovery (Section 3.3, after Algorithm 1): U = GU / G where G > 1e-3,
    U = GU elsewhere.
  * mass projection (a reading; off by default): U <- U + c on
    {g > threshold} with c chosen so that <g U, 1>_h returns to Q0.
"""
from __future__ import annotations

import numpy as np

from .core import Grid


def band_list(phi: np.ndarray, threshold: float) -> np.ndarray:
    flat = np.asarray(phi, dtype=np.float64).reshape(-1)
    return np.flatnonzero(np.abs(2.0 * flat - 1.0) < threshold).astype(np.int32)


def band_list_loop(phi: np.ndarray, threshold: float) -> np.ndarray:
    """The same set by a plain loop (used to pin the vectorized form)."""
    flat = [float(x) for x in np.asarray(phi, dtype=np.float64).reshape(-1)]
    out = []
    for i, x in enumerate(flat):
        if abs(2.0 * x - 1.0) < threshold:
            out.append(i)
    return np.array(out, dtype=np.int32)


def band_mask(phi: np.ndarray, threshold: float) -> np.ndarray:
    return (np.abs(2.0 * np.asarray(phi, dtype=np.float64) - 1.0) < threshold).astype(np.float64)


def recover(GU: np.ndarray, G: np.ndarray, threshold: float = 1e-3) -> np.ndarray:
    safe = np.where(G > threshold, G, 1.0)
    return np.where(G > threshold, GU / safe, GU)


def mass_project(U, g, Q0: float, grid: Grid, threshold: float):
    sel = (g > threshold).astype(np.float64)
    Q = grid.cell * float(np.sum(g * U))
    den = grid.cell * float(np.sum(g * sel))
    if den <= 0.0:
        return U
    return U + ((Q0 - Q) / den) * sel
