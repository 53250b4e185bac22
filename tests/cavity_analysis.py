"""Post-processing of lid-driven cavity fields (Sec. 4.4.1): the stream
function and the vortex centres that Table 1 lists.

The cavity has N x N nodes including the walls; node (i, j) sits at
(i / (N - 1), j / (N - 1)).  The stream function is the integral of u_x up
a column from the bottom wall, psi(x, y) = int_0^y u_x dy', taken with the
composite Simpson rule over node pairs (a trapezoid closes an odd last
interval), and psi = 0 on the bottom wall.  Vortex centres are local extrema
of psi: with the lid moving in +x the primary vortex turns clockwise and is
the global minimum; the counter-rotating corner vortices are local maxima.
"""
from __future__ import annotations

import numpy as np


def stream_function(ux: np.ndarray) -> np.ndarray:
    """psi[j, i] from ux[j, i] (row j = height), spacing h = 1 / (N - 1)."""
    ny = ux.shape[0]
    h = 1.0 / (ny - 1)
    psi = np.zeros_like(ux, dtype=np.float64)
    for j in range(1, ny):
        if j % 2 == 0:
            # Simpson over the pair (j-2, j-1, j)
            psi[j] = psi[j - 2] + h / 3.0 * (ux[j - 2] + 4.0 * ux[j - 1] + ux[j])
        else:
            # odd node: Simpson up to j-1, trapezoid on the last interval
            psi[j] = psi[j - 1] + 0.5 * h * (ux[j - 1] + ux[j])
    return psi


def _argext(psi, region, kind):
    sub = np.where(region, psi, np.nan)
    k = np.nanargmin(sub) if kind == "min" else np.nanargmax(sub)
    j, i = np.unravel_index(k, psi.shape)
    return int(i), int(j)


def vortex_centres(psi: np.ndarray) -> dict:
    """Node indices (i, j) of the primary (global minimum of psi over the
    fluid nodes) and of the lower-left, lower-right and top-left vortices
    (maximum of psi in the corner regions, which holds the corner vortex
    whenever one exists)."""
    n = psi.shape[0]
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    fluid = (ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1)
    x, y = ii / (n - 1), jj / (n - 1)
    out = {"primary": _argext(psi, fluid, "min")}
    out["lower_left"] = _argext(psi, fluid & (x < 0.35) & (y < 0.35), "max")
    out["lower_right"] = _argext(psi, fluid & (x > 0.65) & (y < 0.35), "max")
    out["top_left"] = _argext(psi, fluid & (x < 0.35) & (y > 0.65), "max")
    return out


def load_table(path: str) -> dict:
    """Rows of the vortex-centre fixture: {(re, row): {name: (x, y) or None}}."""
    names = ["primary", "lower_left", "lower_right", "top_left"]
    table = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            re, row, vals = float(tok[0]), tok[1], tok[2:]
            entry = {}
            for k, name in enumerate(names):
                a, b = vals[2 * k], vals[2 * k + 1]
                entry[name] = None if a == "-" else (float(a), float(b))
            table[(re, row)] = entry
    return table
