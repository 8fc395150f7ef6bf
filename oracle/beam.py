"""Divergence of the energetic electrons -- oracle side (numpy, FP64).

TEST INFRASTRUCTURE ONLY: used by the tests; the product library computes its
own with no code in common.

Secs. IV.A-IV.B of the paper compare solvers by the divergence angle
theta_x = atan(p_x / p_z) of the accelerated electrons and by its RMS over the
highest-energy ones.  Readings taken (the paper names no energy cut and no
weighting): the electrons counted are those with Lorentz factor >= gamma_min
(a caller's choice) that move forward (u_z > 0, where atan(p_x/p_z) is the
angle to the axis); the RMS is weighted by the macro-particle charge w.
"""
from __future__ import annotations

import numpy as np


def divergence(p: dict, gamma_min: float) -> dict:
    """Sums over the selected electrons of a particle dict (ux, uy, uz, w):
    w, w theta_x^2, w theta_y^2 and the count, plus the RMS angles."""
    ux, uy, uz, w = (np.asarray(p[k], dtype=np.float64) for k in ("ux", "uy", "uz", "w"))
    sel = (uz > 0) & (ux * ux + uy * uy + uz * uz >= gamma_min * gamma_min - 1.0)
    tx = np.arctan(ux[sel] / uz[sel])
    ty = np.arctan(uy[sel] / uz[sel])
    ws = w[sel]
    sw = float(ws.sum())
    sx, sy = float((ws * tx * tx).sum()), float((ws * ty * ty).sum())
    return {"w": sw, "sum_wtx2": sx, "sum_wty2": sy, "count": int(sel.sum()),
            "rms_x": float(np.sqrt(sx / sw)) if sw > 0 else 0.0, "rms_y": float(np.sqrt(sy / sw)) if sw > 0 else 0.0}
