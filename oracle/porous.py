"""Porous-medium post-processing of a rarefaction sweep (Sec. III), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): written independently of
the library's post-processing, which it checks.

From flow rates Q at several rarefaction parameters delta of one geometry:
  * Kn = sqrt(pi) / (2 delta) and k_a = sqrt(4/pi) Q Kn (Sec. III, first
    equation of the section; reading: delta = sqrt(pi)/(2 Kn));
  * the intrinsic permeability k_inf, defined in Sec. III as the apparent
    permeability in the limit Kn -> 0.  Reading (the paper gives no
    procedure): the least-squares quadratic in Kn through the three samples
    of smallest Kn (an exact fit for three points), evaluated at Kn = 0;
  * H* = H sqrt(12 k_inf / phi) and Kn* = Kn sqrt(phi / (12 k_inf)) (Sec. III,
    the two equations after the flow-rate definition), with H = 1.
"""
from __future__ import annotations

import numpy as np


def permeability_curve(delta, Q, porosity: float) -> dict:
    delta = np.asarray(delta, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    Kn = np.sqrt(np.pi) / (2.0 * delta)
    ka = np.sqrt(4.0 / np.pi) * Q * Kn
    near = np.argsort(Kn)[:3]
    coef = np.polyfit(Kn[near], ka[near], 2)       # highest power first
    k_inf = float(coef[-1])                        # the fit at Kn = 0
    H_star = np.sqrt(12.0 * k_inf / porosity)
    Kn_star = Kn * np.sqrt(porosity / (12.0 * k_inf))
    return {"k_inf": k_inf, "H_star": float(H_star), "Kn_star": Kn_star, "ka_ratio": ka / k_inf,
            "Kn": Kn, "k_a": ka}
