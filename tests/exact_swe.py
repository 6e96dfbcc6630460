"""Analytic solutions of the 1D shallow-water dam break used to pin the oracle.

Stoker (wet downstream bed): left rarefaction, constant middle state, right
shock, from the textbook Riemann relations (Toro 2001, ch. 5):
    rarefaction:  u_m = 2 (c_L - c_m)
    shock:        u_m = (h_m - h_R) sqrt(g (h_m + h_R) / (2 h_m h_R))
Ritter (dry downstream bed): h = (2 c_L - x/t)^2 / (9 g) on -c_L <= x/t <= 2 c_L.
A passive tangential velocity is carried by the contact moving at u_m.
"""
import math

import numpy as np


def stoker_star(hL, hR, g=9.81):
    cL = math.sqrt(g * hL)

    def f(hm):
        return 2.0 * (cL - math.sqrt(g * hm)) - (hm - hR) * math.sqrt(
            g * (hm + hR) / (2.0 * hm * hR))

    lo, hi = hR, hL
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
    hm = 0.5 * (lo + hi)
    um = 2.0 * (cL - math.sqrt(g * hm))
    shock = hm * um / (hm - hR)
    return hm, um, shock


def dam_break_exact(x, t, x0, hL, hR, g=9.81, vL=0.0, vR=0.0):
    """(h, u, v) of the dam break at positions x, time t > 0 (u_L = u_R = 0)."""
    x = np.asarray(x, dtype=np.float64)
    xi = (x - x0) / t
    cL = math.sqrt(g * hL)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    if hR == 0.0:
        left = xi <= -cL
        fan = (xi > -cL) & (xi < 2 * cL)
        h[left] = hL
        u[left] = 0.0
        h[fan] = (2 * cL - xi[fan]) ** 2 / (9 * g)
        u[fan] = 2.0 / 3.0 * (cL + xi[fan])
        dry = xi >= 2 * cL
        h[dry] = 0.0
        u[dry] = 0.0
        um = 2 * cL
    else:
        hm, um, S = stoker_star(hL, hR, g)
        cm = math.sqrt(g * hm)
        left = xi <= -cL
        fan = (xi > -cL) & (xi <= um - cm)
        mid = (xi > um - cm) & (xi < S)
        right = xi >= S
        h[left], u[left] = hL, 0.0
        h[fan] = (2 * cL - xi[fan]) ** 2 / (9 * g)
        u[fan] = 2.0 / 3.0 * (cL + xi[fan])
        h[mid], u[mid] = hm, um
        h[right], u[right] = hR, 0.0
    v = np.where(xi < um, vL, vR)
    return h, u, v
