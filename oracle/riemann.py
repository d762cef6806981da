"""Exact solution of the 1-D Riemann problem for an ideal gas.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Used to check the oracle's
shock-tube run (Sec. 4, the Sod test) against the textbook solution: a
pressure function solved for the star-region pressure by Newton iteration,
then sampling of the self-similar wave pattern (rarefaction fans, contact,
shocks).  Written from the gas-dynamics definitions (Rankine-Hugoniot jump
conditions and isentropic rarefaction relations for a calorically perfect gas).
"""
from __future__ import annotations

import math

import numpy as np


def _pressure_function(p, rho_k, p_k, c_k, gamma):
    """f_k(p) and its derivative: velocity change across the k-wave."""
    if p > p_k:  # shock
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        f = (p - p_k) * s
        df = s * (1.0 - 0.5 * (p - p_k) / (p + B))
    else:  # rarefaction
        pr = p / p_k
        f = 2.0 * c_k / (gamma - 1.0) * (pr ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho_k * c_k) * pr ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(rhoL, uL, pL, rhoR, uR, pR, gamma):
    """Star-region pressure and velocity."""
    cL = math.sqrt(gamma * pL / rhoL)
    cR = math.sqrt(gamma * pR / rhoR)
    p = max(1e-12, 0.5 * (pL + pR))
    for _ in range(200):
        fL, dL = _pressure_function(p, rhoL, pL, cL, gamma)
        fR, dR = _pressure_function(p, rhoR, pR, cR, gamma)
        dp = (fL + fR + (uR - uL)) / (dL + dR)
        pn = max(1e-14, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _pressure_function(p, rhoL, pL, cL, gamma)
    fR, _ = _pressure_function(p, rhoR, pR, cR, gamma)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def waves(rhoL, uL, pL, rhoR, uR, pR, gamma):
    """Star state plus wave speeds (for rarefactions: head and tail)."""
    p, u = star_state(rhoL, uL, pL, rhoR, uR, pR, gamma)
    cL = math.sqrt(gamma * pL / rhoL)
    cR = math.sqrt(gamma * pR / rhoR)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    out = {"p_star": p, "u_star": u}
    if p > pL:
        out["rho_star_L"] = rhoL * ((p / pL + g1) / (g1 * p / pL + 1.0))
        out["left_shock"] = uL - cL * math.sqrt((gamma + 1.0) / (2.0 * gamma) * p / pL + (gamma - 1.0) / (2.0 * gamma))
    else:
        out["rho_star_L"] = rhoL * (p / pL) ** (1.0 / gamma)
        out["left_head"] = uL - cL
        out["left_tail"] = u - cL * (p / pL) ** ((gamma - 1.0) / (2.0 * gamma))
    if p > pR:
        out["rho_star_R"] = rhoR * ((p / pR + g1) / (g1 * p / pR + 1.0))
        out["right_shock"] = uR + cR * math.sqrt((gamma + 1.0) / (2.0 * gamma) * p / pR + (gamma - 1.0) / (2.0 * gamma))
    else:
        out["rho_star_R"] = rhoR * (p / pR) ** (1.0 / gamma)
        out["right_head"] = uR + cR
        out["right_tail"] = u + cR * (p / pR) ** ((gamma - 1.0) / (2.0 * gamma))
    return out


def sample(rhoL, uL, pL, rhoR, uR, pR, gamma, s):
    """Exact (rho, u, p) at similarity coordinates s = (x - x0) / t (array)."""
    s = np.asarray(s, dtype=np.float64)
    w = waves(rhoL, uL, pL, rhoR, uR, pR, gamma)
    p_s, u_s = w["p_star"], w["u_star"]
    cL = math.sqrt(gamma * pL / rhoL)
    cR = math.sqrt(gamma * pR / rhoR)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    for j, x in enumerate(s.ravel()):
        if x <= u_s:  # left of contact
            if p_s > pL:
                if x <= w["left_shock"]:
                    r, v, q = rhoL, uL, pL
                else:
                    r, v, q = w["rho_star_L"], u_s, p_s
            else:
                if x <= w["left_head"]:
                    r, v, q = rhoL, uL, pL
                elif x >= w["left_tail"]:
                    r, v, q = w["rho_star_L"], u_s, p_s
                else:  # inside the left fan
                    v = 2.0 / (gamma + 1.0) * (cL + 0.5 * (gamma - 1.0) * uL + x)
                    c = 2.0 / (gamma + 1.0) * (cL + 0.5 * (gamma - 1.0) * (uL - x))
                    r = rhoL * (c / cL) ** (2.0 / (gamma - 1.0))
                    q = pL * (c / cL) ** (2.0 * gamma / (gamma - 1.0))
        else:
            if p_s > pR:
                if x >= w["right_shock"]:
                    r, v, q = rhoR, uR, pR
                else:
                    r, v, q = w["rho_star_R"], u_s, p_s
            else:
                if x >= w["right_head"]:
                    r, v, q = rhoR, uR, pR
                elif x <= w["right_tail"]:
                    r, v, q = w["rho_star_R"], u_s, p_s
                else:
                    v = 2.0 / (gamma + 1.0) * (-cR + 0.5 * (gamma - 1.0) * uR + x)
                    c = 2.0 / (gamma + 1.0) * (cR - 0.5 * (gamma - 1.0) * (uR - x))
                    r = rhoR * (c / cR) ** (2.0 / (gamma - 1.0))
                    q = pR * (c / cR) ** (2.0 * gamma / (gamma - 1.0))
        rho.flat[j], u.flat[j], p.flat[j] = r, v, q
    return rho, u, p
