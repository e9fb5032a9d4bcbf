"""Macroscopic calibration of the springs' reference strain (host-side input
preparation; the library takes the spring parameters as given).

The multi-spring law of Section 2.1 gives an integration point the stress
K_b tr(eps) m + sum_k c_k tau_k n_k, with tau_k the modified Ramberg-Osgood
skeleton of spring k at its strain gamma_k = n_k . eps.  Under a simple shear
gamma (engineering xy strain) spring k sees n_k,xy gamma, mostly less than
gamma, so a point whose springs all use the soil's reference strain softens
more slowly than the soil: its secant modulus at gamma_ref is above G0 / 2.
``spring_gamma_ref`` returns the spring reference strain for which the
point's secant shear modulus under monotonic simple shear is G0 / 2 at the
soil's gamma_ref, i.e. the point follows the soil's G/G0 curve at its
reference strain.

The skeleton is self-similar (tau / (G0 gamma_ref) depends on gamma /
gamma_ref only), so the ratio spring / soil reference strain depends on the
spring table and h_max alone.
"""
from __future__ import annotations

import numpy as np


def ro_beta(h_max: float) -> float:
    """Exponent of the normalised skeleton e = s (1 + |2s|^beta) whose Masing
    loops reach the damping ratio h_max at large strain."""
    return 2.0 * np.pi * h_max / (2.0 - np.pi * h_max)


def skeleton_s(e: np.ndarray, beta: float) -> np.ndarray:
    """Normalised skeleton stress s (tau / (G0 gamma_ref)) at the normalised
    strains e (gamma / gamma_ref): the root of s (1 + |2s|^beta) = e, by
    Newton from s = e (the residual is convex in s >= 0, so the iterates
    decrease monotonically to the root)."""
    e = np.asarray(e, dtype=np.float64)
    a = np.abs(e)
    s = a.copy()
    for _ in range(200):
        p = np.power(2.0 * s, beta, where=s > 0, out=np.zeros_like(s))
        f = s * (1.0 + p) - a
        ds = f / (1.0 + (1.0 + beta) * p)
        s = s - ds
        if np.all(np.abs(ds) <= 1e-15 * np.maximum(s, 1e-300)):
            break
    return np.sign(e) * s


def point_secant_ratio(gamma: float, gamma_ref_spring: float, h_max: float, dirs: np.ndarray,
                       weights: np.ndarray) -> float:
    """G_sec / G0 of an integration point under a monotonic simple shear
    gamma (xy), every spring with reference strain gamma_ref_spring."""
    nxy = np.asarray(dirs, dtype=np.float64)[:, 3]
    w = np.asarray(weights, dtype=np.float64)
    s = skeleton_s(nxy * gamma / gamma_ref_spring, ro_beta(h_max))
    tau_over_g0 = gamma_ref_spring * s  # tau_k / G0
    return float(np.sum(w * nxy * tau_over_g0) / gamma)


def spring_gamma_ref(gamma_ref: float, h_max: float, dirs: np.ndarray, weights: np.ndarray,
                     rtol: float = 1e-14) -> float:
    """Spring reference strain for which the point's secant shear modulus at
    the soil's gamma_ref is G0 / 2 (bisection in log space: the ratio rises
    monotonically from 0 to its linear value 1 as the spring reference strain
    grows)."""
    if gamma_ref <= 0.0:
        raise ValueError("gamma_ref must be positive")
    nxy = np.asarray(dirs, dtype=np.float64)[:, 3]
    lin = float(np.sum(np.asarray(weights, dtype=np.float64) * nxy * nxy))
    if not lin > 0.5:
        raise ValueError("the spring table has no shear stiffness above G0 / 2 in simple shear")
    lo, hi = gamma_ref * 1e-6, gamma_ref * 1e6
    f = lambda g: point_secant_ratio(gamma_ref, g, h_max, dirs, weights) - 0.5  # noqa: E731
    if not (f(lo) < 0.0 < f(hi)):
        raise ValueError("no spring reference strain within 1e-6..1e6 of gamma_ref reaches G0 / 2")
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
        if hi / lo - 1.0 <= rtol:
            break
    return float(np.sqrt(lo * hi))
