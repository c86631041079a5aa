"""Host-side parameter checks (no GPU).

Weak compressibility (section "A lightning introduction to the method"):
the equation of state uses a fictitious sound speed c0, chosen at least ten
times the largest flow speed U so that the relative density variation,
which scales with the squared Mach number (U/c0)^2, stays near 1%.  For a
free-surface flow under gravity U is at least the free-fall speed
sqrt(2 g H) of the water height H.
"""
from __future__ import annotations

import math


def weak_compressibility(params, height: float, u_max: float = 0.0) -> dict:
    """U = max(u_max, sqrt(2 |g| height)); returns U, the Mach number U/c0,
    the expected relative density variation (U/c0)^2 and ok = c0 >= 10 U."""
    g = math.sqrt(sum(float(v) ** 2 for v in params.g))
    U = max(float(u_max), math.sqrt(2.0 * g * max(float(height), 0.0)))
    c0 = float(params.c0)
    mach = U / c0 if c0 > 0 else math.inf
    return {"U": U, "c0": c0, "mach": mach, "density_variation": mach * mach, "ok": c0 >= 10.0 * U}
