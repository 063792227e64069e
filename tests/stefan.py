"""Analytic Stefan-problem fronts used to pin the oracle (Sec. 4.1).

The front of a film freezing from a wall at T_w below T_m into liquid at
T_0 is s(t) = 2 kappa sqrt(alpha_s t), with kappa the root of

  Ste / (exp(k^2) erf(k))
    - lam_l (T_0 - T_m) sqrt(a_r) Ste / (lam_s (T_m - T_w) exp((sqrt(a_r) k rho_r)^2)
                                         erfc(sqrt(a_r) k rho_r)) = k sqrt(pi),

rho_r = rho_s/rho_l, a_r = alpha_s/alpha_l, Ste = C_s (T_m - T_w)/L.  The
exponential is printed with the square outside its argument; the square
belongs to the argument: the liquid solution is erfc(eta - beta) with
beta = (1 - rho_r) k sqrt(a_r) for the liquid pushed away at (1 - rho_r) ds/dt,
which gives the erfc(sqrt(a_r) k rho_r) and exp(...^2) pair above.
With rho_r = 1 it is the classical two-phase Neumann solution.
"""
import math

from scipy.optimize import brentq
from scipy.special import erf, erfc


def kappa(ste, rho_r=1.0, alpha_r=1.0, lam_l_over_lam_s=1.0, T0=1.0, Tm=0.0, Tw=-1.0):
    a = math.sqrt(alpha_r)

    def fn(k):
        lhs = ste / (math.exp(k * k) * erf(k))
        z = a * k * rho_r
        lhs -= (lam_l_over_lam_s * (T0 - Tm) * a * ste) / ((Tm - Tw) * math.exp(z * z) * erfc(z))
        return lhs - k * math.sqrt(math.pi)

    return brentq(fn, 1e-6, 3.0, xtol=1e-15)


def front(t, kap, alpha_s):
    return 2.0 * kap * math.sqrt(alpha_s * t)
