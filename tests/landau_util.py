"""Closed-form Landau damping rate and the peak fit used by the physics pins."""
import math

import numpy as np


def landau_root(k: float, v_th: float = 1.0):
    """Least-damped root w of the Vlasov-Poisson dispersion relation for a
    Maxwellian,  1 + (1 + zeta Z(zeta)) / (k lambda_D)^2 = 0,
    zeta = w / (sqrt(2) k v_th),  Z(zeta) = i sqrt(pi) w_Faddeeva(zeta)."""
    from scipy.special import wofz

    def D(w):
        zeta = w / (math.sqrt(2.0) * k * v_th)
        Z = 1j * math.sqrt(math.pi) * wofz(zeta)
        return 1.0 + (1.0 + zeta * Z) / (k * v_th) ** 2

    w = complex(math.sqrt(1 + 3 * k * k), -0.15)
    for _ in range(100):
        d = 1e-7
        f = D(w)
        df = (D(w + d) - D(w - d)) / (2 * d)
        step = f / df
        w -= step
        if abs(step) < 1e-14:
            break
    return w


def fit_damping(t, energy, t_min=1.0, t_max=16.0):
    """Least-squares slope of log(energy) through its local maxima; energy
    decays at 2*gamma, so gamma = slope/2."""
    e = np.asarray(energy)
    idx = [i for i in range(1, len(e) - 1) if e[i] > e[i - 1] and e[i] >= e[i + 1]
           and t_min < t[i] < t_max]
    c = np.polyfit(np.asarray(t)[idx], np.log(e[idx]), 1)
    return c[0] / 2.0, len(idx)
