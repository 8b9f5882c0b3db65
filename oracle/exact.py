"""Exact single-mode solutions (oracle; test infrastructure).

Used to pin the order O(tau^k) of the corrected schemes (Lemma 2.2, eq.
err-BDF; Lemma 3.2, eq. err-BDF-frac) on one spatial eigenmode with
eigenvalue mu:
* heat (alpha = 1), y' + mu y = cos t + sin t, y(0) = y0 (every d^l f/dt^l (0)
  is +-1, so every row of Table 1 takes part, and the solution stays bounded):
      y(t) = y0 e^{-mu t} + a (cos t - e^{-mu t}) + b sin t,
      a = (mu - 1)/(1 + mu^2), b = (1 + mu)/(1 + mu^2);
* subdiffusion with alpha = 1/2, f = 0: y(t) = y0 E_{1/2}(-mu t^{1/2}), and
  E_{1/2}(-z) = exp(z^2) erfc(z) = erfcx(z).
"""
import numpy as np
from scipy.special import erfcx


def subdiffusion_half_mode(mu, y0, t):
    t = np.asarray(t, dtype=np.float64)
    return y0 * erfcx(mu * np.sqrt(t))


def heat_trig_mode(mu, y0, t):
    t = np.asarray(t, dtype=np.float64)
    a = (mu - 1.0) / (1.0 + mu ** 2)
    b = (1.0 + mu) / (1.0 + mu ** 2)
    return y0 * np.exp(-mu * t) + a * (np.cos(t) - np.exp(-mu * t)) + b * np.sin(t)
