"""Closed-form values used to pin the oracle (no oracle code is used here).

* Mean exit time of Brownian motion with generator Laplacian (sigma = sqrt(2) I)
  from a rectangle [0, a] x [0, b]: the solution of Lap w = -1, w = 0 on the
  boundary (eq. 26), as its double sine series
      w = sum_{p,q odd} 16 / (pi^2 p q) sin(p pi x / a) sin(q pi y / b)
                         / (pi^2 (p^2/a^2 + q^2/b^2)).
* Harmonic measure of the side y = b of that rectangle (probability of leaving
  through it): the solution of Lap u = 0 with u = 1 on y = b and 0 elsewhere,
      u = sum_{p odd} 4 / (p pi) sin(p pi x / a) sinh(p pi y / a) / sinh(p pi b / a).
"""
import numpy as np


def mean_exit_time_rectangle(x, y, a, b, terms=401):
    p = np.arange(1, terms + 1, 2)[:, None]
    q = np.arange(1, terms + 1, 2)[None, :]
    coef = 16.0 / (np.pi ** 2 * p * q) / (np.pi ** 2 * (p ** 2 / a ** 2 + q ** 2 / b ** 2))
    return float(np.sum(coef * np.sin(p * np.pi * x / a) * np.sin(q * np.pi * y / b)))


def harmonic_measure_top(x, y, a, b, terms=401):
    p = np.arange(1, terms + 1, 2)
    # sinh ratio written with exponentials to avoid overflow
    ratio = np.exp(p * np.pi * (y - b) / a) * (1 - np.exp(-2 * p * np.pi * y / a)) \
        / (1 - np.exp(-2 * p * np.pi * b / a))
    return float(np.sum(4.0 / (p * np.pi) * np.sin(p * np.pi * x / a) * ratio))
