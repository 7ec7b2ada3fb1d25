"""Closed forms the tests hold estimates against (no oracle code)."""
import math

import numpy as np
import scipy.stats


def geometric_asian_closed_form(S0, K, r, sig, T, d):
    """Price, delta, vega, gamma of the discretely monitored geometric Asian
    call (dates jT/d, j = 1..d): ln G is normal with mean
    ln S0 + (r - sig^2/2) mean(t_j) and variance sig^2 (1/d^2) sum min(t_j, t_k)."""
    dt = T / d
    tbar = dt * (d + 1) / 2
    v = sig * math.sqrt(dt * (d + 1) * (2 * d + 1) / (6 * d))
    mu = math.log(S0) + (r - sig**2 / 2) * tbar
    D = math.exp(-r * T)
    F = math.exp(mu + v * v / 2)
    d2 = (mu - math.log(K)) / v
    d1 = d2 + v
    N, n = scipy.stats.norm.cdf, scipy.stats.norm.pdf
    price = D * (F * N(d1) - K * N(d2))
    delta = D * F * N(d1) / S0
    gamma = D * F * n(d1) / (S0 * S0 * v)
    mu_s, v_s = -sig * tbar, v / sig
    vega = D * (F * (mu_s + v * v_s) * N(d1) + K * n(d2) * v_s)
    return np.array([price, delta, vega, gamma])
