"""One generation of the separable natural evolution strategy (SNES) the paper trains
with (Sec. 2.5, citing Schaul, Glasmachers and Schmidhuber 2011), written out in
NumPy float64 from that published algorithm.

TEST INFRASTRUCTURE ONLY (see the package docstring of ``oracle``).

Given the search distribution N(mu, diag(sigma^2)), the population
z_k = mu + sigma * s_k (s_k the standard-normal draws, passed in) and the loss of
every member (lower is better):
  * rank the members by loss (rank 1 = lowest loss, ties by member index);
  * rank-based utilities u_r = max(0, ln(lambda/2 + 1) - ln r) / sum_j max(0,
    ln(lambda/2 + 1) - ln j) - 1/lambda, r = 1..lambda, given to the member of rank r;
  * natural gradients  g_mu = sum_k u_k s_k,  g_sigma = sum_k u_k (s_k^2 - 1);
  * updates  mu <- mu + eta_mu sigma g_mu,  sigma <- sigma exp(eta_sigma g_sigma / 2),
    with the published defaults eta_mu = 1 and eta_sigma = (3 + ln d) / (5 sqrt d).
"""
from __future__ import annotations

import math

import numpy as np


def default_eta_sigma(d: int) -> float:
    return (3.0 + math.log(d)) / (5.0 * math.sqrt(d))


def utilities(lam: int) -> np.ndarray:
    """u[r - 1] for ranks r = 1..lambda (sums to zero)."""
    r = np.arange(1, lam + 1, dtype=np.float64)
    raw = np.maximum(0.0, math.log(lam / 2.0 + 1.0) - np.log(r))
    return raw / raw.sum() - 1.0 / lam


def ranks(loss) -> np.ndarray:
    """0-based rank of every member: the number of members with a lower loss, or an
    equal loss and a lower index."""
    loss = np.asarray(loss, dtype=np.float64)
    lam = loss.shape[0]
    out = np.zeros(lam, dtype=np.int64)
    for k in range(lam):
        for j in range(lam):
            if loss[j] < loss[k] or (loss[j] == loss[k] and j < k):
                out[k] += 1
    return out


def population(mu, sigma, noise) -> np.ndarray:
    """z_k = mu + sigma * s_k for every row s_k of noise [lambda][d]."""
    return np.asarray(mu, dtype=np.float64)[None, :] + np.asarray(sigma, dtype=np.float64)[None, :] * np.asarray(
        noise, dtype=np.float64)


def update(mu, sigma, noise, loss, eta_mu: float = 1.0, eta_sigma: float | None = None):
    """(mu', sigma') after one generation."""
    mu = np.asarray(mu, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    s = np.asarray(noise, dtype=np.float64)
    lam, d = s.shape
    if eta_sigma is None:
        eta_sigma = default_eta_sigma(d)
    u = utilities(lam)[ranks(loss)]  # utility of each member
    g_mu = (u[:, None] * s).sum(0)
    g_sigma = (u[:, None] * (s * s - 1.0)).sum(0)
    return mu + eta_mu * sigma * g_mu, sigma * np.exp(0.5 * eta_sigma * g_sigma)
