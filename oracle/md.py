"""Velocity-Verlet molecular dynamics on the FP64 oracle's forces, with the polarization
current P_dot_a = sum_i sum_b Z_i[a][b] v_i[b] (Sec. 2.4 Eq. 30).

TEST INFRASTRUCTURE ONLY (see the package docstring of ``oracle``).

One step: v += dt/2 F/m; r += dt v; F, Z = forces and Born charges at r; v += dt/2 F/m.
Units: Angstrom, fs, amu, eV; the conversions come from the SI values of the
elementary charge and the atomic mass unit.
"""
from __future__ import annotations

import numpy as np

E_CHARGE = 1.602176634e-19   # C (exact)
AMU = 1.66053906660e-27      # kg (CODATA 2018)
ACC = E_CHARGE / AMU * 1e-10  # (eV / Angstrom) / amu in Angstrom / fs^2
EKIN = AMU / E_CHARGE * 1e10  # amu Angstrom^2 / fs^2 in eV


def run(compute, masses, pos, vel, dt, n_steps):
    """compute(pos) -> (E, F (N,3), Z (N,3,3), P (3,)).  masses (N,) amu, pos and vel (N,3).
    Returns (pos, vel, series[n_steps + 1][8]: E_pot, E_kin, P_dot (3), P (3))."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    series = np.zeros((n_steps + 1, 8))

    def record(k, E, Z, P):
        series[k, 0] = E
        series[k, 1] = 0.5 * EKIN * (m[:, 0] * (vel ** 2).sum(1)).sum()
        series[k, 2:5] = np.einsum("iab,ib->a", Z, vel)
        series[k, 5:8] = P

    E, F, Z, P = compute(pos)
    record(0, E, Z, P)
    for k in range(1, n_steps + 1):
        vel += 0.5 * dt * ACC * F / m
        pos += dt * vel
        E, F, Z, P = compute(pos)
        vel += 0.5 * dt * ACC * F / m
        record(k, E, Z, P)
    return pos, vel, series
