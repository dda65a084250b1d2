"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and lays out arrays: it holds none of the
method's arithmetic (no descriptors, no electrostatics).  Both the FP64 oracle and
the HIP path receive exactly the arrays produced here; positions are rounded to
float32 first so that both sides see bit-identical coordinates.

The paper's training sets are not available, so these boxes stand in for its
workloads (Sec. 3: liquid water, Li7La3Zr2O12, BaTiO3-like perovskite) at their
shapes and densities.  Seeds: ``2601190340 + workload id``, numpy PCG64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 2601190340


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# hyper-parameters (plain records; both sides read them field by field)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class HParams:
    n_types: int
    n_max_R: int = 4          # radial functions n = 0..n_max_R
    n_max_A: int = 4          # angular functions n = 0..n_max_A
    basis_R: int = 8          # Chebyshev terms k = 0..basis_R
    basis_A: int = 8
    l_max: int = 4            # angular orders l = 1..l_max (three-body)
    n_neu: int = 30           # hidden units
    rc_R: float = 6.0
    rc_A: float = 4.0

    @property
    def n_des(self) -> int:
        return (self.n_max_R + 1) + (self.n_max_A + 1) * self.l_max

    def n_theta(self) -> int:
        """Length of the flat parameter vector (count only; the layout is
        interpreted independently by each implementation)."""
        T = self.n_types
        c_r = T * T * (self.n_max_R + 1) * (self.basis_R + 1)
        c_a = T * T * (self.n_max_A + 1) * (self.basis_A + 1)
        per_species = self.n_neu * self.n_des + 3 * self.n_neu + 1
        return c_r + c_a + T * per_species + 2


@dataclasses.dataclass
class ESParams:
    mode: int = 1             # 1: real + reciprocal + self; 2: reciprocal only
    method: int = 0           # 0: Ewald, 1: PPPM
    alpha: float = 0.3        # 1/Angstrom
    rc_coul: float = 9.0      # Angstrom
    kmax: float = 2.0 * math.pi * 0.3
    kmax_inclusive: int = 0
    mesh: tuple = (0, 0, 0)
    order: int = 5
    q_total: float = 0.0
    efield: tuple = (0.0, 0.0, 0.0)  # external electric field, V/Angstrom


@dataclasses.dataclass
class System:
    name: str
    pos: np.ndarray           # (N, 3) float64 holding float32-representable values
    types: np.ndarray         # (N,) int32
    cell: np.ndarray          # (3, 3) float64, rows are the cell vectors a, b, c

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def pos_f32_soa(self) -> np.ndarray:
        return np.ascontiguousarray(self.pos.T.astype(np.float32))


def _finish(name, pos, types, cell) -> System:
    cell = np.asarray(cell, dtype=np.float64)
    # wrap into the cell (fractional coordinates in [0, 1)) and round to float32
    frac = pos @ np.linalg.inv(cell)
    frac -= np.floor(frac)
    pos = frac @ cell
    pos = pos.astype(np.float32).astype(np.float64)
    return System(name, np.ascontiguousarray(pos), np.ascontiguousarray(types, dtype=np.int32), cell)


def _random_rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _grid(n_side, spacing):
    idx = np.arange(n_side)
    g = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3)
    return (g + 0.5) * spacing


def water_box(n_side: int, spacing: float = 3.105, sigma: float = 0.1, seed: int = SEED_BASE,
              n_mol: Optional[int] = None, name: str = "water") -> System:
    """O on a jittered simple-cubic grid, H at 0.96 A and 104.5 deg under a random
    rotation.  Species: O = 0, H = 1.  Atom order: O, H, H per molecule."""
    rng = rng_for(seed)
    L = n_side * spacing
    sites = _grid(n_side, spacing)
    if n_mol is not None and n_mol < sites.shape[0]:
        sites = sites[rng.permutation(sites.shape[0])[:n_mol]]
    n = sites.shape[0]
    O = sites + rng.normal(0.0, sigma, sites.shape)
    R = _random_rotations(rng, n)
    half = math.radians(104.5) / 2.0
    h1 = 0.96 * np.array([math.sin(half), 0.0, math.cos(half)])
    h2 = 0.96 * np.array([-math.sin(half), 0.0, math.cos(half)])
    H1 = O + R @ h1
    H2 = O + R @ h2
    pos = np.stack([O, H1, H2], axis=1).reshape(-1, 3)
    types = np.tile(np.array([0, 1, 1], dtype=np.int32), n)
    return _finish(name, pos, types, np.eye(3) * L)


def perovskite_box(n_cells, a: float = 4.0, sigma: float = 0.08, seed: int = SEED_BASE,
                   name: str = "perovskite") -> System:
    """ABO3: A at (0,0,0), B at (1/2,1/2,1/2), O at the three face centres.
    Species: A = 0, B = 1, O = 2.  ``n_cells`` is an int or a 3-tuple."""
    rng = rng_for(seed)
    nc = (n_cells,) * 3 if np.isscalar(n_cells) else tuple(n_cells)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0.5], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    btype = np.array([0, 1, 2, 2, 2], dtype=np.int32)
    ii, jj, kk = np.meshgrid(np.arange(nc[0]), np.arange(nc[1]), np.arange(nc[2]), indexing="ij")
    origins = np.stack([ii, jj, kk], -1).reshape(-1, 1, 3).astype(np.float64)
    pos = ((origins + basis[None]) * a).reshape(-1, 3)
    pos = pos + rng.normal(0.0, sigma, pos.shape)
    types = np.tile(btype, origins.shape[0])
    return _finish(name, pos, types, np.diag(np.array(nc, dtype=np.float64) * a))


GARNET_DENSITY = 0.08778  # atoms / A^3 for Li7La3Zr2O12 at 5.1 g/cm^3


def garnet_box(n_atoms: int, sigma: float = 0.15, seed: int = SEED_BASE, name: str = "garnet") -> System:
    """Li:La:Zr:O = 7:3:2:12 on the first ``n_atoms`` sites of a shuffled simple-cubic
    grid at 5.1 g/cm^3.  Species: Li = 0, La = 1, Zr = 2, O = 3."""
    assert n_atoms % 24 == 0
    rng = rng_for(seed)
    L = (n_atoms / GARNET_DENSITY) ** (1.0 / 3.0)
    n_side = int(math.ceil(n_atoms ** (1.0 / 3.0) - 1e-9))
    h = L / n_side
    sites = _grid(n_side, h)
    sites = sites[rng.permutation(sites.shape[0])[:n_atoms]]
    pos = sites + rng.normal(0.0, sigma, sites.shape)
    fu = n_atoms // 24
    types = np.concatenate([np.full(7 * fu, 0), np.full(3 * fu, 1), np.full(2 * fu, 2), np.full(12 * fu, 3)])
    types = types[rng.permutation(n_atoms)].astype(np.int32)
    return _finish(name, pos, types, np.eye(3) * L)


def rocksalt(n_cells: int, a0: float = 5.64, jitter: float = 0.0, seed: int = SEED_BASE) -> System:
    """NaCl structure (conventional cubic cell, 8 ions), species Na = 0, Cl = 1."""
    rng = rng_for(seed)
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    cl = base + np.array([0.5, 0, 0])
    basis = np.concatenate([base, cl])
    btype = np.array([0] * 4 + [1] * 4, dtype=np.int32)
    idx = np.arange(n_cells)
    o = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 1, 3)
    pos = ((o + basis[None]) * a0).reshape(-1, 3)
    if jitter:
        pos = pos + rng.normal(0, jitter, pos.shape)
    return _finish("rocksalt", pos, np.tile(btype, o.shape[0]), np.eye(3) * a0 * n_cells)


def theta0(hp: HParams, seed: int, sigma: float = 0.1, s_value: float = 1.5) -> np.ndarray:
    """Random-init parameters ~N(0, sigma^2); the last entry (sqrt(eps_inf)) is fixed."""
    rng = rng_for(seed)
    th = rng.normal(0.0, sigma, hp.n_theta())
    th[-1] = s_value
    return th.astype(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
WATER_HP = HParams(n_types=2, n_max_R=4, n_max_A=4, basis_R=8, basis_A=8, l_max=4, n_neu=30)
GARNET_HP = HParams(n_types=4, n_max_R=8, n_max_A=6, basis_R=8, basis_A=8, l_max=4, n_neu=50)
PEROV_HP = HParams(n_types=3, n_max_R=8, n_max_A=6, basis_R=8, basis_A=8, l_max=4, n_neu=40)


@dataclasses.dataclass
class Workload:
    wid: int
    name: str
    system: System
    hp: HParams
    es: ESParams
    theta: np.ndarray


def workload(wid: int, variant: str = "full") -> Workload:
    """Workloads 0..3 (the batched set is built by ``batch_structures``).

    variant "full" is the stated size, "crop" the same generator at the small size
    used for element-wise parity (still periodic)."""
    seed = SEED_BASE + wid
    if wid == 0:
        sysm = water_box(4, seed=seed, name="water-64")
        L = sysm.cell[0, 0]
        es = ESParams(mode=1, method=0, alpha=0.3, rc_coul=9.0, kmax=2 * math.pi * 6 / L, kmax_inclusive=1)
        return Workload(0, "water-192", sysm, WATER_HP, es, theta0(WATER_HP, seed))
    if wid == 1:
        n = 20 if variant == "full" else 10
        sysm = water_box(n, seed=seed, name=f"water-{n**3}")
        mesh = (64,) * 3 if variant == "full" else (32,) * 3
        es = ESParams(mode=1, method=1, alpha=0.3, rc_coul=9.0, kmax=2 * math.pi * 0.3, mesh=mesh, order=5)
        return Workload(1, f"water-{3 * n**3}", sysm, WATER_HP, es, theta0(WATER_HP, seed))
    if wid == 2:
        n = 153600 if variant == "full" else 768
        sysm = garnet_box(n, seed=seed, name=f"garnet-{n}")
        mesh = (128,) * 3 if variant == "full" else (24,) * 3
        es = ESParams(mode=1, method=1, alpha=0.3, rc_coul=9.0, kmax=2 * math.pi * 0.3, mesh=mesh, order=5)
        return Workload(2, f"garnet-{n}", sysm, GARNET_HP, es, theta0(GARNET_HP, seed))
    if wid == 3:
        n = 58 if variant == "full" else 10
        sysm = perovskite_box(n, seed=seed, name=f"perovskite-{5 * n**3}")
        mesh = (256,) * 3 if variant == "full" else (45,) * 3
        es = ESParams(mode=1, method=1, alpha=0.3, rc_coul=9.0, kmax=2 * math.pi * 0.3, mesh=mesh, order=5)
        return Workload(3, f"perovskite-{5 * n**3}", sysm, PEROV_HP, es, theta0(PEROV_HP, seed))
    raise ValueError(f"unknown workload {wid}")


def batch_structures(n_struct: int = 512, seed: int = SEED_BASE + 4, n_min: int = 24,
                     n_max: int = 768) -> List[System]:
    """Uneven periodic structures, sizes log-uniform in [n_min, n_max]; first half
    water-like (species O = 0, H = 1), second half perovskite-like (A = 2, B = 3,
    O = 0 so that oxygen shares one species across both families)."""
    rng = rng_for(seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_struct))
    out = []
    for s in range(n_struct):
        sub = int(rng.integers(0, 2**31 - 1))
        if s < n_struct // 2:
            nm = max(1, int(round(sizes[s] / 3)))
            side = int(math.ceil(nm ** (1.0 / 3.0) - 1e-9))
            L = (nm * 3 / 0.1002) ** (1.0 / 3.0)
            sysm = water_box(side, spacing=L / side, seed=sub, n_mol=nm, name=f"bw{s}")
        else:
            nc = max(1, int(round(sizes[s] / 5)))
            dims = _most_cubic(nc)
            sysm = perovskite_box(dims, seed=sub, name=f"bp{s}")
            remap = np.array([2, 3, 0], dtype=np.int32)
            sysm = System(sysm.name, sysm.pos, remap[sysm.types], sysm.cell)
        out.append(sysm)
    return out


def _most_cubic(n):
    best = None
    for a in range(1, n + 1):
        if n % a:
            continue
        for b in range(a, n // a + 1):
            if (n // a) % b:
                continue
            c = n // a // b
            if c < b:
                continue
            score = c / a
            if best is None or score < best[0]:
                best = (score, (a, b, c))
    return best[1]


# one four-species model (O, H, A, B) with the hyper-parameters of the water workload
BATCH_HP = HParams(n_types=4, n_max_R=4, n_max_A=4, basis_R=8, basis_A=8, l_max=4, n_neu=30)


@dataclasses.dataclass
class BatchWorkload:
    systems: List[System]
    hp: HParams
    es: ESParams
    theta0: np.ndarray
    thetas: np.ndarray  # [C, n_theta] candidates theta0 + N(0, sigma_c^2)


def batch_workload(n_struct: int = 512, n_cand: int = 64, sigma_c: float = 0.05) -> BatchWorkload:
    """Uneven structures under a population of candidate parameter vectors: Ewald with
    alpha = 0.3, rc = 9 A and kmax = 2 pi alpha; candidates perturb every component
    of theta0 (including s) by N(0, sigma_c^2)."""
    seed = SEED_BASE + 4
    systems = batch_structures(n_struct, seed=seed)
    th0 = theta0(BATCH_HP, seed)
    rng = rng_for(seed + 1000)
    thetas = th0[None, :] + rng.normal(0.0, sigma_c, (n_cand, th0.size))
    thetas = thetas.astype(np.float32).astype(np.float64)
    es = ESParams(mode=1, method=0, alpha=0.3, rc_coul=9.0, kmax=2 * math.pi * 0.3, kmax_inclusive=0)
    return BatchWorkload(systems, BATCH_HP, es, th0, thetas)
