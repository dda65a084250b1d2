"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by
element, on seeded workloads that span several tiles and ragged tails.

Tolerances for the FP32 path (target: forces within 1e-4 eV/A of the
FP64 oracle); the other bounds follow from FP32 rounding of per-atom terms summed
in FP64:
  energy        |dE| / N        <= 2e-6 eV/atom
  forces        max |dF|        <= 1e-4 eV/A
  virial        max |dW| / N    <= 2e-5 eV
  charges       max |dq|        <= 2e-6 e
  Born charges  max |dZ|        <= 1e-4 e
  polarization  max |dP|        <= 8 sqrt(N) eps max|q~'| max|r| e A, eps = 2^-24
The polarization bound is FP32 rounding of its N terms q~'_i r_i (FP64 sum): each
charge carries a relative error of a few units of eps32 = 2^-24 and the errors of
different atoms are independent, so their sum grows like sqrt(N).
"""
import copy
import math
import sys

import numpy as np
import pytest

from paper_2601_19034_amd import inputs

pytestmark = pytest.mark.gpu

# p: the relative rounding unit of one charge (FP32 here) in the polarization bound
TOL = dict(e=2e-6, f=1e-4, w=2e-5, q=2e-6, z=1e-4, p=2.0 ** -24)


def p_bound(n, q_naked, r_max, eps):
    """8 sqrt(N) eps max|q~'| max|r| (see the module docstring)."""
    return 8.0 * math.sqrt(max(n, 1)) * eps * max(np.abs(q_naked).max(initial=0.0), 1e-3) * max(r_max, 1.0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def run_gpu(hp, es, sysm, theta, precision="fp32", per_atom_virial=False):
    from paper_2601_19034_amd.api import ALL_OUTPUTS, DEFAULT_OUTPUTS, QNEP, to_device_inputs

    model = QNEP(hp, precision)
    pos, types, th = to_device_inputs(sysm, theta)
    out = model.compute(pos, types, sysm.cell, th, es, outputs=ALL_OUTPUTS if per_atom_virial else DEFAULT_OUTPUTS)
    flags = model.check_status()
    assert flags == 0, f"device status flags {flags}"
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    g["pos_used"] = np.asarray(sysm.pos, dtype=np.float64)
    return g


def compare(g, r, n, tol=TOL, label=""):
    dE = abs(g["energy"][0] - r.energy) / max(n, 1)
    F = g["forces"].T
    dF = np.abs(F - r.forces).max()
    dW = np.abs(g["virial"].reshape(3, 3) - r.virial).max() / max(n, 1)
    dq = np.abs(g["charges"] - r.q_screened).max()
    dqt = np.abs(g["charges_naked"] - r.q_naked).max()
    Z = g["bec"].T.reshape(n, 3, 3)
    dZ = np.abs(Z - r.bec).max()
    pbound = p_bound(n, r.q_naked, np.abs(g["pos_used"]).max(initial=0.0), tol["p"])
    dP = np.abs(g["polarization"] - r.pol).max()
    _say(f"[{label}] dE/N={dE:.2e} dF={dF:.2e} dW/N={dW:.2e} dq={dq:.2e} dq~={dqt:.2e} dZ={dZ:.2e} dP={dP:.2e} "
         f"(P bound {pbound:.2e}) |F|max={np.abs(r.forces).max():.3f}")
    assert dE <= tol["e"], dE
    assert dF <= tol["f"], dF
    assert dW <= tol["w"], dW
    assert dq <= tol["q"] and dqt <= tol["q"] * 2, (dq, dqt)
    assert dZ <= tol["z"], dZ
    assert dP <= pbound, (dP, pbound)
    t = g["energy_terms"]
    assert abs(t[0] - r.terms[1]) / n <= tol["e"]        # U_NEP
    assert abs(t[2] - r.terms[3]) / n <= tol["e"]        # U_k
    assert abs(t[5] - r.terms[6]) <= 50 * tol["q"] * n ** 0.5  # sum of raw charges


def _oracle(orc, hp, es, sysm, theta):
    return orc.compute(hp, es, sysm.pos, sysm.types, sysm.cell, theta, cells=sysm.n > 1000)


def test_water192_ewald(torch_dev, orc):
    w = inputs.workload(0)
    _say("case water-192 Ewald mode 1")
    g = run_gpu(w.hp, w.es, w.system, w.theta)
    r = _oracle(orc, w.hp, w.es, w.system, w.theta)
    compare(g, r, w.system.n, label="water192-ewald")
    assert g["energy_terms"][7] == r.terms[9]  # same wave-vector set (924)


def test_water192_ewald_many_wave_vectors(torch_dev, orc):
    """A large k-set (|n| up to 32 along every axis): more n2 per row than one
    structure-factor block holds (two blocks of 32) and more (channel, n2) outputs
    than one pass of the per-atom product holds (17 tiles, two passes).  A wide alpha
    keeps the high-k terms above FP32 underflow."""
    w = inputs.workload(0)
    es = copy.copy(w.es)
    es.alpha, es.kmax = 1.5, 2 * math.pi * 2.5
    _say("case water-192 Ewald alpha 1.5, kmax 2 pi 2.5")
    g = run_gpu(w.hp, es, w.system, w.theta)
    r = _oracle(orc, w.hp, es, w.system, w.theta)
    compare(g, r, w.system.n, label="water192-ewald-bigk")
    assert g["energy_terms"][7] == r.terms[9]
    assert r.terms[9] > 60000


def test_water192_mode2_and_charge(torch_dev, orc):
    w = inputs.workload(0)
    for mode, Q in ((2, 0.0), (1, 0.7), (2, -1.1)):
        es = copy.copy(w.es)
        es.mode, es.q_total = mode, Q
        _say(f"case water-192 Ewald mode {mode} Q={Q}")
        g = run_gpu(w.hp, es, w.system, w.theta)
        r = _oracle(orc, w.hp, es, w.system, w.theta)
        compare(g, r, w.system.n, label=f"water192-m{mode}-Q{Q}")
        assert abs(r.q_naked.sum() - Q) < 1e-10


def test_water192_pppm(torch_dev, orc):
    w = inputs.workload(0)
    es = copy.copy(w.es)
    es.method, es.mesh, es.order = 1, (16, 15, 18), 5
    _say("case water-192 PPPM 16x15x18")
    g = run_gpu(w.hp, es, w.system, w.theta)
    r = _oracle(orc, w.hp, es, w.system, w.theta)
    compare(g, r, w.system.n, label="water192-pppm")


@pytest.mark.parametrize("mesh", [(256, 12, 256), (24, 20, 256), (24, 20, 20), (20, 15, 256)])
def test_water192_pppm_transform_forms(torch_dev, orc, mesh):
    """The mesh shapes select the transform: 256 points along c and an even count along
    b take the real-input forward transform and the half spectrum, with 256 points along
    a also the influence function fused with the inverse pass along a ((256, 12, 256));
    (24, 20, 256) the half spectrum without the fusion; (24, 20, 20) and (20, 15, 256)
    (odd along b) the complex transform of (rho, 0)."""
    w = inputs.workload(0)
    es = copy.copy(w.es)
    es.method, es.mesh, es.order = 1, mesh, 5
    _say(f"case water-192 PPPM {mesh}")
    g = run_gpu(w.hp, es, w.system, w.theta)
    r = _oracle(orc, w.hp, es, w.system, w.theta)
    compare(g, r, w.system.n, label=f"water192-pppm-{mesh[0]}x{mesh[1]}x{mesh[2]}")


def test_water3000_pppm_and_ewald(torch_dev, orc):
    w = inputs.workload(1, "crop")
    _say("case water-3000 PPPM 32^3")
    g = run_gpu(w.hp, w.es, w.system, w.theta)
    r = _oracle(orc, w.hp, w.es, w.system, w.theta)
    compare(g, r, w.system.n, label="water3000-pppm")
    es = copy.copy(w.es)
    es.method = 0
    _say("case water-3000 Ewald kmax=2 pi alpha")
    g = run_gpu(w.hp, es, w.system, w.theta)
    r = _oracle(orc, w.hp, es, w.system, w.theta)
    compare(g, r, w.system.n, label="water3000-ewald")


def test_perovskite5000_pppm(torch_dev, orc):
    w = inputs.workload(3, "crop")
    _say("case perovskite-5000 PPPM 45^3")
    g = run_gpu(w.hp, w.es, w.system, w.theta)
    r = _oracle(orc, w.hp, w.es, w.system, w.theta)
    compare(g, r, w.system.n, label="perovskite5000-pppm")


def test_garnet768_pppm(torch_dev, orc):
    w = inputs.workload(2, "crop")
    _say("case garnet-768 PPPM 24^3")
    g = run_gpu(w.hp, w.es, w.system, w.theta)
    r = _oracle(orc, w.hp, w.es, w.system, w.theta)
    compare(g, r, w.system.n, label="garnet768-pppm")


def test_small_ragged_and_triclinic(torch_dev, orc):
    hp = inputs.WATER_HP
    th = inputs.theta0(hp, 17)
    # 37 molecules (111 atoms) in a 10.3 A box: several images of every neighbour
    s = inputs.water_box(4, spacing=10.3 / 4, seed=21, n_mol=37)
    es = inputs.ESParams(mode=1, method=0, alpha=0.35, rc_coul=9.0, kmax=2.2)
    _say("case water-111 small box")
    compare(run_gpu(hp, es, s, th), _oracle(orc, hp, es, s, th), s.n, label="water111")
    # sheared (triclinic) cell, positions re-wrapped
    cell = s.cell.copy()
    cell[1, 0] = 1.7
    cell[2, 0] = -0.9
    cell[2, 1] = 1.1
    t = inputs._finish("tri", s.pos, s.types, cell)
    _say("case water-111 triclinic")
    compare(run_gpu(hp, es, t, th), _oracle(orc, hp, es, t, th), t.n, label="water111-tri")
    es_p = inputs.ESParams(mode=1, method=1, alpha=0.35, rc_coul=9.0, mesh=(12, 12, 12))
    _say("case water-111 triclinic PPPM")
    compare(run_gpu(hp, es_p, t, th), _oracle(orc, hp, es_p, t, th), t.n, label="water111-tri-pppm")


def test_positions_outside_the_cell(torch_dev, orc):
    w = inputs.workload(0)
    s = copy.deepcopy(w.system)
    shift = np.zeros_like(s.pos)
    shift[::3] = s.cell[0] * 2 - s.cell[2]
    s2 = inputs.System("shifted", (s.pos + shift).astype(np.float32).astype(np.float64), s.types, s.cell)
    _say("case water-192 shifted images")
    g = run_gpu(w.hp, w.es, s2, w.theta)
    r = _oracle(orc, w.hp, w.es, s2, w.theta)
    compare(g, r, s.n, tol=dict(TOL, f=2e-4, z=2e-4), label="water192-shifted")


def test_empty_and_single_atom(torch_dev, orc):
    hp = inputs.WATER_HP
    th = inputs.theta0(hp, 3)
    es = inputs.ESParams(mode=1, method=0, alpha=0.3, rc_coul=9.0, kmax=1.9)
    empty = inputs.System("empty", np.zeros((0, 3)), np.zeros(0, dtype=np.int32), np.eye(3) * 10)
    _say("case empty")
    g = run_gpu(hp, es, empty, th)
    assert g["energy"][0] == 0.0 and np.all(g["virial"] == 0) and np.all(g["polarization"] == 0)
    one = inputs.System("one", np.array([[1.0, 2.0, 3.0]]), np.array([1], dtype=np.int32), np.eye(3) * 7.0)
    _say("case single atom")
    compare(run_gpu(hp, es, one, th), _oracle(orc, hp, es, one, th), 1, label="single")


def test_bad_species_flag(torch_dev):
    """A species index outside [0, T) raises QNEP_FLAG_BAD_SPECIES (the kernels clamp it
    internally, so nothing is read out of bounds)."""
    from paper_2601_19034_amd import binding as B
    from paper_2601_19034_amd.api import QNEP, to_device_inputs

    w = inputs.workload(0)
    s = copy.deepcopy(w.system)
    s.types = s.types.copy()
    s.types[5] = 2  # the water model has two species
    model = QNEP(w.hp)
    pos, types, th = to_device_inputs(s, w.theta)
    _say("case bad species")
    model.compute(pos, types, s.cell, th, w.es)
    assert model.check_status() == B.FLAG_BAD_SPECIES
    pos, types, th = to_device_inputs(w.system, w.theta)
    model.compute(pos, types, w.system.cell, th, w.es)
    assert model.check_status() == 0  # the flag is cleared by the next call


def test_water24000_full(torch_dev, orc):
    w = inputs.workload(1)
    _say("case water-24000 PPPM 64^3 (full size)")
    g = run_gpu(w.hp, w.es, w.system, w.theta)
    r = _oracle(orc, w.hp, w.es, w.system, w.theta)
    compare(g, r, w.system.n, label="water24000-pppm")


# BF16 network on the matrix cores (FP32 accumulation), both forms held to the
# target force bound of 5 meV/A.  The forward product splits both operands in
# both forms, so the energy and the charges keep about 16 mantissa bits (p: that
# rounding unit in the polarization bound).
TOL_BF16X3 = dict(e=2e-4, f=5e-3, w=5e-4, q=5e-4, z=5e-3, p=2.0 ** -16)
TOL_BF16 = dict(TOL_BF16X3)


@pytest.mark.parametrize("wid,variant", [(0, "full"), (3, "crop"), (2, "crop")])
@pytest.mark.parametrize("precision", ["bf16x3", "bf16"])
def test_bf16_mlp(torch_dev, orc, wid, variant, precision):
    w = inputs.workload(wid, variant)
    _say(f"case {precision} {w.name}")
    g = run_gpu(w.hp, w.es, w.system, w.theta, precision=precision)
    r = _oracle(orc, w.hp, w.es, w.system, w.theta)
    compare(g, r, w.system.n, tol=TOL_BF16X3 if precision == "bf16x3" else TOL_BF16,
            label=f"{precision}-{w.name}")


# ------------------------------------------------------------------ external field (Eq. 29)
@pytest.mark.parametrize("wid,variant", [(0, "full"), (2, "crop")])
def test_external_field_force(torch_dev, orc, wid, variant):
    """F with a uniform field E against the oracle (same bounds), and the field term
    itself equal to sum_a E_a Z_i[a][:] with the GPU's own Born charges."""
    w = inputs.workload(wid, variant)
    es = copy.copy(w.es)
    es.efield = (0.05, -0.02, 0.035)
    _say(f"case external field {w.name}")
    g0 = run_gpu(w.hp, w.es, w.system, w.theta)
    g = run_gpu(w.hp, es, w.system, w.theta)
    r = _oracle(orc, w.hp, es, w.system, w.theta)
    compare(g, r, w.system.n, label=f"field-{w.name}")
    Z = g["bec"].T.reshape(-1, 3, 3)
    want = np.einsum("a,iab->ib", np.array(es.efield), Z)
    err = np.abs((g["forces"] - g0["forces"]).T - want).max()
    _say(f"[field-{w.name}] F(E) - F(0) vs Z^T E: {err:.2e} (max field force {np.abs(want).max():.3f})")
    assert err <= 2e-6
    assert g["energy"][0] == g0["energy"][0] and np.array_equal(g["virial"], g0["virial"])


# ------------------------------------------------------------------ per-atom virial (Eqs. 12, 20, 39)
@pytest.mark.parametrize("case", ["water192-ewald", "water192-pppm-Q", "garnet768-pppm", "water111-tri"])
def test_per_atom_virial(torch_dev, orc, case):
    """W_i against the oracle's per-atom virial (every partial force, the reciprocal
    per-atom forms and the background share) and sum_i W_i against the total W."""
    if case.startswith("water111"):
        hp, th = inputs.WATER_HP, inputs.theta0(inputs.WATER_HP, 17)
        s = inputs.water_box(4, spacing=10.3 / 4, seed=21, n_mol=37)
        cell = s.cell.copy()
        cell[1, 0], cell[2, 0], cell[2, 1] = 1.7, -0.9, 1.1
        sysm = inputs._finish("tri", s.pos, s.types, cell)
        es = inputs.ESParams(mode=1, method=0, alpha=0.35, rc_coul=9.0, kmax=2.2)
    else:
        w = inputs.workload(0 if case.startswith("water") else 2, "full" if case.startswith("water") else "crop")
        hp, th, sysm, es = w.hp, w.theta, w.system, copy.copy(w.es)
        if case == "water192-pppm-Q":
            es.method, es.mesh, es.q_total = 1, (16, 15, 18), 0.7
    _say(f"case per-atom virial {case}")
    g = run_gpu(hp, es, sysm, th, per_atom_virial=True)
    r = orc.compute(hp, es, sysm.pos, sysm.types, sysm.cell, th, cells=sysm.n > 1000, per_atom_virial=True)
    Va = g["virial_atom"].T.reshape(-1, 3, 3)
    scale = np.abs(r.vatom).max()
    err = np.abs(Va - r.vatom).max()
    dsum = np.abs(Va.sum(0) - g["virial"].reshape(3, 3)).max()
    _say(f"[vatom-{case}] max|dW_i|={err:.2e} (max|W_i| {scale:.2f}) |sum W_i - W|={dsum:.2e}")
    # FP32 partial forces times displacements of a few Angstrom, summed over ~300 pairs
    assert err <= 2e-5 * scale + 1e-5
    assert dsum <= 1e-5 * np.abs(g["virial"]).max() + 1e-4
    # the default outputs are unchanged by the extra work
    g0 = run_gpu(hp, es, sysm, th)
    for k in ("forces", "virial", "bec", "energy"):
        assert np.array_equal(g0[k], g[k]), k


@pytest.mark.parametrize("mesh", [(3, 3, 3), (4, 2, 256)])
def test_spread_atomic_fallback(torch_dev, orc, mesh):
    """A mesh so coarse against the bins that a brick's bin rows or segments would not
    fit the per-work-group tables: the charge assignment takes the atomic path (float
    atomics into a real mesh).  Garnet-768 (20.6 A, bins of 3.4 x 3.4 x 1.6 A) with a
    3^3 mesh: 16 x 16 rows and 32 bins along c per brick, 1024 segments > 512; with
    (4, 2, 256): 14 x 20 = 280 rows > 256.  The 3^3 mesh takes the complex transform of
    (rho, 0); (4, 2, 256) the real-input transform, the atomic spread writing its
    interleaved line pairs."""
    w = inputs.workload(2, "crop")
    es = copy.copy(w.es)
    es.mesh = mesh
    nc = [int(np.floor(w.system.cell[a, a] / (3.0 if a < 2 else 1.5))) for a in range(3)]
    P = [min(16, m) for m in mesh]
    cnt = [int(np.floor((P[a] + 4.02) * nc[a] / mesh[a])) + 2 for a in range(3)]
    rows = cnt[0] * cnt[1]
    assert rows > 256 or rows * ((cnt[2] - 1) // nc[2] + 2) > 512  # the brick tables do not fit
    _say(f"case garnet-768 PPPM {mesh} (atomic charge assignment)")
    g = run_gpu(w.hp, es, w.system, w.theta)
    r = _oracle(orc, w.hp, es, w.system, w.theta)
    compare(g, r, w.system.n, label=f"garnet768-pppm{mesh[0]}x{mesh[1]}x{mesh[2]}-atomic")


# ------------------------------------------------------------------ isolated systems (Eqs. 26, 27)
def _droplet(n_side, radius, box, seed):
    """Water molecules whose oxygen lies within `radius` of the centre of a water box,
    moved to the centre of an empty cubic box of edge `box` (an isolated cluster)."""
    w = inputs.water_box(n_side, seed=seed)
    c = w.cell.diagonal() / 2
    keep = []
    for m in range(w.n // 3):
        if np.linalg.norm(w.pos[3 * m] - c) < radius:
            keep += [3 * m, 3 * m + 1, 3 * m + 2]
    pos = w.pos[keep] - c + box / 2
    return inputs.System("droplet", pos.astype(np.float32).astype(np.float64), w.types[keep].copy(), np.eye(3) * box)


def run_gpu_iso(hp, es, sysm, theta, per_atom_virial=False):
    from paper_2601_19034_amd.api import ALL_OUTPUTS, DEFAULT_OUTPUTS, QNEP, to_device_inputs

    model = QNEP(hp)
    pos, types, th = to_device_inputs(sysm, theta)
    out = model.compute(pos, types, sysm.cell, th, es, periodic=False,
                        outputs=ALL_OUTPUTS if per_atom_virial else DEFAULT_OUTPUTS)
    flags = model.check_status()
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    g["pos_used"] = np.asarray(sysm.pos, dtype=np.float64)
    return g, flags


@pytest.mark.parametrize("radius", [4.0, 11.0])
def test_isolated_droplet(torch_dev, orc, radius):
    """A water droplet in free space (direct Coulomb sum over all pairs, Born charges as
    the derivative of P with absolute positions) against the oracle, with the per-atom
    virial; the default outputs are the same with or without it."""
    hp, th = inputs.WATER_HP, inputs.theta0(inputs.WATER_HP, 31)
    s = _droplet(8, radius, 2 * radius + 2 * 9.5, seed=7)
    es = inputs.ESParams(method=2)
    _say(f"case isolated droplet N={s.n}")
    g, flags = run_gpu_iso(hp, es, s, th, per_atom_virial=True)
    assert flags == 0, flags
    r = orc.compute(hp, es, s.pos, s.types, s.cell, th, periodic=False, per_atom_virial=True)
    compare(g, r, s.n, label=f"droplet-{s.n}")
    Va = g["virial_atom"].T.reshape(-1, 3, 3)
    err = np.abs(Va - r.vatom).max()
    _say(f"[droplet-{s.n}] max|dW_i|={err:.2e} (max|W_i| {np.abs(r.vatom).max():.2f})")
    assert err <= 2e-5 * np.abs(r.vatom).max() + 1e-5
    assert g["energy_terms"][2] == 0.0 and g["energy_terms"][3] == 0.0


def test_isolated_flags(torch_dev):
    """An isolated system must fit its bounding box: an atom outside raises
    QNEP_FLAG_OUTSIDE, and a box so tight that an atom sees a periodic image within a
    cutoff raises QNEP_FLAG_IMAGE."""
    from paper_2601_19034_amd import binding as B

    hp, th = inputs.WATER_HP, inputs.theta0(inputs.WATER_HP, 31)
    s = _droplet(8, 4.0, 30.0, seed=7)
    es = inputs.ESParams(method=2)
    out_of_box = inputs.System("out", s.pos + np.array([0.0, 0.0, 16.0]), s.types, s.cell)
    _say("case isolated flags")
    _, flags = run_gpu_iso(hp, es, out_of_box, th)
    assert flags & B.FLAG_OUTSIDE
    tight = inputs.System("tight", s.pos - 15.0 + 4.5, s.types, np.eye(3) * 9.0)  # images 4 A apart
    _, flags = run_gpu_iso(hp, es, tight, th)
    assert flags & B.FLAG_IMAGE and not flags & B.FLAG_OUTSIDE
