"""GPU adjoint (qnep_backward) against finite differences of the FP64 oracle.

L = gE E + gP . P.  dL/dtheta is compared with central differences of the oracle's E
and P over samples of every parameter block (radial and angular coefficients, W0, b0,
w1E, w1q, b1q per species, b1E, s); dL/dr with the oracle's -gE F + Z^T gP; dL/dh
with a central difference of the oracle energy under a change of the cell at fixed
Cartesian positions (Ewald, with a k-set away from lattice shells and an alpha for
which the real-space truncation is negligible).

Tolerance: |GPU - FD| <= 2e-3 max|FD| + 1e-5 (FP32 sums against an O(h^2) central
difference in FP64).
"""
import copy
import math
import sys

import numpy as np
import pytest

from paper_2601_19034_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _blocks(hp):
    T = hp.n_types
    ncR = T * T * (hp.n_max_R + 1) * (hp.basis_R + 1)
    ncA = T * T * (hp.n_max_A + 1) * (hp.basis_A + 1)
    per = hp.n_neu * hp.n_des + 3 * hp.n_neu + 1
    out = {"cR": (0, ncR), "cA": (ncR, ncR + ncA)}
    for t in range(T):
        b = ncR + ncA + t * per
        H, nd = hp.n_neu, hp.n_des
        out[f"W0_{t}"] = (b, b + H * nd)
        out[f"b0_{t}"] = (b + H * nd, b + H * nd + H)
        out[f"w1E_{t}"] = (b + H * nd + H, b + H * nd + 2 * H)
        out[f"w1q_{t}"] = (b + H * nd + 2 * H, b + H * nd + 3 * H)
        out[f"b1q_{t}"] = (b + H * nd + 3 * H, b + H * nd + 3 * H + 1)
    n = hp.n_theta()
    out["b1E"] = (n - 2, n - 1)
    out["s"] = (n - 1, n)
    return out


def _sample_indices(hp, per_block, seed):
    rng = np.random.default_rng(seed)
    idx = []
    for name, (a, b) in _blocks(hp).items():
        k = min(per_block, b - a)
        idx += list(rng.choice(np.arange(a, b), size=k, replace=False))
    return np.array(sorted(idx))


def _gpu_backward(w, es, gE, gP, sysm=None, want=None):
    from paper_2601_19034_amd.api import QNEP, to_device_inputs

    sysm = sysm or w.system
    model = QNEP(w.hp)
    pos, types, th = to_device_inputs(sysm, w.theta)
    if want is None:  # the cell derivative is formed for the energy term only
        want = ("pos", "theta") if gP is not None else ("pos", "cell", "theta")
    g = model.backward(pos, types, sysm.cell, th, es, gE, gP, want=want)
    return {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}


def _fd_theta(orc, w, es, idx, gE, gP, h=1e-4, sysm=None):
    sysm = sysm or w.system
    out = np.zeros(len(idx))
    for m, k in enumerate(idx):
        vals = []
        for sgn in (+1, -1):
            th = w.theta.copy()
            th[k] += sgn * h
            r = orc.compute(w.hp, es, sysm.pos, sysm.types, sysm.cell, th, forces=False, cells=sysm.n > 1000)
            vals.append(gE * r.energy + (0.0 if gP is None else float(np.dot(gP, r.pol))))
        out[m] = (vals[0] - vals[1]) / (2 * h)
    return out


def _check(gpu, fd, label):
    scale = np.abs(fd).max()
    err = np.abs(gpu - fd)
    worst = int(np.argmax(err))
    _say(f"[{label}] n={len(fd)} max|fd|={scale:.3e} max err={err.max():.3e} (gpu {gpu[worst]:.6e} fd {fd[worst]:.6e})")
    assert np.all(err <= 2e-3 * scale + 1e-5), label


def _es_smooth(L):
    # erfc(alpha rc) ~ 2e-10 and kmax between lattice shells: E is smooth in theta, r and h
    return inputs.ESParams(mode=1, method=0, alpha=0.5, rc_coul=9.0, kmax=2 * math.pi * 6.5 / L)


def test_theta_gradient_energy_water(torch_dev, orc):
    w = inputs.workload(0)
    es = _es_smooth(w.system.cell[0, 0])
    _say("case backward dE/dtheta water-192 Ewald")
    g = _gpu_backward(w, es, 1.0, None)
    idx = _sample_indices(w.hp, 6, 1)
    _check(g["theta"][idx], _fd_theta(orc, w, es, idx, 1.0, None), "dE/dtheta water")


def test_theta_gradient_polarization_water(torch_dev, orc):
    w = inputs.workload(0)
    es = _es_smooth(w.system.cell[0, 0])
    es.q_total = 0.4  # the correction and the s-derivative of P both matter
    gP = np.array([0.7, -0.4, 0.25])
    _say("case backward d(gE E + gP.P)/dtheta water-192, Q = 0.4")
    g = _gpu_backward(w, es, 0.3, gP)
    idx = _sample_indices(w.hp, 5, 2)
    _check(g["theta"][idx], _fd_theta(orc, w, es, idx, 0.3, gP), "dL/dtheta water gP")


def test_theta_gradient_garnet_pppm(torch_dev, orc):
    w = inputs.workload(2, "crop")
    _say("case backward dE/dtheta garnet-768 PPPM (four species)")
    g = _gpu_backward(w, w.es, 1.0, None)
    idx = _sample_indices(w.hp, 3, 3)
    _check(g["theta"][idx], _fd_theta(orc, w, w.es, idx, 1.0, None), "dE/dtheta garnet")


def test_position_and_cell_gradient(torch_dev, orc):
    w = inputs.workload(0)
    es = _es_smooth(w.system.cell[0, 0])
    gP = np.array([0.2, 0.5, -0.3])
    _say("case backward dL/dr, dE/dh water-192")
    g = _gpu_backward(w, es, 1.0, gP, want=("pos",))
    r = orc.compute(w.hp, es, w.system.pos, w.system.types, w.system.cell, w.theta)
    want = -r.forces + np.einsum("a,iab->ib", gP, r.bec)
    err = np.abs(g["pos"].T - want).max()
    _say(f"[dL/dr] max err {err:.2e}")
    assert err < 2e-4
    # cell: central difference of E at fixed Cartesian positions (gP = 0: the cell
    # derivative of P is not formed and is rejected)
    g = _gpu_backward(w, es, 1.0, None, want=("cell",))
    h = 1e-5
    fd = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            vals = []
            for sgn in (+1, -1):
                cell = w.system.cell.copy()
                cell[a, b] += sgn * h
                vals.append(orc.compute(w.hp, es, w.system.pos, w.system.types, cell, w.theta, forces=False).energy)
            fd[a, b] = (vals[0] - vals[1]) / (2 * h)
    err = np.abs(g["cell"] - fd).max()
    _say(f"[dE/dh] max err {err:.2e} (max |fd| {np.abs(fd).max():.3e})")
    assert err < 2e-3 * np.abs(fd).max() + 1e-4


def test_autograd_function(torch_dev, orc):
    import torch

    from paper_2601_19034_amd.api import QNEP, QnepFunction, to_device_inputs

    w = inputs.workload(0)
    es = _es_smooth(w.system.cell[0, 0])
    model = QNEP(w.hp)
    pos, types, th = to_device_inputs(w.system, w.theta)
    pos.requires_grad_(True)
    th.requires_grad_(True)
    cell = torch.tensor(w.system.cell, dtype=torch.float64, requires_grad=False)
    E, P, F, Z, q = QnepFunction.apply(pos, th, cell, model, types, es)
    loss = 2.0 * E + (P * torch.tensor([0.1, 0.2, -0.3], dtype=torch.float64, device=P.device)).sum()
    loss.backward()
    g = model.backward(pos.detach(), types, w.system.cell, th.detach(), es, 2.0, np.array([0.1, 0.2, -0.3]),
                       want=("pos", "theta"))
    assert torch.allclose(pos.grad, g["pos"]) and torch.allclose(th.grad, g["theta"])
    assert torch.allclose(pos.grad, -2.0 * F + torch.einsum("a,abn->bn", torch.tensor(
        [0.1, 0.2, -0.3], device=F.device), Z.reshape(3, 3, -1)), atol=1e-5)
    # the cell gradient of an energy-only loss
    cell = torch.tensor(w.system.cell, dtype=torch.float64, requires_grad=True)
    E, P, F, Z, q = QnepFunction.apply(pos.detach(), th.detach(), cell, model, types, es)
    (2.0 * E).backward()
    g = model.backward(pos.detach(), types, w.system.cell, th.detach(), es, 2.0, None, want=("cell",))
    assert torch.allclose(cell.grad, g["cell"].cpu())
    # P in the loss while the cell needs a gradient: refused, not silently wrong
    cell = torch.tensor(w.system.cell, dtype=torch.float64, requires_grad=True)
    E, P, F, Z, q = QnepFunction.apply(pos.detach(), th.detach(), cell, model, types, es)
    with pytest.raises(NotImplementedError):
        (E + P.sum()).backward()
