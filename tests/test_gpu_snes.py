"""One SNES generation on the GPU (qnep_snes_generation, Sec. 2.5) against the oracle's
generation (oracle/snes.py) on the same standard-normal draws.

The population mu + sigma * s_k is evaluated with the batched loss on both sides (the
oracle's loss from FP64 evaluations of every structure); when the oracle's ranking is
unambiguous at the FP32 loss resolution, the GPU must rank the members the same way
and its updated mean and step sizes must equal the oracle's to FP32 rounding.
"""
import sys

import numpy as np
import pytest

from paper_2601_19034_amd import inputs

pytestmark = pytest.mark.gpu

LAM = (1.0, 2.0, 0.5, 1e-4, 1e-5)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_snes_generation_against_oracle(orc):
    import torch

    from oracle import snes
    from paper_2601_19034_amd.api import QNEP, QNEPBatch
    from test_gpu_batch_grad import _oracle_loss

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    wl = inputs.batch_workload(n_struct=512, n_cand=2)
    systems = [wl.systems[k] for k in (3, 130, 290, 470)]
    refs = [orc.compute(wl.hp, wl.es, s.pos, s.types, s.cell, wl.theta0) for s in systems]
    d = wl.hp.n_theta()
    C = 8
    rng = np.random.default_rng(2601)
    mu = wl.theta0.astype(np.float32)
    sigma = np.full(d, 0.03, dtype=np.float32)
    noise = rng.normal(size=(C, d)).astype(np.float32)
    _say(f"case SNES generation: {len(systems)} structures x {C} members, d = {d}")
    model = QNEP(wl.hp, "fp32")
    batch = QNEPBatch(model, systems, wl.es, max_candidates=C)
    E_ref = torch.tensor([r.energy for r in refs], dtype=torch.float64, device="cuda")
    F_ref = torch.from_numpy(np.ascontiguousarray(np.concatenate([r.forces for r in refs]).T.astype(np.float32))).cuda()
    mu_d, sig_d = torch.from_numpy(mu).cuda(), torch.from_numpy(sigma).cuda()
    out = batch.snes_generation(mu_d, sig_d, torch.from_numpy(noise).cuda(), E_ref, F_ref, lambdas=LAM)
    torch.cuda.synchronize()
    assert batch.check_status() == 0
    loss_gpu = out["loss"].cpu().numpy()
    pop = out["thetas"].cpu().numpy()
    # the population is mu + sigma s in FP32 (one rounding per entry)
    want_pop = snes.population(mu, sigma, noise)
    assert np.abs(pop - want_pop).max() <= 2.0 ** -23 * np.abs(want_pop).max()
    loss_orc = np.array([_oracle_loss(orc, wl.hp, wl.es, systems, refs, want_pop[k], LAM) for k in range(C)])
    _say("[snes] loss gpu " + " ".join(f"{v:.6f}" for v in loss_gpu))
    _say("[snes] loss orc " + " ".join(f"{v:.6f}" for v in loss_orc))
    np.testing.assert_allclose(loss_gpu, loss_orc, rtol=1e-4)
    srt = np.sort(loss_orc)
    assert np.min(np.diff(srt) / srt[1:]) > 1e-3, "ranking too close to call at FP32 resolution"
    np.testing.assert_array_equal(snes.ranks(loss_gpu), snes.ranks(loss_orc))
    mu2, sig2 = snes.update(mu, sigma, noise, loss_orc)
    dmu = np.abs(mu_d.cpu().numpy() - mu2).max()
    dsig = np.abs(sig_d.cpu().numpy() - sig2).max() / sig2.max()
    _say(f"[snes] max |d mu| = {dmu:.2e}, max |d sigma| / sigma = {dsig:.2e}, "
         f"mean step |mu' - mu| = {np.abs(mu2 - mu).mean():.2e}")
    assert dmu <= 4 * 2.0 ** -24 * (np.abs(mu2).max() + 1.0)
    assert dsig <= 1e-6
    assert np.abs(mu2 - mu).mean() > 1e-4  # the generation moved the distribution
