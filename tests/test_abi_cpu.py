"""Host-side checks of the C ABI (no GPU needed): every symbol declared in
include/qnep.h is exported, parameter counting, workspace sizing and argument
validation happen before any device work."""
import math
import os
import re

import numpy as np
import pytest

from paper_2601_19034_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(qnep_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(qlib):
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(qlib, n), n


def test_param_count_matches_layout(qlib):
    from paper_2601_19034_amd import binding as B
    for hp in (inputs.WATER_HP, inputs.GARNET_HP, inputs.PEROV_HP):
        assert B.qnep_param_count(hp) == hp.n_theta()


def test_model_validation(qlib):
    from paper_2601_19034_amd import binding as B
    bad = inputs.HParams(n_types=5)
    with pytest.raises(B.QnepError):
        B.qnep_model_create(bad, 0)
    odd = inputs.HParams(n_types=2, n_max_R=3)
    with pytest.raises(B.QnepError, match="unsupported"):
        B.qnep_model_create(odd, 0)
    with pytest.raises(B.QnepError):
        B.qnep_model_create(inputs.WATER_HP, 7)
    h = B.qnep_model_create(inputs.WATER_HP, 0)
    B.qnep_model_destroy(h)


def test_workspace_and_plan_validation(qlib):
    from paper_2601_19034_amd import binding as B
    w = inputs.workload(0)
    h = B.qnep_model_create(w.hp, 0)
    try:
        es = B.make_es(w.es)
        n = w.system.n
        nb = B.qnep_workspace_size(h, es, B.make_system(n, 0, 0, w.system.cell))
        assert nb > n * 100
        # PPPM workspace grows with the mesh
        es_p = inputs.ESParams(method=1, mesh=(32, 32, 32))
        nb32 = B.qnep_workspace_size(h, B.make_es(es_p), B.make_system(n, 0, 0, w.system.cell))
        es_p.mesh = (64, 64, 64)
        nb64 = B.qnep_workspace_size(h, B.make_es(es_p), B.make_system(n, 0, 0, w.system.cell))
        assert nb64 - nb32 >= 16 * (64 ** 3 - 32 ** 3)  # two complex meshes
        # unsupported mesh (factor 7), singular cell, left-handed cell, thin cell, bad mode
        es_p.mesh = (28, 32, 32)
        with pytest.raises(B.QnepError, match="mesh"):
            B.qnep_workspace_size(h, B.make_es(es_p), B.make_system(n, 0, 0, w.system.cell))
        with pytest.raises(B.QnepError, match="cell"):
            B.qnep_workspace_size(h, es, B.make_system(n, 0, 0, np.zeros((3, 3))))
        lh = w.system.cell.copy()
        lh[2] *= -1
        with pytest.raises(B.QnepError, match="cell"):
            B.qnep_workspace_size(h, es, B.make_system(n, 0, 0, lh))
        with pytest.raises(B.QnepError, match="thinner"):
            B.qnep_workspace_size(h, es, B.make_system(n, 0, 0, np.diag([2.0, 20.0, 20.0])))
        es_bad = inputs.ESParams(mode=3)
        with pytest.raises(B.QnepError, match="mode"):
            B.qnep_workspace_size(h, B.make_es(es_bad), B.make_system(n, 0, 0, w.system.cell))
        with pytest.raises(B.QnepError, match="n_atoms"):
            B.qnep_workspace_size(h, es, B.make_system(1 << 23, 0, 0, w.system.cell))
        # compute refuses a small workspace before touching the device
        outs = B.qnep_outputs()
        with pytest.raises(B.QnepError, match="workspace"):
            B.qnep_compute(h, 1, es, B.make_system(n, 1, 1, w.system.cell), outs, 1, 16, 0)
    finally:
        B.qnep_model_destroy(h)


def test_capacity_factor_validation(qlib):
    from paper_2601_19034_amd import binding as B
    h = B.qnep_model_create(inputs.WATER_HP, 0)
    try:
        with pytest.raises(B.QnepError):
            B.qnep_model_set_capacity_factor(h, 0.5)
        B.qnep_model_set_capacity_factor(h, 2.0)
    finally:
        B.qnep_model_destroy(h)


def test_batch_workspace_and_validation(qlib):
    """Sizing and argument checks of the batched entry points (host only)."""
    import ctypes as C

    from paper_2601_19034_amd import binding as B
    wl = inputs.batch_workload(n_struct=16, n_cand=4)
    h = B.qnep_model_create(wl.hp, 0)
    try:
        sizes = [len(s.types) for s in wl.systems]
        off = (C.c_int64 * 17)(*np.concatenate([[0], np.cumsum(sizes)]).tolist())
        cells = (C.c_double * (9 * 16))(*np.concatenate([s.cell.reshape(9) for s in wl.systems]).tolist())
        es = B.make_es(wl.es)
        b0 = B.make_batch(16, 0, off, cells, 0, 0)
        b1 = B.make_batch(16, B.QNEP_BATCH_VIRIAL, off, cells, 0, 0)
        n0 = B.qnep_batch_workspace_size(h, es, b0, 4)
        n1 = B.qnep_batch_workspace_size(h, es, b1, 4)
        # the virial adds six N x N matrices per structure
        assert n1 - n0 >= 6 * 4 * sum(n * n for n in sizes) - 4096
        assert B.qnep_batch_workspace_size(h, es, b0, 64) > n0
        with pytest.raises(B.QnepError):
            B.qnep_batch_workspace_size(h, es, b0, 0)
        pppm = B.make_es(inputs.ESParams(method=1, mesh=(16, 16, 16)))
        with pytest.raises(B.QnepError, match="unsupported"):
            B.qnep_batch_workspace_size(h, pppm, b0, 4)
        bad = (C.c_int64 * 17)(*([0] + [3000] * 16))
        with pytest.raises(B.QnepError, match="unsupported"):
            B.qnep_batch_workspace_size(h, es, B.make_batch(16, 0, bad, cells, 0, 0), 4)
        empty = (C.c_int64 * 17)(*([0, 0] + [10] * 15))
        with pytest.raises(B.QnepError):
            B.qnep_batch_workspace_size(h, es, B.make_batch(16, 0, empty, cells, 0, 0), 4)
        flat = (C.c_double * (9 * 16))(*([0.0] * 9 * 16))
        with pytest.raises(B.QnepError, match="invalid"):
            B.qnep_batch_workspace_size(h, es, B.make_batch(16, 0, off, flat, 0, 0), 4)
    finally:
        B.qnep_model_destroy(h)
    # the garnet model (10310 parameters) fits the staged-parameter limit; a larger one does not
    big = inputs.HParams(n_types=4, n_max_R=8, n_max_A=6, basis_R=8, basis_A=8, l_max=4, n_neu=64)
    hb = B.qnep_model_create(big, 0)
    try:
        with pytest.raises(B.QnepError, match="unsupported"):
            B.qnep_batch_workspace_size(hb, es, b0, 4)
    finally:
        B.qnep_model_destroy(hb)


def test_new_entry_points_validation(qlib):
    """Host-side checks of the allocation-free call, the MD driver, the SNES generation
    and the field argument: each bad argument is refused before any device work."""
    from paper_2601_19034_amd import binding as B
    w = inputs.workload(0)
    h = B.qnep_model_create(w.hp, 0)
    try:
        n = w.system.n
        es = B.make_es(w.es)
        # field: must be finite; the adjoint refuses a non-zero field
        bad = inputs.ESParams(**{**w.es.__dict__, "efield": (float("nan"), 0.0, 0.0)})
        with pytest.raises(B.QnepError, match="efield"):
            B.qnep_workspace_size(h, B.make_es(bad), B.make_system(n, 0, 0, w.system.cell))
        fld = B.make_es(inputs.ESParams(**{**w.es.__dict__, "efield": (0.1, 0.0, 0.0)}))
        nbw = B.qnep_backward_workspace_size(h, fld, B.make_system(n, 0, 0, w.system.cell))
        with pytest.raises(B.QnepError, match="efield"):
            B.qnep_backward(h, 1, fld, B.make_system(n, 1, 1, w.system.cell), 1.0, None, 0, 0, 0, 1, nbw, 0)
        # the static workspace refuses structures that do not fit in it
        big = inputs.workload(1)
        hb = B.qnep_model_create(big.hp, 0)
        try:
            with pytest.raises(B.QnepError, match="static workspace"):
                B.qnep_compute_static(hb, 1, B.make_es(big.es), B.make_system(big.system.n, 1, 1, big.system.cell),
                                      B.qnep_outputs(), 0, 0)
        finally:
            B.qnep_model_destroy(hb)
        # MD: workspace grows with N; bad time step, masses and sizes are refused
        n1 = B.qnep_md_workspace_size(h, es, n, w.system.cell)
        assert n1 > B.qnep_workspace_size(h, es, B.make_system(n, 0, 0, w.system.cell))
        with pytest.raises(B.QnepError, match="dt"):
            B.qnep_md_nve(h, 1, es, -0.5, 10, [16.0, 1.0], n, 1, w.system.cell, 1, 1, 1, 1, n1, 0)
        with pytest.raises(B.QnepError, match="masses"):
            B.qnep_md_nve(h, 1, es, 0.5, 10, [16.0, 0.0], n, 1, w.system.cell, 1, 1, 1, 1, n1, 0)
        with pytest.raises(B.QnepError, match="workspace"):
            B.qnep_md_nve(h, 1, es, 0.5, 10, [16.0, 1.0], n, 1, w.system.cell, 1, 1, 1, 1, 64, 0)
        # SNES: population size and the prepared batch are checked first
        tg = B.qnep_batch_targets(1, 1, 1.0, 1.0, 1.0, 0.0, 0.0)
        oc = B.qnep_batch_outputs(1, 1, None, None, None, None)
        with pytest.raises(B.QnepError, match="n_candidates"):
            B.qnep_snes_generation(h, 1, 1, 1, 1, 1.0, 0.0, tg, oc, 1, 1, 1 << 20, 0)
        with pytest.raises(B.QnepError, match="prepared"):
            B.qnep_snes_generation(h, 1, 1, 1, 8, 1.0, 0.0, tg, oc, 1, 1, 1 << 20, 0)
        oc_noloss = B.qnep_batch_outputs(1, None, None, None, None, None)
        with pytest.raises(B.QnepError, match="loss"):
            B.qnep_snes_generation(h, 1, 1, 1, 8, 1.0, 0.0, tg, oc_noloss, 1, 1, 1 << 20, 0)
    finally:
        B.qnep_model_destroy(h)


def test_workspace_size_of_tiny_systems(qlib):
    """Sizing an empty or one-atom structure is valid under every electrostatics method
    (the plan's work splits must not divide by a zero atom count)."""
    from paper_2601_19034_amd import binding as B
    w = inputs.workload(0)
    h = B.qnep_model_create(w.hp, 0)
    try:
        cell = w.system.cell
        for es_p in (w.es, inputs.ESParams(method=1, mesh=(16, 16, 16)),
                     inputs.ESParams(**{**w.es.__dict__, "mode": 2})):
            for n in (0, 1):
                assert B.qnep_workspace_size(h, B.make_es(es_p), B.make_system(n, 0, 0, cell)) > 0
        iso = inputs.ESParams(method=2)
        for n in (0, 1):
            assert B.qnep_workspace_size(h, B.make_es(iso), B.make_system(n, 0, 0, cell, periodic=False)) > 0
    finally:
        B.qnep_model_destroy(h)


def test_ewald_rejects_oversized_k_rows(qlib):
    """A cell so long along c that the per-atom Ewald product's LDS stage of n2 values
    would not fit is rejected at sizing, before any device work."""
    from paper_2601_19034_amd import binding as B
    w = inputs.workload(0)
    h = B.qnep_model_create(w.hp, 0)
    try:
        es = B.make_es(w.es)
        cell = np.diag([12.42, 12.42, 12.42 * 40])  # kmax |c| / 2 pi = 6 * 40 > 93
        with pytest.raises(B.QnepError, match="wave vectors"):
            B.qnep_workspace_size(h, es, B.make_system(w.system.n, 0, 0, cell))
    finally:
        B.qnep_model_destroy(h)
