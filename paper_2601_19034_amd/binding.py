"""ctypes binding of libqnep.so: argument marshalling only, one Python function per
C entry point of include/qnep.h (same names).  Every step of the computation runs
in the library's HIP kernels; there is no Python or CPU fallback."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime that libqnep.so links against

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqnep.so")

QNEP_OK = 0
QNEP_MLP_FP32 = 0
QNEP_MLP_BF16 = 1
QNEP_MLP_BF16X3 = 2
N_STAGES = 19
FLAG_RADIAL_OVERFLOW = 1
FLAG_ANGULAR_OVERFLOW = 2
FLAG_COULOMB_OVERFLOW = 4
FLAG_BAD_SPECIES = 8
FLAG_OUTSIDE = 32
FLAG_IMAGE = 64
QNEP_ES_DIRECT = 2


class qnep_hparams(C.Structure):
    _fields_ = [("n_types", C.c_int32), ("n_max_R", C.c_int32), ("n_max_A", C.c_int32), ("basis_R", C.c_int32),
                ("basis_A", C.c_int32), ("l_max", C.c_int32), ("n_neu", C.c_int32), ("rc_R", C.c_double),
                ("rc_A", C.c_double)]


class qnep_es_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("method", C.c_int32), ("alpha", C.c_double), ("rc_coul", C.c_double),
                ("kmax", C.c_double), ("kmax_inclusive", C.c_int32), ("mesh", C.c_int32 * 3), ("order", C.c_int32),
                ("q_total", C.c_double), ("efield", C.c_double * 3)]


class qnep_system(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("pos", C.c_void_p), ("type", C.c_void_p), ("cell", C.c_double * 9),
                ("pbc", C.c_int32 * 3)]


class qnep_outputs(C.Structure):
    _fields_ = [("energy", C.c_void_p), ("forces", C.c_void_p), ("virial", C.c_void_p), ("charges", C.c_void_p),
                ("charges_naked", C.c_void_p), ("bec", C.c_void_p), ("polarization", C.c_void_p),
                ("energy_terms", C.c_void_p), ("virial_atom", C.c_void_p)]


class QnepError(RuntimeError):
    pass


EXPORTED = ["qnep_param_count", "qnep_model_create", "qnep_model_destroy", "qnep_model_set_capacity_factor",
            "qnep_workspace_size", "qnep_compute", "qnep_check_status", "qnep_model_enable_timing",
            "qnep_model_read_timing", "qnep_stage_name", "qnep_backward_workspace_size", "qnep_backward",
            "qnep_status_string", "qnep_last_error"]

_lib = None


def load(path: str = None):
    """Loads the library (raises if it has not been built).  QNEP_LIBRARY in the
    environment selects another build of it (for example one with host sanitizers)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("QNEP_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2601_19034_amd.build`")
    L = C.CDLL(path)
    L.qnep_param_count.restype = C.c_int64
    L.qnep_param_count.argtypes = [C.POINTER(qnep_hparams)]
    L.qnep_model_create.restype = C.c_int
    L.qnep_model_create.argtypes = [C.POINTER(qnep_hparams), C.c_int32, C.POINTER(C.c_void_p)]
    L.qnep_model_destroy.restype = C.c_int
    L.qnep_model_destroy.argtypes = [C.c_void_p]
    L.qnep_model_set_capacity_factor.restype = C.c_int
    L.qnep_model_set_capacity_factor.argtypes = [C.c_void_p, C.c_double]
    L.qnep_workspace_size.restype = C.c_int
    L.qnep_workspace_size.argtypes = [C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_system),
                                      C.POINTER(C.c_size_t)]
    L.qnep_compute.restype = C.c_int
    L.qnep_compute.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_system),
                               C.POINTER(qnep_outputs), C.c_void_p, C.c_size_t, C.c_void_p]
    L.qnep_compute_static.restype = C.c_int
    L.qnep_compute_static.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_system),
                                      C.POINTER(qnep_outputs), C.c_void_p, C.c_void_p]
    L.qnep_check_status.restype = C.c_int
    L.qnep_check_status.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]
    L.qnep_model_enable_timing.restype = C.c_int
    L.qnep_model_enable_timing.argtypes = [C.c_void_p, C.c_int32]
    L.qnep_model_read_timing.restype = C.c_int
    L.qnep_model_read_timing.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int32)]
    L.qnep_stage_name.restype = C.c_char_p
    L.qnep_stage_name.argtypes = [C.c_int32]
    L.qnep_status_string.restype = C.c_char_p
    L.qnep_status_string.argtypes = [C.c_int]
    L.qnep_last_error.restype = C.c_char_p
    L.qnep_last_error.argtypes = []
    _lib = L
    return L


def _check(status: int):
    if status != QNEP_OK:
        L = load()
        raise QnepError(f"{L.qnep_status_string(status).decode()} ({status}): {L.qnep_last_error().decode()}")


def make_hparams(hp) -> qnep_hparams:
    return qnep_hparams(hp.n_types, hp.n_max_R, hp.n_max_A, hp.basis_R, hp.basis_A, hp.l_max, hp.n_neu,
                        float(hp.rc_R), float(hp.rc_A))


def make_es(es) -> qnep_es_params:
    mesh = (C.c_int32 * 3)(*[int(m) for m in es.mesh])
    field = (C.c_double * 3)(*[float(x) for x in getattr(es, "efield", (0.0, 0.0, 0.0))])
    return qnep_es_params(int(es.mode), int(es.method), float(es.alpha), float(es.rc_coul), float(es.kmax),
                          int(es.kmax_inclusive), mesh, int(es.order), float(es.q_total), field)


def make_system(n: int, pos_ptr: int, type_ptr: int, cell, periodic: bool = True) -> qnep_system:
    c = (C.c_double * 9)(*[float(v) for v in list(np.asarray(cell).reshape(-1))])
    p = (C.c_int32 * 3)(*([1, 1, 1] if periodic else [0, 0, 0]))
    return qnep_system(int(n), C.c_void_p(pos_ptr), C.c_void_p(type_ptr), c, p)


def qnep_param_count(hp) -> int:
    return int(load().qnep_param_count(C.byref(make_hparams(hp))))


def qnep_model_create(hp, precision: int) -> int:
    h = C.c_void_p()
    _check(load().qnep_model_create(C.byref(make_hparams(hp)), precision, C.byref(h)))
    return h.value


def qnep_model_destroy(model: int):
    _check(load().qnep_model_destroy(C.c_void_p(model)))


def qnep_model_set_capacity_factor(model: int, factor: float):
    _check(load().qnep_model_set_capacity_factor(C.c_void_p(model), float(factor)))


def qnep_workspace_size(model: int, es: qnep_es_params, sysm: qnep_system) -> int:
    n = C.c_size_t()
    _check(load().qnep_workspace_size(C.c_void_p(model), C.byref(es), C.byref(sysm), C.byref(n)))
    return int(n.value)


def qnep_compute(model: int, theta_ptr: int, es: qnep_es_params, sysm: qnep_system, outs: qnep_outputs,
                 ws_ptr: int, ws_bytes: int, stream: int):
    _check(load().qnep_compute(C.c_void_p(model), C.c_void_p(theta_ptr), C.byref(es), C.byref(sysm),
                               C.byref(outs), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)))


def qnep_compute_static(model: int, theta_ptr: int, es: qnep_es_params, sysm: qnep_system, outs: qnep_outputs,
                        flags_ptr: int, stream: int):
    _check(load().qnep_compute_static(C.c_void_p(model), C.c_void_p(theta_ptr), C.byref(es), C.byref(sysm),
                                      C.byref(outs), C.c_void_p(flags_ptr or None), C.c_void_p(stream)))


QNEP_STATIC_WORKSPACE_BYTES = 64 * 1024 * 1024


def qnep_check_status(ws_ptr: int, stream: int) -> int:
    f = C.c_int32()
    _check(load().qnep_check_status(C.c_void_p(ws_ptr), C.c_void_p(stream), C.byref(f)))
    return int(f.value)


def qnep_model_enable_timing(model: int, enable: bool):
    _check(load().qnep_model_enable_timing(C.c_void_p(model), 1 if enable else 0))


def qnep_model_read_timing(model: int):
    """Returns ({stage name: ms}, {stage name: launches}, calls) since the previous read."""
    ms = (C.c_double * N_STAGES)()
    nl = (C.c_int64 * N_STAGES)()
    calls = C.c_int32()
    _check(load().qnep_model_read_timing(C.c_void_p(model), ms, nl, C.byref(calls)))
    names = [qnep_stage_name(k) for k in range(N_STAGES)]
    return dict(zip(names, list(ms))), dict(zip(names, list(nl))), int(calls.value)


def qnep_stage_name(stage: int) -> str:
    return load().qnep_stage_name(stage).decode()


def _bind_backward(L):
    L.qnep_backward_workspace_size.restype = C.c_int
    L.qnep_backward_workspace_size.argtypes = [C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_system),
                                               C.POINTER(C.c_size_t)]
    L.qnep_backward.restype = C.c_int
    L.qnep_backward.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_system),
                                C.c_double, C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_size_t, C.c_void_p]


def qnep_backward_workspace_size(model: int, es: qnep_es_params, sysm: qnep_system) -> int:
    L = load()
    if not getattr(L, "_bw_bound", False):
        _bind_backward(L)
        L._bw_bound = True
    n = C.c_size_t()
    _check(L.qnep_backward_workspace_size(C.c_void_p(model), C.byref(es), C.byref(sysm), C.byref(n)))
    return int(n.value)


def qnep_backward(model: int, theta_ptr: int, es: qnep_es_params, sysm: qnep_system, gE: float, gP,
                  dpos_ptr: int, dcell_ptr: int, dtheta_ptr: int, ws_ptr: int, ws_bytes: int, stream: int):
    L = load()
    if not getattr(L, "_bw_bound", False):
        _bind_backward(L)
        L._bw_bound = True
    gp = (C.c_double * 3)(*[float(v) for v in gP]) if gP is not None else None
    _check(L.qnep_backward(C.c_void_p(model), C.c_void_p(theta_ptr), C.byref(es), C.byref(sysm), float(gE),
                           gp, C.c_void_p(dpos_ptr or None), C.c_void_p(dcell_ptr or None),
                           C.c_void_p(dtheta_ptr or None), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)))


# ---------------------------------------------------------------- batched evaluation
QNEP_BATCH_VIRIAL = 1
QNEP_BATCH_GRADIENT = 2


class qnep_batch(C.Structure):
    _fields_ = [("n_structures", C.c_int32), ("flags", C.c_int32), ("offsets", C.c_void_p), ("cells", C.c_void_p),
                ("pos", C.c_void_p), ("type", C.c_void_p)]


class qnep_batch_targets(C.Structure):
    _fields_ = [("energy", C.c_void_p), ("forces", C.c_void_p), ("lambda_e", C.c_double), ("lambda_f", C.c_double),
                ("lambda_q", C.c_double), ("lambda_1", C.c_double), ("lambda_2", C.c_double)]


class qnep_batch_outputs(C.Structure):
    _fields_ = [("losses", C.c_void_p), ("loss", C.c_void_p), ("energy", C.c_void_p), ("virial", C.c_void_p),
                ("forces", C.c_void_p), ("charges", C.c_void_p)]


EXPORTED += ["qnep_batch_workspace_size", "qnep_batch_prepare", "qnep_batch_compute", "qnep_batch_gradient",
             "qnep_batch_tune", "qnep_snes_generation"]


def _bind_batch(L):
    if getattr(L, "_batch_bound", False):
        return
    L.qnep_batch_workspace_size.restype = C.c_int
    L.qnep_batch_workspace_size.argtypes = [C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_batch), C.c_int32,
                                            C.POINTER(C.c_size_t)]
    L.qnep_batch_prepare.restype = C.c_int
    L.qnep_batch_prepare.argtypes = [C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_batch), C.c_int32,
                                     C.c_void_p, C.c_size_t, C.c_void_p]
    L.qnep_batch_compute.restype = C.c_int
    L.qnep_batch_compute.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(qnep_batch_targets),
                                     C.POINTER(qnep_batch_outputs), C.c_void_p, C.c_size_t, C.c_void_p]
    L.qnep_batch_gradient.restype = C.c_int
    L.qnep_batch_gradient.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(qnep_batch_targets),
                                      C.POINTER(qnep_batch_outputs), C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_void_p]
    L.qnep_batch_tune.restype = C.c_int
    L.qnep_batch_tune.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(qnep_batch_targets),
                                  C.POINTER(qnep_batch_outputs), C.c_void_p, C.c_size_t, C.c_void_p,
                                  C.POINTER(C.c_int32)]
    L.qnep_snes_generation.restype = C.c_int
    L.qnep_snes_generation.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                       C.c_double, C.POINTER(qnep_batch_targets), C.POINTER(qnep_batch_outputs),
                                       C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    L._batch_bound = True


def make_batch(n_structures: int, flags: int, offsets, cells, pos_ptr: int, type_ptr: int) -> qnep_batch:
    """offsets: ctypes int64 array [S + 1]; cells: ctypes double array [S * 9] (both kept alive by the caller)."""
    return qnep_batch(int(n_structures), int(flags), C.cast(offsets, C.c_void_p), C.cast(cells, C.c_void_p),
                      C.c_void_p(pos_ptr), C.c_void_p(type_ptr))


def qnep_batch_workspace_size(model: int, es: qnep_es_params, batch: qnep_batch, max_candidates: int) -> int:
    L = load()
    _bind_batch(L)
    n = C.c_size_t()
    _check(L.qnep_batch_workspace_size(C.c_void_p(model), C.byref(es), C.byref(batch), int(max_candidates),
                                       C.byref(n)))
    return int(n.value)


def qnep_batch_prepare(model: int, es: qnep_es_params, batch: qnep_batch, max_candidates: int, ws_ptr: int,
                       ws_bytes: int, stream: int):
    L = load()
    _bind_batch(L)
    _check(L.qnep_batch_prepare(C.c_void_p(model), C.byref(es), C.byref(batch), int(max_candidates),
                                C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)))


def qnep_batch_compute(model: int, thetas_ptr: int, n_candidates: int, targets: qnep_batch_targets,
                       outputs: qnep_batch_outputs, ws_ptr: int, ws_bytes: int, stream: int):
    L = load()
    _bind_batch(L)
    _check(L.qnep_batch_compute(C.c_void_p(model), C.c_void_p(thetas_ptr), int(n_candidates), C.byref(targets),
                                C.byref(outputs), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)))


def qnep_batch_tune(model: int, thetas_ptr: int, n_candidates: int, targets: qnep_batch_targets,
                    outputs: qnep_batch_outputs, ws_ptr: int, ws_bytes: int, stream: int):
    L = load()
    _bind_batch(L)
    choice = (C.c_int32 * 5)()
    _check(L.qnep_batch_tune(C.c_void_p(model), C.c_void_p(thetas_ptr), int(n_candidates), C.byref(targets),
                             C.byref(outputs), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream), choice))
    return [int(v) for v in choice]


def qnep_batch_gradient(model: int, thetas_ptr: int, n_candidates: int, targets: qnep_batch_targets,
                        outputs: qnep_batch_outputs, dthetas_ptr: int, ws_ptr: int, ws_bytes: int, stream: int):
    L = load()
    _bind_batch(L)
    _check(L.qnep_batch_gradient(C.c_void_p(model), C.c_void_p(thetas_ptr), int(n_candidates), C.byref(targets),
                                 C.byref(outputs), C.c_void_p(dthetas_ptr), C.c_void_p(ws_ptr), ws_bytes,
                                 C.c_void_p(stream)))


def qnep_snes_generation(model: int, mu_ptr: int, sigma_ptr: int, noise_ptr: int, n_candidates: int, eta_mu: float,
                         eta_sigma: float, targets: qnep_batch_targets, outputs: qnep_batch_outputs, thetas_ptr: int,
                         ws_ptr: int, ws_bytes: int, stream: int):
    L = load()
    _bind_batch(L)
    _check(L.qnep_snes_generation(C.c_void_p(model), C.c_void_p(mu_ptr), C.c_void_p(sigma_ptr),
                                  C.c_void_p(noise_ptr), int(n_candidates), float(eta_mu), float(eta_sigma),
                                  C.byref(targets), C.byref(outputs), C.c_void_p(thetas_ptr), C.c_void_p(ws_ptr),
                                  ws_bytes, C.c_void_p(stream)))


class qnep_md_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_steps", C.c_int32), ("masses", C.c_void_p)]


EXPORTED += ["qnep_md_workspace_size", "qnep_md_nve"]


def _bind_md(L):
    if getattr(L, "_md_bound", False):
        return
    L.qnep_md_workspace_size.restype = C.c_int
    L.qnep_md_workspace_size.argtypes = [C.c_void_p, C.POINTER(qnep_es_params), C.c_int64, C.c_void_p,
                                         C.POINTER(C.c_size_t)]
    L.qnep_md_nve.restype = C.c_int
    L.qnep_md_nve.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(qnep_es_params), C.POINTER(qnep_md_params),
                              C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_size_t, C.c_void_p]
    L._md_bound = True


def qnep_md_workspace_size(model: int, es: qnep_es_params, n_atoms: int, cell) -> int:
    L = load()
    _bind_md(L)
    c = (C.c_double * 9)(*[float(v) for v in list(cell.reshape(-1))])
    n = C.c_size_t()
    _check(L.qnep_md_workspace_size(C.c_void_p(model), C.byref(es), int(n_atoms), C.cast(c, C.c_void_p),
                                    C.byref(n)))
    return int(n.value)


def qnep_md_nve(model: int, theta_ptr: int, es: qnep_es_params, dt: float, n_steps: int, masses, n_atoms: int,
                type_ptr: int, cell, pos_ptr: int, vel_ptr: int, series_ptr: int, ws_ptr: int, ws_bytes: int,
                stream: int):
    L = load()
    _bind_md(L)
    m = (C.c_double * len(masses))(*[float(v) for v in masses])
    md = qnep_md_params(float(dt), int(n_steps), C.cast(m, C.c_void_p))
    c = (C.c_double * 9)(*[float(v) for v in list(cell.reshape(-1))])
    _check(L.qnep_md_nve(C.c_void_p(model), C.c_void_p(theta_ptr), C.byref(es), C.byref(md), int(n_atoms),
                         C.c_void_p(type_ptr), C.cast(c, C.c_void_p), C.c_void_p(pos_ptr), C.c_void_p(vel_ptr),
                         C.c_void_p(series_ptr), C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream)))
