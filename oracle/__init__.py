"""FP64 CPU oracle of the qNEP force evaluation (arXiv:2601.19034).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only code allowed to import it.
The product path (``paper_2601_19034_amd``) never imports, links or runs it.

The arithmetic lives in ``qnep_oracle.c`` (plain C, double precision); this module
only compiles it with gcc and marshals numpy arrays through ctypes.

Pins (see ``tests/test_oracle_*.py``): the rock-salt Madelung constant,
alpha-independence of U_ES, central finite differences of E for forces, virial
and (through the cluster identity) Born charges, the P = 5 alias sum, B-spline
properties, the addition theorem for the angular descriptor, PPPM -> Ewald
convergence and the invariances.  No GPUMD code or model is available here, so
equality with GPUMD's NEP descriptors is parity unpinned.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qnep_oracle.c")
_LIB = os.path.join(_HERE, "libqnep_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _HP(C.Structure):
    _fields_ = [("n_types", C.c_int), ("n_max_R", C.c_int), ("n_max_A", C.c_int), ("basis_R", C.c_int),
                ("basis_A", C.c_int), ("l_max", C.c_int), ("n_neu", C.c_int), ("rc_R", C.c_double),
                ("rc_A", C.c_double)]


class _ES(C.Structure):
    _fields_ = [("mode", C.c_int), ("method", C.c_int), ("alpha", C.c_double), ("rc_coul", C.c_double),
                ("kmax", C.c_double), ("kmax_inclusive", C.c_int), ("mesh", C.c_int * 3), ("order", C.c_int),
                ("q_total", C.c_double), ("efield", C.c_double * 3)]


_DP = C.POINTER(C.c_double)


class _OUT(C.Structure):
    _fields_ = [(name, _DP) for name in ("terms", "forces", "virial", "q_screened", "q_naked", "q_raw", "bec",
                                         "pol", "desc", "site_energy", "phi", "vatom")]


def lib():
    """The compiled oracle (QNEP_ORACLE_LIBRARY in the environment selects another
    build of the same source, for example one with sanitizers)."""
    global _lib
    if _lib is None:
        path = os.environ.get("QNEP_ORACLE_LIBRARY")
        if not path:
            path = _LIB
            if not os.path.exists(path):
                build()
        L = C.CDLL(path)
        L.oq_compute.restype = C.c_int
        L.oq_compute.argtypes = [C.POINTER(_HP), C.POINTER(_ES), C.c_int, _DP, C.POINTER(C.c_int), _DP, _DP,
                                 C.c_int, C.c_int, C.POINTER(_OUT), C.c_int]
        L.oq_theta_count.restype = C.c_int64
        L.oq_theta_count.argtypes = [C.POINTER(_HP)]
        L.oq_radial_basis.restype = None
        L.oq_radial_basis.argtypes = [C.c_double, C.c_double, C.c_int, _DP, _DP]
        L.oq_assign_weight.restype = C.c_double
        L.oq_assign_weight.argtypes = [C.c_int, C.c_double]
        L.oq_alias_poly5.restype = C.c_double
        L.oq_alias_poly5.argtypes = [C.c_double]
        L.oq_dft3.restype = None
        L.oq_dft3.argtypes = [_DP, _DP, C.POINTER(C.c_int), C.c_int]
        L.oq_set_ablation.restype = None
        L.oq_set_ablation.argtypes = [C.c_int]
        L.oq_neighbors.restype = C.c_int
        L.oq_neighbors.argtypes = [C.c_int, C.c_int, _DP, _DP, C.c_double, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int), _DP, C.c_int]
        _lib = L
    return _lib


def _hp(hp) -> _HP:
    return _HP(hp.n_types, hp.n_max_R, hp.n_max_A, hp.basis_R, hp.basis_A, hp.l_max, hp.n_neu, hp.rc_R, hp.rc_A)


def _es(es) -> _ES:
    m = (C.c_int * 3)(*[int(x) for x in es.mesh])
    E = (C.c_double * 3)(*[float(x) for x in getattr(es, "efield", (0.0, 0.0, 0.0))])
    return _ES(es.mode, es.method, es.alpha, es.rc_coul, es.kmax, es.kmax_inclusive, m, es.order, es.q_total, E)


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return _DP()
    return a.ctypes.data_as(_DP)


@dataclass
class OracleResult:
    energy: float
    terms: np.ndarray          # E, U_NEP, U_r, U_k, U_s, U_bg, sum q_raw, mean phi, sum q~', n_k
    forces: Optional[np.ndarray]
    virial: Optional[np.ndarray]
    q_screened: np.ndarray
    q_naked: np.ndarray
    q_raw: np.ndarray
    bec: Optional[np.ndarray]
    pol: np.ndarray
    desc: np.ndarray
    site_energy: np.ndarray
    phi: np.ndarray
    vatom: Optional[np.ndarray] = None  # (N, 3, 3) per-atom virial W_i[a][b]


def theta_count(hp) -> int:
    h = _hp(hp)
    return int(lib().oq_theta_count(C.byref(h)))


def compute(hp, es, pos, types, cell, theta, forces: bool = True, cells: bool = False,
            per_atom_virial: bool = False, periodic: bool = True) -> OracleResult:
    """Evaluate E, F, W, q, Z*, P (and intermediates) in FP64.

    pos (N, 3) Angstrom, types (N,) int, cell (3, 3) rows a, b, c, theta flat vector.
    ``cells`` selects the cell-list neighbour search instead of brute force;
    ``per_atom_virial`` also returns W_i (needs ``forces``).  A non-zero ``es.efield``
    adds the external-field force to the forces.  ``periodic=False`` evaluates an
    isolated system (no images; es.method must be 2, the direct Coulomb sum; the cell
    only bounds the cluster) with the Born charges of Eq. 27."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    types = np.ascontiguousarray(types, dtype=np.int32)
    cell = np.ascontiguousarray(cell, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = pos.shape[0]
    ndes = (hp.n_max_R + 1) + (hp.n_max_A + 1) * hp.l_max
    terms = np.zeros(10)
    F = np.zeros((n, 3)) if forces else None
    W = np.zeros((3, 3)) if forces else None
    Z = np.zeros((n, 3, 3)) if forces else None
    qs, qt, qr = np.zeros(n), np.zeros(n), np.zeros(n)
    P = np.zeros(3)
    D = np.zeros((n, ndes))
    U = np.zeros(n)
    phi = np.zeros(n)
    Va = np.zeros((n, 3, 3)) if (forces and per_atom_virial) else None
    out = _OUT(_ptr(terms), _ptr(F), _ptr(W), _ptr(qs), _ptr(qt), _ptr(qr), _ptr(Z), _ptr(P), _ptr(D), _ptr(U),
               _ptr(phi), _ptr(Va))
    h, e = _hp(hp), _es(es)
    rc = lib().oq_compute(C.byref(h), C.byref(e), n, _ptr(pos), types.ctypes.data_as(C.POINTER(C.c_int)),
                          _ptr(cell), _ptr(theta), 1 if cells else 0, 1 if forces else 0, C.byref(out),
                          1 if periodic else 0)
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return OracleResult(terms[0], terms, F, W, qs, qt, qr, Z, P, D, U, phi, Va)


def set_ablation(flags: int) -> None:
    """Test-only mistake switch (0 = off): bit 1 makes the forces use chi_i = phi_i
    instead of phi_i - mean(phi)."""
    lib().oq_set_ablation(int(flags))


def neighbors(pos, cell, rc, cells: bool = False, cap: int = 0):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    cell = np.ascontiguousarray(cell, dtype=np.float64)
    n = pos.shape[0]
    counts = np.zeros(n, dtype=np.int32)
    js = np.zeros((n, cap), dtype=np.int32) if cap else None
    ds = np.zeros((n, cap)) if cap else None
    ov = lib().oq_neighbors(1 if cells else 0, n, _ptr(pos), _ptr(cell), rc,
                            counts.ctypes.data_as(C.POINTER(C.c_int)),
                            js.ctypes.data_as(C.POINTER(C.c_int)) if cap else C.POINTER(C.c_int)(),
                            _ptr(ds), cap)
    if ov:
        raise ValueError("neighbour capacity exceeded")
    return counts, js, ds


def radial_basis(r: float, rc: float, nb: int):
    f, df = np.zeros(nb + 1), np.zeros(nb + 1)
    lib().oq_radial_basis(r, rc, nb, _ptr(f), _ptr(df))
    return f, df


def assign_weight(P: int, x: float) -> float:
    return float(lib().oq_assign_weight(P, x))


def alias_poly5(z: float) -> float:
    return float(lib().oq_alias_poly5(z))


def dft3(x: np.ndarray, sign: int = -1) -> np.ndarray:
    re = np.ascontiguousarray(x.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(x.imag, dtype=np.float64).copy()
    N = (C.c_int * 3)(*x.shape)
    lib().oq_dft3(_ptr(re), _ptr(im), N, sign)
    return re + 1j * im
