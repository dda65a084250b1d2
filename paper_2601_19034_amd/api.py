"""Python front end of libqnep: device memory and streams come from PyTorch, every
computation runs in the library's HIP kernels.

    model = QNEP(hp, precision="fp32")
    out = model.compute(pos, types, cell, theta, es)   # dict of device tensors
"""
from __future__ import annotations

from typing import Dict, Optional

import ctypes as C

import numpy as np
import torch

from . import binding as B

ALL_OUTPUTS = ("energy", "forces", "virial", "charges", "charges_naked", "bec", "polarization", "energy_terms",
               "virial_atom")
DEFAULT_OUTPUTS = ALL_OUTPUTS[:-1]  # the per-atom virial costs extra work and is requested explicitly


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("qnep needs a ROCm GPU: no device is visible")


class QNEP:
    """A model handle (hyper-parameters and MLP precision) plus a cached workspace."""

    def __init__(self, hp, precision: str = "fp32", capacity_factor: Optional[float] = None):
        B.load()
        self.hp = hp
        self.precision = precision
        prec = {"fp32": B.QNEP_MLP_FP32, "bf16": B.QNEP_MLP_BF16, "bf16x3": B.QNEP_MLP_BF16X3}[precision]
        self.handle = B.qnep_model_create(hp, prec)
        if capacity_factor is not None:
            B.qnep_model_set_capacity_factor(self.handle, capacity_factor)
        self._ws: Optional[torch.Tensor] = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                B.qnep_model_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def n_theta(self) -> int:
        return B.qnep_param_count(self.hp)

    def workspace_bytes(self, es, n_atoms: int, cell, periodic: bool = True) -> int:
        sysm = B.make_system(n_atoms, 0, 0, np.asarray(cell, dtype=np.float64), periodic)
        return B.qnep_workspace_size(self.handle, B.make_es(es), sysm)

    def workspace(self, nbytes: int, device) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes or self._ws.device != device:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self._ws

    def compute(self, pos: torch.Tensor, types: torch.Tensor, cell, theta: torch.Tensor, es,
                outputs=DEFAULT_OUTPUTS, out: Optional[Dict[str, torch.Tensor]] = None,
                stream: Optional[torch.cuda.Stream] = None, periodic: bool = True) -> Dict[str, torch.Tensor]:
        """pos: float32 device tensor [3, N] (SoA); types: int32 [N]; cell: (3, 3) rows a, b, c;
        theta: float32 device [n_theta].  Returns device tensors (energy, virial, polarization in
        float64; forces [3, N]; bec [9, N]; charges [N]) enqueued on ``stream``.  periodic=False
        evaluates an isolated system in the bounding box ``cell`` (es.method = 2)."""
        _require_gpu()
        assert pos.dtype == torch.float32 and pos.is_cuda and pos.dim() == 2 and pos.shape[0] == 3
        assert pos.is_contiguous() and types.dtype == torch.int32 and types.is_contiguous()
        assert theta.dtype == torch.float32 and theta.is_contiguous() and theta.numel() == self.n_theta
        n = pos.shape[1]
        dev = pos.device
        cell = np.asarray(cell, dtype=np.float64)
        es_c = B.make_es(es)
        sysm = B.make_system(n, pos.data_ptr(), types.data_ptr(), cell, periodic)
        nbytes = B.qnep_workspace_size(self.handle, es_c, sysm)
        ws = self.workspace(nbytes, dev)
        if out is None:
            out = {}
            shapes = {"energy": ((1,), torch.float64), "forces": ((3, n), torch.float32),
                      "virial": ((9,), torch.float64), "charges": ((n,), torch.float32),
                      "charges_naked": ((n,), torch.float32), "bec": ((9, n), torch.float32),
                      "polarization": ((3,), torch.float64), "energy_terms": ((8,), torch.float64),
                      "virial_atom": ((9, n), torch.float32)}
            for k in outputs:
                shp, dt = shapes[k]
                out[k] = torch.empty(shp, dtype=dt, device=dev)
        ptr = {k: (v.data_ptr() if v is not None else 0) for k, v in out.items()}
        outs = B.qnep_outputs(*[ptr.get(k, 0) or None for k in ALL_OUTPUTS])
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        B.qnep_compute(self.handle, theta.data_ptr(), es_c, sysm, outs, ws.data_ptr(), ws.numel(), s.cuda_stream)
        self._last_stream = s
        return out

    def enable_timing(self, on: bool = True):
        B.qnep_model_enable_timing(self.handle, on)

    def read_timing(self):
        """({stage: total ms}, {stage: launches}, calls) since the previous read."""
        return B.qnep_model_read_timing(self.handle)

    def check_status(self) -> int:
        """Synchronizes the last stream and returns the device status bits (0 = fine)."""
        return B.qnep_check_status(self._ws.data_ptr(), self._last_stream.cuda_stream)


def _md_nve(self, pos: torch.Tensor, vel: torch.Tensor, types: torch.Tensor, cell, theta: torch.Tensor, es,
            masses, dt: float, n_steps: int, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """n_steps velocity-Verlet steps (qnep_md_nve); pos and vel (float32 [3, N], Angstrom
    and Angstrom/fs) are advanced in place.  Returns the series float64 [n_steps + 1, 8]
    (E_pot, E_kin, P_dot, P) as a device tensor.  masses: per species, amu."""
    _require_gpu()
    assert pos.dtype == torch.float32 and vel.dtype == torch.float32 and pos.is_contiguous() and vel.is_contiguous()
    assert pos.shape == vel.shape and pos.shape[0] == 3 and types.dtype == torch.int32
    n = pos.shape[1]
    cell = np.asarray(cell, dtype=np.float64)
    es_c = B.make_es(es)
    nbytes = B.qnep_md_workspace_size(self.handle, es_c, n, cell)
    ws = self.workspace(nbytes, pos.device)
    series = torch.empty((n_steps + 1, 8), dtype=torch.float64, device=pos.device)
    s = stream if stream is not None else torch.cuda.current_stream(pos.device)
    B.qnep_md_nve(self.handle, theta.data_ptr(), es_c, dt, n_steps, list(masses), n, types.data_ptr(), cell,
                  pos.data_ptr(), vel.data_ptr(), series.data_ptr(), ws.data_ptr(), ws.numel(), s.cuda_stream)
    self._last_stream = s
    return series


QNEP.md_nve = _md_nve


def to_device_inputs(system, theta: np.ndarray, device="cuda"):
    """Seeded host arrays -> the device tensors ``QNEP.compute`` takes."""
    pos = torch.from_numpy(system.pos_f32_soa()).to(device)
    types = torch.from_numpy(system.types.astype(np.int32)).to(device)
    th = torch.from_numpy(np.asarray(theta, dtype=np.float32)).to(device)
    return pos, types, th


def _backward(self, pos, types, cell, theta, es, gE: float = 1.0, gP=None, want=("pos", "cell", "theta"),
              stream=None, periodic: bool = True):
    """Adjoint of ``compute`` for L = gE E + gP . P.  Returns a dict with
    ``pos`` ([3, N] float32, dL/dr), ``cell`` ([3, 3] float64, dE/dh at fixed positions;
    only with gP = 0, the library rejects the cell derivative of P) and ``theta`` ([n_theta] float32, exact dL/dtheta), all device tensors."""
    _require_gpu()
    n = pos.shape[1]
    dev = pos.device
    cell = np.asarray(cell, dtype=np.float64)
    es_c = B.make_es(es)
    sysm = B.make_system(n, pos.data_ptr(), types.data_ptr(), cell, periodic)
    nbytes = B.qnep_backward_workspace_size(self.handle, es_c, sysm)
    ws = self.workspace(nbytes, dev)
    out = {}
    if "pos" in want:
        out["pos"] = torch.empty((3, n), dtype=torch.float32, device=dev)
    if "cell" in want:
        out["cell"] = torch.empty((3, 3), dtype=torch.float64, device=dev)
    if "theta" in want:
        out["theta"] = torch.empty(theta.numel(), dtype=torch.float32, device=dev)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    B.qnep_backward(self.handle, theta.data_ptr(), es_c, sysm, gE, gP,
                    out["pos"].data_ptr() if "pos" in out else 0, out["cell"].data_ptr() if "cell" in out else 0,
                    out["theta"].data_ptr() if "theta" in out else 0, ws.data_ptr(), ws.numel(), s.cuda_stream)
    self._last_stream = s
    return out


QNEP.backward = _backward


class QnepFunction(torch.autograd.Function):
    """E and P of one structure as differentiable functions of the positions ([3, N]),
    the parameter vector and the cell ((3, 3) float64 tensor).  Forces, Born charges and
    charges come back as non-differentiable extras.

        E, P, extras = QnepFunction.apply(pos, theta, cell, model, types, es)
    """

    @staticmethod
    def forward(ctx, pos, theta, cell, model, types, es):
        cell_np = cell.detach().cpu().numpy()
        out = model.compute(pos.detach(), types, cell_np, theta.detach(), es)
        ctx.model, ctx.types, ctx.es, ctx.cell_np = model, types, es, cell_np
        ctx.save_for_backward(pos, theta)
        ctx.mark_non_differentiable(out["forces"], out["bec"], out["charges"])
        return out["energy"][0], out["polarization"], out["forces"], out["bec"], out["charges"]

    @staticmethod
    def backward(ctx, gE, gP, *unused):
        pos, theta = ctx.saved_tensors
        ge = float(gE.detach().cpu()) if gE is not None else 0.0
        gp = gP.detach().cpu().numpy().astype(np.float64) if gP is not None else None
        if ctx.needs_input_grad[2] and gp is not None and np.any(gp != 0.0):
            raise NotImplementedError("the cell gradient covers the energy only: P enters the loss while the "
                                      "cell requires a gradient")
        want = ("pos", "theta", "cell") if ctx.needs_input_grad[2] else ("pos", "theta")
        g = ctx.model.backward(pos.detach(), ctx.types, ctx.cell_np, theta.detach(), ctx.es, ge, gp, want=want)
        dcell = g["cell"].to("cpu") if ctx.needs_input_grad[2] else None
        return g["pos"], g["theta"], dcell, None, None, None


class QNEPBatch:
    """Many structures x many candidate parameter vectors (qnep_batch_*).

        batch = QNEPBatch(model, systems, es, max_candidates=64)
        out = batch.compute(thetas, E_ref, F_ref)          # dict of device tensors

    ``systems`` carry ``pos`` (N, 3), ``types`` (N,) and ``cell`` (3, 3); the geometry
    (lists and Ewald pair matrices) is built once here, on the device."""

    def __init__(self, model: QNEP, systems, es, max_candidates: int, virial: bool = False, gradient: bool = False,
                 device="cuda"):
        _require_gpu()
        self.model = model
        self.S = len(systems)
        self.max_candidates = int(max_candidates)
        sizes = [len(s.types) for s in systems]
        self.offsets_np = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n_total = int(self.offsets_np[-1])
        self.sizes = np.asarray(sizes)
        self._offsets = (C.c_int64 * (self.S + 1))(*self.offsets_np.tolist())
        cells = np.concatenate([np.asarray(s.cell, dtype=np.float64).reshape(9) for s in systems])
        self._cells = (C.c_double * (9 * self.S))(*cells.tolist())
        pos = np.concatenate([np.asarray(s.pos, dtype=np.float64) for s in systems]).astype(np.float32)
        self.pos = torch.from_numpy(np.ascontiguousarray(pos.T)).to(device)
        self.types = torch.from_numpy(np.concatenate([s.types for s in systems]).astype(np.int32)).to(device)
        self.es = B.make_es(es)
        self.flags = (B.QNEP_BATCH_VIRIAL if virial else 0) | (B.QNEP_BATCH_GRADIENT if gradient else 0)
        self.cbatch = B.make_batch(self.S, self.flags, self._offsets, self._cells, self.pos.data_ptr(),
                                   self.types.data_ptr())
        nbytes = B.qnep_batch_workspace_size(model.handle, self.es, self.cbatch, self.max_candidates)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.device = self.pos.device
        s = torch.cuda.current_stream(self.device)
        B.qnep_batch_prepare(model.handle, self.es, self.cbatch, self.max_candidates, self.ws.data_ptr(),
                             self.ws.numel(), s.cuda_stream)
        self._stream = s

    def _args(self, thetas, E_ref, F_ref, lambdas, outputs):
        C_ = thetas.shape[0]
        assert thetas.dtype == torch.float32 and thetas.is_contiguous() and thetas.shape[1] == self.model.n_theta
        assert E_ref.dtype == torch.float64 and E_ref.numel() == self.S
        assert F_ref.dtype == torch.float32 and F_ref.shape == (3, self.n_total) and F_ref.is_contiguous()
        dev = self.device
        shapes = {"losses": ((self.S, C_, 3), torch.float32), "loss": ((C_,), torch.float64),
                  "energy": ((self.S, C_), torch.float64), "virial": ((self.S, C_, 9), torch.float64),
                  "forces": ((C_, 3, self.n_total), torch.float32), "charges": ((C_, self.n_total), torch.float32)}
        out = {k: torch.empty(shapes[k][0], dtype=shapes[k][1], device=dev) for k in ("losses",) + tuple(outputs)}
        lam = list(lambdas) + [0.0] * (5 - len(lambdas))
        tg = B.qnep_batch_targets(C.c_void_p(E_ref.data_ptr()), C.c_void_p(F_ref.data_ptr()), *[float(v) for v in lam])
        ptr = lambda k: C.c_void_p(out[k].data_ptr()) if k in out else None
        oc = B.qnep_batch_outputs(ptr("losses"), ptr("loss"), ptr("energy"), ptr("virial"), ptr("forces"),
                                  ptr("charges"))
        return C_, tg, oc, out

    def compute(self, thetas: torch.Tensor, E_ref: torch.Tensor, F_ref: torch.Tensor,
                lambdas=(1.0, 1.0, 1.0, 0.0, 0.0), outputs=("loss", "energy"),
                stream: Optional[torch.cuda.Stream] = None) -> Dict[str, torch.Tensor]:
        """thetas: float32 [C, n_theta]; E_ref float64 [S]; F_ref float32 [3, n_total]."""
        C_, tg, oc, out = self._args(thetas, E_ref, F_ref, lambdas, outputs)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        B.qnep_batch_compute(self.model.handle, thetas.data_ptr(), C_, tg, oc, self.ws.data_ptr(), self.ws.numel(),
                             s.cuda_stream)
        self._stream = s
        return out

    def gradient(self, thetas: torch.Tensor, E_ref: torch.Tensor, F_ref: torch.Tensor,
                 lambdas=(1.0, 1.0, 1.0, 0.0, 0.0), outputs=("loss",),
                 stream: Optional[torch.cuda.Stream] = None):
        """(outputs, dL/dtheta [C, n_theta]) for the total loss of every candidate."""
        C_, tg, oc, out = self._args(thetas, E_ref, F_ref, lambdas, outputs)
        d = torch.empty_like(thetas)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        B.qnep_batch_gradient(self.model.handle, thetas.data_ptr(), C_, tg, oc, d.data_ptr(), self.ws.data_ptr(),
                              self.ws.numel(), s.cuda_stream)
        self._stream = s
        return out, d

    def snes_generation(self, mu: torch.Tensor, sigma: torch.Tensor, noise: torch.Tensor, E_ref: torch.Tensor,
                        F_ref: torch.Tensor, lambdas=(1.0, 1.0, 1.0, 0.0, 0.0), eta_mu: float = 1.0,
                        eta_sigma: float = 0.0, outputs=("loss",),
                        stream: Optional[torch.cuda.Stream] = None) -> Dict[str, torch.Tensor]:
        """One SNES generation: mu, sigma (float32 [n_theta]) are updated in place from
        the population mu + sigma * noise (noise float32 [C, n_theta]); returns the
        outputs (``loss`` per member always) and the population under ``thetas``."""
        assert mu.dtype == torch.float32 and sigma.dtype == torch.float32 and noise.dtype == torch.float32
        assert mu.is_contiguous() and sigma.is_contiguous() and noise.is_contiguous()
        thetas = torch.empty_like(noise)
        outs = tuple(outputs) if "loss" in outputs else ("loss",) + tuple(outputs)
        C_, tg, oc, out = self._args(thetas, E_ref, F_ref, lambdas, outs)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        B.qnep_snes_generation(self.model.handle, mu.data_ptr(), sigma.data_ptr(), noise.data_ptr(), C_, eta_mu,
                               eta_sigma, tg, oc, thetas.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                               s.cuda_stream)
        self._stream = s
        out["thetas"] = thetas
        return out

    def tune(self, thetas, E_ref, F_ref, lambdas=(1.0, 1.0, 1.0, 0.0, 0.0)):
        """Autotunes lanes per atom (per size class) and workgroups per CU; returns the choice."""
        C_, tg, oc, out = self._args(thetas, E_ref, F_ref, lambdas, ("loss",))
        s = torch.cuda.current_stream(self.device)
        return B.qnep_batch_tune(self.model.handle, thetas.data_ptr(), C_, tg, oc, self.ws.data_ptr(),
                                 self.ws.numel(), s.cuda_stream)

    def check_status(self) -> int:
        return B.qnep_check_status(self.ws.data_ptr(), self._stream.cuda_stream)
