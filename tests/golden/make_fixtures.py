"""Writes FP64 oracle fixtures for the GPU tests and the benchmark's error report.
Calls only the oracle and the seeded input generator.

    python tests/golden/make_fixtures.py [name ...]

  garnet153600       garnet-like box, 153,600 atoms, PPPM 128^3: global outputs and
                     every per-atom output at 512 seeded sample atoms (about a minute)
  water24000_ewald   water-like box, 24,000 atoms, direct Ewald with kmax = 2 pi alpha
                     (27,200 wave vectors): the same (about a minute on 8 cores)
  perovskite5000     the 5,000-atom perovskite crop, PPPM 45^3: every output of every
                     atom (the per-form errors of the benchmark)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from make_perovskite975560 import input_digest  # noqa: E402
from paper_2601_19034_amd import inputs  # noqa: E402

N_SAMPLE = 512


def workload(name):
    if name == "garnet153600":
        return inputs.workload(2, "full")
    if name == "water24000_ewald":
        w = inputs.workload(1, "full")
        w.es.method = 0  # alpha 0.3, rc 9 A, kmax = 2 pi alpha (the PPPM fields stay unused)
        return w
    if name == "perovskite5000":
        return inputs.workload(3, "crop")
    raise ValueError(name)


def write(name):
    w = workload(name)
    s = w.system
    r = oracle.compute(w.hp, w.es, s.pos, s.types, s.cell, w.theta, cells=True)
    common = dict(digest=np.array(input_digest(s, w.theta)), n=np.array(s.n), energy=np.array(r.energy),
                  terms=r.terms, virial=r.virial, pol=r.pol)
    if name == "perovskite5000":
        np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), forces=r.forces, q_naked=r.q_naked,
                            bec=r.bec, **common)
    else:
        idx = np.sort(np.random.default_rng(s.n).choice(s.n, N_SAMPLE, replace=False))
        np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), idx=idx, forces=r.forces[idx],
                            q_screened=r.q_screened[idx], q_naked=r.q_naked[idx], bec=r.bec[idx], **common)
    print(name, "energy", r.energy, "k vectors", r.terms[9])


if __name__ == "__main__":
    oracle.build(force=False)
    for nm in sys.argv[1:] or ["perovskite5000", "garnet153600", "water24000_ewald"]:
        write(nm)
