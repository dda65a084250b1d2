"""Writes perovskite975560_oracle.npz: the FP64 oracle on the full 975,560-atom
perovskite workload (58^3 cells, PPPM 256^3, order 5, alpha 0.3, rc 9 A) — the global
outputs and every per-atom output at 512 seeded sample atoms.  Calls only the oracle
and the seeded input generator; takes a few minutes on 8 cores.

    python tests/golden/make_perovskite975560.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2601_19034_amd import inputs  # noqa: E402

N_SAMPLE = 512


def input_digest(sysm, theta) -> str:
    h = hashlib.sha256()
    for a in (sysm.pos, sysm.types, sysm.cell, theta):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    oracle.build(force=False)
    w = inputs.workload(3, "full")
    s = w.system
    r = oracle.compute(w.hp, w.es, s.pos, s.types, s.cell, w.theta, cells=True)
    idx = np.sort(np.random.default_rng(975560).choice(s.n, N_SAMPLE, replace=False))
    np.savez_compressed(
        os.path.join(HERE, "perovskite975560_oracle.npz"),
        digest=np.array(input_digest(s, w.theta)), n=np.array(s.n), energy=np.array(r.energy), terms=r.terms,
        virial=r.virial, pol=r.pol, idx=idx, forces=r.forces[idx], q_screened=r.q_screened[idx],
        q_naked=r.q_naked[idx], bec=r.bec[idx], phi=r.phi[idx], sum_abs_qnaked=np.array(np.abs(r.q_naked).sum()))
    print("energy", r.energy, "samples", N_SAMPLE)


if __name__ == "__main__":
    main()
