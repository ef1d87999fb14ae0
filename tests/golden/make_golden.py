"""Writes the stored Poisson data of the synthetic workloads.

For each workload: l1 = A1 f_true with the oracle (C = 1), the calibration
constant C = 1e4 / max(l1) (counts scaled to a maximum mean of 1e4), and
integer counts y ~ Poisson(C l1) with the workload's noise seed; and the work
census of the workload's geometry.  Calls only ``oracle`` and the seeded input
generators.

    python tests/golden/make_golden.py [slice32 slice128 ... batch64]

``batch64`` writes only the per-scan work census of the 64-scan uneven batch
(its counts are drawn at run time).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1603_06400_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def make(name: str) -> str:
    w = inputs.workload(name)
    f = inputs.phantom(w.geom, w.phantom_seed, w.n_rect)
    l1 = oracle.Oracle(w.geom.with_(C=1.0)).forward(f)
    C = 1e4 / float(l1.max())
    y = inputs.poisson_counts(C * l1, w.noise_seed)
    path = os.path.join(HERE, f"{name}_counts.npz")
    np.savez_compressed(path, y=y.astype(np.float32), C=np.float64(C), l1_max=np.float64(l1.max()))
    return path


def census(name: str) -> str:
    """Work census of the direct evaluation (pairs, pairs with an open mask
    cell, open triples whose Bragg energy falls in the spectrum band)."""
    w = inputs.workload(name)
    c = oracle.Oracle(w.geom).census()
    c = {k: float(v) for k, v in c.items()}
    c.update(workload=name, nvox=w.geom.nvox, npix=w.geom.npix, nq=w.geom.nq)
    path = os.path.join(HERE, f"{name}_census.json")
    with open(path, "w") as fh:
        json.dump(c, fh, indent=1)
    return path


def batch_census(n_scans: int = 64) -> str:
    """Per-scan work census of the uneven batch (same fields as census())."""
    out = []
    for s in inputs.batch_scans(n_scans):
        c = {k: float(v) for k, v in oracle.Oracle(s.geom).census().items()}
        c.update(n=s.geom.nx, nvox=s.geom.nvox, npix=s.geom.npix, nq=s.geom.nq,
                 phantom_seed=s.phantom_seed)
        out.append(c)
    path = os.path.join(HERE, f"batch{n_scans}_census.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    return path


if __name__ == "__main__":
    for n in (sys.argv[1:] or ["slice32", "slice128", "slice128_open1", "slice128_open01", "batch64"]):
        if n.startswith("batch"):
            print(batch_census(int(n[5:])))
            continue
        print(make(n))
        print(census(n))
