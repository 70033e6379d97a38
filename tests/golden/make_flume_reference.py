"""Write the stored oracle reference of one full-size wave flume (2048 x 512).

The oracle (FP64, single thread) needs about ten minutes for two steps of one
2048 x 512 flume of the 16-sample flume batch (its first amplitude), too long
for a GPU test run, so this script runs
it once and stores what the GPU test compares against: the values of every
state field at seeded samples of cells and faces, the fields' full L2 norms,
and the oracle's solver statistics.  Inputs come from the seeded workload
generator; only the oracle computes the stored values.

    python tests/golden/make_flume_reference.py   (writes flume2048_2steps.npz)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.join(ROOT, "oracle")]

import oracle as O  # noqa: E402
from paper_2003_08374_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "flume2048_2steps.npz")
NSTEPS = 2
NSAMPLE = 4096


def case():
    """The first sample of the 16-sample flume batch (amplitudes seed 7):
    2048 x 512 cells of 5 mm, dt 1 ms."""
    return W.flume_batch(16)[0]


def main():
    c = case()
    nc = c.ncells
    nf = sum(O.nfaces(c.shape))
    rng = np.random.default_rng(12345)
    cells = np.sort(rng.choice(nc, NSAMPLE, replace=False))
    faces = np.sort(rng.choice(nf, NSAMPLE, replace=False))
    t0 = time.time()
    out, info = O.step(c.replace(p_tol=1e-14, p_maxit=200000), O.initial_state(c), NSTEPS)
    F = np.concatenate(out["F"])
    np.savez_compressed(
        OUT, cells=cells, faces=faces, nsteps=NSTEPS,
        alpha=out["alpha"][cells], U=out["U"][:, cells], p_rgh=out["p_rgh"][cells],
        p=out["p"][cells], F=F[faces],
        norm_alpha=np.linalg.norm(out["alpha"]), norm_U=np.linalg.norm(out["U"]),
        norm_p_rgh=np.linalg.norm(out["p_rgh"]), norm_F=np.linalg.norm(F),
        p_iters=np.array(info["p_iters"]), mom_sweeps=info["mom_sweeps"],
        max_div=info["max_div"], oracle_seconds=time.time() - t0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s; p_iters {info['p_iters']}")


if __name__ == "__main__":
    main()
