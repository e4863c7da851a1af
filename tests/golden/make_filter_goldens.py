"""Writes the oracle's end-to-end filter results that the GPU filter tests compare against.

Every value stored here comes from the FP64 CPU oracle (``oracle.filter.run_filter``: the Sec. 2.2.2
procedure with the Sec. 6 local restart) on seeded synthetic inputs from
``paper_2509_16896_amd.workloads`` (truth and observation paths only; that module holds none of the
filter's arithmetic).  Nothing is read from the GPU library.

    python tests/golden/make_filter_goldens.py [name ...]

Cases (each file ``filter_<name>.npz`` holds the per-step posterior means, logZ_k, ESS and clamp
counts, plus the workload's sizes for a consistency check):

* ``cubic_r1000_n4096``  -- the r = 1000 cubic sensor with n reduced to 4096, all 50 steps;
* ``cubic_r100_n16384``  -- the r = 100 cubic sensor, all 100 steps;
* ``batch64_run<b>``     -- runs of the 64-run batch workload (r ~ U{10..200}, n = 2^U{11..15}),
  all 100 steps, for the cheapest runs and two with r above the matrix-core K step;
* ``batch6_run<b>``      -- the six uneven runs of the batch tests over 8 steps.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import filter as ofilter  # noqa: E402
from paper_2509_16896_amd import workloads as W  # noqa: E402

# runs of batch_runs(64) whose oracle finishes in minutes: the four cheapest (r = 11, 19, 24, 25 at
# n = 2048) and two above one 32-wide K step (r = 68 and 115 at n = 2048)
BATCH64_RUNS = (21, 48, 3, 53, 2, 13)
# the six uneven runs of tests/test_gpu_batch.py (r, n), K = 8
BATCH6_SHAPES = ((10, 2048), (33, 1024), (64, 4096), (100, 2048), (150, 1024), (200, 8192))


def batch6_workloads(K: int = 8):
    out = []
    for b, (r, n) in enumerate(BATCH6_SHAPES):
        out.append(W.Workload(f"batch_r{r}_n{n}", r=r, n=n, dt=0.01, K=K, drift=W.F_COS, obs=W.H_CUBE, q=0.09,
                              rho2=0.09, scales=(1.0, 2.0, 4.0), box_half=0.3 + 0.1 * b, restart_every=2, R=0.3,
                              seed=b + 1))
    return out


def cases():
    out = {
        "cubic_r1000_n4096": W.shrink(W.cubic_r1000(), n=4096, name="cubic_r1000_n4096"),
        "cubic_r100_n16384": W.cubic_r100(),
    }
    runs = W.batch_runs(64)
    for b in BATCH64_RUNS:
        out[f"batch64_run{b}"] = runs[b]
    for b, w in enumerate(batch6_workloads()):
        out[f"batch6_run{b}"] = w
    return out


def path_of(name: str) -> str:
    return os.path.join(HERE, f"filter_{name}.npz")


def write(name: str, w) -> None:
    t0 = time.time()
    _, dys = W.simulate(w)
    ref = ofilter.run_filter(w, dys)
    np.savez_compressed(path_of(name), means=ref["means"], logZ=ref["logZ"], ess=ref["ess"],
                        clamps=ref["clamps"], r=w.r, n=w.n, K=w.K, dt=w.dt, seed=w.seed)
    print(f"{name}: r={w.r} n={w.n} K={w.K} in {time.time() - t0:.0f} s", flush=True)


def main(argv):
    oracle.build(force=False)
    todo = cases()
    names = argv or list(todo)
    for name in names:
        write(name, todo[name])


if __name__ == "__main__":
    main(sys.argv[1:])
