"""Writes mask_fd_128.txt: FP64 central finite differences of the
mask-design objective at the mask-design workload's shapes.

The objective (the mean phase-aligned relative squared error after 20
unrolled GD steps of Eq. (2), on intensities of Eq. (1)) is evaluated by the
FP64 oracle only, on the first two problems of the seeded mask-design inputs
(128^2 signals padded to 256^2, L = 2, shared masks), at theta +- eps d for
32 seeded N(0,1) directions d and eps = 1e-6.  Each evaluation takes seconds,
so the values are stored; the tests regenerate the same inputs and
directions from the same seeds.

Usage: python tests/golden/make_mask_fd.py [workers]
"""
from __future__ import annotations

import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import sr_inputs  # noqa: E402

SEED_INPUTS = 3     # sr_inputs.mask_design seed
SEED_DIRS = 128     # sr_inputs.fd_directions seed
NDIR = 32
NPROB = 2
EPS = 1e-6
OUT = os.path.join(HERE, "mask_fd_128.txt")


def case():
    d = sr_inputs.mask_design(SEED_INPUTS)
    th = d["theta"].astype(np.float64)
    dirs = sr_inputs.fd_directions(SEED_DIRS, NDIR, th.shape)
    return d, th, dirs


def _loss(args):
    k, sign = args
    d, th, dirs = case()
    t = th + sign * EPS * dirs[k]
    return oracle.unrolled_gd_loss(t, d["x_star"][:NPROB], d["x0"][:NPROB], d["steps"], d["mu"])


def main(workers: int) -> None:
    d, th, dirs = case()
    jobs = [(k, s) for k in range(NDIR) for s in (1.0, -1.0)]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        vals = list(ex.map(_loss, jobs))
    loss = oracle.unrolled_gd_loss(th, d["x_star"][:NPROB], d["x0"][:NPROB], d["steps"], d["mu"])
    with open(OUT, "w") as f:
        f.write("# Central finite differences (l(theta + eps d) - l(theta - eps d)) / (2 eps) of the\n")
        f.write("# mask-design objective (mean phase-aligned relative squared error after unrolled GD,\n")
        f.write("# Eq. (2) on y = |A x*|^2 of Eq. (1)), FP64 oracle, written by make_mask_fd.py.\n")
        f.write(f"# inputs: sr_inputs.mask_design({SEED_INPUTS}), first {NPROB} problems, "
                f"{d['steps']} steps, mu {d['mu']}\n")
        f.write(f"# directions: sr_inputs.fd_directions({SEED_DIRS}, {NDIR}, theta.shape); eps {EPS}\n")
        f.write(f"loss {float(loss)!r}\n")
        for k in range(NDIR):
            fd = (vals[2 * k] - vals[2 * k + 1]) / (2 * EPS)
            f.write(f"fd {k} {float(fd)!r}\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else min(8, os.cpu_count() or 1))
