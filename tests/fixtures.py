"""Readers of the stored test fixtures under tests/golden."""
import os

import numpy as np

import sr_inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_mask_fd():
    """The stored FP64 central differences (tests/golden/mask_fd_128.txt,
    written by tests/golden/make_mask_fd.py from the oracle alone) and the
    inputs and directions they were taken on, regenerated from their seeds."""
    loss, fd = None, {}
    with open(os.path.join(GOLDEN, "mask_fd_128.txt")) as f:
        for line in f:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "loss":
                loss = float(p[1])
            elif p[0] == "fd":
                fd[int(p[1])] = float(p[2])
    d = sr_inputs.mask_design(3)
    dirs = sr_inputs.fd_directions(128, len(fd), d["theta"].shape)
    return d, loss, np.array([fd[k] for k in range(len(fd))]), dirs
