"""Shared builders for tests: one seeded workload fed to both the oracle and the GPU path."""
from __future__ import annotations

import math

import numpy as np

import workloads as W

FP64_TOL = 1e-10   # relative L2 bar for the FP64 path


def lattice_case(n, jitter=0.2, seed=11, lo=(0.0, 0.0), hi=(1.0, 1.0), rfac=2.0):
    x, dx = W.jittered_lattice((n, n), lo, hi, jitter, seed)
    R = np.full(x.shape[0], rfac * dx)
    return x, R, dx


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def absorber_dir(theta=0.3):
    return math.cos(theta), math.sin(theta)
