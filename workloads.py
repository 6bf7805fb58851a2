"""Seeded synthetic workloads shared by the tests, the smoke check and the
benchmark.  This module holds sizes, seeds and plain random-input
generators only; none of the method's arithmetic lives here.

Each configuration restates one benchmark system of the project:
  tfim10     1D transverse-field Ising, open chain N=10, J=h=1; 1D pRNN
             d_h=16; N_s=64; one step, lambda=1e-3, eta=0.01, mu=0
  tfim64     1D TFIM periodic N=64, J=h=1; 1D pRNN d_h=64 (13058 params);
             N_s=1024, N+1 connected configurations per sample; eta=0.05,
             lambda=1e-3, mu=0.7 (the N=200 step size 0.5 drives this
             smaller chain into the ferromagnetic product state)
  cluster100 periodic cluster chain -sum Z X Z, N=100; 1D cRNN d_h=128
             (50948 params); N_s=2048; checkpoints every 10 sites
  heis10x10  open 10x10 Heisenberg; 2D pRNN d_h=128 with Marshall sign and
             zero-magnetisation masking; N_s=4096; pseudo-inverse 1e-8
  j1j2batch  16 open J1-J2 (J2=0.5) lattices 6x6..12x12, 2D cRNN d_h=128,
             N_s 512..4096
Seeds: Philox key = 1000 + index, parameter seed = 2000 + index.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    Lx: int
    Ly: int
    dim: int
    H: int
    complex_head: bool
    marshall: bool
    zero_mag: bool
    ham: str
    J: float
    h: float
    J2: float
    pbc: bool
    Ns: int
    eta: float
    lam: float
    mu: float
    pinv_cutoff: float
    ckpt_every: int
    key: int
    seed: int
    E0: float = float("nan")          # exact ground energy where known


WORKLOADS = {
    "tfim10": Workload("tfim10", 10, 1, 1, 16, False, False, False, "tfim", 1.0, 1.0, 0.0, False,
                       64, 0.01, 1e-3, 0.0, 0.0, 1, 1001, 2001, -12.381489999654756),
    "tfim64": Workload("tfim64", 64, 1, 1, 64, False, False, False, "tfim", 1.0, 1.0, 0.0, True,
                       1024, 0.05, 1e-3, 0.7, 0.0, 1, 1002, 2002, -81.49551266892574),
    "cluster100": Workload("cluster100", 100, 1, 1, 128, True, False, False, "cluster", 1.0, 0.0, 0.0, True,
                           2048, 5e-3, 1e-3, 0.1, 0.0, 10, 1003, 2003, -100.0),
    "heis10x10": Workload("heis10x10", 10, 10, 2, 128, False, True, True, "j1j2", 1.0, 0.0, 0.0, False,
                          4096, 0.06, 0.0, 0.75, 1e-8, 10, 1004, 2004),
}


def j1j2_batch():
    """Instances k = 0..15 of the batched J1-J2 workload: L = 6 + k mod 7,
    N_s = 512 * 2^(k mod 4)."""
    out = []
    for k in range(16):
        L = 6 + (k % 7)
        out.append(Workload(f"j1j2_{k}", L, L, 2, 128, True, True, False, "j1j2", 1.0, 0.0, 0.5, False,
                            512 * 2 ** (k % 4), 0.1, 0.1, 0.1, 0.0, 1, 1005 + 100 * k, 2005 + 100 * k))
    return out


def random_configs(rng_seed, ns, n, zero_mag=False):
    """Uniformly random spin configurations (uint8, 0/1), optionally with
    exactly n/2 ones per row."""
    rng = np.random.default_rng(rng_seed)
    if not zero_mag:
        return rng.integers(0, 2, size=(ns, n), dtype=np.uint8)
    out = np.zeros((ns, n), dtype=np.uint8)
    for s in range(ns):
        out[s, rng.permutation(n)[: n // 2]] = 1
    return out


def random_vector(rng_seed, n, scale=1.0):
    return np.random.default_rng(rng_seed).normal(size=n) * scale
