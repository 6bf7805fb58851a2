"""Connected configurations and local energies.

Local energy (Sec. 2.3):  eps(sigma) = sum_{sigma'} H_{sigma sigma'} Psi(sigma') / Psi(sigma).

Hamiltonians (spin value 0 <-> z = +1, z = 1 - 2 sigma):
  * TFIM (Sec. 3.1):  -J sum_b Z_a Z_b - h sum_i X_i; bonds (i, i+1), plus
    (N-1, 0) with periodic boundaries.  Off-diagonal: single flip i, -h.
  * cluster (periodic form -sum_i Z_{i-1} X_i Z_{i+1}; Sec. 3.2 uses an open
    chain with boundary terms, this project uses the periodic chain):
    flip i with element -z_{i-1} z_{i+1}, read on the unflipped neighbours.
  * J1-J2 on an open square lattice (Sec. 3.3):  (J_b/4) sigma_a . sigma_b
    per bond; diagonal (J_b/4) z_a z_b, exchange of an antiparallel pair
    with element J_b/2.  J2 = 0 is the Heisenberg model.

Each off-diagonal amplitude ratio is obtained by evaluating log Psi of the
whole flipped configuration from scratch (no prefix sharing) and
exponentiating the difference.
"""
from dataclasses import dataclass

import numpy as np

from . import model


@dataclass(frozen=True)
class Ham:
    kind: str              # "tfim", "cluster", "j1j2"
    J: float = 1.0         # TFIM J, J1-J2 J1
    h: float = 1.0         # TFIM transverse field
    J2: float = 0.0        # J1-J2 next-nearest coupling
    pbc: bool = False      # TFIM boundary; cluster is always periodic


def bonds_2d(spec):
    """Nearest and next-nearest bonds of the open Lx x Ly lattice, as pairs
    of path positions."""
    nn, nnn = [], []
    for j in range(spec.Ly):
        for i in range(spec.Lx):
            a = model.path_index(spec, i, j)
            if i + 1 < spec.Lx:
                nn.append((a, model.path_index(spec, i + 1, j)))
            if j + 1 < spec.Ly:
                nn.append((a, model.path_index(spec, i, j + 1)))
            if i + 1 < spec.Lx and j + 1 < spec.Ly:
                nnn.append((a, model.path_index(spec, i + 1, j + 1)))
            if i - 1 >= 0 and j + 1 < spec.Ly:
                nnn.append((a, model.path_index(spec, i - 1, j + 1)))
    return nn, nnn


def terms(spec, ham, sigma):
    """Diagonal element (Ns,) and list of (flip positions, element (Ns,))."""
    sigma = np.asarray(sigma, dtype=np.int64)
    z = 1.0 - 2.0 * sigma
    N = spec.N
    off = []
    if ham.kind == "tfim":
        bonds = [(i, i + 1) for i in range(N - 1)]
        if ham.pbc and N > 2:
            bonds.append((N - 1, 0))
        diag = -ham.J * sum(z[:, a] * z[:, b] for a, b in bonds)
        for i in range(N):
            off.append(((i,), np.full(sigma.shape[0], -ham.h)))
    elif ham.kind == "cluster":
        diag = np.zeros(sigma.shape[0])
        for i in range(N):
            off.append(((i,), -z[:, (i - 1) % N] * z[:, (i + 1) % N]))
    elif ham.kind == "j1j2":
        nn, nnn = bonds_2d(spec)
        diag = np.zeros(sigma.shape[0])
        for J, bl in ((ham.J, nn), (ham.J2, nnn)):
            if J == 0.0:
                continue
            for a, b in bl:
                diag = diag + (J / 4.0) * z[:, a] * z[:, b]
                anti = sigma[:, a] != sigma[:, b]
                off.append(((a, b), np.where(anti, J / 2.0, 0.0)))
    else:
        raise ValueError(ham.kind)
    return diag, off


def local_energy(spec, theta, ham, sigma, logpsi=None):
    """eps(sigma) (Ns,) complex128."""
    sigma = np.asarray(sigma, dtype=np.int64)
    if logpsi is None:
        logpsi = model.log_psi(spec, theta, sigma)
    diag, off = terms(spec, ham, sigma)
    eps = diag.astype(np.complex128)
    for flips, mel in off:
        nz = mel != 0.0
        if not np.any(nz):
            continue
        sp = sigma[nz].copy()
        for f in flips:
            sp[:, f] = 1 - sp[:, f]
        lp2 = model.log_psi(spec, theta, sp)
        eps[nz] += mel[nz] * np.exp(lp2 - logpsi[nz])
    return eps
