"""Independent references for pinning the oracle: dense Hamiltonians built
from Kronecker products of Pauli matrices, exact enumeration of all
configurations, exact diagonalisation and closed forms.  Nothing here calls
the oracle's local-energy or Jacobian code."""
import itertools

import numpy as np

X = np.array([[0.0, 1.0], [1.0, 0.0]])
Y = np.array([[0.0, -1j], [1j, 0.0]])
Z = np.array([[1.0, 0.0], [0.0, -1.0]])   # basis state 0 is z = +1
I2 = np.eye(2)


def all_configs(N):
    """All 2^N configurations, row b has bit k of b (MSB first) at position k."""
    return np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.int64)


def op_on(N, ops):
    """Kronecker product with ops = {position: 2x2 matrix}, identity elsewhere."""
    m = np.array([[1.0 + 0j]])
    for k in range(N):
        m = np.kron(m, ops.get(k, I2))
    return m


def dense_tfim(N, J, h, pbc):
    H = np.zeros((2 ** N, 2 ** N), dtype=complex)
    bonds = [(i, i + 1) for i in range(N - 1)] + ([(N - 1, 0)] if pbc and N > 2 else [])
    for a, b in bonds:
        H -= J * op_on(N, {a: Z, b: Z})
    for i in range(N):
        H -= h * op_on(N, {i: X})
    return H


def dense_cluster_pbc(N):
    H = np.zeros((2 ** N, 2 ** N), dtype=complex)
    for i in range(N):
        H -= op_on(N, {(i - 1) % N: Z, i: X, (i + 1) % N: Z})
    return H


def lattice_bonds(Lx, Ly, pidx):
    """NN and NNN bonds of the open Lx x Ly lattice as path-index pairs;
    pidx(i, j) maps lattice coordinates to path positions."""
    nn, nnn = [], []
    for j in range(Ly):
        for i in range(Lx):
            for (di, dj, lst) in ((1, 0, nn), (0, 1, nn), (1, 1, nnn), (-1, 1, nnn)):
                i2, j2 = i + di, j + dj
                if 0 <= i2 < Lx and 0 <= j2 < Ly:
                    lst.append((pidx(i, j), pidx(i2, j2)))
    return nn, nnn


def snake(Lx):
    return lambda i, j: j * Lx + (i if j % 2 == 0 else Lx - 1 - i)


def dense_j1j2(Lx, Ly, J1, J2):
    N = Lx * Ly
    nn, nnn = lattice_bonds(Lx, Ly, snake(Lx))
    H = np.zeros((2 ** N, 2 ** N), dtype=complex)
    for J, bl in ((J1, nn), (J2, nnn)):
        for a, b in bl:
            for P in (X, Y, Z):
                H += (J / 4.0) * op_on(N, {a: P, b: P})
    return H


def tfim_obc_free_fermion(N, J=1.0, h=1.0):
    """Ground energy of the open TFIM from its free-fermion solution:
    E0 = -sum of the singular values of the N x N bidiagonal matrix with h
    on the diagonal and J on the superdiagonal, times 1 (Pfeuty 1970)."""
    M = np.diag(np.full(N, h)) + np.diag(np.full(N - 1, J), 1)
    return -np.sum(np.linalg.svd(M, compute_uv=False))


def tfim_pbc_critical(N):
    """Ground energy of the periodic critical chain (J = h = 1)."""
    return -2.0 / np.sin(np.pi / (2 * N))
