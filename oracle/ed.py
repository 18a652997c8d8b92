"""Exact-diagonalisation Hamiltonians used to pin the oracle (oracle).

These are built from the model definitions directly (Kronecker products of
local operators, or fermionic Fock-space operators), never from an MPO, so
that an MPO or contraction mistake cannot cancel against them.
"""
from __future__ import annotations

import itertools
import math
from typing import List, Tuple

import numpy as np

from paper_2007_14822_amd.inputs import aklt_bond_operator, cylinder_bonds, spin_ops


def _site_op(op: np.ndarray, i: int, N: int) -> np.ndarray:
    d = op.shape[0]
    out = np.array([[1.0]])
    for k in range(N):
        out = np.kron(out, op if k == i else np.eye(d))
    return out


def heisenberg_dense(N: int, two_s: int = 1, J: float = 1.0) -> np.ndarray:
    """H = J sum_i S_i . S_{i+1} (Eq. Heis of Sec. 7.1), open chain."""
    o = spin_ops(two_s)
    d = two_s + 1
    H = np.zeros((d ** N, d ** N))
    for i in range(N - 1):
        H += J * (_site_op(o["Sz"], i, N) @ _site_op(o["Sz"], i + 1, N))
        H += 0.5 * J * (_site_op(o["S+"], i, N) @ _site_op(o["S-"], i + 1, N))
        H += 0.5 * J * (_site_op(o["S-"], i, N) @ _site_op(o["S+"], i + 1, N))
    return H


def aklt_dense(N: int) -> np.ndarray:
    h = aklt_bond_operator()
    d = 3
    H = np.zeros((d ** N, d ** N))
    for i in range(N - 1):
        H += np.kron(np.kron(np.eye(d ** i), h), np.eye(d ** (N - i - 2)))
    return H


# ----------------------------------------------------------------------------
# Fermions: modes ordered (site 0 up, site 0 dn, site 1 up, ...)
# ----------------------------------------------------------------------------
def _mode_annihilators(nmodes: int) -> List[np.ndarray]:
    """Jordan-Wigner annihilators on 2^nmodes, mode 0 most significant."""
    a = np.array([[0.0, 1.0], [0.0, 0.0]])  # |0> <- |1>, basis (|0>, |1>)
    z = np.diag([1.0, -1.0])
    out = []
    for j in range(nmodes):
        op = np.array([[1.0]])
        for k in range(nmodes):
            op = np.kron(op, z if k < j else (a if k == j else np.eye(2)))
        out.append(op)
    return out


def hubbard_dense(Lx: int, Ly: int, t: float = 1.0, U: float = 8.0) -> np.ndarray:
    """Full Fock-space Hubbard Hamiltonian on the cylinder (column-major
    sites), modes ordered up-then-down on each site, returned in the site
    basis (|0>, |up>, |dn>, |up dn>) of the MPO inputs."""
    return hubbard_dense_bonds(Lx * Ly, cylinder_bonds(Lx, Ly), t, U)


def hubbard_dense_bonds(N: int, bonds, t: float = 1.0, U: float = 8.0) -> np.ndarray:
    """As hubbard_dense for an explicit list of hopping bonds (i < j)."""
    c = _mode_annihilators(2 * N)
    dim = 4 ** N
    H = np.zeros((dim, dim))
    for (i, j) in bonds:
        for s in range(2):
            ci, cj = c[2 * i + s], c[2 * j + s]
            H += -t * (ci.T @ cj + cj.T @ ci)
    for i in range(N):
        nu = c[2 * i].T @ c[2 * i]
        nd = c[2 * i + 1].T @ c[2 * i + 1]
        H += U * nu @ nd
    # The Kronecker basis of the two modes of a site, up mode more
    # significant, is (|0>, |dn>, |up>, |up dn>) with |up dn> = c+_up c+_dn|0>;
    # reorder every site to (|0>, |up>, |dn>, |up dn>) (a pure permutation).
    loc = [0, 2, 1, 3]
    perm = np.zeros(dim, dtype=np.int64)
    for k in range(dim):
        digits = [(k // 4 ** (N - 1 - i)) % 4 for i in range(N)]
        perm[k] = sum(loc[dg] * 4 ** (N - 1 - i) for i, dg in enumerate(digits))
    return H[np.ix_(perm, perm)]


def hubbard_sector_ground_energy(Lx: int, Ly: int, n_up: int, n_dn: int,
                                 t: float = 1.0, U: float = 8.0) -> float:
    """Lowest eigenvalue in the sector (N_up, N_dn) by building the sector
    Hamiltonian from occupation bit strings (mode 0 = most significant bit,
    modes ordered (site, spin) as above)."""
    N = Lx * Ly
    M = 2 * N
    states = []
    for bits in range(1 << M):
        nu = sum((bits >> (M - 1 - (2 * i))) & 1 for i in range(N))
        nd = sum((bits >> (M - 1 - (2 * i + 1))) & 1 for i in range(N))
        if nu == n_up and nd == n_dn:
            states.append(bits)
    index = {s: k for k, s in enumerate(states)}
    H = np.zeros((len(states), len(states)))

    def occ(bits, mode):
        return (bits >> (M - 1 - mode)) & 1

    def sign_before(bits, mode):
        # number of occupied modes strictly before `mode`
        cnt = 0
        for k in range(mode):
            cnt += occ(bits, k)
        return -1.0 if cnt % 2 else 1.0

    for k, s in enumerate(states):
        for i in range(N):
            if occ(s, 2 * i) and occ(s, 2 * i + 1):
                H[k, k] += U
        for (i, j) in cylinder_bonds(Lx, Ly):
            for sp in range(2):
                for (p, q) in ((2 * i + sp, 2 * j + sp), (2 * j + sp, 2 * i + sp)):
                    # c+_p c_q |s>
                    if not occ(s, q) or (occ(s, p) and p != q):
                        continue
                    sg = sign_before(s, q)
                    s1 = s ^ (1 << (M - 1 - q))
                    if occ(s1, p):
                        continue
                    sg *= sign_before(s1, p)
                    s2 = s1 | (1 << (M - 1 - p))
                    H[index[s2], k] += -t * sg
    return float(np.linalg.eigvalsh(H)[0])


def free_fermion_cylinder_energy(Lx: int, Ly: int, n_up: int, n_dn: int, t: float = 1.0) -> float:
    """U = 0 closed form: single-particle levels
    eps(n, m) = -2t cos(pi n / (Lx+1)) - 2t cos(2 pi m / Ly)
    (open in x, periodic in y); fill the lowest levels of each spin."""
    eps = []
    for n in range(1, Lx + 1):
        for m in range(Ly):
            ex = -2.0 * t * math.cos(math.pi * n / (Lx + 1))
            if Ly == 1:
                ey = 0.0
            elif Ly == 2:
                ey = -t * math.cos(math.pi * m)  # a single bond in y
            else:
                ey = -2.0 * t * math.cos(2.0 * math.pi * m / Ly)
            eps.append(ex + ey)
    eps.sort()
    return float(sum(eps[:n_up]) + sum(eps[:n_dn]))
