"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only *specifies problems*: local operator matrices, the MPO
tensors of the model Hamiltonians, random MPS tensors and QN sector tables.
It contains none of the arithmetic of the effective-Hamiltonian method
(no environment, no matvec, no block selection by flux), so that the oracle
and the GPU library can share it without sharing method code.

Conventions (the paper's MPS formula in Sec. 7.3 and the operator element
convention of the hard-core boson example in Sec. 8.3):
  * MPS site tensor   A[a_{i-1}, s_i, a_i]
  * MPO site tensor   W[m_{i-1}, m_i, s', s]   with op[s', s] = <s'|op|s>
  * Lower-triangular finite-state MPOs: the left boundary selects the last
    MPO channel (w-1, "nothing placed yet") and the right boundary selects
    channel 0 ("every term completed").
  * Spin basis: highest S^z first (the S=3/2 operator listing of Sec. 10.2).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

BASE_SEED = 14822


def seed_for(config: int, chi: int) -> int:
    """Seed of a workload: 14822 + 1000*config + chi."""
    return BASE_SEED + 1000 * int(config) + int(chi)


def rng_for(config: int, chi: int) -> np.random.Generator:
    return np.random.default_rng(seed_for(config, chi))


# ----------------------------------------------------------------------------
# Local operators
# ----------------------------------------------------------------------------
def spin_ops(two_s: int) -> Dict[str, np.ndarray]:
    """Spin-S operators, basis m = S, S-1, ..., -S (highest S^z first)."""
    d = two_s + 1
    S = two_s / 2.0
    m = np.array([S - k for k in range(d)])
    Sz = np.diag(m)
    Sp = np.zeros((d, d))
    for k in range(1, d):
        # <m+1| S+ |m> = sqrt(S(S+1) - m(m+1)); row k-1 holds m+1
        mm = m[k]
        Sp[k - 1, k] = math.sqrt(S * (S + 1) - mm * (mm + 1))
    Sm = Sp.T.copy()
    return {"Sz": Sz, "S+": Sp, "S-": Sm, "Id": np.eye(d)}


def hubbard_ops() -> Dict[str, np.ndarray]:
    """Spinful-fermion site, basis (|0>, |up>, |dn>, |up dn>) with
    |up dn> = c+_up c+_dn |0>  (up mode ordered before dn within a site).

    The annihilators are site-local: they carry the sign of the modes that
    precede them *on the same site* but no Jordan-Wigner string from other
    sites; F = (-1)^(n_up + n_dn) is that string's per-site factor.
    """
    Cup = np.zeros((4, 4))
    Cdn = np.zeros((4, 4))
    # c_up |up> = |0>;  c_up |up dn> = c_up c+_up c+_dn|0> = |dn>
    Cup[0, 1] = 1.0
    Cup[2, 3] = 1.0
    # c_dn |dn> = |0>;  c_dn |up dn> = c_dn c+_up c+_dn |0> = -c+_up c_dn c+_dn|0> = -|up>
    Cdn[0, 2] = 1.0
    Cdn[1, 3] = -1.0
    Nup = np.diag([0.0, 1.0, 0.0, 1.0])
    Ndn = np.diag([0.0, 0.0, 1.0, 1.0])
    F = np.diag([1.0, -1.0, -1.0, 1.0])
    return {
        "Id": np.eye(4), "F": F, "Cup": Cup, "Cdn": Cdn,
        "Cdagup": Cup.T.copy(), "Cdagdn": Cdn.T.copy(),
        "Nup": Nup, "Ndn": Ndn, "Nupdn": Nup @ Ndn,
    }


# ----------------------------------------------------------------------------
# MPOs (problem definitions; each is checked against exact diagonalisation)
# ----------------------------------------------------------------------------
def heisenberg_mpo(N: int, two_s: int = 1, J: float = 1.0) -> List[np.ndarray]:
    """Nearest-neighbour Heisenberg chain, the bond-dimension-5 MPO of
    Eq. (Heis) in Sec. 7.1:  H = sum_i Sz Sz + 1/2 (S+ S- + S- S+)."""
    o = spin_ops(two_s)
    d = two_s + 1
    w = 5
    W = np.zeros((w, w, d, d))
    W[0, 0] = o["Id"]
    W[1, 0] = o["S+"]
    W[2, 0] = o["S-"]
    W[3, 0] = o["Sz"]
    W[4, 1] = 0.5 * J * o["S-"]
    W[4, 2] = 0.5 * J * o["S+"]
    W[4, 3] = J * o["Sz"]
    W[4, 4] = o["Id"]
    return [W.copy() for _ in range(N)]


def aklt_bond_operator() -> np.ndarray:
    """h = S.S + (S.S)^2 / 3 for two spin-1 sites, as a (9 x 9) matrix on
    |s1 s2> (row = s1' s2')."""
    o = spin_ops(2)
    ss = (np.kron(o["Sz"], o["Sz"]) + 0.5 * np.kron(o["S+"], o["S-"])
          + 0.5 * np.kron(o["S-"], o["S+"]))
    return ss + ss @ ss / 3.0


def aklt_mpo(N: int) -> List[np.ndarray]:
    """Spin-1 AKLT chain H = sum_i h_{i,i+1} as a lower-triangular MPO.

    The bond operator is written as sum_k P_k (x) Q_k by an operator-Schmidt
    decomposition (rank 9), giving w = 2 + 9 = 11.
    """
    d = 3
    h = aklt_bond_operator().reshape(d, d, d, d)  # [s1', s2', s1, s2]
    # regroup to (s1' s1) x (s2' s2)
    M = h.transpose(0, 2, 1, 3).reshape(d * d, d * d)
    U, s, Vt = np.linalg.svd(M)
    r = int(np.sum(s > 1e-12 * s[0]))
    w = r + 2
    W = np.zeros((w, w, d, d))
    W[0, 0] = np.eye(d)
    W[w - 1, w - 1] = np.eye(d)
    for k in range(r):
        P = (U[:, k] * s[k]).reshape(d, d)
        Q = Vt[k].reshape(d, d)
        W[w - 1, 1 + k] = P
        W[1 + k, 0] = Q
    return [W.copy() for _ in range(N)]


def cylinder_bonds(Lx: int, Ly: int) -> List[Tuple[int, int]]:
    """Nearest-neighbour bonds of an Lx x Ly cylinder (open in x, periodic
    in y for Ly > 2) in column-major ("snaked") order n = Ly*x + y."""
    bonds = set()
    for x in range(Lx):
        for y in range(Ly):
            n = Ly * x + y
            if Ly > 1:
                yy = (y + 1) % Ly
                if y + 1 < Ly or Ly > 2:
                    m = Ly * x + yy
                    bonds.add((min(n, m), max(n, m)))
            if x + 1 < Lx:
                m = Ly * (x + 1) + y
                bonds.add((n, m))
    return sorted(bonds)


def hubbard_mpo(Lx: int, Ly: int, t: float = 1.0, U: float = 8.0) -> List[np.ndarray]:
    """Hubbard model on an Lx x Ly cylinder, column-major order.

    H = -t sum_<ij>,s (c+_is c_js + h.c.) + U sum_i n_i,up n_i,dn

    Finite-state MPO: four open-operator kinds
      0: c+_up F, 1: c+_dn F, 2: F c_up, 3: F c_dn
    each carried through delay channels r = 1..rmax (string F on every
    site passed), closed at distance r by c_up, c_dn, c+_up, c+_dn with
    amplitude -t if (i-r, i) is a bond. w = 2 + 4*rmax.
    """
    o = hubbard_ops()
    N = Lx * Ly
    bonds = set(cylinder_bonds(Lx, Ly))
    rmax = max(j - i for i, j in bonds) if bonds else 1
    w = 2 + 4 * rmax
    # For i < j, with c_i = F_0..F_{i-1} C_i in the tensor-product basis:
    #   c+_i c_j = (C+ F)_i  F ... F  (C)_j
    #   c+_j c_i = (F C)_i   F ... F  (C+)_j
    start = [o["Cdagup"] @ o["F"], o["Cdagdn"] @ o["F"],
             o["F"] @ o["Cup"], o["F"] @ o["Cdn"]]
    close = [o["Cup"], o["Cdn"], o["Cdagup"], o["Cdagdn"]]

    def ch(kind: int, r: int) -> int:
        return 1 + kind * rmax + (r - 1)

    Ws = []
    for i in range(N):
        W = np.zeros((w, w, 4, 4))
        W[0, 0] = o["Id"]
        W[w - 1, w - 1] = o["Id"]
        W[w - 1, 0] = U * o["Nupdn"]
        for k in range(4):
            W[w - 1, ch(k, 1)] = start[k]
            for r in range(1, rmax):
                W[ch(k, r), ch(k, r + 1)] = o["F"]
            for r in range(1, rmax + 1):
                if (i - r, i) in bonds:
                    W[ch(k, r), 0] = -t * close[k]
        Ws.append(W)
    return Ws


# ----------------------------------------------------------------------------
# MPS inputs
# ----------------------------------------------------------------------------
def random_product_state(N: int, d: int, rng: np.random.Generator) -> List[np.ndarray]:
    """Each site a normalised Gaussian d-vector, drawn in site order."""
    out = []
    for _ in range(N):
        v = rng.standard_normal(d)
        v /= np.linalg.norm(v)
        out.append(v.reshape(1, d, 1))
    return out


def neel_product_state(N: int, d: int, up: int = 0, dn: int = 1) -> List[np.ndarray]:
    out = []
    for n in range(N):
        v = np.zeros(d)
        v[up if n % 2 == 0 else dn] = 1.0
        out.append(v.reshape(1, d, 1))
    return out


def mps_bond_dims(N: int, d: int, chi: int) -> List[int]:
    """D_k = min(d^k, d^(N-k), chi) for k = 0..N."""
    return [int(min(d ** k, d ** (N - k), chi)) for k in range(N + 1)]


def random_canonical_mps(N: int, d: int, chi: int, center: int,
                         rng: np.random.Generator) -> List[np.ndarray]:
    """Gaussian site tensors; sites left of `center` are made left-
    orthonormal by QR, sites right of it right-orthonormal by QR of the
    transpose (an LQ).  Tensors are drawn in site order."""
    D = mps_bond_dims(N, d, chi)
    As = []
    for i in range(N):
        A = rng.standard_normal((D[i], d, D[i + 1]))
        if i < center:
            Q, _ = np.linalg.qr(A.reshape(D[i] * d, D[i + 1]))
            A = Q.reshape(D[i], d, D[i + 1])
        elif i > center:
            Q, _ = np.linalg.qr(A.reshape(D[i], d * D[i + 1]).T)
            A = Q.T.reshape(D[i], d, D[i + 1])
        else:
            A /= np.linalg.norm(A)
        As.append(A)
    return As


def aklt_site_tensors() -> np.ndarray:
    """AKLT MPS tensor A[s] (2x2) for s = +1, 0, -1:
    A+ = sqrt(2/3) sigma+, A0 = -sqrt(1/3) sigma_z, A- = -sqrt(2/3) sigma-."""
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    sz = np.array([[1.0, 0.0], [0.0, -1.0]])
    A = np.zeros((2, 3, 2))
    A[:, 0, :] = math.sqrt(2.0 / 3.0) * sp
    A[:, 1, :] = -math.sqrt(1.0 / 3.0) * sz
    A[:, 2, :] = -math.sqrt(2.0 / 3.0) * sp.T
    return A


def aklt_mps(N: int, left: Sequence[float], right: Sequence[float]) -> List[np.ndarray]:
    A = aklt_site_tensors()
    As = [A.copy() for _ in range(N)]
    As[0] = np.einsum("a,asb->sb", np.asarray(left, float), A)[None]
    As[-1] = np.einsum("asb,b->as", A, np.asarray(right, float))[..., None]
    return As


def gaussian(shape, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal(shape)


def unit_gaussian(shape, rng: np.random.Generator) -> np.ndarray:
    x = rng.standard_normal(shape)
    return x / np.linalg.norm(x)


# ----------------------------------------------------------------------------
# QN inputs
# ----------------------------------------------------------------------------
def block_values(seed: int, key: Sequence[int], shape) -> np.ndarray:
    """Gaussian values of one block, keyed by (seed, key) so that any
    enumeration order gives the same numbers."""
    g = np.random.default_rng([int(seed)] + [int(k) + (1 << 20) for k in key])
    return g.standard_normal(tuple(int(s) for s in shape))


def c3_sector_dims(nsec: int = 25, total: int = 4096, peak: int = 800,
                   floor: int = 8, sigma: float = 1.996) -> List[Tuple[int, int]]:
    """Binomial-shaped U(1) sectors of a bond at the centre of a long S=1/2
    chain: 2Sz in {-(nsec-1), ..., nsec-1} step 2, size
    max(floor, round(peak*exp(-(q/2)^2/(2 sigma^2)))), with the residual to
    `total` added to the central sector."""
    half = nsec // 2
    qs = [2 * (k - half) for k in range(nsec)]
    dims = [max(floor, int(round(peak * math.exp(-((q / 2) ** 2) / (2 * sigma * sigma)))))
            for q in qs]
    dims[half] += total - sum(dims)
    return list(zip(qs, dims))


def c4_sector_dims(total: int = 4096, sigma: float = 2.0) -> List[Tuple[Tuple[int, int], int]]:
    """(dN, 2Sz) sectors relative to a half-filled half cylinder with
    dN = 2Sz (mod 2); size proportional to exp(-dN^2/(2s^2) - (2Sz)^2/(2s^2)),
    scaled to `total`, zeros dropped, the residual put on (0, 0)."""
    cand = []
    for dn in range(-12, 13):
        for sz in range(-12, 13):
            if (dn - sz) % 2:
                continue
            cand.append(((dn, sz), math.exp(-(dn * dn) / (2 * sigma ** 2) - (sz * sz) / (2 * sigma ** 2))))
    z = sum(v for _, v in cand)
    out = []
    for q, v in cand:
        n = int(round(total * v / z))
        if n > 0:
            out.append((q, n))
    idx = [q for q, _ in out].index((0, 0))
    q0, n0 = out[idx]
    out[idx] = (q0, n0 + total - sum(n for _, n in out))
    return out


def sectors_from_basis_qns(qns: Sequence) -> Tuple[List[Tuple[int, ...]], List[int]]:
    """Run-length encoding of a basis' QN list into (sector QNs, sector dims):
    maximal runs of equal QN in basis order (equal QNs may repeat)."""
    q_out: List[Tuple[int, ...]] = []
    d_out: List[int] = []
    for q in qns:
        q = tuple(int(x) for x in (q if isinstance(q, (tuple, list)) else (q,)))
        if q_out and q_out[-1] == q:
            d_out[-1] += 1
        else:
            q_out.append(q)
            d_out.append(1)
    return q_out, d_out


def long_range_hubbard_mpo(N: int, rmax: int, t: float = 1.0, U: float = 8.0) -> List[np.ndarray]:
    """Synthetic Hubbard chain with equal hopping at every distance 1..rmax
    (a charge-conserving MPO of w = 2 + 4 rmax, used as a shape)."""
    o = hubbard_ops()
    w = 2 + 4 * rmax
    start = [o["Cdagup"] @ o["F"], o["Cdagdn"] @ o["F"], o["F"] @ o["Cup"], o["F"] @ o["Cdn"]]
    close = [o["Cup"], o["Cdn"], o["Cdagup"], o["Cdagdn"]]

    def ch(kind: int, r: int) -> int:
        return 1 + kind * rmax + (r - 1)

    Ws = []
    for i in range(N):
        W = np.zeros((w, w, 4, 4))
        W[0, 0] = o["Id"]
        W[w - 1, w - 1] = o["Id"]
        W[w - 1, 0] = U * o["Nupdn"]
        for k in range(4):
            W[w - 1, ch(k, 1)] = start[k]
            for r in range(1, rmax):
                W[ch(k, r), ch(k, r + 1)] = o["F"]
            for r in range(1, rmax + 1):
                if i - r >= 0:
                    W[ch(k, r), 0] = -t * close[k]
        Ws.append(W)
    return Ws


def heisenberg_site_qn(two_s: int = 1) -> List[int]:
    """2Sz of each basis state (highest first)."""
    return [two_s - 2 * k for k in range(two_s + 1)]


def heisenberg_mpo_link_qn() -> List[int]:
    """2Sz of each Heisenberg MPO channel, read with the arrows
    W[m_in:Out, m_out:In, s':Out, s:In] and zero flux, i.e.
    q(m_out) = q(m_in) + q(s') - q(s), with q(channel 4) = 0:
    channel 1 follows S- (-2), channel 2 follows S+ (+2)."""
    return [0, -2, 2, 0, 0]


def hubbard_mpo_link_qn(w: int) -> List[Tuple[int, int]]:
    """(N, 2Sz) of each channel of hubbard_mpo: kinds 0..3 follow
    c+_up, c+_dn, c_up, c_dn."""
    rmax = (w - 2) // 4
    kind_q = [(1, 1), (1, -1), (-1, -1), (-1, 1)]
    out = [(0, 0)] * w
    for k in range(4):
        for r in range(1, rmax + 1):
            out[1 + k * rmax + (r - 1)] = kind_q[k]
    return out


def hubbard_site_qn() -> List[Tuple[int, int]]:
    """(N, 2Sz) of the basis (|0>, |up>, |dn>, |up dn>)."""
    return [(0, 0), (1, 1), (1, -1), (2, 0)]


# ---------------------------------------------------- Z_N momentum labels
# A third QN component with Z_4 addition (a k_y-like momentum label around a
# 4-leg cylinder).  Structure only: the operands built on it are synthetic.

def c4z4_sector_dims(total: int = 4096, n: int = 4) -> List[Tuple[Tuple[int, int, int], int]]:
    """Every (dN, 2Sz) sector of c4_sector_dims split into n momentum
    sectors k = 0..n-1 of near-equal size (zero sizes dropped)."""
    out = []
    for (dn, sz), d in c4_sector_dims(total):
        for k in range(n):
            m = d // n + (1 if k < d % n else 0)
            if m > 0:
                out.append(((dn, sz, k), m))
    return out


def hubbard_momentum_site_qn(k: int = 1, n: int = 4) -> List[Tuple[int, int, int]]:
    """(N, 2Sz, momentum mod n) of (|0>, |up>, |dn>, |up dn>) for an orbital
    of momentum k."""
    return [(0, 0, 0), (1, 1, k % n), (1, -1, k % n), (2, 0, (2 * k) % n)]


def hubbard_momentum_link_qn(w: int, k: int = 1, n: int = 4) -> List[Tuple[int, int, int]]:
    """hubbard_mpo_link_qn with a momentum component: creation channels carry
    +k, annihilation channels -k (mod n)."""
    kinds = {(1, 1): k, (1, -1): k, (-1, -1): -k, (-1, 1): -k, (0, 0): 0}
    return [(a, b, kinds[(a, b)] % n) for a, b in hubbard_mpo_link_qn(w)]
