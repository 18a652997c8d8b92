"""Environments and the two-site effective Hamiltonian (oracle).

The paper names the two costs of a DMRG step, forming the environment
tensors and diagonalising the local effective Hamiltonian (Sec. 7.2), and
cites the standard formulation of two-site DMRG for them.  Written out with
the index conventions of the MPS formula (Sec. 7.3) and the operator
element convention op[s', s] of Sec. 8.3:

  L_i[a', m', a] = sum L_{i-1}[a'', m, a'''] A_i[a'', s', a'] W_i[m, m', s', s] A_i[a''', s, a]
  R_i[b', m, b]  = sum A_i[b', s', b''] W_i[m, m', s', s] A_i[b, s, b'''] R_{i+1}[b'', m', b''']
  (H_eff psi)[a', s1', s2', b'] =
      sum L[a', m0, a] W1[m0, m1, s1', s1] W2[m1, m2, s2', s2] R[b', m2, b] psi[a, s1, s2, b]

Boundaries (lower-triangular MPO): L_0[0, m, 0] = delta(m, w-1) and
R_{N+1}[0, m, 0] = delta(m, 0).  All data is real, so the bra layer needs
no conjugation.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def _es(sub, *ops):
    return np.einsum(sub, *[np.asarray(o, np.float64) for o in ops], optimize=False)


def left_boundary(w: int) -> np.ndarray:
    L = np.zeros((1, w, 1))
    L[0, w - 1, 0] = 1.0
    return L


def right_boundary(w: int) -> np.ndarray:
    R = np.zeros((1, w, 1))
    R[0, 0, 0] = 1.0
    return R


def env_left(L: np.ndarray, A: np.ndarray, W: np.ndarray) -> np.ndarray:
    """One left environment step, three pairwise contractions."""
    T1 = _es("xmy,ysa->xmsa", L, A)          # sum over a'''
    T2 = _es("xmsa,mnts->xtna", T1, W)       # sum over m, s
    return _es("xtna,xtb->bna", T2, A)       # sum over a'', s'


def env_right(R: np.ndarray, A: np.ndarray, W: np.ndarray) -> np.ndarray:
    """One right environment step, three pairwise contractions."""
    T1 = _es("xny,bsy->xnbs", R, A)          # sum over b'''
    T2 = _es("xnbs,mnts->xtmb", T1, W)       # sum over m', s
    return _es("xtmb,ctx->cmb", T2, A)       # sum over b'', s'


def heff_stage1(L, psi):
    """X[a', m0, s1, s2, b] = sum_a L[a', m0, a] psi[a, s1, s2, b]."""
    return _es("xma,astb->xmstb", L, psi)


def heff_wstage(X, W1, W2):
    """Z[a', s1', s2', m2, b] = sum_{m0, s1, m1, s2} X W1[m0,m1,s1',s1] W2[m1,m2,s2',s2],
    as two contractions (first over m0, s1; then over m1, s2)."""
    Y = _es("xmstb,mnus->xnutb", X, W1)       # [a', m1, s1', s2, b]
    return _es("xnutb,nkvt->xuvkb", Y, W2)    # [a', s1', s2', m2, b]


def heff_stage4(Z, R):
    """(H psi)[a', s1', s2', b'] = sum_{m2, b} Z[a', s1', s2', m2, b] R[b', m2, b]."""
    return _es("xuvkb,ckb->xuvc", Z, R)


def heff_apply(L, W1, W2, R, psi) -> np.ndarray:
    return heff_stage4(heff_wstage(heff_stage1(L, psi), W1, W2), R)


def heff_apply_rows(L, W1, W2, R, psi, rows: Sequence[int]) -> np.ndarray:
    """Output rows a' in `rows` only (the row a' of the result depends on
    L[a', :, :] alone), for spot checks at sizes where the full matvec is
    too slow."""
    Ls = np.asarray(L)[list(rows)]
    return heff_apply(Ls, W1, W2, R, psi)


def heff_matrix(L, W1, W2, R) -> np.ndarray:
    """Dense H_eff[(a' s1' s2' b'), (a s1 s2 b)] from the operator alone
    (no psi): L W1, then W2, then R, pairwise.  Small sizes only."""
    T = _es("xma,mnuv->xaunv", L, W1)              # [a', a, s1', m1, s1]
    T = _es("xaunv,nkpt->xauvkpt", T, W2)          # [a', a, s1', s1, m2, s2', s2]
    T = _es("xauvkpt,ckb->xauvptcb", T, R)         # [a', a, s1', s1, s2', s2, b', b]
    T = T.transpose(0, 2, 4, 6, 1, 3, 5, 7)        # [a', s1', s2', b', a, s1, s2, b]
    n = L.shape[0] * W1.shape[2] * W2.shape[2] * R.shape[0]
    return np.ascontiguousarray(T).reshape(n, n)


def heff_flops(chi_l: int, chi_r: int, d: int, w: int, nv: int = 1) -> float:
    """Multiply-add count x2 of the order stage1 -> W (two steps) -> stage4."""
    s1 = 2.0 * (w * chi_l) * chi_l * (d * d * chi_r)
    sw = 2.0 * chi_l * chi_r * (w * d * d) * (w * d) + 2.0 * chi_l * chi_r * (w * d * d) * (w * d)
    s4 = 2.0 * (d * d * chi_l) * (w * chi_r) * chi_r
    return nv * (s1 + sw + s4)


# ----------------------------------------------------------------------------
# Whole-chain helpers
# ----------------------------------------------------------------------------
def mpo_to_dense(Ws: Sequence[np.ndarray]) -> np.ndarray:
    """Sum over MPO channels with the lower-triangular boundaries."""
    w = Ws[0].shape[0]
    v = np.zeros(w)
    v[w - 1] = 1.0
    # T[m, S', S] accumulated left to right
    T = np.einsum("m,mnts->nts", v, Ws[0], optimize=False)
    for W in Ws[1:]:
        T = np.einsum("mab,mnts->natbs", T, W, optimize=False)
        n, a, t, b, s = T.shape
        T = T.reshape(n, a * t, b * s)
    return T[0]


def mps_to_dense(As: Sequence[np.ndarray]) -> np.ndarray:
    psi = np.asarray(As[0])
    for A in As[1:]:
        psi = np.einsum("xsa,atb->xstb", psi.reshape(psi.shape[0], -1, psi.shape[-1]), A,
                        optimize=False)
        psi = psi.reshape(psi.shape[0], -1, psi.shape[-1])
    return psi.reshape(-1)


def left_envs(As, Ws) -> List[np.ndarray]:
    """envs[k] = L_k built from sites 0..k-1 (envs[0] = boundary)."""
    w = Ws[0].shape[0]
    out = [left_boundary(w)]
    for A, W in zip(As, Ws):
        out.append(env_left(out[-1], A, W))
    return out


def right_envs(As, Ws) -> List[np.ndarray]:
    """envs[k] = R built from sites k..N-1 (envs[N] = boundary)."""
    N = len(As)
    w = Ws[0].shape[0]
    out = [None] * (N + 1)
    out[N] = right_boundary(w)
    for k in range(N - 1, -1, -1):
        out[k] = env_right(out[k + 1], As[k], Ws[k])
    return out


def mps_energy(As, Ws) -> float:
    """<psi|H|psi> / <psi|psi> from a full left environment sweep."""
    Ls = left_envs(As, Ws)
    num = Ls[-1][0, 0, 0]
    # norm: environment of the identity
    N = np.ones((1, 1))
    for A in As:
        N = np.einsum("xy,xsa,ysb->ab", N, A, A, optimize=False)
    return float(num / N[0, 0])


def canonicalize(As, center: int) -> List[np.ndarray]:
    """Mixed-canonical form with the orthogonality centre on `center`:
    QR from the left up to it, QR of the transpose (an LQ) from the right."""
    As = [np.array(A, dtype=np.float64) for A in As]
    N = len(As)
    for i in range(center):
        a, d, b = As[i].shape
        Q, Rm = np.linalg.qr(As[i].reshape(a * d, b))
        As[i] = Q.reshape(a, d, Q.shape[1])
        As[i + 1] = np.einsum("xy,ysb->xsb", Rm, As[i + 1], optimize=False)
    for i in range(N - 1, center, -1):
        a, d, b = As[i].shape
        Q, Rm = np.linalg.qr(As[i].reshape(a, d * b).T)
        As[i] = Q.T.reshape(Q.shape[1], d, b)
        As[i - 1] = np.einsum("asx,yx->asy", As[i - 1], Rm, optimize=False)
    return As


def heff_apply_sum(terms, psi: np.ndarray) -> np.ndarray:
    """Sec. 7.2: a Hamiltonian given as a sum of MPOs H = sum_k H_k acts on the
    two-site wavefunction as the sum of the terms' effective Hamiltonians;
    terms = [(L_k, W1_k, W2_k, R_k), ...] (each with its own MPO bond
    dimension)."""
    out = np.zeros_like(psi, dtype=np.float64)
    for L, W1, W2, R in terms:
        out = out + heff_apply(L, W1, W2, R, psi)
    return out
