"""Two-site DMRG, step by step (oracle).

Sec. 7.2 gives the algorithm's inputs (an MPO Hamiltonian, an initial MPS,
a schedule of sweeps with a maximum bond dimension and a cutoff per sweep)
and its two costs (environments, local eigensolve); Sec. 5 fixes the
truncation semantics of the SVD.  The steps below are the standard two-site
algorithm in that notation:

  1. start from a right-canonical MPS, build every right environment;
  2. per sweep, left->right over bonds (0,1)..(N-2,N-1): form the two-site
     tensor, find the lowest eigenpair of H_eff, split it by a truncated SVD
     keeping U left-orthonormal and S V^T on the right site, extend the left
     environment; then right->left over the same bonds with V^T kept
     right-orthonormal and U S on the left site, extending the right
     environment;
  3. the sweep's energy is the eigenvalue at the last bond it visits.

Readings where the paper is silent: two-site updates, a sweep is a full
left->right->left round trip, truncation on relative squared singular values
with the kept spectrum renormalised, and an exact dense eigensolve when the
local space has at most 4096 states (FP64 Davidson otherwise).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Sequence, Tuple

import numpy as np

from . import heff as hf

EXACT_EIGH_MAX = 4096


@dataclass
class TruncationResult:
    keep: int
    discarded_weight: float


def truncation_count(s: np.ndarray, cutoff: float, maxdim: int, mindim: int = 1) -> TruncationResult:
    """Sec. 5: sum squared singular values from the smallest up while the
    sum stays within the cutoff, and keep at most maxdim.  Weights are taken
    relative to the total; at least `mindim` values are kept."""
    s = np.asarray(s, np.float64)
    p = s * s
    tot = float(p.sum())
    if tot == 0.0:
        return TruncationResult(max(1, mindim), 0.0)
    p = p / tot
    n = len(p)
    keep = n
    disc = 0.0
    # discard from the smallest while the running discarded weight stays <= cutoff
    while keep > 1 and disc + p[keep - 1] <= cutoff:
        disc += p[keep - 1]
        keep -= 1
    keep = min(keep, int(maxdim))
    keep = max(keep, min(int(mindim), n))
    disc = float(p[keep:].sum())
    return TruncationResult(keep, disc)


def split_bond(psi: np.ndarray, cutoff: float, maxdim: int, to_right: bool,
               mindim: int = 1):
    """Truncated SVD of psi[a, s1, s2, b] as the matrix [(a s1), (s2 b)].

    Returns (A_left, A_right, discarded_weight, singular_values_kept).
    Moving right: A_left = U (left-orthonormal), A_right = S V^T.
    Moving left:  A_left = U S, A_right = V^T (right-orthonormal).
    The kept singular values are renormalised to unit 2-norm.
    """
    cl, d1, d2, cr = psi.shape
    M = psi.reshape(cl * d1, d2 * cr)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    tr = truncation_count(s, cutoff, maxdim, mindim)
    k = tr.keep
    sk = s[:k] / np.linalg.norm(s[:k])
    if to_right:
        Al = U[:, :k].reshape(cl, d1, k)
        Ar = (sk[:, None] * Vt[:k]).reshape(k, d2, cr)
    else:
        Al = (U[:, :k] * sk[None, :]).reshape(cl, d1, k)
        Ar = Vt[:k].reshape(k, d2, cr)
    return Al, Ar, tr.discarded_weight, sk


def davidson(apply: Callable[[np.ndarray], np.ndarray], v0: np.ndarray,
             krylovdim: int = 8, maxiter: int = 200, tol: float = 1e-12):
    """Lowest eigenpair by Davidson with the identity preconditioner and
    full re-orthogonalisation (equivalently a restarted Lanczos)."""
    shape = v0.shape
    x = v0.ravel().astype(np.float64)
    x = x / np.linalg.norm(x)
    V = [x]
    AV = [apply(x.reshape(shape)).ravel()]
    theta = 0.0
    for _ in range(maxiter):
        Vm = np.stack(V, 1)
        AVm = np.stack(AV, 1)
        Hk = Vm.T @ AVm
        Hk = 0.5 * (Hk + Hk.T)
        ev, ey = np.linalg.eigh(Hk)
        theta = float(ev[0])
        y = ey[:, 0]
        x = Vm @ y
        ax = AVm @ y
        r = ax - theta * x
        rn = float(np.linalg.norm(r))
        if rn <= tol * max(1.0, abs(theta)):
            break
        t = r.copy()
        for _rep in range(2):
            for v in V:
                t -= (v @ t) * v
        tn = np.linalg.norm(t)
        if tn < 1e-14:
            break
        t /= tn
        if len(V) >= krylovdim:
            V = [x / np.linalg.norm(x)]
            AV = [ax / np.linalg.norm(x)]
            for _rep in range(2):
                t -= (V[0] @ t) * V[0]
            t /= np.linalg.norm(t)
        V.append(t)
        AV.append(apply(t.reshape(shape)).ravel())
    return theta, (x / np.linalg.norm(x)).reshape(shape)


def overlap_env_left(LO, A, B):
    """<psi|phi> environment one site further right: LO'[b', b] =
    sum_{a', a, s} A[a', s, b'] LO[a', a] B[a, s, b] (A of psi, B of phi)."""
    return np.einsum("xsy,xa,asb->yb", A, LO, B, optimize=False)


def overlap_env_right(RO, A, B):
    """The mirror image: RO'[a', a] = sum_{b', b, s} A[a', s, b'] RO[b', b] B[a, s, b]."""
    return np.einsum("xsy,yb,asb->xa", A, RO, B, optimize=False)


def projected_state(LO, B1, B2, RO):
    """A previous state phi seen from the two-site space of psi at the bond:
    v[a', s1, s2, b'] = sum LO[a', a] B1[a, s1, m] B2[m, s2, b] RO[b', b]."""
    return np.einsum("xa,asm,mtb,yb->xsty", LO, B1, B2, RO, optimize=False)


def local_ground_state(L, W1, W2, R, psi0, penalty=()):
    """Lowest eigenpair of H_eff + sum_k w |v_k><v_k| (penalty = [(w, v_k)])."""
    n = psi0.size
    if n <= EXACT_EIGH_MAX:
        H = hf.heff_matrix(L, W1, W2, R)
        for wt, v in penalty:
            H = H + wt * np.outer(v.ravel(), v.ravel())
        H = 0.5 * (H + H.T)
        ev, evec = np.linalg.eigh(H)
        return float(ev[0]), evec[:, 0].reshape(psi0.shape)

    def apply(x):
        y = hf.heff_apply(L, W1, W2, R, x)
        for wt, v in penalty:
            y = y + wt * float(np.vdot(v, x)) * v
        return y
    return davidson(apply, psi0)


@dataclass
class SweepRecord:
    sweep: int
    energy: float
    max_bond: int
    max_trunc: float


@dataclass
class DMRGResult:
    energy: float
    mps: List[np.ndarray]
    records: List[SweepRecord] = field(default_factory=list)


def dmrg(Ws: Sequence[np.ndarray], As0: Sequence[np.ndarray],
         sweeps: Sequence[Tuple[int, float]], mindim: int = 1, ortho: Sequence = (),
         weight: float = 0.0) -> DMRGResult:
    """Two-site DMRG.  `As0` must be right-canonical with its norm on site 0
    (a normalised product state is).  `ortho`: previously found states (lists
    of site tensors) whose projectors, times the energy penalty `weight`, are
    added to the Hamiltonian (Sec. 7.2, excited states)."""
    As = [np.array(A, dtype=np.float64) for A in As0]
    N = len(As)
    w = Ws[0].shape[0]
    Lenv: List = [None] * (N + 1)
    Renv: List = [None] * (N + 1)
    Lenv[0] = hf.left_boundary(w)
    Renv[N] = hf.right_boundary(w)
    for k in range(N - 1, 0, -1):
        Renv[k] = hf.env_right(Renv[k + 1], As[k], Ws[k])
    # overlap environments <psi|phi_j>, left and right of the bond
    LO = [[None] * (N + 1) for _ in ortho]
    RO = [[None] * (N + 1) for _ in ortho]
    for j, Bs in enumerate(ortho):
        LO[j][0] = np.ones((1, 1))
        RO[j][N] = np.ones((1, 1))
        for k in range(N - 1, 0, -1):
            RO[j][k] = overlap_env_right(RO[j][k + 1], As[k], Bs[k])

    def penalty(i):
        return [(weight, projected_state(LO[j][i], Bs[i], Bs[i + 1], RO[j][i + 2]))
                for j, Bs in enumerate(ortho)]
    records = []
    energy = 0.0
    for sw, (maxdim, cutoff) in enumerate(sweeps):
        maxtr = 0.0
        for i in range(0, N - 1):
            psi = np.einsum("asb,btc->astc", As[i], As[i + 1], optimize=False)
            energy, psi = local_ground_state(Lenv[i], Ws[i], Ws[i + 1], Renv[i + 2], psi, penalty(i))
            As[i], As[i + 1], tw, _ = split_bond(psi, cutoff, maxdim, True, mindim)
            maxtr = max(maxtr, tw)
            Lenv[i + 1] = hf.env_left(Lenv[i], As[i], Ws[i])
            for j, Bs in enumerate(ortho):
                LO[j][i + 1] = overlap_env_left(LO[j][i], As[i], Bs[i])
        for i in range(N - 2, -1, -1):
            psi = np.einsum("asb,btc->astc", As[i], As[i + 1], optimize=False)
            energy, psi = local_ground_state(Lenv[i], Ws[i], Ws[i + 1], Renv[i + 2], psi, penalty(i))
            As[i], As[i + 1], tw, _ = split_bond(psi, cutoff, maxdim, False, mindim)
            maxtr = max(maxtr, tw)
            Renv[i + 1] = hf.env_right(Renv[i + 2], As[i + 1], Ws[i + 1])
            for j, Bs in enumerate(ortho):
                RO[j][i + 1] = overlap_env_right(RO[j][i + 2], As[i + 1], Bs[i + 1])
        records.append(SweepRecord(sw, energy, max(A.shape[2] for A in As), maxtr))
    return DMRGResult(energy, As, records)
