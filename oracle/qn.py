"""Quantum-number block-sparse tensors (oracle).

Sec. 8: an index is an ordered list of sectors (a QN and a dimension) with
an arrow, Out or In.  A block (one sector per index) is stored iff the
arrow-weighted sum of its QNs equals the tensor's flux (Out adds, In
subtracts); contracted index pairs must have opposite arrows; the flux of a
product is the sum of the operands' fluxes.  Sec. 9.2 stores a block-sparse
tensor as one array plus a map from block to offset.

A QN component may obey Z_N addition instead of integer addition (Sec. 8,
fermion parity being the example, Z_2): its values are taken modulo N.  An
index carries the modulus of every component (`mod`, 0 = integer addition,
empty = all integer); QN values are stored reduced, in [0, N).

Block layout used for packing (a reading; the paper's tuples are 1-based):
blocks are 0-based sector tuples sorted lexicographically with the first
index most significant, each block row-major, offsets the exclusive prefix
sum of block sizes.

Two independent routes compute H_eff psi: a loop over allowed block pairs
(`heff_apply_blocks`), and embedding every operand densely, applying the
dense oracle and reading the blocks back (`heff_apply_embedded`).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import heff as hf

QN = Tuple[int, ...]


def qn(*vals) -> QN:
    return tuple(int(v) for v in vals)


def qn_add(a: QN, b: QN) -> QN:
    return tuple(x + y for x, y in zip(a, b))


def qn_scale(a: QN, s: int) -> QN:
    return tuple(s * x for x in a)


def qn_reduce(a: QN, mod: Sequence[int]) -> QN:
    """Components with modulus N > 0 taken modulo N (into [0, N))."""
    if not mod:
        return tuple(a)
    return tuple(x % m if m else x for x, m in zip(a, mod))


@dataclass(frozen=True)
class QNIndex:
    sectors: Tuple[Tuple[QN, int], ...]
    arrow: int = +1  # +1 Out, -1 In
    mod: Tuple[int, ...] = ()  # per-component modulus, 0 = integer addition

    @property
    def dim(self) -> int:
        return sum(n for _, n in self.sectors)

    @property
    def nsec(self) -> int:
        return len(self.sectors)

    def offsets(self) -> List[int]:
        out, o = [], 0
        for _, n in self.sectors:
            out.append(o)
            o += n
        return out

    def dag(self) -> "QNIndex":
        return QNIndex(self.sectors, -self.arrow, self.mod)

    def with_arrow(self, arrow: int) -> "QNIndex":
        return QNIndex(self.sectors, arrow, self.mod)

    def qn(self, k: int) -> QN:
        return self.sectors[k][0]

    def sdim(self, k: int) -> int:
        return self.sectors[k][1]


def make_index(pairs: Sequence[Tuple[Sequence[int], int]], arrow: int = +1,
               mod: Sequence[int] = ()) -> QNIndex:
    mod = tuple(int(m) for m in mod)
    return QNIndex(tuple((qn_reduce(tuple(int(x) for x in q), mod), int(n)) for q, n in pairs), arrow,
                   mod)


def index_from_basis_qns(qns: Sequence[Sequence[int]], arrow: int = +1,
                         mod: Sequence[int] = ()) -> QNIndex:
    """Sectors as maximal runs of equal QN in basis order (runs of the same
    QN need not be merged)."""
    mod = tuple(int(m) for m in mod)
    pairs: List[Tuple[QN, int]] = []
    for q in qns:
        q = qn_reduce(tuple(int(x) for x in (q if isinstance(q, (tuple, list)) else (q,))), mod)
        if pairs and pairs[-1][0] == q:
            pairs[-1] = (q, pairs[-1][1] + 1)
        else:
            pairs.append((q, 1))
    return QNIndex(tuple(pairs), arrow, mod)


def common_mod(inds: Sequence[QNIndex]) -> Tuple[int, ...]:
    mods = {ind.mod for ind in inds}
    if len(mods) != 1:
        raise ValueError("indices of one tensor need the same QN moduli")
    return mods.pop()


def block_flux(inds: Sequence[QNIndex], blk: Sequence[int]) -> QN:
    nq = len(inds[0].qn(0))
    tot = (0,) * nq
    for ind, k in zip(inds, blk):
        tot = qn_add(tot, qn_scale(ind.qn(k), ind.arrow))
    return qn_reduce(tot, common_mod(inds))


def allowed_blocks(inds: Sequence[QNIndex], flux: QN) -> List[Tuple[int, ...]]:
    """Every sector tuple whose arrow-weighted QN sum equals the flux, in
    lexicographic order."""
    want = qn_reduce(tuple(flux), common_mod(inds))
    out = []
    for blk in itertools.product(*[range(ind.nsec) for ind in inds]):
        if block_flux(inds, blk) == want:
            out.append(tuple(blk))
    return out


@dataclass
class BlockTensor:
    inds: List[QNIndex]
    flux: QN
    blocks: Dict[Tuple[int, ...], np.ndarray] = field(default_factory=dict)

    def block_shape(self, blk) -> Tuple[int, ...]:
        return tuple(ind.sdim(k) for ind, k in zip(self.inds, blk))

    def to_dense(self) -> np.ndarray:
        T = np.zeros([ind.dim for ind in self.inds])
        offs = [ind.offsets() for ind in self.inds]
        for blk, arr in self.blocks.items():
            sl = tuple(slice(offs[i][k], offs[i][k] + self.inds[i].sdim(k)) for i, k in enumerate(blk))
            T[sl] = arr
        return T

    def norm(self) -> float:
        return float(np.sqrt(sum(float((a * a).sum()) for a in self.blocks.values())))

    def packed(self):
        """(sorted block list, offsets, flat data) in the packing layout."""
        keys = sorted(self.blocks)
        offs, data, o = [], [], 0
        for k in keys:
            offs.append(o)
            data.append(self.blocks[k].ravel())
            o += self.blocks[k].size
        flat = np.concatenate(data) if data else np.zeros(0)
        return keys, offs, flat


def from_dense(T: np.ndarray, inds: Sequence[QNIndex], flux: QN) -> BlockTensor:
    offs = [ind.offsets() for ind in inds]
    out = BlockTensor(list(inds), qn_reduce(tuple(flux), common_mod(inds)))
    for blk in allowed_blocks(inds, flux):
        sl = tuple(slice(offs[i][k], offs[i][k] + inds[i].sdim(k)) for i, k in enumerate(blk))
        out.blocks[blk] = np.array(T[sl], dtype=np.float64)
    return out


def outside_blocks_max(T: np.ndarray, inds: Sequence[QNIndex], flux: QN) -> float:
    """Largest |entry| of a dense array outside the allowed blocks."""
    mask = np.ones(T.shape, bool)
    offs = [ind.offsets() for ind in inds]
    for blk in allowed_blocks(inds, flux):
        sl = tuple(slice(offs[i][k], offs[i][k] + inds[i].sdim(k)) for i, k in enumerate(blk))
        mask[sl] = False
    return float(np.abs(T[mask]).max()) if mask.any() else 0.0


def random_blocks(inds: Sequence[QNIndex], flux: QN, seed: int, block_values) -> BlockTensor:
    """Fill every allowed block with `block_values(seed, key, shape)`."""
    out = BlockTensor(list(inds), qn_reduce(tuple(flux), common_mod(inds)))
    for blk in allowed_blocks(inds, flux):
        out.blocks[blk] = block_values(seed, blk, out.block_shape(blk))
    return out


def contract_blocks(A: BlockTensor, la: Sequence[int], B: BlockTensor, lb: Sequence[int],
                    lc: Sequence[int]) -> BlockTensor:
    """Sec. 9.4: a block-sparse contraction is a set of dense contractions of
    block pairs whose contracted sectors match; pairs that land on the same
    output block are summed (in ascending order of the pair list, which is
    sorted)."""
    la, lb, lc = list(la), list(lb), list(lc)
    common = [l for l in la if l in lb]
    for l in common:
        ia, ib = A.inds[la.index(l)], B.inds[lb.index(l)]
        if ia.arrow == ib.arrow:
            raise ValueError("contracted QN indices need opposite arrows")
        if ia.sectors != ib.sectors or ia.mod != ib.mod:
            raise ValueError("contracted QN indices have different sectors")
    free_a = [l for l in la if l not in lb]
    free_b = [l for l in lb if l not in la]
    if sorted(lc) != sorted(free_a + free_b):
        raise ValueError("bad output labels")
    ind_of = {}
    for l, ind in zip(la, A.inds):
        ind_of[l] = ind
    for l, ind in zip(lb, B.inds):
        if l not in ind_of:
            ind_of[l] = ind
    out = BlockTensor([ind_of[l] for l in lc],
                      qn_reduce(qn_add(A.flux, B.flux), common_mod(list(A.inds) + list(B.inds))))
    letters = "abcdefghijklmnopqrstuvwxyz"
    allv = sorted(set(la) | set(lb))
    m = {l: letters[k] for k, l in enumerate(allv)}
    sub = "".join(m[l] for l in la) + "," + "".join(m[l] for l in lb) + "->" + "".join(m[l] for l in lc)
    # B's blocks by their contracted sectors: the pairs visited, and their
    # order (ascending ka, then ascending kb), are those of a full double loop
    # that skips pairs whose contracted sectors differ.
    by_sec: Dict[Tuple[int, ...], List[Tuple[int, ...]]] = {}
    for kb in sorted(B.blocks):
        by_sec.setdefault(tuple(kb[lb.index(l)] for l in common), []).append(kb)
    for ka in sorted(A.blocks):
        for kb in by_sec.get(tuple(ka[la.index(l)] for l in common), []):
            sec = {}
            for l, k in zip(la, ka):
                sec[l] = k
            for l, k in zip(lb, kb):
                sec[l] = k
            kc = tuple(sec[l] for l in lc)
            val = np.einsum(sub, A.blocks[ka], B.blocks[kb], optimize=False)
            if kc in out.blocks:
                out.blocks[kc] = out.blocks[kc] + val
            else:
                out.blocks[kc] = val
    return out


# labels: a'=0 m0=1 a=2 s1=3 s2=4 b=5 m1=6 s1'=7 s2'=8 m2=9 b'=10
def heff_apply_blocks(L: BlockTensor, W1: BlockTensor, W2: BlockTensor, R: BlockTensor,
                      psi: BlockTensor) -> BlockTensor:
    """Blockwise H_eff psi in the dense oracle's order: L, then W1, W2, R."""
    X = contract_blocks(L, [0, 1, 2], psi, [2, 3, 4, 5], [0, 1, 3, 4, 5])
    Y = contract_blocks(X, [0, 1, 3, 4, 5], W1, [1, 6, 7, 3], [0, 6, 7, 4, 5])
    Z = contract_blocks(Y, [0, 6, 7, 4, 5], W2, [6, 9, 8, 4], [0, 7, 8, 9, 5])
    return contract_blocks(Z, [0, 7, 8, 9, 5], R, [10, 9, 5], [0, 7, 8, 10])


def heff_apply_embedded(L: BlockTensor, W1: BlockTensor, W2: BlockTensor, R: BlockTensor,
                        psi: BlockTensor):
    """Dense route: embed, apply the dense oracle, return (dense result,
    blocks read back with psi's indices and flux)."""
    y = hf.heff_apply(L.to_dense(), W1.to_dense(), W2.to_dense(), R.to_dense(), psi.to_dense())
    return y, from_dense(y, psi.inds, psi.flux)


def mpo_blocks(W: np.ndarray, link_in: QNIndex, link_out: QNIndex, site: QNIndex) -> BlockTensor:
    """An MPO tensor W[m_in:Out, m_out:In, s':Out, s:In] with zero flux."""
    inds = [link_in.with_arrow(+1), link_out.with_arrow(-1), site.with_arrow(+1),
            site.with_arrow(-1)]
    nq = len(site.qn(0))
    return from_dense(W, inds, (0,) * nq)


def heff_qn_operands(bond_l: Sequence[Tuple[QN, int]], bond_r: Sequence[Tuple[QN, int]],
                     site_qns: Sequence, link_qns: Sequence, W1: np.ndarray, W2: np.ndarray,
                     seed: int, block_values, psi_flux: QN | None = None):
    """Synthetic QN operands of one H_eff: L[a':Out, m:In, a:In] and
    R[b':In, m:Out, b:Out] Gaussian on every allowed block, psi[a:Out,
    s1:Out, s2:Out, b:In] Gaussian on every allowed block and unit norm,
    W as block tensors.  Block values come from `block_values` keyed by
    (seed + tensor tag, sector tuple)."""
    site = index_from_basis_qns(site_qns)
    link = index_from_basis_qns(link_qns)
    al = make_index(bond_l, +1)
    ar = make_index(bond_r, +1)
    L, R, psi = _env_and_psi(al, ar, site, link, seed, block_values, psi_flux)
    w1 = mpo_blocks(W1, link, link, site)
    w2 = mpo_blocks(W2, link, link, site)
    return L, w1, w2, R, psi


def _env_and_psi(al: QNIndex, ar: QNIndex, site: QNIndex, link: QNIndex, seed: int, block_values,
                 psi_flux):
    zero = (0,) * len(site.qn(0))
    L = random_blocks([al, link.with_arrow(-1), al.with_arrow(-1)], zero, seed + 1, block_values)
    R = random_blocks([ar.with_arrow(-1), link.with_arrow(+1), ar.with_arrow(+1)], zero, seed + 2,
                      block_values)
    psi = random_blocks([al, site, site, ar.with_arrow(-1)], psi_flux or zero, seed + 3, block_values)
    nrm = psi.norm()
    for k in psi.blocks:
        psi.blocks[k] = psi.blocks[k] / nrm
    return L, R, psi


def heff_qn_operands_random_w(bond_l: Sequence[Tuple[QN, int]], bond_r: Sequence[Tuple[QN, int]],
                              site_qns: Sequence, link_qns: Sequence, mod: Sequence[int], seed: int,
                              block_values, psi_flux: QN | None = None):
    """As heff_qn_operands, for QNs with the given moduli, with the two MPO
    tensors also Gaussian on every allowed block (a symmetric but otherwise
    synthetic W).  Returns (L, w1, w2, R, psi, W1 dense, W2 dense)."""
    site = index_from_basis_qns(site_qns, +1, mod)
    link = index_from_basis_qns(link_qns, +1, mod)
    al = make_index(bond_l, +1, mod)
    ar = make_index(bond_r, +1, mod)
    L, R, psi = _env_and_psi(al, ar, site, link, seed, block_values, psi_flux)
    winds = [link.with_arrow(+1), link.with_arrow(-1), site.with_arrow(+1), site.with_arrow(-1)]
    zero = (0,) * len(site.qn(0))
    w1 = random_blocks(winds, zero, seed + 4, block_values)
    w2 = random_blocks(winds, zero, seed + 5, block_values)
    return L, w1, w2, R, psi, w1.to_dense(), w2.to_dense()
