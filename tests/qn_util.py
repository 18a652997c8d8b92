"""Helpers turning oracle QN tensors into the binding's descriptors (tests)."""
import numpy as np

from paper_2007_14822_amd import inputs as inp
from oracle import qn as Q


def space(ind: Q.QNIndex):
    sp = ([q for q, _ in ind.sectors], [n for _, n in ind.sectors], ind.arrow)
    return sp + (ind.mod,) if ind.mod else sp


def desc(bt: Q.BlockTensor, data=None, with_data=True):
    keys, offs, flat = bt.packed()
    d = {"spaces": [space(i) for i in bt.inds], "blocks": keys, "offsets": offs}
    if with_data:
        d["data"] = flat if data is None else data
    return d, flat


def mpo_desc(W: np.ndarray, wb: Q.BlockTensor):
    return {"spaces": [space(i) for i in wb.inds], "data": np.ascontiguousarray(W, np.float64)}


def small_u1(seed=77):
    bl = [((-2,), 3), ((0,), 5), ((2,), 4)]
    br = [((-2,), 2), ((0,), 4), ((2,), 5), ((4,), 3)]
    W = inp.heisenberg_mpo(3)[1]
    ops = Q.heff_qn_operands(bl, br, inp.heisenberg_site_qn(1), inp.heisenberg_mpo_link_qn(), W, W,
                             seed, inp.block_values)
    return ops, W, W


def small_u1u1(seed=99):
    bl = [((0, 0), 2), ((1, 1), 3), ((1, -1), 2), ((2, 0), 4)]
    br = [((1, 1), 2), ((2, 0), 3), ((3, 1), 2), ((2, 2), 1), ((3, -1), 2)]
    Ws = inp.hubbard_mpo(2, 4)
    ops = Q.heff_qn_operands(bl, br, inp.hubbard_site_qn(), inp.hubbard_mpo_link_qn(Ws[0].shape[0]),
                             Ws[5], Ws[6], seed, inp.block_values)
    return ops, Ws[5], Ws[6]


def c3_operands(seed=None):
    secs = [((q,), n) for q, n in inp.c3_sector_dims()]
    W = inp.heisenberg_mpo(3)[1]
    seed = inp.seed_for(3, 4096) if seed is None else seed
    ops = Q.heff_qn_operands(secs, secs, inp.heisenberg_site_qn(1), inp.heisenberg_mpo_link_qn(),
                             W, W, seed, inp.block_values)
    return ops, W, W


def large_u1(seed=31):
    """Sectors of a few hundred states (none a multiple of 8): block GEMMs large
    enough for the 256-tile path, with ragged M, N and K."""
    bl = [((-2,), 197), ((0,), 301), ((2,), 229)]
    br = [((-2,), 203), ((0,), 263), ((2,), 311), ((4,), 199)]
    W = inp.heisenberg_mpo(3)[1]
    ops = Q.heff_qn_operands(bl, br, inp.heisenberg_site_qn(1), inp.heisenberg_mpo_link_qn(), W, W,
                             seed, inp.block_values)
    return ops, W, W


def zn_u1z4(seed=41, scale=1):
    """U(1) x Z_4 operands (Z_4 as a momentum-like label) with a synthetic
    symmetric W (Gaussian on every allowed block); sector sizes times
    `scale`.  Returns (ops, W1 dense, W2 dense)."""
    bond = [((0, 0), 2), ((1, 1), 3), ((1, 3), 2), ((2, 2), 2), ((0, 2), 1), ((2, 0), 3), ((1, 2), 2)]
    bond = [(q, n * scale) for q, n in bond]
    site = [(0, 0), (1, 1), (1, 3), (2, 0)]
    link = [(0, 0), (1, 1), (-1, 3), (0, 2), (0, 0)]
    L, w1, w2, R, psi, W1, W2 = Q.heff_qn_operands_random_w(bond, bond, site, link, (0, 4), seed,
                                                            inp.block_values)
    return (L, w1, w2, R, psi), W1, W2
