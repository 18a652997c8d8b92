"""Helpers turning oracle QN tensors into the binding's descriptors (tests)."""
import numpy as np

from paper_2007_14822_amd import inputs as inp
from oracle import qn as Q


def space(ind: Q.QNIndex):
    return ([q for q, _ in ind.sectors], [n for _, n in ind.sectors], ind.arrow)


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
