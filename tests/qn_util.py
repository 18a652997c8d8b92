"""Helpers turning oracle QN tensors into the binding's descriptors (tests)."""
import numpy as np

from paper_2007_14822_amd import inputs as inp
from oracle import qn as Q


def space(ind: Q.QNIndex):
    sp = ([q for q, _ in ind.sectors], [n for _, n in ind.sectors], ind.arrow)
    return sp + (ind.mod,) if ind.mod else sp


def desc(bt: Q.BlockTensor, data=None, with_data=True):
    keys, offs, flat = bt.packed()
    d = {"spaces": [space(i) for i in bt.inds], "blocks": keys, "offsets": offs,
         "flux": list(bt.flux)}
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


def u1_degenerate_site(seed=67):
    """U(1) (particle number only) operands whose site sectors hold more than
    one state (the two singly occupied states share N = 1), so a psi block
    has several (s1, s2) column runs per b; bond sectors are not multiples of
    8.  Synthetic symmetric W (Gaussian on every allowed block)."""
    bl = [((0,), 3), ((1,), 5), ((2,), 4)]
    br = [((1,), 2), ((2,), 5), ((3,), 3), ((4,), 2)]
    site = [(0,), (1,), (1,), (2,)]
    link = [(0,), (1,), (-1,), (1,), (-1,), (0,)]
    L, w1, w2, R, psi, W1, W2 = Q.heff_qn_operands_random_w(bl, br, site, link, (0,), seed,
                                                            inp.block_values)
    return (L, w1, w2, R, psi), W1, W2


def small_u1u1z4(seed=53):
    """U(1) x U(1) x Z_4 operands: (dN, 2Sz, momentum mod 4) sectors of a
    small bond, the Hubbard momentum site basis, the w = 6 channel charges of
    a nearest-neighbour hopping MPO with momentum labels, and a synthetic
    symmetric W (Gaussian on every allowed block)."""
    bl = [((0, 0, 0), 2), ((1, 1, 1), 2), ((1, -1, 1), 3), ((2, 0, 2), 2), ((1, 1, 0), 1),
          ((0, 0, 2), 2)]
    br = [((1, 1, 1), 2), ((2, 0, 2), 3), ((2, 2, 2), 1), ((3, 1, 3), 2), ((2, 0, 0), 2),
          ((3, -1, 3), 1), ((1, -1, 1), 2)]
    site = inp.hubbard_momentum_site_qn()
    link = inp.hubbard_momentum_link_qn(6)
    L, w1, w2, R, psi, W1, W2 = Q.heff_qn_operands_random_w(bl, br, site, link, (0, 0, 4), seed,
                                                            inp.block_values)
    return (L, w1, w2, R, psi), W1, W2


def _bench_blocks(inds, flux, seed, key_prefix=()):
    """Every allowed block filled with block_values(seed, key_prefix + block)
    (the keys the benchmark uses for its operands)."""
    out = Q.BlockTensor(list(inds), Q.qn_reduce(tuple(flux), Q.common_mod(inds)))
    for blk in Q.allowed_blocks(inds, flux):
        out.blocks[blk] = inp.block_values(seed, tuple(key_prefix) + tuple(blk),
                                           out.block_shape(blk))
    return out


def c4_operands(which: str = "c4", nv: int = 1):
    """The U(1) x U(1) Hubbard cylinder bond of the benchmark as oracle
    tensors, with the benchmark's structure and values:
      c4     chi = 4096 in 81 (dN, 2Sz) sectors, w = 18 (column-major 4 x 32
             cylinder, the bulk tensors of sites 62, 63)
      c4w38  the same sectors, the w = 38 long-range shape
      c4z4   the 81 sectors split by a Z_4 momentum label (324 sectors),
             synthetic symmetric W (Gaussian on the allowed blocks)
    Returns ((L, w1, w2, R, [psi_v for v < nv]), W1, W2)."""
    if which == "c4z4":
        bond = list(inp.c4z4_sector_dims())
        site_q = inp.hubbard_momentum_site_qn()
        link_q = inp.hubbard_momentum_link_qn(18)
        mod = (0, 0, 4)
        seed = inp.seed_for(5, 4096)
    else:
        bond = list(inp.c4_sector_dims())
        site_q = inp.hubbard_site_qn()
        mod = ()
        seed = inp.seed_for(4, 4096)
        if which == "c4":
            Ws = inp.hubbard_mpo(32, 4)
            W1, W2 = Ws[62], Ws[63]
        else:
            Ws = inp.long_range_hubbard_mpo(8, 9)
            W1, W2 = Ws[6], Ws[7]
        link_q = inp.hubbard_mpo_link_qn(W1.shape[0])
    site = Q.index_from_basis_qns(site_q, +1, mod)
    link = Q.index_from_basis_qns(link_q, +1, mod)
    al = Q.make_index(bond, +1, mod)
    zero = (0,) * len(site.qn(0))
    L = _bench_blocks([al, link.with_arrow(-1), al.with_arrow(-1)], zero, seed + 1, (0,))
    R = _bench_blocks([al.with_arrow(-1), link.with_arrow(+1), al.with_arrow(+1)], zero, seed + 2,
                      (0,))
    psis = []
    for v in range(nv):
        p = _bench_blocks([al, site, site, al.with_arrow(-1)], zero, seed + 3, (v,))
        nrm = p.norm()
        for k in p.blocks:
            p.blocks[k] = p.blocks[k] / nrm
        psis.append(p)
    winds = [link.with_arrow(+1), link.with_arrow(-1), site.with_arrow(+1), site.with_arrow(-1)]
    if which == "c4z4":
        w1 = _bench_blocks(winds, zero, seed + 4)
        w2 = _bench_blocks(winds, zero, seed + 5)
        W1, W2 = w1.to_dense(), w2.to_dense()
    else:
        w1 = Q.from_dense(W1, winds, zero)
        w2 = Q.from_dense(W2, winds, zero)
    return (L, w1, w2, R, psis), W1, W2


def abs_blocks(bt: Q.BlockTensor) -> Q.BlockTensor:
    """The same blocks with absolute values (scale of the rounding bound)."""
    return Q.BlockTensor(bt.inds, bt.flux, {k: np.abs(v) for k, v in bt.blocks.items()})
