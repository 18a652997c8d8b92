"""Pins of the oracle's quantum-number block-sparse layer (Sec. 8, 9.2)."""
import json
import os

import numpy as np
import pytest

from paper_2007_14822_amd import inputs as inp
from oracle import qn as Q

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def _idx(entry, arrow=+1):
    return Q.make_index([(tuple(q), n) for q, n in entry], arrow)


def test_paper_index_examples():
    for key in ("qn_index_i", "qn_index_j", "qn_index_three_sectors"):
        g = GOLD[key]
        assert _idx(g["sectors"]).dim == g["dim"]


def test_paper_element_flux():
    gi, gj, ge = GOLD["qn_index_i"], GOLD["qn_index_j"], GOLD["qn_element_flux"]
    i, j = _idx(gi["sectors"]), _idx(gj["sectors"])
    def sector_of(ind, pos1):
        offs = ind.offsets()
        return max(k for k in range(ind.nsec) if offs[k] <= pos1 - 1)
    blk = (sector_of(i, ge["element_1based"][0]), sector_of(j, ge["element_1based"][1]))
    assert list(blk) == ge["sectors_0based"]
    assert list(Q.block_flux([i, j], blk)) == ge["flux"]
    # a tensor of that flux stores this block and the other flux-2 block
    assert Q.allowed_blocks([i, j], tuple(ge["flux"])) == [(0, 1), (1, 0)]


def test_qn_arithmetic():
    g = GOLD["qn_add"]
    assert list(Q.qn_add(tuple(g["a"]), tuple(g["b"]))) == g["sum"]
    assert list(Q.qn_add(tuple(g["b"]), tuple(g["b"]))) == g["b_plus_b"]


def test_hardcore_boson_operators():
    g = GOLD["hardcore_boson"]
    s = _idx(g["site_sectors"])
    inds = [s, s.dag()]  # a = ITensor(s', dag(s))
    a = np.zeros((2, 2))
    r, c = g["a_nonzero_1based"]
    a[r - 1, c - 1] = 1.0
    blocks_a = Q.allowed_blocks(inds, tuple(g["a_flux"]))
    assert len(blocks_a) == 1
    ta = Q.from_dense(a, inds, tuple(g["a_flux"]))
    assert sum(b.size for b in ta.blocks.values()) == g["a_stored_elements"]
    assert Q.outside_blocks_max(a, inds, tuple(g["a_flux"])) == 0.0
    n = np.diag([0.0, 1.0])
    assert len(Q.allowed_blocks(inds, tuple(g["n_flux"]))) == g["n_blocks"]
    assert Q.outside_blocks_max(n, inds, tuple(g["n_flux"])) == 0.0


def test_ndtensors_block_layout():
    g = GOLD["ndtensors_blocksparse"]
    # plain block sparsity: give the two indices charges that allow exactly nzblocks
    i = Q.make_index([((0,), g["blockdims"][0][0]), ((1,), g["blockdims"][0][1])], +1)
    j = Q.make_index([((1,), g["blockdims"][1][0]), ((0,), g["blockdims"][1][1])], -1)
    blocks = Q.allowed_blocks([i, j], (0,))
    assert [tuple(x + 1 for x in b) for b in blocks] == [tuple(b) for b in g["nzblocks_1based"]]
    assert [i.dim, j.dim] == g["dims"]
    T = Q.random_blocks([i, j], (0,), 1, inp.block_values)
    keys, offs, flat = T.packed()
    assert keys == [(0, 1), (1, 0)]
    assert offs == [0, 2 * 3]  # block (0,1) is 2x3
    assert flat.size == 2 * 2 + 2 * 3


def test_contract_arrow_rule():
    i = Q.make_index([((0,), 2), ((1,), 1)], +1)
    A = Q.random_blocks([i, i.dag()], (0,), 1, inp.block_values)
    B = Q.random_blocks([i, i.dag()], (0,), 2, inp.block_values)
    Q.contract_blocks(A, [1, 2], B, [2, 3], [1, 3])  # In meets Out: fine
    with pytest.raises(ValueError):
        Q.contract_blocks(A, [1, 2], B, [3, 2], [1, 3])  # In meets In


def test_heisenberg_mpo_respects_link_charges():
    W = inp.heisenberg_mpo(3)[1]
    link = Q.index_from_basis_qns(inp.heisenberg_mpo_link_qn())
    site = Q.index_from_basis_qns(inp.heisenberg_site_qn(1))
    inds = [link, link.dag(), site, site.dag()]
    assert Q.outside_blocks_max(W, inds, (0,)) == 0.0


def test_hubbard_mpo_respects_link_charges():
    Ws = inp.hubbard_mpo(2, 4)
    link = Q.index_from_basis_qns(inp.hubbard_mpo_link_qn(Ws[0].shape[0]))
    site = Q.index_from_basis_qns(inp.hubbard_site_qn())
    inds = [link, link.dag(), site, site.dag()]
    for W in Ws:
        assert Q.outside_blocks_max(W, inds, (0, 0)) == 0.0


def _small_u1():
    bl = [((-2,), 3), ((0,), 5), ((2,), 4)]
    br = [((-2,), 2), ((0,), 4), ((2,), 5), ((4,), 3)]
    W = inp.heisenberg_mpo(3)[1]
    return Q.heff_qn_operands(bl, br, inp.heisenberg_site_qn(1), inp.heisenberg_mpo_link_qn(),
                              W, W, 77, inp.block_values, psi_flux=None)


def _small_u1u1():
    bl = [((0, 0), 2), ((1, 1), 3), ((1, -1), 2), ((2, 0), 4)]
    br = [((1, 1), 2), ((2, 0), 3), ((3, 1), 2), ((2, 2), 1), ((3, -1), 2)]
    Ws = inp.hubbard_mpo(2, 4)
    return Q.heff_qn_operands(bl, br, inp.hubbard_site_qn(),
                              inp.hubbard_mpo_link_qn(Ws[0].shape[0]), Ws[5], Ws[6], 99,
                              inp.block_values)


@pytest.mark.parametrize("make", [_small_u1, _small_u1u1])
def test_blockwise_equals_embedded(make):
    L, W1, W2, R, psi = make()
    assert len(psi.blocks) > 0
    y = Q.heff_apply_blocks(L, W1, W2, R, psi)
    yd, ye = Q.heff_apply_embedded(L, W1, W2, R, psi)
    # flux conservation: nothing outside psi's blocks, exactly
    assert Q.outside_blocks_max(yd, psi.inds, psi.flux) == 0.0
    assert sorted(y.blocks) == sorted(psi.blocks)
    for k in psi.blocks:
        np.testing.assert_allclose(y.blocks[k], ye.blocks[k], rtol=0, atol=1e-13)


def _c3_psi_stats():
    secs = inp.c3_sector_dims()
    bond = Q.make_index([((q,), n) for q, n in secs], +1)
    site = Q.index_from_basis_qns(inp.heisenberg_site_qn(1))
    inds = [bond, site, site, bond.dag()]
    # the C3 bond at the chain centre: psi's right bond carries the same sectors
    blks = Q.allowed_blocks(inds, (0,))
    nel = sum(np.prod([inds[i].sdim(k) for i, k in enumerate(b)]) for b in blks)
    link = Q.index_from_basis_qns(inp.heisenberg_mpo_link_qn())
    L_inds = [bond, link.dag(), bond.dag()]
    lb = Q.allowed_blocks(L_inds, (0,))
    nl = sum(np.prod([L_inds[i].sdim(k) for i, k in enumerate(b)]) for b in lb)
    return len(blks), int(nel), int(nl)


def test_c3_block_counts():
    nb, nel, nl = _c3_psi_stats()
    assert nb == 98
    assert abs(nel - 8.79e6) / 8.79e6 < 0.01
    assert abs(nl - 11.05e6) / 11.05e6 < 0.01


# ------------------------------------------------------- Z_N quantum numbers
def test_zn_paper_parity_example():
    """Sec. 8: with Z_2 addition, P=1 plus P=1 is P=0; a combined (N, Sz, P)
    QN adds componentwise with only P taken modulo 2."""
    assert Q.qn_reduce(Q.qn_add((1,), (1,)), (2,)) == (0,)
    a, b = (1, -1, 1), (2, 1, 1)
    assert Q.qn_reduce(Q.qn_add(a, b), (0, 0, 2)) == (3, 0, 0)
    assert Q.make_index([((5,), 1), ((-3,), 2)], +1, (4,)).sectors == (((1,), 1), ((1,), 2))


def _group_average(T, inds, flux, n_u1=64):
    """Projection of a dense array onto the tensors with the given flux under
    the symmetry group of the indices' QNs, by averaging the group action
    e^{i theta q} over the group (Z_N: its N elements; U(1): n_u1 equally
    spaced angles, exact for charge sums of magnitude below n_u1)."""
    mod = inds[0].mod or (0,) * len(inds[0].qn(0))
    out = T.astype(complex)
    for c, m in enumerate(mod):
        n = m if m else n_u1
        acc = np.zeros_like(out)
        for g in range(n):
            th = 2 * np.pi * g / n
            G = out.copy()
            for a, ind in enumerate(inds):
                ph = np.concatenate([np.full(nk, np.exp(1j * th * ind.arrow * q[c]))
                                     for q, nk in ind.sectors])
                shape = [1] * T.ndim
                shape[a] = -1
                G = G * ph.reshape(shape)
            acc += G * np.exp(-1j * th * flux[c])
        out = acc / n
    return out


@pytest.mark.parametrize("mod,flux", [((4,), (0,)), ((4,), (3,)), ((0, 3), (1, 2)), ((2, 0, 4), (0, 1, 1))])
def test_zn_allowed_blocks_match_group_projection(mod, flux):
    """A random dense array projected onto the symmetric subspace by group
    averaging equals its restriction to the allowed blocks (and nothing of it
    lies outside them)."""
    rng = np.random.default_rng(5)
    nq = len(mod)
    def idx(arrow, seed):
        r = np.random.default_rng(seed)
        return Q.make_index([(tuple(int(x) for x in r.integers(-3, 5, nq)), int(r.integers(1, 3)))
                             for _ in range(4)], arrow, mod)
    inds = [idx(+1, 1), idx(-1, 2), idx(+1, 3)]
    # distinct QNs per index (merge duplicates by building from unique QNs)
    inds = [Q.QNIndex(tuple({q: n for q, n in ind.sectors}.items()), ind.arrow, ind.mod) for ind in inds]
    T = rng.standard_normal([ind.dim for ind in inds])
    P = _group_average(T, inds, flux)
    assert np.abs(P.imag).max() < 1e-12
    B = Q.from_dense(T, inds, flux).to_dense()
    assert np.allclose(P.real, B, atol=1e-12)
    assert Q.outside_blocks_max(P.real, inds, flux) < 1e-12


def test_zn_contract_matches_dense():
    mod = (0, 4)
    a = Q.make_index([((0, 0), 2), ((1, 1), 3), ((1, 3), 1), ((2, 2), 2)], +1, mod)
    m = Q.make_index([((0, 0), 1), ((1, 1), 2), ((-1, 3), 1), ((0, 2), 2)], +1, mod)
    A = Q.random_blocks([a, m.dag(), a.dag()], (0, 0), 11, inp.block_values)
    B = Q.random_blocks([a, m, a.dag()], (1, 3), 12, inp.block_values)
    C = Q.contract_blocks(A, [1, 2, 3], B, [3, 4, 5], [1, 2, 4, 5])
    D = np.einsum("abc,cde->abde", A.to_dense(), B.to_dense())
    assert C.flux == (1, 3)
    assert np.allclose(C.to_dense(), D, atol=1e-12)
    assert Q.outside_blocks_max(D, C.inds, C.flux) < 1e-12


def test_zn_heff_blocks_match_embedded():
    """U(1) x Z_4 operands with a synthetic symmetric W: the blockwise H_eff
    equals the dense route, and the result keeps psi's flux."""
    bond = [((0, 0), 2), ((1, 1), 3), ((1, 3), 2), ((2, 2), 2), ((0, 2), 1)]
    site = [(0, 0), (1, 1), (1, 3), (2, 0)]
    link = [(0, 0), (1, 1), (-1, 3), (0, 2), (0, 0)]
    L, w1, w2, R, psi, W1, W2 = Q.heff_qn_operands_random_w(bond, bond, site, link, (0, 4), 21,
                                                            inp.block_values)
    yb = Q.heff_apply_blocks(L, w1, w2, R, psi)
    yd, ye = Q.heff_apply_embedded(L, w1, w2, R, psi)
    assert np.allclose(yb.to_dense(), yd, atol=1e-12)
    assert Q.outside_blocks_max(yd, psi.inds, psi.flux) < 1e-12
    assert len(psi.blocks) > 0 and W1.shape == (5, 5, 4, 4)
