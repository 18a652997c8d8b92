"""GPU parity of the block-sparse labelled contraction (itn_contract with QN
operands) against the oracle's blockwise contraction (Sec. 8, 9.4)."""
import numpy as np
import pytest
import torch

import paper_2007_14822_amd as itn
from paper_2007_14822_amd import inputs as inp
from oracle import qn as Q
from tests import qn_util as U
from tests.workloads import rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module")
def h():
    hd = itn.Handle(0)
    yield hd
    hd.close()


def _dev_desc(bt, dtype=torch.float64):
    d, flat = U.desc(bt, with_data=False)
    d["data"] = torch.as_tensor(flat, dtype=dtype, device=DEV)
    return d


def _out_desc(inds, flux, blocks=None, dtype=torch.float64):
    """C descriptor: the given blocks (default every allowed block), filled
    with NaN so that unwritten elements show."""
    blocks = Q.allowed_blocks(inds, flux) if blocks is None else blocks
    sizes = [int(np.prod([inds[i].sdim(k) for i, k in enumerate(b)])) for b in blocks]
    offs = [int(x) for x in np.cumsum([0] + sizes)[:len(sizes)]]
    d = {"spaces": [U.space(i) for i in inds], "blocks": blocks, "offsets": offs,
         "flux": list(Q.qn_reduce(tuple(flux), Q.common_mod(inds)) if inds else flux),
         "data": torch.full((max(1, sum(sizes)),), float("nan"), dtype=dtype, device=DEV)}
    return d


def _check(h, A, la, B, lb, lc, prec="f64", cdt=torch.float64, extra_blocks=False):
    ref = Q.contract_blocks(A, la, B, lb, lc)
    blocks = sorted(ref.blocks) if not extra_blocks else None
    Cd = _out_desc(ref.inds, ref.flux, blocks, cdt)
    h.contract_blocks(_dev_desc(A), la, _dev_desc(B), lb, Cd, lc, prec=prec)
    torch.cuda.synchronize()
    got = Cd["data"].double().cpu().numpy()
    keys = Cd["blocks"]
    offs = Cd["offsets"]
    assert not np.isnan(got[:sum(int(np.prod(ref.block_shape(k))) for k in keys)]).any()
    gvals, rvals = [], []
    for k, o in zip(keys, offs):
        n = int(np.prod(ref.block_shape(k)))
        g = got[o:o + n]
        r = ref.blocks[k].ravel() if k in ref.blocks else np.zeros(n)
        if k not in ref.blocks:
            assert np.all(g == 0.0), k  # blocks no pair reaches are zero
        gvals.append(g)
        rvals.append(r)
    e = rel_err(np.concatenate(gvals), np.concatenate(rvals))
    assert e <= max(TOL[prec], 1e-6 if cdt == torch.float32 else 0), (prec, e)
    return ref


def test_paper_hardcore_boson_number_operator(h):
    """Sec. 8.3: a (flux -1, one stored element) contracted with a^dagger
    gives n = a^dagger a, flux zero, two blocks, diag(0, 1)."""
    s = Q.make_index([((0,), 1), ((1,), 1)], +1)
    a = Q.from_dense(np.array([[0.0, 1.0], [0.0, 0.0]]), [s, s.dag()], (-1,))
    adag = Q.from_dense(np.array([[0.0, 0.0], [1.0, 0.0]]), [s, s.dag()], (1,))
    ref = _check(h, adag, [1, 2], a, [2, 3], [1, 3])
    assert np.allclose(ref.to_dense(), np.diag([0.0, 1.0]))


def test_label_example_with_sectors(h):
    """The Sec. 9.1 contraction contract(A,(-1,1,-2),B,(2,-2,-1)) with A
    [3,7,2], B [4,2,3] -> C [7,4], its indices split into U(1) sectors."""
    i3 = Q.make_index([((0,), 1), ((1,), 2)], +1)
    i7 = Q.make_index([((-1,), 2), ((0,), 3), ((1,), 2)], +1)
    i2 = Q.make_index([((0,), 1), ((2,), 1)], +1)
    i4 = Q.make_index([((0,), 2), ((1,), 1), ((3,), 1)], +1)
    A = Q.random_blocks([i3, i7.dag(), i2], (1,), 5, inp.block_values)
    B = Q.random_blocks([i4, i2.dag(), i3.dag()], (0,), 6, inp.block_values)
    ref = _check(h, A, [-1, 1, -2], B, [2, -2, -1], [1, 2])
    assert [ind.dim for ind in ref.inds] == [7, 4]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("lc", [[1, 2, 5, 6], [6, 2, 1, 5]])
def test_u1u1_rank4_mixed_arrows(h, prec, lc):
    """U(1) x U(1) rank-4 tensors with fluxes, both arrow directions on the
    contracted pair, several pairs per output block, natural and permuted
    output orders."""
    a = Q.make_index([((0, 0), 3), ((1, 1), 5), ((1, -1), 4), ((2, 0), 6), ((0, 2), 2)], +1)
    b = Q.make_index([((0, 0), 2), ((1, 1), 3), ((-1, 1), 2), ((1, -1), 4)], +1)
    c = Q.make_index([((0, 0), 7), ((1, 1), 9), ((1, -1), 5), ((2, 0), 3)], +1)
    A = Q.random_blocks([a, b.dag(), c, a.dag()], (1, 1), 7, inp.block_values)
    B = Q.random_blocks([c.dag(), b, a, b.dag()], (0, 0), 8, inp.block_values)
    # labels 3 (c Out on A, In on B) and 4 (a In on A, Out on B) contracted
    _check(h, A, [1, 2, 3, 4], B, [3, 5, 4, 6], lc, prec)


def test_zn_contraction(h):
    mod = (0, 4)
    a = Q.make_index([((0, 0), 2), ((1, 1), 3), ((1, 3), 1), ((2, 2), 2)], +1, mod)
    m = Q.make_index([((0, 0), 1), ((1, 1), 2), ((-1, 3), 1), ((0, 2), 2)], +1, mod)
    A = Q.random_blocks([a, m.dag(), a.dag()], (0, 0), 11, inp.block_values)
    B = Q.random_blocks([a, m, a.dag()], (1, 3), 12, inp.block_values)
    ref = _check(h, A, [1, 2, 3], B, [3, 4, 5], [1, 2, 4, 5])
    assert ref.flux == (1, 3)


def test_outer_and_full_contraction(h):
    i = Q.make_index([((0,), 3), ((1,), 2), ((2,), 4)], +1)
    j = Q.make_index([((0,), 2), ((1,), 5)], +1)
    A = Q.random_blocks([i, j.dag()], (0,), 13, inp.block_values)
    B = Q.random_blocks([j, i.dag()], (-1,), 14, inp.block_values)
    _check(h, A, [1, 2], B, [3, 4], [3, 1, 4, 2])  # outer product, permuted
    ref = _check(h, A, [1, 2], B, [2, 3], [1, 3])  # matrix product, flux -1
    assert ref.flux == (-1,)
    B0 = Q.random_blocks([j, i.dag()], (0,), 15, inp.block_values)
    full = Q.contract_blocks(A, [1, 2], B0, [2, 1], [])
    Cd = {"spaces": [], "blocks": [()], "offsets": [0], "flux": [0],
          "data": torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)}
    h.contract_blocks(_dev_desc(A), [1, 2], _dev_desc(B0), [2, 1], Cd, [])
    torch.cuda.synchronize()
    got = float(Cd["data"].cpu()[0])
    assert abs(got - float(full.blocks[()].ravel()[0])) <= 1e-12 * max(1.0, abs(got))


def test_unreached_output_blocks_are_zeroed(h):
    """C may list flux-allowed blocks no pair reaches: they come back zero."""
    i = Q.make_index([((0,), 3), ((1,), 2), ((2,), 4)], +1)
    j = Q.make_index([((0,), 2), ((3,), 5)], +1)
    A = Q.random_blocks([i, j.dag()], (-1,), 16, inp.block_values)
    B = Q.random_blocks([j, i.dag()], (0,), 17, inp.block_values)
    _check(h, A, [1, 2], B, [2, 3], [1, 3], extra_blocks=True)


def test_large_sectors_grouped(h):
    """Sectors of a few hundred states (several 128x128 tiles per block
    product, several pairs summed per output block) in f64 and bf16."""
    a = Q.make_index([((-2,), 197), ((0,), 301), ((2,), 229)], +1)
    m = Q.make_index([((-2,), 1), ((0,), 3), ((2,), 1)], +1)
    L = Q.random_blocks([a, m.dag(), a.dag()], (0,), 18, inp.block_values)
    P = Q.random_blocks([a, m, a.dag()], (0,), 19, inp.block_values)
    for prec in ("f64", "bf16"):
        _check(h, L, [1, 2, 3], P, [3, 2, 4], [1, 4], prec)
