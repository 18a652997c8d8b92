"""GPU parity of the block-sparse (QN) H_eff against the oracle's blockwise
route, through the C ABI (planner + grouped launches + hipGraph replay)."""
import numpy as np
import pytest
import torch

import paper_2007_14822_amd as itn
from oracle import qn as Q
from paper_2007_14822_amd import inputs as inp
from tests import qn_util as U
from tests.workloads import elementwise_ratio, group_rel_err, heff_error_factor, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-2}
GTOL = {"f64": 1e-9, "f32": 1e-4, "bf16": 3e-2}
TDT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


@pytest.fixture(scope="module")
def h():
    return itn.Handle(0)


def _gpu_desc(bt, dtype):
    d, flat = U.desc(bt, with_data=False)
    d["data"] = torch.as_tensor(flat, dtype=dtype, device=DEV)
    return d


def _run(h, ops, W1, W2, prec, nv, psis):
    """psis: list of nv oracle psi BlockTensors (same structure)."""
    L, w1, w2, R, psi = ops
    Ld, Rd = _gpu_desc(L, TDT[prec]), _gpu_desc(R, TDT[prec])
    Pd, _ = U.desc(psi, with_data=False)
    flat = np.concatenate([p.packed()[2] for p in psis])
    Pd["data"] = torch.as_tensor(flat, device=DEV)
    Od = dict(Pd)
    Od["data"] = torch.zeros_like(Pd["data"])
    plan = h.qn_plan(Ld, U.mpo_desc(W1, w1), U.mpo_desc(W2, w2), Rd, Pd, nv=nv, prec=prec)
    h.qn_apply(plan, Ld, Rd, Pd, Od)
    torch.cuda.synchronize()
    return plan, (Ld, Rd, Pd, Od), Od["data"].cpu().numpy()


def _ref(ops, psis):
    L, w1, w2, R, _ = ops
    return np.concatenate([Q.heff_apply_blocks(L, w1, w2, R, p).packed()[2] for p in psis])


def _perturbed(psi, seed):
    rng = np.random.default_rng(seed)
    out = Q.BlockTensor(psi.inds, psi.flux)
    for k, v in psi.blocks.items():
        out.blocks[k] = rng.standard_normal(v.shape)
    return out


@pytest.mark.parametrize("make", [U.small_u1, U.small_u1u1])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nv", [1, 3])
def test_qn_heff_parity(h, make, prec, nv):
    ops, W1, W2 = make()
    psis = [ops[4]] + [_perturbed(ops[4], 10 + v) for v in range(nv - 1)]
    _, _, got = _run(h, ops, W1, W2, prec, nv, psis)
    assert rel_err(got, _ref(ops, psis)) <= TOL[prec]


def test_qn_graph_replay_new_operands(h):
    """The captured graph is replayed with new psi/out buffers."""
    ops, W1, W2 = U.small_u1u1()
    plan, (Ld, Rd, Pd, Od), got = _run(h, ops, W1, W2, "f64", 1, [ops[4]])
    assert rel_err(got, _ref(ops, [ops[4]])) <= 1e-10
    for seed in (1, 2, 3):
        p2 = _perturbed(ops[4], seed)
        P2 = dict(Pd)
        P2["data"] = torch.as_tensor(p2.packed()[2], device=DEV)
        O2 = dict(Od)
        O2["data"] = torch.full_like(P2["data"], float("nan"))
        h.qn_apply(plan, Ld, Rd, P2, O2)
        torch.cuda.synchronize()
        assert rel_err(O2["data"].cpu().numpy(), _ref(ops, [p2])) <= 1e-10


def test_qn_deterministic(h):
    ops, W1, W2 = U.small_u1()
    plan, (Ld, Rd, Pd, Od), a = _run(h, ops, W1, W2, "bf16", 2, [ops[4], _perturbed(ops[4], 4)])
    h.qn_apply(plan, Ld, Rd, Pd, Od)
    torch.cuda.synchronize()
    b = Od["data"].cpu().numpy()
    assert np.array_equal(a, b)


def test_qn_structure_mismatch_rejected(h):
    ops, W1, W2 = U.small_u1()
    plan, (Ld, Rd, Pd, Od), _ = _run(h, ops, W1, W2, "f64", 1, [ops[4]])
    bad = dict(Rd)
    bad["blocks"] = Rd["blocks"][:-1]
    bad["offsets"] = Rd["offsets"][:-1]
    with pytest.raises(itn.ItnError) as e:
        h.qn_apply(plan, Ld, bad, Pd, Od)
    assert e.value.name == "ITN_E_SHAPE"


def _sector_refs(L, w1, w2, R, psi, chosen):
    """The oracle's output blocks of the a'-sectors in `chosen` (L restricted
    to those rows), and the same for the absolute values of every operand."""
    def restrict(Lt):
        return Q.BlockTensor(Lt.inds, Lt.flux, {k: v for k, v in Lt.blocks.items() if k[0] in chosen})
    ref = Q.heff_apply_blocks(restrict(L), w1, w2, R, psi)
    aref = Q.heff_apply_blocks(restrict(U.abs_blocks(L)), U.abs_blocks(w1), U.abs_blocks(w2),
                               U.abs_blocks(R), U.abs_blocks(psi))
    return ref, aref


def _check_sectors(got, psi, ref, aref, chosen, prec, c, what):
    """Every output block of the chosen a'-sectors: relative error per block
    (blocks of 16+ elements), element-wise rounding bound, 16-element runs."""
    keys, offs, _ = psi.packed()
    g_all, r_all, a_all = [], [], []
    worst_blk = 0.0
    for k, o in zip(keys, offs):
        if k[0] not in chosen:
            continue
        n = psi.blocks[k].size
        r = ref.blocks[k].ravel() if k in ref.blocks else np.zeros(n)
        a = aref.blocks[k].ravel() if k in aref.blocks else np.zeros(n)
        g = got[o:o + n]
        if n >= 16:
            worst_blk = max(worst_blk, rel_err(g, r))
        g_all.append(g)
        r_all.append(r)
        a_all.append(a)
        # runs of 16 inside the block (the last axis is b, rows are (a', s1', s2'))
        assert group_rel_err(g.reshape(-1, psi.blocks[k].shape[-1]),
                             r.reshape(-1, psi.blocks[k].shape[-1])) <= GTOL[prec], (what, k)
    g_all, r_all, a_all = map(np.concatenate, (g_all, r_all, a_all))
    e = rel_err(g_all, r_all)
    q = elementwise_ratio(g_all, r_all, a_all, c)
    print("qn", what, prec, "rel %.2e  worst block %.2e  elementwise %.3f of bound"
          % (e, worst_blk, q))
    assert e <= TOL[prec], (what, e)
    assert worst_blk <= 5 * TOL[prec], (what, worst_blk)
    assert q <= 1.0, (what, q)


def _qn_factor(prec, L, w1, R, psi):
    """Rounding-error factor of a QN apply: the dense bound's stages with
    the full bond dimensions as the sum lengths (upper bounds of every
    block sum), X stored in the operand type (five rounded operands)."""
    chil, w, chir = L.inds[0].dim, w1.inds[0].dim, R.inds[0].dim
    d2 = psi.inds[1].dim * psi.inds[2].dim
    return heff_error_factor(prec, chil, w * d2, w * chir, op_roundings=5, w=w)


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_c3_full_size_sampled_sectors(h, prec):
    """U(1) chi=4096 in 25 sectors (the benchmark workload): every output
    block of three a'-sectors against the oracle restricted to those rows."""
    ops, W1, W2 = U.c3_operands()
    L, w1, w2, R, psi = ops
    _, _, got = _run(h, ops, W1, W2, prec, 1, [psi])
    chosen = {0, 7, 17}  # dims 8, 35, 107
    ref, aref = _sector_refs(L, w1, w2, R, psi, chosen)
    _check_sectors(got, psi, ref, aref, chosen, prec, _qn_factor(prec, L, w1, R, psi), "c3")


@pytest.mark.parametrize("which", ["c4", "c4w38", "c4z4"])
def test_c4_full_size_sampled_sectors(h, which):
    """The Hubbard cylinder bond at full size and nv = 4, as the benchmark
    launches it (chi = 4096 in 81 (dN, 2Sz) sectors with w = 18 or the
    w = 38 shape; or 272 sectors with a Z_4 momentum label): every output
    block of four a'-sectors of the first and last vector against the oracle
    restricted to those rows, in FP64 and bf16."""
    ops, W1, W2 = U.c4_operands(which, nv=4)
    L, w1, w2, R, psis = ops
    nsec = L.inds[0].nsec
    if which == "c4z4":
        chosen = {134, 79, 102, 10}  # (0,0,0): 81, (-2,-2,1): 30, (-1,-3,1): 23, (-5,-5,0): 1
    else:
        chosen = {40, 24, 31, 5}  # (0,0): 324, (-2,-2): 120, (-1,-3): 93, (-5,-5): 1
    assert max(chosen) < nsec
    refs = {v: _sector_refs(L, w1, w2, R, psis[v], chosen) for v in (0, 3)}
    n1 = sum(b.size for b in psis[0].blocks.values())
    for prec in ("f64", "bf16"):
        _, _, got = _run(h, (L, w1, w2, R, psis[0]), W1, W2, prec, 4, psis)
        c = _qn_factor(prec, L, w1, R, psis[0])
        for v in (0, 3):
            _check_sectors(got[v * n1:(v + 1) * n1], psis[v], *refs[v], chosen, prec, c,
                           (which, v))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nv", [1, 2])
def test_zn_three_component_parity(h, prec, nv):
    """U(1) x U(1) x Z_4 QNs ((dN, 2Sz, momentum mod 4), the cylinder's
    three-component structure at small size) with a synthetic symmetric W."""
    ops, W1, W2 = U.small_u1u1z4()
    psis = [ops[4]] + [_perturbed(ops[4], 60 + v) for v in range(nv - 1)]
    _, _, got = _run(h, ops, W1, W2, prec, nv, psis)
    assert rel_err(got, _ref(ops, psis)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("which", ["large_u1", "zn_u1z4_x20"])
def test_qn_launch_modes_parity(h, monkeypatch, prec, which):
    """Every grouped launch mode, forced, against the oracle: sectors of a
    few hundred states (ragged M, N, K: the 256-tile path with K tails), and
    U(1) x Z_4 sectors of 20-60 states, whose Z x R products are narrow
    (N < 96 on the 256 x 64 tiles of mode 6)."""
    ops, W1, W2 = U.large_u1() if which == "large_u1" else U.zn_u1z4(scale=20)
    ref = _ref(ops, [ops[4]])
    for mode in ("0,0", "1,1", "2,2", "3,3", "2,3", "3,2", "4,4", "5,5", "4,5", "6,6", "5,6", "7,7"):
        monkeypatch.setenv("ITN_QN_TILE_MODE", mode)
        plan, _, got = _run(h, ops, W1, W2, prec, 1, [ops[4]])
        assert plan.info()["n_tiles"] > 0
        assert rel_err(got, ref) <= TOL[prec], (mode, prec)
        del plan


def test_qn_bf16_operand_rounds_once(h):
    """psi's FP64 -> bf16 conversion on the block-sparse path is one rounding
    to nearest, ties to even.  With identity environments (L, R = 1 on every
    diagonal block) and a one-channel identity MPO, H_eff psi = psi, and
    every later step is exact in bf16 / f32 (products with 1, sums of one
    term), so the output is psi rounded to bf16: values just above and below
    bf16 midpoints (where rounding to FP32 first lands on the midpoint and
    then ties to even) and random values, against the exact reference."""
    bl = [((-2,), 3), ((0,), 5), ((2,), 4)]
    br = [((-2,), 2), ((0,), 4), ((2,), 5), ((4,), 3)]
    W = np.zeros((1, 1, 2, 2))
    W[0, 0] = np.eye(2)
    L, w1, w2, R, psi = Q.heff_qn_operands(bl, br, inp.heisenberg_site_qn(1), [0], W, W, 5,
                                           inp.block_values)
    for env in (L, R):
        for k in env.blocks:
            assert k[0] == k[2]
            env.blocks[k] = np.eye(env.blocks[k].shape[0]).reshape(env.blocks[k].shape)
    rng = np.random.default_rng(17)
    ulp = 2.0 ** -7
    for k, blk in psi.blocks.items():
        base = (1.0 + rng.integers(0, 127, blk.shape) * ulp) * rng.choice([-1.0, 1.0], blk.shape)
        kind = rng.integers(0, 4, blk.shape)
        off = np.choose(kind, [0.5 * ulp, 0.5 * ulp + 2.0 ** -30, 0.5 * ulp - 2.0 ** -30,
                               rng.random(blk.shape) * ulp])
        psi.blocks[k] = (base + np.sign(base) * off) * 2.0 ** rng.integers(-4, 4, blk.shape)
    flat = psi.packed()[2]
    e = np.floor(np.log2(np.abs(flat)))
    q = 2.0 ** (e - 7)
    ref = np.rint(flat / q) * q
    _, _, got = _run(h, (L, w1, w2, R, psi), W, W, "bf16", 1, [psi])
    assert np.array_equal(got, ref), np.flatnonzero(got != ref)[:8]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nv", [1, 3])
def test_zn_heff_parity(h, prec, nv):
    """U(1) x Z_4 QNs (Z_N addition, Sec. 8) with a synthetic symmetric W."""
    ops, W1, W2 = U.zn_u1z4()
    psis = [ops[4]] + [_perturbed(ops[4], 30 + v) for v in range(nv - 1)]
    _, _, got = _run(h, ops, W1, W2, prec, nv, psis)
    assert rel_err(got, _ref(ops, psis)) <= TOL[prec]


@pytest.mark.parametrize("mode", ["0,0", "2,3", "4,5"])
def test_zn_large_sectors_parity(h, monkeypatch, mode):
    """U(1) x Z_4 sectors of 100-300 states (the 256-row tiles, K tails)."""
    monkeypatch.setenv("ITN_QN_TILE_MODE", mode)
    ops, W1, W2 = U.zn_u1z4(scale=100)
    for prec in ("f64", "bf16"):
        _, _, got = _run(h, ops, W1, W2, prec, 1, [ops[4]])
        assert rel_err(got, _ref(ops, [ops[4]])) <= TOL[prec], (mode, prec)


@pytest.mark.parametrize("wk", ["64", "128", "256"])
@pytest.mark.parametrize("make", [U.small_u1u1, U.zn_u1z4, U.u1_degenerate_site])
def test_qn_wstage_kernels_parity(h, monkeypatch, wk, make):
    """Every W-stage work-item size (one wave with one, two or four vectors
    per lane) gives the oracle's result, with b-sectors that are not
    multiples of the 16-byte vector (padded columns)."""
    monkeypatch.setenv("ITN_QN_WSTAGE", wk)
    ops, W1, W2 = make()
    for prec in ("f64", "bf16"):
        _, _, got = _run(h, ops, W1, W2, prec, 2, [ops[4], _perturbed(ops[4], 7)])
        assert rel_err(got, _ref(ops, [ops[4], _perturbed(ops[4], 7)])) <= TOL[prec], (wk, prec)


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_qn_prepared_environments(h, prec):
    """Applies with environments prepared once (itn_qn_prepare_env, L = R =
    NULL) give the same output as applies that pass L and R, across new psi
    buffers and a second environment pair; a prepared apply on a fresh plan,
    or with only one environment, is an argument error."""
    ops, W1, W2 = U.small_u1u1()
    L, w1, w2, R, psi = ops
    Ld, Rd = _gpu_desc(L, TDT[prec]), _gpu_desc(R, TDT[prec])
    Pd, _ = U.desc(psi, with_data=False)
    Pd["data"] = torch.as_tensor(psi.packed()[2], device=DEV)
    Od = dict(Pd)
    Od["data"] = torch.zeros_like(Pd["data"])
    plan = h.qn_plan(Ld, U.mpo_desc(W1, w1), U.mpo_desc(W2, w2), Rd, Pd, nv=1, prec=prec)
    with pytest.raises(itn.ItnError):
        h.qn_apply(plan, None, None, Pd, Od)  # nothing prepared yet
    with pytest.raises(itn.ItnError):
        h.qn_apply(plan, Ld, None, Pd, Od)
    # a second environment pair of the same structure (scaled values)
    L2d, R2d = dict(Ld), dict(Rd)
    L2d["data"] = Ld["data"] * 0.5
    R2d["data"] = Rd["data"] * 2.0
    for envs in ((Ld, Rd), (L2d, R2d)):
        plan.prepare_env(*envs)
        for seed in (1, 2):
            p2 = _perturbed(psi, seed)
            P2 = dict(Pd)
            P2["data"] = torch.as_tensor(p2.packed()[2], device=DEV)
            Oa, Ob = dict(Od), dict(Od)
            Oa["data"] = torch.full_like(P2["data"], float("nan"))
            Ob["data"] = torch.full_like(P2["data"], float("nan"))
            h.qn_apply(plan, None, None, P2, Oa)
            h.qn_apply(plan, envs[0], envs[1], P2, Ob)
            torch.cuda.synchronize()
            a, b = Oa["data"].cpu().numpy(), Ob["data"].cpu().numpy()
            assert np.array_equal(a, b), (prec, seed)
            # (0.5 L, 2 R): exact power-of-two scalings, the same H_eff
            ref = Q.heff_apply_blocks(L, w1, w2, R, p2).packed()[2]
            assert rel_err(a, ref) <= TOL[prec], (prec, seed)


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_splitblocks_mpo_sectors_parity(h, prec):
    """The sparse-MPO form (every MPO channel its own link sector, so equal
    charges repeat): the planner and grouped launches against the oracle on
    the Hubbard MPO."""
    from oracle import qn as Qn
    from paper_2007_14822_amd import inputs as inp
    Ws = inp.hubbard_mpo(2, 4)
    link_q = inp.hubbard_mpo_link_qn(Ws[0].shape[0])
    link = Qn.make_index([(q, 1) for q in link_q], +1)
    site = Qn.index_from_basis_qns(inp.hubbard_site_qn())
    bl = [((0, 0), 2), ((1, 1), 3), ((1, -1), 2), ((2, 0), 4)]
    br = [((1, 1), 2), ((2, 0), 3), ((3, 1), 2), ((2, 2), 1), ((3, -1), 2)]
    al, ar = Qn.make_index(bl, +1), Qn.make_index(br, +1)
    L, R, psi = Qn._env_and_psi(al, ar, site, link, 99, inp.block_values, None)
    w1 = Qn.mpo_blocks(Ws[5], link, link, site)
    w2 = Qn.mpo_blocks(Ws[6], link, link, site)
    ops = (L, w1, w2, R, psi)
    assert link.nsec == Ws[0].shape[0]
    _, _, got = _run(h, ops, Ws[5], Ws[6], prec, 2, [psi, _perturbed(psi, 3)])
    assert rel_err(got, _ref(ops, [psi, _perturbed(psi, 3)])) <= TOL[prec]


@pytest.mark.parametrize("make", [U.small_u1, U.small_u1u1, U.zn_u1z4, U.small_u1u1z4])
def test_qn_heff_diag_matches_oracle_unit_vectors(h, make):
    """itn_qn_heff_diag (block Davidson's preconditioner) equals the diagonal
    of the oracle's block-sparse H_eff, read off entry by entry by applying
    it to every unit vector of psi's block layout (brute force), to 1e-12
    relative; under U(1), U(1) x U(1), U(1) x Z_4 and three-component rules."""
    ops, W1, W2 = make()[:3]
    L, w1, w2, R, psi = ops
    Ld, Rd = _gpu_desc(L, torch.float64), _gpu_desc(R, torch.float64)
    Pd, _ = U.desc(psi, with_data=False)
    keys, offs, flat = psi.packed()
    Od = dict(Pd)
    Od["data"] = torch.full((flat.size,), float("nan"), dtype=torch.float64, device=DEV)
    h.qn_heff_diag(Ld, U.mpo_desc(W1, w1), U.mpo_desc(W2, w2), Rd, Od)
    torch.cuda.synchronize()
    got = Od["data"].cpu().numpy()
    ref = np.empty(flat.size)
    for k, o in zip(keys, offs):
        shape = psi.blocks[k].shape
        for j in range(int(np.prod(shape))):
            e = Q.BlockTensor(psi.inds, psi.flux, {kk: np.zeros(v.shape) for kk, v in psi.blocks.items()})
            e.blocks[k].flat[j] = 1.0
            out = Q.heff_apply_blocks(L, w1, w2, R, e).blocks.get(k)
            ref[o + j] = 0.0 if out is None else out.flat[j]
    assert np.all(np.isfinite(got))
    scale = np.abs(ref).max()
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)
