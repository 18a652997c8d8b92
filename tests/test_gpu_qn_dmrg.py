"""GPU two-site DMRG on block-sparse (QN) MPS through the C ABI: block-sparse
H_eff, per-sector bond split, block-sparse environments; against exact
diagonalisation, with the total QN conserved."""
import numpy as np
import pytest

import paper_2007_14822_amd as itn
from paper_2007_14822_amd import inputs as inp
from oracle import dmrg as odmrg, ed, heff as hf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    hd = itn.Handle(0)
    yield hd
    hd.close()


def _state_qn(sites, site_qn):
    """Total QN of every basis state of the dense state vector (site order)."""
    d = len(site_qn)
    tot = np.zeros((d,) * len(sites) + (len(site_qn[0]),))
    grids = np.meshgrid(*[np.arange(d)] * len(sites), indexing="ij")
    sq = np.array(site_qn)
    for g in grids:
        tot += sq[g]
    return tot


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_u1_heisenberg_matches_ed(h, prec):
    """S=1/2 chain, N = 10, U(1) 2Sz sectors, Neel start (total 2Sz = 0),
    maxdim 32 (exact): the energy equals ED to 1e-10, the state stays in
    the 2Sz = 0 sector, and its energy from the returned tensors agrees."""
    N = 10
    e0 = float(np.linalg.eigvalsh(ed.heisenberg_dense(N))[0])
    site_qn = [(q,) for q in inp.heisenberg_site_qn(1)]
    mps = h.qn_mps(site_qn, [k % 2 for k in range(N)])
    mpo = h.mpo(inp.heisenberg_mpo(N))
    link_qn = [(q,) for q in inp.heisenberg_mpo_link_qn()]
    recs = h.qn_dmrg_sweep(mps, mpo, link_qn, [(32, 1e-14)] * 5, prec=prec, eig_tol=1e-12,
                           krylovdim=12, maxiter=400)
    E = recs[-1]["energy"]
    print("qn heis", prec, E - e0, [r["energy"] for r in recs], h.qn_mps_bonds(mps))
    assert abs(E - e0) / abs(e0) <= 1e-10
    assert h.qn_mps_link(mps, N) == [((0,), 1)] and h.qn_mps_link(mps, 0) == [((0,), 1)]
    sites = h.qn_mps_sites(mps)
    psi = hf.mps_to_dense(sites).reshape((2,) * N)
    qtot = _state_qn(sites, site_qn)[..., 0]
    assert np.abs(psi[qtot != 0]).max(initial=0.0) == 0.0
    assert abs(hf.mps_energy(sites, inp.heisenberg_mpo(N)) - E) <= 1e-9 * abs(E)
    if prec != "f64":
        assert sum(r["matvecs"] for r in recs) > sum(r["matvecs_f64"] for r in recs)


def test_spin1_chain_matches_ed(h):
    N = 6
    e0 = float(np.linalg.eigvalsh(ed.heisenberg_dense(N, 2))[0])
    site_qn = [(q,) for q in inp.heisenberg_site_qn(2)]
    mps = h.qn_mps(site_qn, [0, 2] * (N // 2))
    mpo = h.mpo(inp.heisenberg_mpo(N, 2))
    recs = h.qn_dmrg_sweep(mps, mpo, [(q,) for q in inp.heisenberg_mpo_link_qn()], [(27, 1e-14)] * 5,
                           eig_tol=1e-12, krylovdim=12, maxiter=400)
    assert abs(recs[-1]["energy"] - e0) / abs(e0) <= 1e-10


def test_hubbard_2x2_u1u1_matches_ed(h):
    """U(1) x U(1) (N, 2Sz): the 2 x 2 Hubbard cluster at half filling, Neel
    start; the energy equals ED in the (N_up, N_dn) = (2, 2) sector (the
    global minimum of the Fock space lies at N = 2, which a dense sweep can
    drift to through rounding; the block-sparse one cannot), and N = 4,
    2Sz = 0 are conserved."""
    Lx, Ly = 2, 2
    e0 = float(ed.hubbard_sector_ground_energy(Lx, Ly, 2, 2, U=8.0))
    assert e0 > float(np.linalg.eigvalsh(ed.hubbard_dense(Lx, Ly, U=8.0))[0]) + 1.0
    Ws = inp.hubbard_mpo(Lx, Ly, U=8.0)
    mps = h.qn_mps(inp.hubbard_site_qn(), [1, 2, 1, 2])
    mpo = h.mpo(Ws)
    recs = h.qn_dmrg_sweep(mps, mpo, inp.hubbard_mpo_link_qn(Ws[0].shape[0]), [(64, 1e-14)] * 4,
                           eig_tol=1e-12, krylovdim=12, maxiter=400)
    assert abs(recs[-1]["energy"] - e0) / abs(e0) <= 1e-10
    assert h.qn_mps_link(mps, 4) == [((4, 0), 1)]


def test_hubbard_4x1_half_filling(h):
    """The 4-site Hubbard chain from a Neel state stays at half filling: its
    energy is the (2, 2) sector's ED ground energy."""
    Ws = inp.hubbard_mpo(4, 1, U=8.0)
    e0 = float(ed.hubbard_sector_ground_energy(4, 1, 2, 2, U=8.0))
    mps = h.qn_mps(inp.hubbard_site_qn(), [1, 2, 1, 2])
    recs = h.qn_dmrg_sweep(mps, h.mpo(Ws), inp.hubbard_mpo_link_qn(Ws[0].shape[0]), [(64, 1e-14)] * 3,
                           eig_tol=1e-12, krylovdim=12, maxiter=400)
    assert abs(recs[-1]["energy"] - e0) / abs(e0) <= 1e-10


def test_truncated_u1_sweep_tracks_dense(h):
    """N = 16 chain with maxdim 16 then 24 (truncating): the block-sparse sweep
    keeps the sector structure, respects maxdim, and its converged energy
    agrees with the dense GPU sweep at the same schedule to 1e-8."""
    N = 16
    sched = [(16, 1e-10), (24, 1e-10), (24, 1e-10), (24, 1e-10)]
    site_qn = [(q,) for q in inp.heisenberg_site_qn(1)]
    mps = h.qn_mps(site_qn, [k % 2 for k in range(N)])
    mpo = h.mpo(inp.heisenberg_mpo(N))
    rq = h.qn_dmrg_sweep(mps, mpo, [(q,) for q in inp.heisenberg_mpo_link_qn()], sched, eig_tol=1e-11,
                         krylovdim=12, maxiter=400)
    dmps = h.mps(inp.neel_product_state(N, 2))
    rd = h.dmrg_sweep(dmps, mpo, sched, eig_tol=1e-11, krylovdim=12, maxiter=400)
    print("trunc", [r["energy"] for r in rq], [r["energy"] for r in rd], h.qn_mps_bonds(mps))
    assert max(h.qn_mps_bonds(mps)) <= 24
    assert rq[-1]["max_trunc"] > 0.0
    assert abs(rq[-1]["energy"] - rd[-1]["energy"]) <= 1e-8 * abs(rd[-1]["energy"])
    for k in range(N + 1):  # every link's sectors sum to its dimension; charges distinct
        secs = h.qn_mps_link(mps, k)
        assert len({q for q, _ in secs}) == len(secs)


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_hubbard_3x2_block_davidson_matches_ed(h, prec):
    """Block Davidson on block-sparse sweeps (4 residuals per step,
    preconditioned with the block-sparse H_eff diagonal, one batched matvec
    per step): the 3 x 2 Hubbard cylinder at half filling reaches the
    (3, 3)-sector ED energy; N = 6, 2Sz = 0 stay conserved; in bf16 most
    matvecs run in bf16 and the FP64 restarts bring the energy to the FP64
    one."""
    Lx, Ly = 3, 2
    e0 = float(ed.hubbard_sector_ground_energy(Lx, Ly, 3, 3, U=8.0))
    Ws = inp.hubbard_mpo(Lx, Ly, U=8.0)
    mps = h.qn_mps(inp.hubbard_site_qn(), [1, 2] * 3)
    recs = h.qn_dmrg_sweep(mps, h.mpo(Ws), inp.hubbard_mpo_link_qn(Ws[0].shape[0]), [(64, 1e-14)] * 5,
                           prec=prec, eig_tol=1e-12, krylovdim=16, maxiter=400, block=4)
    E = recs[-1]["energy"]
    print("qn block", prec, E - e0, [r["energy"] for r in recs],
          [(r["matvecs"], r["matvecs_f64"]) for r in recs])
    assert abs(E - e0) / abs(e0) <= 1e-10
    assert h.qn_mps_link(mps, Lx * Ly) == [((6, 0), 1)]
    if prec != "f64":
        mv = sum(r["matvecs"] for r in recs)
        assert mv - sum(r["matvecs_f64"] for r in recs) >= 0.5 * mv


def test_block_davidson_matches_single_vector_sweep(h):
    """The same truncating schedule on the N = 16 S=1/2 chain with block = 4
    and block = 1 converges to the same energy (to 1e-9) and bond sizes."""
    N = 16
    sched = [(16, 1e-10), (24, 1e-10), (24, 1e-10), (24, 1e-10), (24, 1e-10)]
    site_qn = [(q,) for q in inp.heisenberg_site_qn(1)]
    lq = [(q,) for q in inp.heisenberg_mpo_link_qn()]
    mpo = h.mpo(inp.heisenberg_mpo(N))
    out = []
    for block in (1, 4):
        mps = h.qn_mps(site_qn, [k % 2 for k in range(N)])
        r = h.qn_dmrg_sweep(mps, mpo, lq, sched, eig_tol=1e-11, krylovdim=12, maxiter=400, block=block)
        out.append((r[-1]["energy"], h.qn_mps_bonds(mps)))
    print("block vs single", out)
    assert abs(out[0][0] - out[1][0]) <= 1e-9 * abs(out[0][0])
    assert max(out[1][1]) <= 24


@pytest.mark.parametrize("sched", [[(4, 0.0), (8, 0.0), (8, 0.0)], [(16, 1e-6), (16, 1e-8), (32, 1e-10)],
                                   [(8, 1e-10), (12, 1e-10), (12, 1e-10)]])
def test_truncating_qn_sweeps_match_oracle(h, sched):
    """The per-sector bond split against the oracle's dense one (N = 12 S=1/2
    chain from the Neel state, maxdim 4 .. 32, cutoffs 0 .. 1e-6; the
    oracle's states stay at total 2Sz = 0): per sweep the largest bond
    dimension equals the oracle's, the largest discarded weight agrees to
    1e-8 relative and the energy to 1e-10; the final bond dimensions match
    site by site."""
    N = 12
    ref = odmrg.dmrg(inp.heisenberg_mpo(N), inp.neel_product_state(N, 2), sched)
    site_qn = [(q,) for q in inp.heisenberg_site_qn(1)]
    mps = h.qn_mps(site_qn, [k % 2 for k in range(N)])
    recs = h.qn_dmrg_sweep(mps, h.mpo(inp.heisenberg_mpo(N)), [(q,) for q in inp.heisenberg_mpo_link_qn()],
                           sched, eig_tol=1e-13, krylovdim=12, maxiter=800, allow_unconverged=True)
    for r, o in zip(recs, ref.records):
        print("sweep", o.sweep, r["max_bond"], o.max_bond, r["max_trunc"], o.max_trunc, r["energy"], o.energy)
        assert r["max_bond"] == o.max_bond
        assert abs(r["max_trunc"] - o.max_trunc) <= 1e-8 * o.max_trunc + 1e-14
        assert abs(r["energy"] - o.energy) <= 1e-10 * abs(o.energy)
    assert h.qn_mps_bonds(mps) == [1] + [A.shape[2] for A in ref.mps]
