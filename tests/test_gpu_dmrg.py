"""GPU two-site DMRG sweeps (FP64 Davidson, rocSOLVER bond split) through
the C ABI, against exact diagonalisation and the oracle."""
import numpy as np
import pytest

import paper_2007_14822_amd as itn
from paper_2007_14822_amd import inputs as inp
from oracle import dmrg as odmrg, ed, heff as hf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    return itn.Handle(0)


@pytest.fixture(scope="module")
def e_ed10():
    return float(np.linalg.eigvalsh(ed.heisenberg_dense(10))[0])


def run(h, Ws, As0, sweeps, **kw):
    mpo = h.mpo(Ws)
    mps = h.mps(As0)
    recs = h.dmrg_sweep(mps, mpo, sweeps, **kw)
    return recs, mps


@pytest.mark.parametrize("block", [1, 4])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_c0_heisenberg_matches_ed(h, e_ed10, prec, block):
    """N=10 S=1/2, maxdim 32 (an exact representation), 5 sweeps, random
    product start: |E - E_ED| / |E_ED| <= 1e-10 (FP64), and the same for the
    mixed-precision runs (low-precision expansions, each restart vector
    applied in FP64); single-vector and block (4 vectors per batched matvec)
    Davidson."""
    N = 10
    As0 = inp.random_product_state(N, 2, inp.rng_for(0, 32))
    recs, mps = run(h, inp.heisenberg_mpo(N), As0, [(32, 1e-14)] * 5, prec=prec, eig_tol=1e-12,
                    krylovdim=12, maxiter=400, block=block)
    print("c0", prec, block, recs[-1]["energy"] - e_ed10, recs[-1]["matvecs"],
          recs[-1]["matvecs_f64"])
    E = recs[-1]["energy"]
    assert abs(E - e_ed10) / abs(e_ed10) <= 1e-10, (prec, E, e_ed10)
    bonds = h.mps_bonds(mps)
    assert max(bonds) <= 32
    # the returned state carries that energy
    sites = h.mps_sites(mps)
    assert abs(hf.mps_energy(sites, inp.heisenberg_mpo(N)) - E) / abs(E) <= 1e-9
    tot = sum(r["matvecs"] for r in recs)
    f64 = sum(r["matvecs_f64"] for r in recs)
    if prec != "f64":
        assert tot > f64 > 0
    else:
        assert tot == f64


def test_c0_matches_oracle_dmrg_per_converged_sweep(h):
    N = 10
    As0 = inp.random_product_state(N, 2, inp.rng_for(0, 32))
    ref = odmrg.dmrg(inp.heisenberg_mpo(N), As0, [(32, 1e-14)] * 5)
    recs, _ = run(h, inp.heisenberg_mpo(N), As0, [(32, 1e-14)] * 5, eig_tol=1e-12, krylovdim=12,
                  maxiter=400)
    assert abs(recs[-1]["energy"] - ref.energy) / abs(ref.energy) <= 1e-10


def test_aklt_exact_energy(h):
    N = 8
    As0 = inp.random_product_state(N, 3, np.random.default_rng(8))
    recs, _ = run(h, inp.aklt_mpo(N), As0, [(16, 1e-12)] * 4, eig_tol=1e-11, krylovdim=12,
                  maxiter=400)
    assert abs(recs[-1]["energy"] + 2.0 / 3.0 * (N - 1)) < 1e-9


def test_spin1_chain_matches_ed(h):
    N = 6
    e = float(np.linalg.eigvalsh(ed.heisenberg_dense(N, 2))[0])
    As0 = inp.random_product_state(N, 3, np.random.default_rng(6))
    recs, _ = run(h, inp.heisenberg_mpo(N, 2), As0, [(27, 1e-14)] * 4, eig_tol=1e-12,
                  krylovdim=12, maxiter=400)
    assert abs(recs[-1]["energy"] - e) / abs(e) <= 1e-10


def test_hubbard_2x2_matches_ed(h):
    Lx, Ly = 2, 2
    e = float(np.linalg.eigvalsh(ed.hubbard_dense(Lx, Ly, U=8.0))[0])
    As0 = inp.neel_product_state(Lx * Ly, 4, up=1, dn=2)
    recs, _ = run(h, inp.hubbard_mpo(Lx, Ly, U=8.0), As0, [(64, 1e-14)] * 4, eig_tol=1e-12,
                  krylovdim=12, maxiter=400)
    assert abs(recs[-1]["energy"] - e) / abs(e) <= 1e-10


def test_truncation_respects_maxdim(h):
    N = 12
    As0 = inp.random_product_state(N, 2, np.random.default_rng(3))
    recs, mps = run(h, inp.heisenberg_mpo(N), As0, [(4, 0.0), (8, 0.0)], eig_tol=1e-10,
                    krylovdim=8, maxiter=200)
    assert max(h.mps_bonds(mps)) <= 8
    assert recs[0]["max_bond"] <= 4
    assert recs[-1]["max_trunc"] > 0.0


@pytest.mark.parametrize("sched", [[(4, 0.0), (8, 0.0), (8, 0.0)], [(16, 1e-6), (16, 1e-8), (32, 1e-10)]])
def test_truncating_sweeps_match_oracle(h, sched):
    """Sweeps that truncate (N = 12 S=1/2 chain; maxdim 4 then 8, and cutoffs
    1e-6 .. 1e-10): per sweep, the largest bond dimension equals the
    oracle's, the largest discarded weight agrees to 1e-8 relative, and the
    energies agree to 1e-10 relative; the final bond dimensions match site
    by site."""
    N = 12
    As0 = inp.random_product_state(N, 2, np.random.default_rng(3))
    ref = odmrg.dmrg(inp.heisenberg_mpo(N), As0, sched)
    recs, mps = run(h, inp.heisenberg_mpo(N), As0, sched, eig_tol=1e-13, krylovdim=12,
                    maxiter=800, allow_unconverged=True)
    for r, o in zip(recs, ref.records):
        print("sweep", o.sweep, r["max_bond"], o.max_bond, r["max_trunc"], o.max_trunc,
              r["energy"], o.energy)
        assert r["max_bond"] == o.max_bond
        assert abs(r["max_trunc"] - o.max_trunc) <= 1e-8 * o.max_trunc + 1e-14
        assert abs(r["energy"] - o.energy) <= 1e-10 * abs(o.energy)
    assert h.mps_bonds(mps) == [1] + [A.shape[2] for A in ref.mps]


def test_mismatched_mpo_rejected(h):
    As0 = inp.random_product_state(6, 2, np.random.default_rng(1))
    mps = h.mps(As0)
    mpo = h.mpo(inp.heisenberg_mpo(7))
    with pytest.raises(itn.ItnError) as e:
        h.dmrg_sweep(mps, mpo, [(8, 0.0)])
    assert e.value.name == "ITN_E_SHAPE"


def test_sweep_phase_timing(h):
    """With timing on, the per-phase seconds are filled, non-negative and
    within the sweep's wall time; the energy is unaffected."""
    N = 10
    As0 = inp.random_product_state(N, 2, inp.rng_for(0, 32))
    kw = dict(eig_tol=1e-12, krylovdim=12, maxiter=400)
    recs_t, _ = run(h, inp.heisenberg_mpo(N), As0, [(32, 1e-14)] * 2, timing=True, **kw)
    recs, _ = run(h, inp.heisenberg_mpo(N), As0, [(32, 1e-14)] * 2, **kw)
    for r in recs_t:
        parts = [r[k] for k in ("t_matvec", "t_solver", "t_split", "t_env")]
        assert all(x >= 0.0 for x in parts)
        assert r["t_matvec"] > 0.0 and r["t_split"] > 0.0
        assert sum(parts) <= r["seconds"] * 1.01 + 1e-3
    assert "t_matvec" not in recs[0]
    assert abs(recs_t[-1]["energy"] - recs[-1]["energy"]) <= 1e-12 * abs(recs[-1]["energy"])


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_excited_state_by_energy_penalty(h, prec):
    """Sec. 7.2: the ground state found first, the next sweep with its
    projector times a penalty finds the first excited level (ED, N = 8), and
    a third with both projectors the level after."""
    N = 8
    ev = np.linalg.eigvalsh(ed.heisenberg_dense(N))
    levels = [ev[0]]
    for e in ev[1:]:
        if e > levels[-1] + 1e-8:
            levels.append(e)
    kw = dict(prec=prec, eig_tol=1e-12, krylovdim=12, maxiter=400)
    sweeps = [(16, 1e-14)] * 6
    mpo = h.mpo(inp.heisenberg_mpo(N))
    gs = h.mps(inp.random_product_state(N, 2, np.random.default_rng(1)))
    r0 = h.dmrg_sweep(gs, mpo, sweeps, **kw)
    assert abs(r0[-1]["energy"] - levels[0]) < 1e-9
    x1 = h.mps(inp.random_product_state(N, 2, np.random.default_rng(2)))
    r1 = h.dmrg_sweep(x1, mpo, sweeps, ortho=[gs], weight=10.0, **kw)
    assert abs(r1[-1]["energy"] - levels[1]) < 1e-8, (prec, r1[-1]["energy"], levels[:3])
    v0 = hf.mps_to_dense(h.mps_sites(gs)).ravel()
    v1 = hf.mps_to_dense(h.mps_sites(x1)).ravel()
    assert abs(v0 @ v1) < 1e-5
    # the oracle's penalty DMRG from the same states agrees
    ref = odmrg.dmrg(inp.heisenberg_mpo(N), inp.random_product_state(N, 2, np.random.default_rng(2)),
                     sweeps, ortho=[h.mps_sites(gs)], weight=10.0)
    assert abs(ref.energy - r1[-1]["energy"]) < 1e-8


def test_excited_state_rejects_bad_ortho(h):
    mpo = h.mpo(inp.heisenberg_mpo(6))
    a = h.mps(inp.random_product_state(6, 2, np.random.default_rng(1)))
    b = h.mps(inp.random_product_state(7, 2, np.random.default_rng(1)))
    with pytest.raises(itn.ItnError) as e:
        h.dmrg_sweep(a, mpo, [(8, 0.0)], ortho=[b], weight=1.0)
    assert e.value.name == "ITN_E_SHAPE"
    with pytest.raises(itn.ItnError) as e:
        h.dmrg_sweep(a, mpo, [(8, 0.0)], ortho=[a], weight=1.0)
    assert e.value.name == "ITN_E_ARG"


@pytest.mark.parametrize("maxdim", [32, 100, 200])
def test_bond_split_eigensolvers_agree(h, monkeypatch, maxdim):
    """The bond split's density-matrix eigensolver: the cooperative
    Householder path (one launch over workgroups holding the matrix rows in
    LDS; density matrices of 96, 300 and 600 rows use 8, 16 and 32
    workgroups) and the
    library's full symmetric solver give the same sweep energies, bond
    dimensions and truncation weights (spin-1 chain, N=20, FP64)."""
    N = 20
    As0 = inp.random_product_state(N, 3, inp.rng_for(5, maxdim))
    out = {}
    for mode in ("library", "coop"):
        if mode == "library":
            monkeypatch.setenv("ITN_EIG", "library")
        else:
            monkeypatch.delenv("ITN_EIG", raising=False)
        recs, _ = run(h, inp.heisenberg_mpo(N, 2), As0, [(maxdim, 1e-12)] * 3, prec="f64",
                      eig_tol=1e-9, krylovdim=8, maxiter=200, allow_unconverged=True)
        out[mode] = recs
    for a, b in zip(out["library"], out["coop"]):
        assert abs(a["energy"] - b["energy"]) <= 1e-10 * abs(a["energy"]), (a, b)
        assert a["max_bond"] == b["max_bond"], (a, b)
        assert abs(a["max_trunc"] - b["max_trunc"]) <= 1e-12, (a, b)


@pytest.mark.parametrize("block", [1, 4])
def test_mixed_precision_sweeps_mostly_low_precision(h, block):
    """Spin-1 chain (N = 20, maxdim 64, 9 sweeps), bf16 expansions with FP64 restart
    vectors and a small Davidson budget per bond (4 vectors, 8 matvecs; four
    times that with blocks of 4): at least 70 % of the matvecs run in bf16,
    at most 2.5 FP64 matvecs per bond on average (5 with blocks, whose
    restarts apply all four kept vectors in FP64), and the converged energy
    agrees with the FP64 run to 1e-9 relative."""
    N = 20
    As0 = inp.random_product_state(N, 3, inp.rng_for(2, 64))
    sched = [(64, 1e-10)] * 9
    kw = dict(eig_tol=1e-9, krylovdim=4 * block, maxiter=8 * block, allow_unconverged=True,
              block=block)
    r64, _ = run(h, inp.heisenberg_mpo(N, 2), As0, sched, prec="f64", **kw)
    rbf, _ = run(h, inp.heisenberg_mpo(N, 2), As0, sched, prec="bf16", **kw)
    bonds = 2 * (N - 1)
    tot = sum(r["matvecs"] for r in rbf)
    f64 = sum(r["matvecs_f64"] for r in rbf)
    print("mixed", block, tot, f64, f64 / (len(rbf) * bonds), rbf[-1]["energy"], r64[-1]["energy"])
    print("  sweeps f64 ", [r["energy"] for r in r64])
    print("  sweeps bf16", [r["energy"] for r in rbf])
    assert (tot - f64) / tot >= 0.70
    # single-vector: a restart cycle is one FP64 and three bf16 matvecs; a
    # block cycle is four FP64 (the kept block) and twelve bf16 matvecs
    assert f64 / (len(rbf) * bonds) <= (2.5 if block == 1 else 5.0)
    assert abs(rbf[-1]["energy"] - r64[-1]["energy"]) <= 1e-9 * abs(r64[-1]["energy"])
