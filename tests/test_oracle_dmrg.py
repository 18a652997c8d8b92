"""Pins of the oracle's truncation, bond split, Davidson and sweeps."""
import numpy as np
import pytest

from paper_2007_14822_amd import inputs as inp
from oracle import dmrg as dm, ed, heff as hf


def test_truncation_examples():
    s = np.array([4.0, 2.0, 1.0, 0.5])  # weights 16, 4, 1, 0.25 of 21.25
    tot = 21.25
    r = dm.truncation_count(s, 0.0, 10)
    assert r.keep == 4 and r.discarded_weight == 0.0
    r = dm.truncation_count(s, 0.25 / tot, 10)          # tie counts as discardable
    assert r.keep == 3 and abs(r.discarded_weight - 0.25 / tot) < 1e-16
    r = dm.truncation_count(s, 1.2 / tot, 10)
    assert r.keep == 3
    r = dm.truncation_count(s, 1.25 / tot, 10)
    assert r.keep == 2 and abs(r.discarded_weight - 1.25 / tot) < 1e-15
    r = dm.truncation_count(s, 0.0, 1)
    assert r.keep == 1 and abs(r.discarded_weight - 5.25 / tot) < 1e-15
    r = dm.truncation_count(s, 1.0, 10)                  # never below one state
    assert r.keep == 1


@pytest.mark.parametrize("to_right", [True, False])
def test_split_exact_and_truncated(to_right):
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((3, 2, 2, 5))
    psi /= np.linalg.norm(psi)
    Al, Ar, tw, s = dm.split_bond(psi, 0.0, 100, to_right)
    np.testing.assert_allclose(np.einsum("asb,btc->astc", Al, Ar), psi, atol=1e-13)
    assert tw == 0.0
    if to_right:
        M = Al.reshape(-1, Al.shape[2])
        np.testing.assert_allclose(M.T @ M, np.eye(M.shape[1]), atol=1e-13)
    else:
        M = Ar.reshape(Ar.shape[0], -1)
        np.testing.assert_allclose(M @ M.T, np.eye(M.shape[0]), atol=1e-13)
    Al, Ar, tw, s = dm.split_bond(psi, 0.0, 2, to_right)
    assert Al.shape[2] == 2
    sv = np.linalg.svd(psi.reshape(6, 10), compute_uv=False)
    assert abs(tw - (sv[2:] ** 2).sum() / (sv ** 2).sum()) < 1e-14
    approx = np.einsum("asb,btc->astc", Al, Ar)
    # truncated and renormalised: equals the best rank-2 approximation, scaled
    U, S, Vt = np.linalg.svd(psi.reshape(6, 10))
    best = (U[:, :2] * S[:2]) @ Vt[:2] / np.linalg.norm(S[:2])
    np.testing.assert_allclose(approx.reshape(6, 10), best, atol=1e-13)


def test_davidson_matches_eigh():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((300, 300))
    A = A + A.T
    th, v = dm.davidson(lambda x: A @ x, rng.standard_normal(300), krylovdim=30, maxiter=2000,
                        tol=1e-11)
    ev = np.linalg.eigvalsh(A)
    assert abs(th - ev[0]) < 1e-9
    assert np.linalg.norm(A @ v - th * v) < 1e-8


def test_dmrg_c0_matches_exact_diagonalisation():
    """N=10 S=1/2 chain, maxdim 32 (exact representation), 5 sweeps."""
    N = 10
    e_ed = np.linalg.eigvalsh(ed.heisenberg_dense(N))[0]
    As0 = inp.random_product_state(N, 2, inp.rng_for(0, 32))
    res = dm.dmrg(inp.heisenberg_mpo(N), As0, [(32, 1e-14)] * 5)
    assert abs(res.energy - e_ed) / abs(e_ed) <= 1e-10
    assert abs(hf.mps_energy(res.mps, inp.heisenberg_mpo(N)) - e_ed) / abs(e_ed) <= 1e-10
    assert res.records[-1].max_bond <= 32


def test_dmrg_aklt_exact_energy():
    N = 8
    As0 = inp.random_product_state(N, 3, np.random.default_rng(8))
    res = dm.dmrg(inp.aklt_mpo(N), As0, [(16, 1e-12)] * 4)
    assert abs(res.energy + 2.0 / 3.0 * (N - 1)) < 1e-9


def test_dmrg_spin1_matches_ed():
    N = 6
    e_ed = np.linalg.eigvalsh(ed.heisenberg_dense(N, 2))[0]
    As0 = inp.random_product_state(N, 3, np.random.default_rng(6))
    res = dm.dmrg(inp.heisenberg_mpo(N, 2), As0, [(27, 1e-14)] * 4)
    assert abs(res.energy - e_ed) / abs(e_ed) <= 1e-10


def test_dmrg_hubbard_small_cylinder():
    """2x2 Hubbard (U=8): dense DMRG is free to change particle number, so
    it must reach the lowest eigenvalue of the whole Fock space."""
    Lx, Ly = 2, 2
    e_ed = np.linalg.eigvalsh(ed.hubbard_dense(Lx, Ly, U=8.0))[0]
    As0 = inp.neel_product_state(Lx * Ly, 4, up=1, dn=2)
    res = dm.dmrg(inp.hubbard_mpo(Lx, Ly, U=8.0), As0, [(64, 1e-14)] * 4)
    assert abs(res.energy - e_ed) / abs(e_ed) <= 1e-10


def test_excited_states_by_energy_penalty_match_ed():
    """Sec. 7.2 excited states: with the ground state's projector added times
    a penalty larger than the gap, DMRG finds the first excited level, and
    with both found states penalised the next level (ED spectrum, N = 8)."""
    N = 8
    Ws = inp.heisenberg_mpo(N)
    ev = np.linalg.eigvalsh(ed.heisenberg_dense(N))
    levels = [ev[0]]
    for e in ev[1:]:
        if e > levels[-1] + 1e-8:
            levels.append(e)
    sweeps = [(16, 1e-14)] * 6
    r0 = dm.dmrg(Ws, inp.random_product_state(N, 2, np.random.default_rng(1)), sweeps)
    assert abs(r0.energy - levels[0]) < 1e-10
    r1 = dm.dmrg(Ws, inp.random_product_state(N, 2, np.random.default_rng(2)), sweeps,
                    ortho=[r0.mps], weight=10.0)
    assert abs(r1.energy - levels[1]) < 1e-9
    # the excited state is orthogonal to the ground state
    v0 = hf.mps_to_dense(r0.mps).ravel()
    v1 = hf.mps_to_dense(r1.mps).ravel()
    assert abs(v0 @ v1) < 1e-6 and abs(np.linalg.norm(v1) - 1) < 1e-9


def test_projected_state_is_the_overlap():
    """<phi|psi> over the whole chain equals v . psi_bond at any bond, with v
    the projected state built from the overlap environments."""
    N, i = 6, 2
    rng = np.random.default_rng(3)
    As = inp.random_canonical_mps(N, 2, 4, i, rng)
    Bs = inp.random_canonical_mps(N, 2, 3, 0, rng)
    LO, RO = np.ones((1, 1)), np.ones((1, 1))
    for k in range(i):
        LO = dm.overlap_env_left(LO, As[k], Bs[k])
    for k in range(N - 1, i + 1, -1):
        RO = dm.overlap_env_right(RO, As[k], Bs[k])
    v = dm.projected_state(LO, Bs[i], Bs[i + 1], RO)
    psi = np.einsum("asb,btc->astc", As[i], As[i + 1])
    full = hf.mps_to_dense(As).ravel() @ hf.mps_to_dense(Bs).ravel()
    assert abs(float(np.vdot(v, psi)) - full) < 1e-12
