"""Pins of the model inputs (MPOs, operators) against exact diagonalisation."""
import json
import os

import numpy as np
import pytest

from paper_2007_14822_amd import inputs as inp
from oracle import ed, heff as hf

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_spin_three_halves_listing():
    g = GOLD["spin_three_halves"]
    o = inp.spin_ops(3)
    np.testing.assert_allclose(np.diag(o["Sz"]), g["Sz"], atol=1e-15)
    np.testing.assert_allclose(np.diag(o["S+"], 1), g["Splus_superdiag"], atol=1e-15)
    assert np.count_nonzero(o["S+"]) == 3
    np.testing.assert_allclose(o["S-"], o["S+"].T)


@pytest.mark.parametrize("two_s", [1, 2, 3])
def test_spin_algebra(two_s):
    o = inp.spin_ops(two_s)
    np.testing.assert_allclose(o["S+"] @ o["S-"] - o["S-"] @ o["S+"], 2 * o["Sz"], atol=1e-14)
    S = two_s / 2
    sx = 0.5 * (o["S+"] + o["S-"])
    sy = -0.5j * (o["S+"] - o["S-"])
    cas = sx @ sx + (sy @ sy).real + o["Sz"] @ o["Sz"]
    np.testing.assert_allclose(cas, S * (S + 1) * np.eye(two_s + 1), atol=1e-13)


def test_heisenberg_mpo_bond_dim_is_paper_value():
    assert inp.heisenberg_mpo(4)[0].shape[0] == GOLD["heisenberg_mpo_bond_dim"]["value"]


@pytest.mark.parametrize("N,two_s", [(2, 1), (6, 1), (4, 2), (3, 3)])
def test_heisenberg_mpo_equals_kronecker(N, two_s):
    H_mpo = hf.mpo_to_dense(inp.heisenberg_mpo(N, two_s))
    H_ed = ed.heisenberg_dense(N, two_s)
    np.testing.assert_allclose(H_mpo, H_ed, atol=1e-13)


def test_two_site_heisenberg_spectrum():
    ev = np.linalg.eigvalsh(ed.heisenberg_dense(2))
    np.testing.assert_allclose(ev, [-0.75, 0.25, 0.25, 0.25], atol=1e-14)


def test_aklt_mpo():
    Ws = inp.aklt_mpo(4)
    assert Ws[0].shape[0] == 11
    np.testing.assert_allclose(hf.mpo_to_dense(Ws), ed.aklt_dense(4), atol=1e-12)
    # AKLT ground energy of an open chain: -(2/3)(N-1), four-fold degenerate
    ev = np.linalg.eigvalsh(ed.aklt_dense(4))
    np.testing.assert_allclose(ev[:4], -2.0 / 3.0 * 3, atol=1e-12)
    assert ev[4] > ev[0] + 1e-3


def test_aklt_mps_exact_eigenstate():
    N = 5
    H = ed.aklt_dense(N)
    for lv, rv in [((1, 0), (0, 1)), ((0.3, -1.2), (0.7, 0.4))]:
        v = hf.mps_to_dense(inp.aklt_mps(N, lv, rv))
        v /= np.linalg.norm(v)
        Hv = H @ v
        e = v @ Hv
        assert abs(e + 2.0 / 3.0 * (N - 1)) < 1e-12
        assert np.linalg.norm(Hv - e * v) < 1e-12


@pytest.mark.parametrize("Lx,Ly", [(2, 3), (3, 2), (1, 4)])
def test_hubbard_mpo_equals_fock_space(Lx, Ly):
    """Operator equality pins the Jordan-Wigner strings for hops of every
    distance present, including the periodic wrap in y."""
    H_mpo = hf.mpo_to_dense(inp.hubbard_mpo(Lx, Ly, t=1.0, U=8.0))
    H_ed = ed.hubbard_dense(Lx, Ly, t=1.0, U=8.0)
    np.testing.assert_allclose(H_mpo, H_ed, atol=1e-12)


def test_hubbard_cylinder_channel_count():
    # column-major snake of a width-4 cylinder: hop distances 1, 3, 4
    Ws = inp.hubbard_mpo(3, 4)
    assert Ws[0].shape[0] == 2 + 4 * 4 == 18
    dists = sorted({j - i for i, j in inp.cylinder_bonds(32, 4)})
    assert dists == [1, 3, 4]


def test_free_fermion_closed_form_matches_sector_ed():
    for (Lx, Ly) in [(2, 3), (3, 2)]:
        N = Lx * Ly
        nup = N // 2
        e_ed = ed.hubbard_sector_ground_energy(Lx, Ly, nup, nup, t=1.0, U=0.0)
        e_cf = ed.free_fermion_cylinder_energy(Lx, Ly, nup, nup, t=1.0)
        assert abs(e_ed - e_cf) < 1e-10


def test_sector_ed_matches_full_fock():
    Lx, Ly = 2, 2
    H = ed.hubbard_dense(Lx, Ly, U=8.0)
    # restrict to (N_up, N_dn) = (2, 2) using the Fock-space number operators
    c = ed._mode_annihilators(2 * Lx * Ly)
    nup = sum(c[2 * i].T @ c[2 * i] for i in range(Lx * Ly))
    ndn = sum(c[2 * i + 1].T @ c[2 * i + 1] for i in range(Lx * Ly))
    idx = [k for k in range(H.shape[0]) if round(nup[k, k]) == 2 and round(ndn[k, k]) == 2]
    e_full = np.linalg.eigvalsh(H[np.ix_(idx, idx)])[0]
    e_sec = ed.hubbard_sector_ground_energy(Lx, Ly, 2, 2, U=8.0)
    assert abs(e_full - e_sec) < 1e-11


def test_c3_sector_table():
    secs = inp.c3_sector_dims()
    assert [n for _, n in secs] == [8, 8, 8, 8, 8, 8, 9, 35, 107, 259, 484, 706, 800, 706, 484,
                                    259, 107, 35, 9, 8, 8, 8, 8, 8, 8]
    assert sum(n for _, n in secs) == 4096


def test_c4_sector_table():
    secs = inp.c4_sector_dims()
    dims = [n for _, n in secs]
    assert sum(dims) == 4096
    assert len(secs) == 81 and max(dims) == 324 and min(dims) == 1


def test_long_range_hubbard_mpo_equals_fock_space():
    N, rmax = 5, 3
    bonds = [(i, j) for i in range(N) for j in range(i + 1, min(N, i + rmax + 1))]
    H_mpo = hf.mpo_to_dense(inp.long_range_hubbard_mpo(N, rmax, t=0.7, U=3.0))
    H_ed = ed.hubbard_dense_bonds(N, bonds, t=0.7, U=3.0)
    np.testing.assert_allclose(H_mpo, H_ed, atol=1e-12)
    assert inp.long_range_hubbard_mpo(4, 9)[0].shape[0] == 38


def test_sector_runs():
    q, d = inp.sectors_from_basis_qns(inp.heisenberg_mpo_link_qn())
    assert q == [(0,), (-2,), (2,), (0,)] and d == [1, 1, 1, 2]
