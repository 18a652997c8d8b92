"""Pins of the oracle's environments and two-site H_eff."""
import numpy as np
import pytest

from paper_2007_14822_amd import inputs as inp
from oracle import ed, heff as hf


def test_two_site_heff_is_bond_operator():
    """N=2 with boundary environments: H_eff is S.S, spectrum (-3/4, 1/4 x3)."""
    Ws = inp.heisenberg_mpo(2)
    H = hf.heff_matrix(hf.left_boundary(5), Ws[0], Ws[1], hf.right_boundary(5))
    np.testing.assert_allclose(H, ed.heisenberg_dense(2), atol=1e-15)
    np.testing.assert_allclose(np.linalg.eigvalsh(H), [-0.75, 0.25, 0.25, 0.25], atol=1e-14)


@pytest.mark.parametrize("model", ["heis", "spin1", "aklt"])
def test_full_rank_envs_give_ed_spectrum(model):
    """N=4, bond (1,2), with unitary (full-rank) outer sites: the
    environments are exact and H_eff is unitarily equivalent to H."""
    if model == "heis":
        Ws, Hd, d = inp.heisenberg_mpo(4), ed.heisenberg_dense(4), 2
    elif model == "spin1":
        Ws, Hd, d = inp.heisenberg_mpo(4, 2), ed.heisenberg_dense(4, 2), 3
    else:
        Ws, Hd, d = inp.aklt_mpo(4), ed.aklt_dense(4), 3
    rng = np.random.default_rng(5)
    Q0, _ = np.linalg.qr(rng.standard_normal((d, d)))
    Q3, _ = np.linalg.qr(rng.standard_normal((d, d)))
    A0 = Q0.reshape(1, d, d)
    A3 = Q3.T.reshape(d, d, 1)
    L = hf.env_left(hf.left_boundary(Ws[0].shape[0]), A0, Ws[0])
    R = hf.env_right(hf.right_boundary(Ws[0].shape[0]), A3, Ws[3])
    H = hf.heff_matrix(L, Ws[1], Ws[2], R)
    np.testing.assert_allclose(np.linalg.eigvalsh(H), np.linalg.eigvalsh(Hd), atol=1e-12)
    # the matvec route agrees with the matrix route
    psi = rng.standard_normal((d, d, d, d))
    np.testing.assert_allclose(hf.heff_apply(L, Ws[1], Ws[2], R, psi).ravel(), H @ psi.ravel(),
                               atol=1e-12)


def test_heff_matches_dense_projection():
    """H_eff = P^T H P with P the isometry of the mixed-canonical MPS."""
    N, d = 6, 2
    rng = np.random.default_rng(7)
    As = inp.random_canonical_mps(N, d, 4, center=2, rng=rng)
    Ws = inp.heisenberg_mpo(N)
    Ls, Rs = hf.left_envs(As, Ws), hf.right_envs(As, Ws)
    L, R = Ls[2], Rs[4]
    H = hf.heff_matrix(L, Ws[2], Ws[3], R)
    # isometry: left block (sites 0,1) and right block (sites 4,5)
    Lm = np.einsum("asb,btc->astc", As[0], As[1]).reshape(d * d, -1)   # [(s0 s1), a]
    Rm = np.einsum("asb,btc->astc", As[4], As[5]).reshape(-1, d * d)   # [b, (s4 s5)]
    cl, cr = Lm.shape[1], Rm.shape[0]
    # build P column by column: P[:, (a s2 s3 b)] = |L_a> (x) |s2> (x) |s3> (x) |R_b>
    cols = []
    for a in range(cl):
        for s2 in range(d):
            for s3 in range(d):
                for b in range(cr):
                    e2 = np.eye(d)[s2]
                    e3 = np.eye(d)[s3]
                    cols.append(np.kron(np.kron(np.kron(Lm[:, a], e2), e3), Rm[b]))
    P = np.stack(cols, 1)
    np.testing.assert_allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-12)
    np.testing.assert_allclose(H, P.T @ ed.heisenberg_dense(N) @ P, atol=1e-12)


def test_heff_hermitian_on_built_envs():
    N, d = 8, 2
    rng = np.random.default_rng(11)
    As = inp.random_canonical_mps(N, d, 8, center=3, rng=rng)
    Ws = inp.heisenberg_mpo(N)
    L, R = hf.left_envs(As, Ws)[3], hf.right_envs(As, Ws)[5]
    phi = rng.standard_normal((L.shape[0], d, d, R.shape[0]))
    psi = rng.standard_normal(phi.shape)
    a = np.vdot(phi, hf.heff_apply(L, Ws[3], Ws[4], R, psi))
    b = np.vdot(hf.heff_apply(L, Ws[3], Ws[4], R, phi), psi)
    assert abs(a - b) <= 1e-12 * np.linalg.norm(phi) * np.linalg.norm(psi) * 10


def test_env_identity_channels():
    N, d = 7, 3
    rng = np.random.default_rng(3)
    As = inp.random_canonical_mps(N, d, 9, center=N - 1, rng=rng)
    Ws = inp.heisenberg_mpo(N, 2)
    for k, L in enumerate(hf.left_envs(As, Ws)[1:N]):
        np.testing.assert_allclose(L[:, 4, :], np.eye(L.shape[0]), atol=1e-13)
    As = inp.random_canonical_mps(N, d, 9, center=0, rng=rng)
    for R in hf.right_envs(As, Ws)[1:N]:
        np.testing.assert_allclose(R[:, 0, :], np.eye(R.shape[0]), atol=1e-13)


@pytest.mark.parametrize("N,two_s", [(6, 1), (5, 2)])
def test_energy_from_envs_matches_dense(N, two_s):
    d = two_s + 1
    rng = np.random.default_rng(N)
    As = [rng.standard_normal((1 if i == 0 else 3, d, 1 if i == N - 1 else 3)) for i in range(N)]
    Ws = inp.heisenberg_mpo(N, two_s)
    v = hf.mps_to_dense(As)
    e_dense = v @ ed.heisenberg_dense(N, two_s) @ v / (v @ v)
    assert abs(hf.mps_energy(As, Ws) - e_dense) < 1e-12 * max(1, abs(e_dense))


@pytest.mark.parametrize("bond", [0, 2, 4])
def test_aklt_eigenstate_at_any_bond(bond):
    """AKLT MPS is exact: H_eff psi = E psi with E = -(2/3)(N-1)."""
    N = 7
    As = hf.canonicalize(inp.aklt_mps(N, (0.6, -0.8), (0.3, 1.1)), bond)
    Ws = inp.aklt_mpo(N)
    L, R = hf.left_envs(As, Ws)[bond], hf.right_envs(As, Ws)[bond + 2]
    psi = np.einsum("asb,btc->astc", As[bond], As[bond + 1])
    psi /= np.linalg.norm(psi)
    Hpsi = hf.heff_apply(L, Ws[bond], Ws[bond + 1], R, psi)
    E = -2.0 / 3.0 * (N - 1)
    assert np.linalg.norm(Hpsi - E * psi) <= 1e-12
    assert abs(np.vdot(psi, Hpsi) - E) <= 1e-12


def test_stage_order_equals_matrix_definition():
    rng = np.random.default_rng(9)
    cl, cr, d, w = 3, 4, 2, 5
    L = rng.standard_normal((cl, w, cl))
    R = rng.standard_normal((cr, w, cr))
    W1 = rng.standard_normal((w, w, d, d))
    W2 = rng.standard_normal((w, w, d, d))
    psi = rng.standard_normal((cl, d, d, cr))
    y = hf.heff_apply(L, W1, W2, R, psi)
    # brute-force eight nested sums
    yb = np.zeros_like(y)
    for ap in range(cl):
        for u in range(d):
            for v in range(d):
                for bp in range(cr):
                    acc = 0.0
                    for m0 in range(w):
                        for m1 in range(w):
                            for m2 in range(w):
                                for a in range(cl):
                                    for s1 in range(d):
                                        for s2 in range(d):
                                            for b in range(cr):
                                                acc += (L[ap, m0, a] * W1[m0, m1, u, s1] *
                                                        W2[m1, m2, v, s2] * R[bp, m2, b] *
                                                        psi[a, s1, s2, b])
                    yb[ap, u, v, bp] = acc
    np.testing.assert_allclose(y, yb, rtol=1e-12, atol=1e-12)
    rows = [2, 0]
    np.testing.assert_allclose(hf.heff_apply_rows(L, W1, W2, R, psi, rows), y[rows], atol=1e-13)


# ------------------------------------------------------------ sums of MPOs
def _split_heisenberg(N):
    """The S=1/2 Heisenberg chain as two MPOs: flip-flop (w=4) and ZZ (w=3),
    same convention as the library's MPO (left boundary row w-1, right
    boundary column 0)."""
    ops = inp.spin_ops(1)
    Sp, Sm, Sz, I = ops["S+"], ops["S-"], ops["Sz"], ops["Id"]
    Wf = np.zeros((4, 4, 2, 2))
    Wf[0, 0], Wf[1, 0], Wf[2, 0] = I, Sp, Sm
    Wf[3, 1], Wf[3, 2], Wf[3, 3] = 0.5 * Sm, 0.5 * Sp, I
    Wz = np.zeros((3, 3, 2, 2))
    Wz[0, 0], Wz[1, 0], Wz[2, 1], Wz[2, 2] = I, Sz, Sz, I
    return [Wf.copy() for _ in range(N)], [Wz.copy() for _ in range(N)]


def test_heff_sum_of_split_mpos_equals_full_mpo():
    """Sec. 7.2: H given as a sum of MPOs.  Projecting H = H_ff + H_zz onto the
    two-site space of an MPS is linear, so the sum of the two terms' H_eff
    (each with its own environments) equals the full MPO's H_eff."""
    N, i = 8, 3
    As = inp.random_canonical_mps(N, 2, 6, i, np.random.default_rng(4))
    Wfull = inp.heisenberg_mpo(N)
    Wf, Wz = _split_heisenberg(N)
    def operands(Ws):
        return hf.left_envs(As, Ws)[i], Ws[i], Ws[i + 1], hf.right_envs(As, Ws)[i + 2]
    psi = np.einsum("asm,mtb->astb", As[i], As[i + 1])
    full = hf.heff_apply(*operands(Wfull), psi)
    summed = hf.heff_apply_sum([operands(Wf), operands(Wz)], psi)
    assert np.allclose(summed, full, atol=1e-12)
    # the split MPOs sum to the chain Hamiltonian (dense, small chain)
    Hs = hf.mpo_to_dense(Wf[:6]) + hf.mpo_to_dense(Wz[:6])
    assert np.allclose(Hs, ed.heisenberg_dense(6), atol=1e-12)


def test_heff_sum_equals_direct_sum_mpo():
    """A sum of terms equals one H_eff whose MPO tensors are the block-diagonal
    direct sum of the terms' (environments concatenated along m)."""
    rng = np.random.default_rng(9)
    cl, cr, d = 5, 4, 3
    ws = [3, 5, 2]
    terms = [(rng.standard_normal((cl, w, cl)), rng.standard_normal((w, w, d, d)),
              rng.standard_normal((w, w, d, d)), rng.standard_normal((cr, w, cr))) for w in ws]
    psi = rng.standard_normal((cl, d, d, cr))
    W = sum(ws)
    Lds = np.concatenate([t[0] for t in terms], axis=1)
    Rds = np.concatenate([t[3] for t in terms], axis=1)
    W1ds, W2ds = np.zeros((W, W, d, d)), np.zeros((W, W, d, d))
    o = 0
    for (_, W1, W2, _), w in zip(terms, ws):
        W1ds[o:o + w, o:o + w], W2ds[o:o + w, o:o + w] = W1, W2
        o += w
    assert np.allclose(hf.heff_apply_sum(terms, psi), hf.heff_apply(Lds, W1ds, W2ds, Rds, psi),
                       atol=1e-10)
