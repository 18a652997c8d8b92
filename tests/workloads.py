"""Seeded workloads of the dense H_eff benchmark family, built with the
oracle (tests only)."""
import math

import numpy as np

from paper_2007_14822_amd import inputs as inp
from oracle import heff as hf


def c1_chain(chi: int, d: int = 2, config: int = 1):
    """Random canonical MPS of N_c = 2 log2(chi) + 2 sites with its centre
    on the bond (c, c+1), c = N_c/2 - 1, and the Heisenberg MPO."""
    n = int(round(math.log2(chi)))
    Nc = 2 * n + 2
    c = Nc // 2 - 1
    rng = inp.rng_for(config, chi)
    As = inp.random_canonical_mps(Nc, d, chi, center=c, rng=rng)
    Ws = inp.heisenberg_mpo(Nc, d - 1)
    return As, Ws, c, rng


def c1_operands(chi: int, d: int = 2, config: int = 1):
    """(L, W1, W2, R, psi) of the centre bond; L, R by the oracle."""
    As, Ws, c, rng = c1_chain(chi, d, config)
    L = hf.left_envs(As[:c], Ws[:c])[-1]
    R = hf.right_envs(As[c + 2:], Ws[c + 2:])[0]
    psi = inp.unit_gaussian((L.shape[0], d, d, R.shape[0]), rng)
    return L, Ws[c], Ws[c + 1], R, psi


def rel_err(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))
