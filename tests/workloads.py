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


# ------------------------------------------------------------ error bounds
# Unit roundoff (round to nearest) of the operand and accumulator formats:
# bf16 keeps 8 significant bits, float 24, double 53.
UNIT = {"bf16": 2.0 ** -8, "f32": 2.0 ** -24, "f64": 2.0 ** -53}


def gamma(n: int, u: float) -> float:
    """Higham's gamma_n = n u / (1 - n u): a sum of n + 1 terms in any order
    is within gamma_n * (sum of |terms|) of the exact sum."""
    return n * u / (1.0 - n * u)


def heff_error_factor(prec: str, k1: int, kw: int, k4: int, op_roundings: int = 4,
                      w: int = 1) -> float:
    """c with |y - y_ref| <= c * A element-wise, A the H_eff contraction of
    the absolute values |L| |W1| |W2| |R| |psi|, for the three-stage order
    (stage 1 over k1 terms, W-stage over kw, stage 4 over k4).  Counted:
    each operand or stored intermediate rounded once to the operand format
    (L, psi, R, Z; X too where it is stored), the W12 coefficients rounded to
    float (FP64 in the FP64 path), accumulation in float (FP64 in the FP64
    path), and the FP64 reference's own rounding (products of w W1 W2 terms,
    then the three sums)."""
    uo = UNIT[prec]
    ua = UNIT["f64"] if prec == "f64" else UNIT["f32"]
    u64 = UNIT["f64"]
    c = ((1 + uo) ** op_roundings * (1 + ua) * (1 + gamma(w, u64)) * (1 + gamma(k1, ua))
         * (1 + gamma(kw, ua)) * (1 + gamma(k4, ua)) - 1.0)
    c_ref = gamma(k1 + w + kw + k4, u64)
    return (c + c_ref) * (1.0 + 1e-6)


def elementwise_ratio(got, ref, absref, c: float) -> float:
    """max |got - ref| / (c * absref); at most 1 when the bound holds (an
    element whose bound is 0 must match exactly)."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    bnd = c * np.asarray(absref, np.float64).ravel()
    err = np.abs(got - ref)
    if np.any((bnd == 0) & (err != 0)):
        return float("inf")
    nz = bnd > 0
    return float(np.max(err[nz] / bnd[nz])) if nz.any() else 0.0


def group_rel_err(got, ref, g: int = 16) -> float:
    """Largest relative error over runs of g consecutive elements (the last
    axis split into whole runs, a shorter tail ignored; a lost or misplaced
    16-wide tile column shows up here even when the global norm hardly
    moves)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    n = (got.shape[-1] // g) * g
    if n == 0:  # rows shorter than a run: the element-wise bound covers them
        return 0.0
    a = got[..., :n].reshape(-1, g)
    b = ref[..., :n].reshape(-1, g)
    nb = np.linalg.norm(b, axis=1)
    keep = nb > 0
    ea = np.linalg.norm(a - b, axis=1)
    if np.any(~keep & (ea > 0)):
        return float("inf")
    return float(np.max(ea[keep] / nb[keep])) if keep.any() else 0.0
