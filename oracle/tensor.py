"""Labelled dense contraction (oracle).

Follows the product operator of Sec. 4: indices that appear in both
operands are summed, every other index survives; no shared index gives an
outer product, all indices shared gives a scalar.  Indices are integer
labels as in the NDTensors interface of Sec. 9.1; the caller fixes the
output order (the result of Sec. 4 does not depend on input index order).
"""
from __future__ import annotations

import itertools
from typing import Sequence

import numpy as np

_LETTERS = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"


def output_labels(la: Sequence[int], lb: Sequence[int]) -> list:
    """Uncontracted labels: those of A not in B, then those of B not in A."""
    return [l for l in la if l not in lb] + [l for l in lb if l not in la]


def contract(A: np.ndarray, la: Sequence[int], B: np.ndarray, lb: Sequence[int],
             lc: Sequence[int] | None = None) -> np.ndarray:
    la, lb = list(la), list(lb)
    if len(set(la)) != len(la) or len(set(lb)) != len(lb):
        raise ValueError("repeated label within one operand")
    if lc is None:
        lc = output_labels(la, lb)
    lc = list(lc)
    if sorted(lc) != sorted(output_labels(la, lb)):
        raise ValueError("output labels must be exactly the uncontracted labels")
    for l in set(la) & set(lb):
        if A.shape[la.index(l)] != B.shape[lb.index(l)]:
            raise ValueError("contracted extents differ")
    allv = sorted(set(la) | set(lb))
    m = {l: _LETTERS[k] for k, l in enumerate(allv)}
    sub = "".join(m[l] for l in la) + "," + "".join(m[l] for l in lb) + "->" + "".join(m[l] for l in lc)
    return np.einsum(sub, np.asarray(A, np.float64), np.asarray(B, np.float64), optimize=False)


def contract_bruteforce(A, la, B, lb, lc) -> np.ndarray:
    """Nested loops over every index value (tiny shapes only)."""
    la, lb, lc = list(la), list(lb), list(lc)
    ext = {}
    for l, n in zip(la, A.shape):
        ext[l] = n
    for l, n in zip(lb, B.shape):
        ext[l] = n
    summed = [l for l in la if l in lb]
    C = np.zeros([ext[l] for l in lc])
    for cidx in itertools.product(*[range(ext[l]) for l in lc]):
        val = dict(zip(lc, cidx))
        acc = 0.0
        for sidx in itertools.product(*[range(ext[l]) for l in summed]):
            val.update(zip(summed, sidx))
            acc += A[tuple(val[l] for l in la)] * B[tuple(val[l] for l in lb)]
        C[cidx] = acc
    return C
