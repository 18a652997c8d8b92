"""Pins of the oracle's labelled contraction (Sec. 4 product, Sec. 9.1 labels)."""
import json
import os

import numpy as np
import pytest

from oracle.tensor import contract, contract_bruteforce, output_labels

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


@pytest.mark.parametrize("seed", range(6))
def test_contract_matches_bruteforce(seed):
    rng = np.random.default_rng(seed)
    labels = list(range(6))
    rng.shuffle(labels)
    la = labels[:3]
    lb = [labels[2], labels[3], labels[0], labels[4]][: 2 + seed % 3]
    ext = {l: int(rng.integers(1, 4)) for l in labels}
    A = rng.standard_normal([ext[l] for l in la])
    B = rng.standard_normal([ext[l] for l in lb])
    lc = output_labels(la, lb)
    rng.shuffle(lc)
    C = contract(A, la, B, lb, lc)
    Cb = contract_bruteforce(A, la, B, lb, lc)
    assert C.shape == Cb.shape
    np.testing.assert_allclose(C, Cb, rtol=1e-13, atol=1e-13)


def test_outer_inner_and_partial():
    rng = np.random.default_rng(1)
    v, w = rng.standard_normal(3), rng.standard_normal(4)
    np.testing.assert_allclose(contract(v, [1], w, [2]), np.outer(v, w), rtol=0, atol=1e-15)
    A = rng.standard_normal((2, 3, 4))
    B = A.transpose(2, 0, 1).copy() * 0.5 + 1.0  # indices k,i,j: order differs
    s = contract(A, [1, 2, 3], B, [3, 1, 2], [])
    assert s.shape == ()
    np.testing.assert_allclose(s, np.dot(A.ravel(), B.transpose(1, 2, 0).ravel()), rtol=1e-14)
    T = rng.standard_normal((2, 3, 4))
    M = rng.standard_normal((4, 5))
    np.testing.assert_allclose(contract(T, [1, 2, 3], M, [3, 4]),
                               (T.reshape(6, 4) @ M).reshape(2, 3, 5), rtol=1e-13)


def test_appendix_shapes():
    g = GOLD["appendix_contraction"]
    dims = g["dims"]
    lab = {k: n for n, k in enumerate(sorted(dims))}
    rng = np.random.default_rng(2)
    A = rng.standard_normal([dims[x] for x in g["A"]])
    B = rng.standard_normal([dims[x] for x in g["B"]])
    C = contract(A, [lab[x] for x in g["A"]], B, [lab[x] for x in g["B"]])
    assert sorted(output_labels([lab[x] for x in g["A"]], [lab[x] for x in g["B"]])) == \
        sorted(lab[x] for x in g["C_has"])
    assert sorted(C.shape) == sorted(dims[x] for x in g["C_has"])


def test_ndtensors_label_example():
    g = GOLD["ndtensors_contract"]
    rng = np.random.default_rng(3)
    A = rng.standard_normal(g["A_dims"])
    B = rng.standard_normal(g["B_dims"])
    C = contract(A, g["A_labels"], B, g["B_labels"])
    assert list(C.shape) == g["C_dims"]
    Cb = contract_bruteforce(A, g["A_labels"], B, g["B_labels"], [1, 2])
    np.testing.assert_allclose(C, Cb, rtol=1e-13, atol=1e-14)


def test_bad_labels_rejected():
    A = np.zeros((2, 3))
    B = np.zeros((4, 5))
    with pytest.raises(ValueError):
        contract(A, [1, 2], B, [2, 3])  # extents 3 vs 4
    with pytest.raises(ValueError):
        contract(A, [1, 1], np.zeros((2,)), [1])
