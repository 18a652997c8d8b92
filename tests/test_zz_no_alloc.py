"""The allocation-free H_eff entry point (itn_heff_apply_noalloc) against
itn_heff_apply through the C ABI: bit-identical outputs on two calls in a
row (the second smaller, on another code path), parity with the oracle, and
a request beyond the fixed scratch rejected before any work."""
import numpy as np
import pytest
import torch

import paper_2007_14822_amd as itn
from paper_2007_14822_amd import inputs as inp
from oracle import heff as hf
from tests.workloads import rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-2}


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _case(cl, cr, d, w, nv, seed, mpo):
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((cl, w, cl)) / cl
    R = rng.standard_normal((cr, w, cr)) / cr
    if mpo == "heis":
        W1 = W2 = inp.heisenberg_mpo(3, d - 1)[1]
    else:
        W1 = rng.standard_normal((w, w, d, d)) * (rng.random((w, w, 1, 1)) < 0.4)
        W2 = rng.standard_normal((w, w, d, d)) * (rng.random((w, w, 1, 1)) < 0.4)
    psi = rng.standard_normal((nv, cl, d, d, cr))
    return L, W1, W2, R, psi


# a large fused-kernel call, then a smaller one on the unfused path (w = 11:
# W-stage tables for a separate W-stage kernel, also held in the scratch)
CALLS = [(384, 320, 2, 5, 2, "heis"), (40, 52, 3, 11, 1, "rand")]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_noalloc_matches_heff_apply(prec):
    h = itn.Handle(0)
    try:
        for k, (cl, cr, d, w, nv, mpo) in enumerate(CALLS):
            L, W1, W2, R, psi = _case(cl, cr, d, w, nv, 500 + k, mpo)
            edt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[prec]
            Ld, Rd, pd = dev(L, edt), dev(R, edt), dev(psi)
            a = torch.full(psi.shape, float("nan"), dtype=torch.float64, device=DEV)
            b = torch.full(psi.shape, float("nan"), dtype=torch.float64, device=DEV)
            h.heff_apply(Ld, W1, W2, Rd, pd, a, nv=nv, prec=prec)
            h.heff_apply_noalloc(Ld, W1, W2, Rd, pd, b, nv=nv, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(a, b), (prec, k)
            ref = np.stack([hf.heff_apply(L, W1, W2, R, psi[v]) for v in range(nv)])
            assert rel_err(b.cpu().numpy(), ref) <= TOL[prec], (prec, k)
    finally:
        h.close()


def test_noalloc_rejects_oversized_request():
    h = itn.Handle(0)
    try:
        cap = h.heff_noalloc_max_bytes()
        assert cap == 64 << 20
        cl = cr = 1536  # bf16 W-stage output alone: 1536^2 * 20 * 2 bytes > 64 MiB
        W = inp.heisenberg_mpo(3)[1]
        Ld = torch.zeros((cl, 5, cl), dtype=torch.bfloat16, device=DEV)
        Rd = torch.zeros((cr, 5, cr), dtype=torch.bfloat16, device=DEV)
        pd = torch.zeros((cl, 2, 2, cr), dtype=torch.float64, device=DEV)
        out = torch.full_like(pd, 7.0)
        with pytest.raises(itn.ItnError) as e:
            h.heff_apply_noalloc(Ld, W, W, Rd, pd, out, prec="bf16")
        assert e.value.name == "ITN_E_WORKSPACE"
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())  # nothing was written
        # the entry point still works after the rejection
        L, W1, W2, R, psi = _case(64, 64, 2, 5, 1, 9, "heis")
        a = torch.zeros(psi.shape, dtype=torch.float64, device=DEV)
        b = torch.zeros(psi.shape, dtype=torch.float64, device=DEV)
        h.heff_apply(dev(L), W1, W2, dev(R), dev(psi), a, prec="f64")
        h.heff_apply_noalloc(dev(L), W1, W2, dev(R), dev(psi), b, prec="f64")
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    finally:
        h.close()
