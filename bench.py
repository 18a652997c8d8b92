#!/usr/bin/env python3
"""Benchmark of the two-site DMRG effective-Hamiltonian matvec on one MI355X.

One step = one dense H_eff*psi (stage-1 MFMA GEMM with L, the sparse
W-stage, stage-4 MFMA GEMM with R, including the conversion/transposition of
the FP64 input vector) at chi = 2048, d = 2, w = 5 (Heisenberg MPO), the
environments built on the GPU from a seeded random canonical MPS.  The
headline `value` is the mixed-precision (bf16 operands, fp32 accumulation)
throughput in TFLOP/s of algorithmic work; f32 and the plain FP64 GPU form of
the same path are timed beside it, with their error against FP64.

    python bench.py [--steps K] [--warmup W] [--chi 2048] [--no-cpu-baseline]

Prints one JSON line.  Only one GPU is used; --gpus > 1 is refused.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = ("H_eff·psi TFLOP/s (% MFMA peak), mixed vs FP64; DMRG sweep time at 1e-8 ΔE")
PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "f64": 78.6}
# the sources each timed kernel is compiled from (its HBM-traffic record is
# valid only for this code); of the shared declarations header only the
# kernel's argument struct counts
KERNEL_SOURCES = {
    "heff_stage1_fused": (["paper_2007_14822_amd/csrc/heff_fused.hip",
                           "paper_2007_14822_amd/csrc/gemm_core.h",
                           "paper_2007_14822_amd/csrc/common.h"], "struct HeffFusedArgs"),
    "heff_stage4_gemm": (["paper_2007_14822_amd/csrc/gemm.hip", "paper_2007_14822_amd/csrc/gemm_core.h",
                          "paper_2007_14822_amd/csrc/common.h"], "struct GemmArgs"),
}
KERNEL_DECLS = "paper_2007_14822_amd/csrc/kernels.h"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(kernel: str = "heff_stage1_fused") -> str:
    srcs, decl = KERNEL_SOURCES[kernel]
    hsh = hashlib.sha256()
    for p in srcs:
        fp = os.path.join(ROOT, p)
        if os.path.exists(fp):
            hsh.update(open(fp, "rb").read())
    fp = os.path.join(ROOT, KERNEL_DECLS)
    if os.path.exists(fp):
        text = open(fp, "rb").read().decode()
        i = text.find(decl)
        if i >= 0:
            hsh.update(text[i:text.index("};", i)].encode())
    return hsh.hexdigest()[:16]


def heff_flops(chi_l, chi_r, d, w, nv=1):
    """Algorithmic flops of one H_eff*psi: 4 w d^2 chi^3 (two GEMM stages)
    plus 4 w^2 d^3 chi^2 (the W-stage as two K = w d contractions)."""
    return nv * (2.0 * w * d * d * chi_l * chi_l * chi_r + 2.0 * w * d * d * chi_l * chi_r * chi_r
                 + 4.0 * w * w * d ** 3 * chi_l * chi_r)


def kernel_work(chi_l, chi_r, d, w, nv=1):
    """Algorithmic work per launch of each kernel of one H_eff*psi:
    flops for the matrix-core stages, HBM bytes for the memory-bound ones
    (operand sizes at the precision in use are filled in by the caller)."""
    s1 = 2.0 * w * d * d * chi_l * chi_l * chi_r * nv
    sw = 4.0 * w * w * d ** 3 * chi_l * chi_r * nv
    s4 = 2.0 * w * d * d * chi_l * chi_r * chi_r * nv
    return {"heff_stage1_fused": s1 + sw, "heff_stage1_gemm": s1, "heff_stage4_gemm": s4}


def build_workload(h, chi, d, torch, np, inp):
    """Random canonical MPS of N_c = 2 log2 chi + 2 sites, Heisenberg MPO;
    L = environment of the sites left of the centre bond, R of those right
    of it, both built on the GPU (FP64 environment steps); psi unit Gaussian."""
    n = int(round(math.log2(chi)))
    Nc = 2 * n + 2
    c = Nc // 2 - 1
    rng = inp.rng_for(1, chi)
    As = inp.random_canonical_mps(Nc, d, chi, center=c, rng=rng)
    Ws = inp.heisenberg_mpo(Nc, d - 1)
    w = Ws[0].shape[0]
    dev = "cuda:0"
    Lg = torch.zeros((1, w, 1), dtype=torch.float64, device=dev)
    Lg[0, w - 1, 0] = 1.0
    for k in range(c):
        A = torch.as_tensor(np.ascontiguousarray(As[k]), device=dev)
        nxt = torch.empty((A.shape[2], w, A.shape[2]), dtype=torch.float64, device=dev)
        h.env_update(Lg, A, Ws[k], "left", nxt)
        Lg = nxt
    Rg = torch.zeros((1, w, 1), dtype=torch.float64, device=dev)
    Rg[0, 0, 0] = 1.0
    for k in range(Nc - 1, c + 1, -1):
        A = torch.as_tensor(np.ascontiguousarray(As[k]), device=dev)
        nxt = torch.empty((A.shape[0], w, A.shape[0]), dtype=torch.float64, device=dev)
        h.env_update(Rg, A, Ws[k], "right", nxt)
        Rg = nxt
    psi = inp.unit_gaussian((Lg.shape[0], d, d, Rg.shape[0]), rng)
    torch.cuda.synchronize()
    return Lg, Ws[c], Ws[c + 1], Rg, torch.as_tensor(np.ascontiguousarray(psi), device=dev)


def sum_leg(h, torch, np, inp, chi, steps, warmup):
    """H = H_ff + H_zz: the S=1/2 Heisenberg chain as two MPOs (flip-flop,
    w=4; ZZ, w=3) applied as a sum of H_eff terms at bond dimension chi (bf16
    operands; environments Gaussian of the right shapes, as only the time is
    taken here; the parity tests check the values)."""
    ops = inp.spin_ops(1)
    Sp, Sm, Sz, I = ops["S+"], ops["S-"], ops["Sz"], ops["Id"]
    Wf = np.zeros((4, 4, 2, 2))
    Wf[0, 0], Wf[1, 0], Wf[2, 0], Wf[3, 1], Wf[3, 2], Wf[3, 3] = I, Sp, Sm, 0.5 * Sm, 0.5 * Sp, I
    Wz = np.zeros((3, 3, 2, 2))
    Wz[0, 0], Wz[1, 0], Wz[2, 1], Wz[2, 2] = I, Sz, Sz, I
    g = torch.Generator(device="cuda:0").manual_seed(inp.seed_for(1, chi) + 7)
    terms = []
    for W in (Wf, Wz):
        w = W.shape[0]
        Le = (torch.randn((chi, w, chi), generator=g, device="cuda:0") / chi).to(torch.bfloat16)
        Re = (torch.randn((chi, w, chi), generator=g, device="cuda:0") / chi).to(torch.bfloat16)
        terms.append((Le, W, W, Re))
    psi = torch.randn((chi, 2, 2, chi), generator=g, device="cuda:0", dtype=torch.float64)
    out = torch.empty_like(psi)
    for _ in range(warmup):
        h.heff_apply_sum(terms, psi, out, prec="bf16")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        h.heff_apply_sum(terms, psi, out, prec="bf16")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    flops = 0.0
    for W in (Wf, Wz):
        kw = kernel_work(chi, chi, 2, W.shape[0])
        flops += kw["heff_stage1_fused"] + kw["heff_stage4_gemm"]
    return {"terms": "Heisenberg flip-flop (w=4) + ZZ (w=3)", "chi": chi, "ms_per_apply": ms,
            "flop_per_apply": flops, "tflops": flops / (ms * 1e-3) / 1e12, "precision": "bf16"}


def excited_leg(h, np, inp, N=40, maxdim=64):
    """Ground state, then the first excited state with the ground state's
    projector times an energy penalty added (bf16 matvecs, FP64 refinement):
    energies, gap, wall time and matvecs of each run."""
    mpo = h.mpo(inp.heisenberg_mpo(N))
    sweeps = [(16, 1e-10), (32, 1e-10)] + [(maxdim, 1e-10)] * 4
    kw = dict(prec="bf16", eig_tol=1e-9, krylovdim=8, maxiter=60, refine=True, allow_unconverged=True)
    out = {"model": "S=1/2 Heisenberg chain, N=%d, maxdim %d, penalty weight 4" % (N, maxdim)}
    gs = h.mps(inp.random_product_state(N, 2, inp.rng_for(2, 40)))
    t0 = time.perf_counter()
    r0 = h.dmrg_sweep(gs, mpo, sweeps, **kw)
    out["ground"] = {"energy": r0[-1]["energy"], "seconds": time.perf_counter() - t0,
                     "matvecs": int(sum(r["matvecs"] for r in r0))}
    x1 = h.mps(inp.random_product_state(N, 2, inp.rng_for(2, 41)))
    t0 = time.perf_counter()
    r1 = h.dmrg_sweep(x1, mpo, sweeps, ortho=[gs], weight=4.0, **kw)
    out["excited"] = {"energy": r1[-1]["energy"], "seconds": time.perf_counter() - t0,
                      "matvecs": int(sum(r["matvecs"] for r in r1))}
    out["gap"] = r1[-1]["energy"] - r0[-1]["energy"]
    return out


def time_heff(h, torch, Lp, W1, W2, Rp, psi, out, prec, steps, warmup):
    for _ in range(warmup):
        h.heff_apply(Lp, W1, W2, Rp, psi, out, prec=prec)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        h.heff_apply(Lp, W1, W2, Rp, psi, out, prec=prec)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def size_leg(h, torch, np, inp, chi, d, steps, warmup, precs=("bf16", "f32", "f64")):
    """The dense matvec at another bond dimension / local dimension (same
    workload recipe as the headline): ms, TFLOP/s and fraction of the
    precision's MFMA peak per precision, per-kernel times, error vs FP64."""
    L64, W1, W2, R64, psi = build_workload(h, chi, d, torch, np, inp)
    w = W1.shape[0]
    flops = heff_flops(chi, chi, d, w)
    work = kernel_work(chi, chi, d, w)
    tdt = {"bf16": torch.bfloat16, "f32": torch.float32, "f64": torch.float64}
    res, outs = {}, {}
    for prec in precs:
        if prec == "f64":
            Lp, Rp = L64, R64
        else:
            Lp = torch.empty(L64.shape, dtype=tdt[prec], device="cuda:0")
            Rp = torch.empty(R64.shape, dtype=tdt[prec], device="cuda:0")
            h.cast(L64, Lp)
            h.cast(R64, Rp)
        out = torch.zeros_like(psi)
        st = steps if prec != "f64" else max(2, steps // 4)
        ms = time_heff(h, torch, Lp, W1, W2, Rp, psi, out, prec, st, warmup)
        prof = profile_heff(h, torch, Lp, W1, W2, Rp, psi, out, prec, max(2, st // 2))
        for k, v in prof.items():
            if k in work:
                v["tflops"] = work[k] / (v["avg_ms"] * 1e-3) / 1e12
                v["frac_of_peak"] = v["tflops"] / PEAK_TFLOPS[prec]
        tf = flops / (ms * 1e-3) / 1e12
        res[prec] = {"ms_per_step": ms, "tflops": tf, "frac_of_peak": tf / PEAK_TFLOPS[prec],
                     "steps": st, "kernels": prof}
        outs[prec] = out
        del Lp, Rp
    if "f64" in outs:
        for prec in outs:
            if prec != "f64":
                res[prec]["rel_err_vs_f64"] = float(torch.linalg.vector_norm(outs[prec] - outs["f64"]) /
                                                    torch.linalg.vector_norm(outs["f64"]))
    return {"chi": chi, "d": d, "w": w, "flop_per_step": flops, "by_precision": res}


def profile_heff(h, torch, Lp, W1, W2, Rp, psi, out, prec, steps):
    h.profile(True)
    for _ in range(steps):
        h.heff_apply(Lp, W1, W2, Rp, psi, out, prec=prec)
    rep = h.profile_report()
    h.profile(False)
    return {k: {"avg_ms": v[0] / max(1, v[1]), "launches": v[1]} for k, v in rep.items()}


def traffic_record(kernel: str, workload: str):
    """HBM bytes per launch measured by rocprofv3 --pmc (FETCH_SIZE,
    WRITE_SIZE) and calibrated with a plain copy, stored with the hash of
    the kernel sources it was taken on; None if absent or stale."""
    fp = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(fp):
        return None
    rec = json.load(open(fp))
    if kernel not in KERNEL_SOURCES or rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def ttgt(tensordot, L, W1, W2, R, psi):
    """H_eff psi as the paper's TTGT contraction (Sec. 9.4): every pairwise
    contraction a permutation plus one library GEMM (tensordot).  A comparator
    only: W1[m0, m1, s1', s1], W2[m1, m2, s2', s2], R[b', m2, b]."""
    T1 = tensordot(L, psi, ([2], [0]))              # [a', m0, s1, s2, b]
    T2 = tensordot(T1, W1, ([1, 2], [0, 3]))        # [a', s2, b, m1, s1']
    T3 = tensordot(T2, W2, ([1, 3], [3, 0]))        # [a', b, s1', m2, s2']
    T4 = tensordot(T3, R, ([1, 3], [2, 1]))         # [a', s1', s2', b']
    return T4


def ttgt_gpu(torch, L, W1, W2, R, psi, flops, steps):
    """TTGT with PyTorch FP64 (rocBLAS/hipBLASLt DGEMMs and permute copies)."""
    W1t = torch.as_tensor(W1, device=L.device)
    W2t = torch.as_tensor(W2, device=L.device)
    td = lambda a, b, dims: torch.tensordot(a, b, dims=dims)
    y = ttgt(td, L, W1t, W2t, R, psi)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        y = ttgt(td, L, W1t, W2t, R, psi)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"ms_per_step": ms, "tflops": flops / (ms * 1e-3) / 1e12, "steps": steps,
            "method": "torch.tensordot chain L, W1, W2, R in FP64 (permute + library GEMM each)"}


def ttgt_cpu(np, L, W1, W2, R, psi, flops):
    """TTGT on the host BLAS with every core (numpy tensordot, FP64), one matvec."""
    import os
    Lh, Rh, ph = L.cpu().numpy(), R.cpu().numpy(), psi.cpu().numpy()
    td = lambda a, b, dims: np.tensordot(a, b, axes=dims)
    t0 = time.perf_counter()
    ttgt(td, Lh, W1, W2, Rh, ph)
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "seconds": dt,
            "cores": len(os.sched_getaffinity(0)),
            "method": "numpy.tensordot chain in FP64 on the host BLAS, one full matvec"}


def cpu_baseline(L, W1, W2, R, psi, chi, d, w, budget_s):
    """The oracle (plain einsum, one thread) on a bounded sample: the first k
    output rows a' of the same matvec; throughput scaled by k/chi."""
    import numpy as np
    from oracle import heff as hf
    t0 = time.perf_counter()
    hf.heff_apply_rows(L, W1, W2, R, psi, [0])
    t1 = time.perf_counter() - t0
    k = int(max(1, min(chi, budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    hf.heff_apply_rows(L, W1, W2, R, psi, list(range(k)))
    dt = time.perf_counter() - t0
    fl = heff_flops(chi, chi, d, w) * k / chi
    return {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d output rows a' of the chi=%d matvec (oracle heff_apply_rows, "
                      "numpy einsum optimize=False, single thread), %.1f s" % (k, chi, chi, dt)}


# ----------------------------------------------------------------- QN legs
def qn_workload(h, torch, np, inp, which, prec, nv, split_mpo=False):
    """Block-sparse H_eff operands.  Structure from the library's block
    enumeration, values from the seeded per-block generator.  split_mpo:
    every MPO channel its own link sector (the sparse-MPO "splitblocks"
    form: zero W blocks between channels of equal charge are never formed;
    the same operator, finer groups).
      c3: U(1) S=1/2 chain bond, chi=4096 in 25 binomial-shaped sectors, w=5
      c4: U(1)xU(1) Hubbard 4x32 cylinder bond, chi=4096 in 81 sectors,
          w=18 (column-major snake) or the synthetic w=38 shape"""
    if which == "c3":
        bond = [((q,), n) for q, n in inp.c3_sector_dims()]
        site_q = inp.heisenberg_site_qn(1)
        W = inp.heisenberg_mpo(3)[1]
        W1 = W2 = W
        link_q = inp.heisenberg_mpo_link_qn()
        seed = inp.seed_for(3, 4096)
    elif which == "c4z4":
        bond = list(inp.c4z4_sector_dims())
        site_q = inp.hubbard_momentum_site_qn()
        link_q = inp.hubbard_momentum_link_qn(18)
        W1 = W2 = None  # Gaussian on the allowed blocks, built below
        seed = inp.seed_for(5, 4096)
    else:
        bond = list(inp.c4_sector_dims())
        site_q = inp.hubbard_site_qn()
        if which == "c4":
            Ws = inp.hubbard_mpo(32, 4)
            W1, W2 = Ws[62], Ws[63]
        else:  # c4w38
            Ws = inp.long_range_hubbard_mpo(8, 9)
            W1, W2 = Ws[6], Ws[7]
        link_q = [None] * W1.shape[0]
        # channel charges: kinds 0..3 follow c+up, c+dn, cup, cdn
        rmax = (W1.shape[0] - 2) // 4
        kind_q = [(1, 1), (1, -1), (-1, -1), (-1, 1)]
        link_q = [(0, 0)] + [kind_q[k] for k in range(4) for _ in range(rmax)] + [(0, 0)]
        seed = inp.seed_for(4, 4096)
    mod = (0, 0, 4) if which == "c4z4" else None
    bq = [tuple(q) if isinstance(q, tuple) else (q,) for q, _ in bond]
    bd = [n for _, n in bond]
    sq, sd = inp.sectors_from_basis_qns(site_q)
    if split_mpo:
        lq = [tuple(int(x) for x in (q if isinstance(q, (tuple, list)) else (q,))) for q in link_q]
        ld = [1] * len(lq)
    else:
        lq, ld = inp.sectors_from_basis_qns(link_q)
    spaces = {
        "L": [(bq, bd, +1), (lq, ld, -1), (bq, bd, -1)],
        "R": [(bq, bd, -1), (lq, ld, +1), (bq, bd, +1)],
        "psi": [(bq, bd, +1), (sq, sd, +1), (sq, sd, +1), (bq, bd, -1)],
        "W": [(lq, ld, +1), (lq, ld, -1), (sq, sd, +1), (sq, sd, -1)],
    }
    if mod:
        spaces = {k: [sp + (mod,) for sp in v] for k, v in spaces.items()}
    tdt = {"bf16": torch.bfloat16, "f32": torch.float32, "f64": torch.float64}[prec]
    dev = "cuda:0"

    def fill(name, tag, nvec=1):
        blocks, offs, tot = h.qn_allowed_blocks(spaces[name])
        sizes = [int(np.prod([spaces[name][i][1][k] for i, k in enumerate(b)])) for b in blocks]
        flat = np.empty(nvec * tot)
        for v in range(nvec):
            for b, o, sz in zip(blocks, offs, sizes):
                flat[v * tot + o:v * tot + o + sz] = inp.block_values(seed + tag, (v,) + tuple(b),
                                                                     (sz,))
        return {"spaces": spaces[name], "blocks": blocks, "offsets": offs}, flat, tot

    Ld, Lf, _ = fill("L", 1)
    Rd, Rf, _ = fill("R", 2)
    Pd, Pf, tot = fill("psi", 3, nv)
    for v in range(nv):
        Pf[v * tot:(v + 1) * tot] /= np.linalg.norm(Pf[v * tot:(v + 1) * tot])
    Ld["data"] = torch.as_tensor(Lf, dtype=tdt, device=dev)
    Rd["data"] = torch.as_tensor(Rf, dtype=tdt, device=dev)
    Pd["data"] = torch.as_tensor(Pf, device=dev)
    Od = dict(Pd)
    Od["data"] = torch.zeros_like(Pd["data"])
    if W1 is None:  # synthetic symmetric MPO tensors: Gaussian on their allowed blocks
        Wds = []
        for tag in (4, 5):
            blocks, offs, _ = h.qn_allowed_blocks(spaces["W"])
            dims = [spaces["W"][i][1] for i in range(4)]
            starts = [np.concatenate([[0], np.cumsum(dd)[:-1]]) for dd in dims]
            Wd = np.zeros([int(sum(dd)) for dd in dims])
            for b in blocks:
                shp = tuple(int(dims[i][b[i]]) for i in range(4))
                sl = tuple(slice(int(starts[i][b[i]]), int(starts[i][b[i]]) + shp[i]) for i in range(4))
                Wd[sl] = inp.block_values(seed + tag, tuple(b), shp)
            Wds.append(Wd)
        W1, W2 = Wds
    W1d = {"spaces": spaces["W"], "data": np.ascontiguousarray(W1)}
    W2d = {"spaces": spaces["W"], "data": np.ascontiguousarray(W2)}
    return Ld, W1d, W2d, Rd, Pd, Od


def time_qn(h, torch, np, inp, which, prec, nv, steps, warmup, split_mpo=False):
    Ld, W1d, W2d, Rd, Pd, Od = qn_workload(h, torch, np, inp, which, prec, nv, split_mpo)
    t0 = time.perf_counter()
    plan = h.qn_plan(Ld, W1d, W2d, Rd, Pd, nv=nv, prec=prec)
    tplan = time.perf_counter() - t0
    apply = plan.bind(Ld, Rd, Pd, Od)  # descriptors marshalled once
    for _ in range(warmup):
        apply()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        apply()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # as inside an eigensolver: environments repacked once per bond
    plan.prepare_env(Ld, Rd)
    apply_pe = plan.bind(None, None, Pd, Od)
    for _ in range(max(1, warmup // 2)):
        apply_pe()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        apply_pe()
    e1.record()
    torch.cuda.synchronize()
    ms_pe = e0.elapsed_time(e1) / steps
    info = plan.info()
    h.profile(True)
    for _ in range(max(2, steps // 4)):
        apply()
    rep = h.profile_report()
    h.profile(False)
    out = Od["data"].clone()
    del Ld, Rd, Pd, Od
    kern = {k: {"avg_ms": v[0] / max(1, v[1]), "launches": v[1]} for k, v in rep.items()}
    # roofline of each stage: block-sparse flops of the grouped GEMMs against
    # the MFMA peak of the precision; the W-stage's compulsory bytes (read X
    # once, write Z once, in their stored types) against HBM
    es = {"bf16": 2, "f32": 4, "f64": 8}[prec]
    xs = es  # X is stored in the operand type (bf16 applies accumulate it in f32)
    work = {"qn_stage1_grouped": ("mfma", info["flops_stage1"]),
            "qn_stage4_grouped": ("mfma", info["flops"] - info["flops_stage1"]),
            "qn_wstage": ("hbm", nv * (info["x_elems"] * xs + info["z_elems"] * es))}
    roof = {}
    for k, (bound, amount) in work.items():
        if k not in kern:
            continue
        t = kern[k]["avg_ms"] * 1e-3
        if bound == "mfma":
            ach = amount / t / 1e12
            roof[k] = {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[prec],
                       "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS[prec], "flop_per_launch": amount}
        else:
            ach = amount / t / 1e9
            roof[k] = {"bound": "hbm", "achieved": ach, "peak": 8000.0, "unit": "GB/s",
                       "frac": ach / 8000.0, "bytes_per_launch": amount}
    return {"ms_per_apply": ms, "tflops": info["flops"] / (ms * 1e-3) / 1e12,
            "frac_of_peak": info["flops"] / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
            "roofline": roof,
            "ms_per_apply_prepared_env": ms_pe,
            "tflops_prepared_env": info["flops"] / (ms_pe * 1e-3) / 1e12,
            "flop_per_apply": info["flops"], "out_blocks": info["out_nblocks"],
            "stage1_groups": info["n_groups_stage1"], "stage4_segments": info["n_pairs_stage4"],
            "plan_seconds": tplan, "nv": nv,
            "launch_modes": [info["mode_stage1"], info["mode_stage4"]],
            "wstage_tile": info["wstage_tile"], "kernels": kern}, out


# ---------------------------------------------------------------- DMRG leg
# Davidson budget per bond: a few matvecs per local solve (the sweeps, not the
# local solve, carry the convergence), and a tight budget for the reference run
# that fixes the converged energy.
DAVIDSON = {"krylovdim": 4, "maxiter": 8}
DAVIDSON_TIGHT = {"krylovdim": 8, "maxiter": 60}
# block Davidson (dense and block-sparse sweeps): 4 residuals per step, two
# steps between restarts (8 basis vectors), 12 vectors applied per bond
DAVIDSON_BLOCK4 = {"krylovdim": 8, "maxiter": 12}


def dmrg_leg(h, np, inp, prec, sweeps, N=100, timing=False, davidson=None, block=1):
    """Spin-1 Heisenberg chain (d=3, w=5), random product start, the given
    (maxdim, cutoff) schedule; per-sweep time, energy, matvecs (all, and
    those in FP64), and with timing the per-phase split (adds stream
    waits).  block > 1: block Davidson, `block` vectors per batched matvec
    (Krylov budget `davidson`, else DAVIDSON_BLOCK4 for block 4 and the
    small budget scaled by the block otherwise)."""
    mpo = h.mpo(inp.heisenberg_mpo(N, 2))
    mps = h.mps(inp.random_product_state(N, 3, inp.rng_for(2, 64)))
    if davidson is not None:
        dv = dict(davidson)
    elif block == 4:
        dv = dict(DAVIDSON_BLOCK4)
    elif block > 1:
        dv = {"krylovdim": DAVIDSON["krylovdim"] * block, "maxiter": DAVIDSON["maxiter"] * block}
    else:
        dv = dict(DAVIDSON)
    t0 = time.perf_counter()
    recs = h.dmrg_sweep(mps, mpo, sweeps, prec=prec, eig_tol=1e-9, refine=True,
                        allow_unconverged=True, timing=timing, block=block, **dv)
    secs = time.perf_counter() - t0
    mps.close()
    mpo.close()
    tot = sum(r["matvecs"] for r in recs)
    f64 = sum(r["matvecs_f64"] for r in recs)
    bonds = 2 * (N - 1) * len(recs)
    return {"total_seconds": secs, "sweeps": recs, "block": block, "davidson": dv,
            "matvecs": tot, "matvecs_f64": f64, "low_precision_fraction": (tot - f64) / tot,
            "f64_matvecs_per_bond": f64 / bonds}


def qn_dmrg_leg(h, inp, prec, Lx=8, Ly=4, maxdims=(128, 512, 1024, 2048, 2048), block=1, davidson=None):
    """Block-sparse two-site sweeps on the U(1) x U(1) Hubbard cylinder
    (Lx x Ly, U/t = 8, half filling from a Neel product state, cutoff 1e-8),
    the bench's small Davidson budget; per sweep energy, time and the
    phase split.  block > 1: block Davidson, `block` vectors per batched
    matvec (the Krylov budget `davidson`, else the small one scaled by the
    block)."""
    Ws = inp.hubbard_mpo(Lx, Ly, U=8.0)
    N = Lx * Ly
    mps = h.qn_mps(inp.hubbard_site_qn(), [1 + (k % 2) for k in range(N)])
    mpo = h.mpo(Ws)
    dv = dict(davidson or DAVIDSON)
    if block > 1 and davidson is None:
        dv = {"krylovdim": dv["krylovdim"] * block, "maxiter": dv["maxiter"] * block}
    t0 = time.perf_counter()
    recs = h.qn_dmrg_sweep(mps, mpo, inp.hubbard_mpo_link_qn(Ws[0].shape[0]),
                           [(m, 1e-8) for m in maxdims], prec=prec, eig_tol=1e-10,
                           allow_unconverged=True, timing=True, block=block, **dv)
    secs = time.perf_counter() - t0
    total_qn = h.qn_mps_link(mps, N)  # the last link carries the state's (N, 2Sz)
    mps.close()
    mpo.close()
    tot = sum(r["matvecs"] for r in recs)
    f64 = sum(r["matvecs_f64"] for r in recs)
    return {"model": "Hubbard %dx%d cylinder, U/t=8, U(1)xU(1) (N, 2Sz), w=%d" % (Lx, Ly, Ws[0].shape[0]),
            "schedule": [(m, 1e-8) for m in maxdims], "block": block, "davidson": dv,
            "total_seconds": secs, "sweeps": recs,
            "matvecs": tot, "matvecs_f64": f64, "low_precision_fraction": (tot - f64) / tot,
            "total_qn": [list(q) for q, _ in total_qn]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--chi", type=int, default=2048)
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--only", choices=["bf16", "f32", "f64"], default=None,
                    help="time one precision only (profiling runs)")
    ap.add_argument("--no-qn", action="store_true")
    ap.add_argument("--no-dmrg", action="store_true")
    ap.add_argument("--no-sum", action="store_true")
    ap.add_argument("--qn-only", action="store_true",
                    help="run the block-sparse legs only (profiling runs; prints their JSON)")
    ap.add_argument("--qn-which", default="c3,c4,c4w38,c4z4",
                    help="block-sparse workloads of --qn-only (comma list)")
    ap.add_argument("--qn-prec", default="bf16,f64", help="precisions of --qn-only (comma list)")
    ap.add_argument("--qn-dmrg-only", action="store_true",
                    help="run the block-sparse Hubbard sweeps only, precisions of --qn-prec (profiling runs)")
    ap.add_argument("--qn-dmrg-block", type=int, default=1, help="Davidson block of --qn-dmrg-only")
    ap.add_argument("--no-splitblocks", action="store_true",
                    help="--qn-only without the one-sector-per-channel MPO legs")
    ap.add_argument("--dmrg-large", action="store_true",
                    help="with --dmrg-only: spin-1 chain N=40, cutoff 0, maxdim 256 then 1024 x 3 "
                         "(density matrices of up to 3072 rows)")
    ap.add_argument("--dmrg-only", action="store_true",
                    help="run the DMRG legs only (profiling runs; prints their JSON)")
    ap.add_argument("--no-sizes", action="store_true",
                    help="skip the other dense sizes (chi 256/512/1024 at d=2, chi 2048 at d=3)")
    ap.add_argument("--dmrg-maxdim", type=int, default=256)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the timed work, copy a buffer of this many bytes 3 times "
                         "(a plain copy kernel of known size, to calibrate HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2007_14822_amd as itn
    from paper_2007_14822_amd import inputs as inp

    chi, d = args.chi, args.d
    h = itn.Handle(0)
    if args.qn_only or args.dmrg_only or args.qn_dmrg_only:
        out = {}
        if args.qn_dmrg_only:  # the block-sparse Hubbard sweeps alone (profiling runs)
            for prec in args.qn_prec.split(","):
                log("[bench] block-sparse DMRG, Hubbard 8x4 cylinder %s, block %d" % (prec, args.qn_dmrg_block))
                out["qn_dmrg_" + prec] = qn_dmrg_leg(
                    h, inp, prec, block=args.qn_dmrg_block,
                    davidson=DAVIDSON_BLOCK4 if args.qn_dmrg_block == 4 else None)
                log("[bench]   %.1f s" % out["qn_dmrg_" + prec]["total_seconds"])
        if args.qn_only:
            nvs = {"c3": 1, "c4": 4, "c4w38": 4, "c4z4": 4}
            for which in args.qn_which.split(","):
                nv = nvs[which]
                for prec in args.qn_prec.split(","):
                    log("[bench] QN %s %s nv=%d" % (which, prec, nv))
                    out["%s_%s" % (which, prec)] = time_qn(h, torch, np, inp, which, prec, nv, 10, 3)[0]
                if which in ("c3", "c4") and "bf16" in args.qn_prec and not args.no_splitblocks:
                    log("[bench] QN %s bf16, one link sector per MPO channel" % which)
                    out["%s_bf16_splitblocks" % which] = time_qn(h, torch, np, inp, which, "bf16", nv, 10,
                                                                 3, split_mpo=True)[0]
        if args.dmrg_only and args.dmrg_large:
            sched = [(256, 0.0), (1024, 0.0), (1024, 0.0), (1024, 0.0)]
            for prec in ("bf16", "f64"):
                log("[bench] DMRG spin-1 N=40 %s, cutoff 0, maxdim up to 1024" % prec)
                out["dmrg_large_" + prec] = dmrg_leg(h, np, inp, prec, sched, N=40, timing=True)
                log("[bench]   %.1f s" % out["dmrg_large_" + prec]["total_seconds"])
        elif args.dmrg_only:
            md = args.dmrg_maxdim
            sched = [(min(64, md), 1e-10), (min(128, md), 1e-10)] + [(md, 1e-10)] * 4
            for prec in ("f64", "bf16"):
                log("[bench] DMRG spin-1 N=100 %s" % prec)
                out["dmrg_" + prec] = dmrg_leg(h, np, inp, prec, sched)
        h.close()
        print(json.dumps(out), flush=True)
        return
    log("[bench] building chi=%d workload" % chi)
    t0 = time.perf_counter()
    L64, W1, W2, R64, psi = build_workload(h, chi, d, torch, np, inp)
    w = W1.shape[0]
    log("[bench] workload ready in %.1f s" % (time.perf_counter() - t0))
    flops = heff_flops(chi, chi, d, w)
    gemm_flops = 2.0 * w * d * d * chi ** 3  # one GEMM stage
    precs = [args.only] if args.only else ["bf16", "f32", "f64"]
    tdt = {"bf16": torch.bfloat16, "f32": torch.float32, "f64": torch.float64}
    results = {}
    outs = {}
    for prec in precs:
        if prec == "f64":
            Lp, Rp = L64, R64
        else:
            Lp = torch.empty(L64.shape, dtype=tdt[prec], device="cuda:0")
            Rp = torch.empty(R64.shape, dtype=tdt[prec], device="cuda:0")
            h.cast(L64, Lp)
            h.cast(R64, Rp)
        out = torch.zeros_like(psi)
        steps = args.steps if prec != "f64" else max(2, args.steps // 4)
        log("[bench] %s: %d warmup + %d timed steps" % (prec, args.warmup, steps))
        ms = time_heff(h, torch, Lp, W1, W2, Rp, psi, out, prec, steps, args.warmup)
        prof = profile_heff(h, torch, Lp, W1, W2, Rp, psi, out, prec, max(2, steps // 2))
        outs[prec] = out.clone()
        results[prec] = {"ms_per_step": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                         "frac_of_peak": flops / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                         "steps": steps, "kernels": prof}
        log("[bench] %s: %.3f ms/step, %.1f TFLOP/s" % (prec, ms, results[prec]["tflops"]))
        del Lp, Rp
    if "f64" in outs:
        ref = outs["f64"]
        for prec in precs:
            if prec != "f64":
                results[prec]["rel_err_vs_f64"] = float(
                    torch.linalg.vector_norm(outs[prec] - ref) / torch.linalg.vector_norm(ref))
    head = precs[0]
    r = results[head]
    # dominant kernel and its roofline
    work = kernel_work(chi, chi, d, w)
    kern = max(r["kernels"].items(), key=lambda kv: kv[1]["avg_ms"])
    kname, kst = kern[0], kern[1]
    fl = work.get(kname)
    achieved = fl / (kst["avg_ms"] * 1e-3) / 1e12 if fl else None
    roof = {"bound": "mfma", "kernel": kname, "achieved": achieved, "peak": PEAK_TFLOPS[head],
            "unit": "TFLOP/s", "frac": (achieved / PEAK_TFLOPS[head]) if achieved else None,
            "traffic": traffic_record(kname, "c1_chi%d_%s" % (chi, head)),
            "avg_ms": kst["avg_ms"], "flop_per_launch": fl}
    for k, v in r["kernels"].items():
        if k in work:
            v["tflops"] = work[k] / (v["avg_ms"] * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": r["tflops"], "unit": "TFLOP/s", "n_gpus": 1,
        "steps": r["steps"], "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": head,
        "data": "synthetic",
        "config": {"workload": "dense two-site H_eff*psi, chi=%d, d=%d, w=%d (S=1/2 Heisenberg "
                               "MPO), nv=1, environments of a seeded random canonical MPS" %
                               (chi, d, w),
                   "chi": chi, "d": d, "w": w, "nv": 1, "flop_per_step": flops,
                   "precision": "%s operands, %s accumulation" %
                                (head, "fp64" if head == "f64" else "fp32")},
        "roofline": roof,
        "by_precision": {k: {kk: vv for kk, vv in v.items() if kk != "kernels"} for k, v in
                         results.items()},
        "kernels": {k: v["kernels"] for k, v in results.items()},
    }
    if "f64" in results and head != "f64":
        line["speedup_vs_fp64_gpu"] = results["f64"]["ms_per_step"] / r["ms_per_step"]
    if not args.only and not args.no_sizes:
        sizes = {}
        for cs, ds in ((256, 2), (512, 2), (1024, 2), (2048, 3)):
            if (cs, ds) == (chi, d):
                continue
            log("[bench] dense chi=%d d=%d" % (cs, ds))
            sizes["chi%d_d%d" % (cs, ds)] = size_leg(h, torch, np, inp, cs, ds, args.steps,
                                                     args.warmup)
            b = sizes["chi%d_d%d" % (cs, ds)]["by_precision"]
            log("[bench]   " + ", ".join("%s %.3f ms (%.1f%% of peak)" % (p, v["ms_per_step"],
                                                                        100 * v["frac_of_peak"])
                                        for p, v in b.items()))
        line["dense_sizes"] = sizes
    if not args.only:
        log("[bench] TTGT comparators (library GEMMs + permutes, FP64)")
        line["ttgt_gpu_f64"] = ttgt_gpu(torch, L64, W1, W2, R64, psi, flops, args.steps // 4 + 2)
        if not args.no_cpu_baseline:
            line["ttgt_cpu_f64"] = ttgt_cpu(np, L64, W1, W2, R64, psi, flops)
    if not args.no_qn and not args.only:
        qn = {}
        for which, nv in (("c3", 1), ("c4", 4), ("c4w38", 4), ("c4z4", 4)):
            for prec in ("bf16", "f64"):
                log("[bench] QN %s %s nv=%d" % (which, prec, nv))
                r_qn, out = time_qn(h, torch, np, inp, which, prec, nv, 10, 3)
                qn["%s_%s" % (which, prec)] = r_qn
                if prec == "f64":
                    ref = out
                    lo = qn["%s_bf16" % which]
                    lo["rel_err_vs_f64"] = float(torch.linalg.vector_norm(lo_out - ref) /
                                                 torch.linalg.vector_norm(ref))
                else:
                    lo_out = out
                log("[bench]   %.3f ms, %.1f TFLOP/s" % (r_qn["ms_per_apply"], r_qn["tflops"]))
        for which in ("c3", "c4"):  # the same operators with every MPO channel its own sector
            log("[bench] QN %s bf16, one link sector per MPO channel" % which)
            r_qn, _ = time_qn(h, torch, np, inp, which, "bf16", 1 if which == "c3" else 4, 10, 3,
                              split_mpo=True)
            qn["%s_bf16_splitblocks" % which] = r_qn
            log("[bench]   %.3f ms, %.1f TFLOP/s" % (r_qn["ms_per_apply"], r_qn["tflops"]))
        line["qn"] = qn
    if not args.no_sum and not args.only:
        line["mpo_sum"] = sum_leg(h, torch, np, inp, chi, args.steps, args.warmup)
    if not args.no_dmrg and not args.only:
        md = args.dmrg_maxdim
        sched = [(min(64, md), 1e-10), (min(128, md), 1e-10)] + [(md, 1e-10)] * 4
        dm = {}
        for prec, blk in (("f64", 1), ("bf16", 1), ("f64", 4), ("bf16", 4)):
            key = prec if blk == 1 else "%s_block%d" % (prec, blk)
            log("[bench] DMRG spin-1 N=100 %s, block %d, maxdim up to %d" % (prec, blk, md))
            dm[key] = dmrg_leg(h, np, inp, prec, sched, block=blk)
            log("[bench]   %.1f s, E=%.12f, %d matvecs (%d FP64)" % (
                dm[key]["total_seconds"], dm[key]["sweeps"][-1]["energy"], dm[key]["matvecs"],
                dm[key]["matvecs_f64"]))
        log("[bench] DMRG reference: FP64, tight Davidson budget %s" % DAVIDSON_TIGHT)
        ref_run = dmrg_leg(h, np, inp, "f64", sched, davidson=DAVIDSON_TIGHT)
        e_conv = ref_run["sweeps"][-1]["energy"]
        e64 = dm["f64"]["sweeps"][-1]["energy"]
        for prec in dm:
            ss = dm[prec]["sweeps"]
            t = 0.0
            reached = within = None
            for k, rec in enumerate(ss):
                t += rec["seconds"]
                if k > 0 and abs(rec["energy"] - ss[k - 1]["energy"]) < 1e-8 * abs(rec["energy"]):
                    reached = t if reached is None else reached
                if abs(rec["energy"] - e_conv) < 1e-8 * abs(e_conv):
                    within = t if within is None else within
            dm[prec]["seconds_to_dE_1e-8"] = reached
            dm[prec]["seconds_to_within_1e-8_of_converged"] = within
            dm[prec]["rel_err_vs_f64_run"] = abs(ss[-1]["energy"] - e64) / abs(e64)
            dm[prec]["rel_err_vs_converged"] = abs(ss[-1]["energy"] - e_conv) / abs(e_conv)
        dm["davidson"] = DAVIDSON
        dm["reference"] = {"davidson": DAVIDSON_TIGHT, "energy": e_conv,
                           "total_seconds": ref_run["total_seconds"],
                           "sweep_energies": [r["energy"] for r in ref_run["sweeps"]]}
        # time split of the last sweep, from a separate run with phase timers
        log("[bench] DMRG bf16 time split (phase-timed run)")
        sp = dmrg_leg(h, np, inp, "bf16", sched, timing=True)["sweeps"][-1]
        split = {k: sp[k] for k in ("seconds", "t_matvec", "t_solver", "t_split", "t_env", "matvecs",
                                    "matvecs_f64", "max_bond")}
        line["dmrg"] = {"model": "spin-1 Heisenberg chain, N=100, d=3, w=5",
                        "schedule": sched, **dm, "bf16_last_sweep_split": split}
    if not args.no_dmrg and not args.only:
        qd = {}
        for prec in ("f64", "bf16"):
            log("[bench] block-sparse DMRG, Hubbard 8x4 cylinder %s, maxdim up to 2048" % prec)
            qd[prec] = qn_dmrg_leg(h, inp, prec)
            log("[bench]   %.1f s, E=%.10f" % (qd[prec]["total_seconds"], qd[prec]["sweeps"][-1]["energy"]))
        e64 = qd["f64"]["sweeps"][-1]["energy"]
        qd["bf16"]["rel_err_vs_f64_run"] = abs(qd["bf16"]["sweeps"][-1]["energy"] - e64) / abs(e64)
        log("[bench] block-sparse DMRG, Hubbard 8x4 cylinder bf16, block Davidson (4 vectors per launch)")
        qd["bf16_block4"] = qn_dmrg_leg(h, inp, "bf16", block=4, davidson=DAVIDSON_BLOCK4)
        log("[bench]   %.1f s, E=%.10f" % (qd["bf16_block4"]["total_seconds"],
                                          qd["bf16_block4"]["sweeps"][-1]["energy"]))
        line["qn_dmrg"] = qd
        log("[bench] excited state by energy penalty, S=1/2 chain N=40")
        line["excited_state"] = excited_leg(h, np, inp)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(L64.cpu().numpy(), W1, W2, R64.cpu().numpy(),
                                            psi.cpu().numpy(), chi, d, w, args.cpu_budget)
    else:
        line["cpu_baseline"] = None
    if args.copy_probe > 0:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = n * 4
    h.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
