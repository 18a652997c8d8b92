"""Python binding of libitn (two-site DMRG H_eff on MI355X / gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libitn.so.  Device tensors are torch tensors on a ROCm device;
MPO tensors are host float64 numpy arrays.  Importing the package does not
load the library; the first call does, and raises if it is missing.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref
from typing import Optional, Sequence

import numpy as np

from . import _lib as L

__all__ = ["ItnError", "Handle", "PREC", "load"]

PREC = {"f64": L.ITN_P_F64, "f32": L.ITN_P_F32, "bf16": L.ITN_P_BF16}


def load():
    return L.load()


class ItnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (L.STATUS_NAMES.get(status, str(status)), msg))
        self.status = status
        self.name = L.STATUS_NAMES.get(status, str(status))


def _dtype_code(t) -> int:
    import torch
    if isinstance(t, np.ndarray):
        if t.dtype == np.float64:
            return L.ITN_F64
        if t.dtype == np.float32:
            return L.ITN_F32
        raise TypeError("unsupported numpy dtype %s" % t.dtype)
    m = {torch.float64: L.ITN_F64, torch.float32: L.ITN_F32, torch.bfloat16: L.ITN_BF16}
    if t.dtype not in m:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return m[t.dtype]


class _Keep:
    """Holds ctypes buffers alive for the duration of a call."""

    def __init__(self):
        self.items = []

    def arr(self, ctype, values):
        a = (ctype * max(1, len(values)))(*values)
        self.items.append(a)
        return a


def _dense(keep: _Keep, t, labels: Optional[Sequence[int]] = None, shape=None) -> L.itn_tensor:
    """itn_tensor for a dense torch tensor (device) or numpy array (host)."""
    if isinstance(t, np.ndarray):
        if not t.flags.c_contiguous:
            raise ValueError("host arrays must be C-contiguous")
        ptr = t.ctypes.data
    else:
        if not t.is_contiguous():
            raise ValueError("device tensors must be contiguous")
        ptr = t.data_ptr()
    dims = list(shape if shape is not None else t.shape)
    tt = L.itn_tensor()
    tt.rank = len(dims)
    tt.dims = keep.arr(C.c_int64, dims)
    if labels is not None:
        tt.label = keep.arr(C.c_int32, list(labels))
    tt.dtype = _dtype_code(t)
    tt.data = C.c_void_p(ptr)
    tt.nblocks = 0
    return tt


# Library objects still alive at interpreter exit are freed by an atexit hook
# (registered when the first handle is created, so it runs before torch's own
# exit handlers and while the HIP runtime is still up): plans and MPS/MPO
# objects first, then the handles that own their device resources.  After
# that, and during interpreter finalisation, __del__ does nothing.
_live_objects: "weakref.WeakSet" = weakref.WeakSet()
_live_handles: "weakref.WeakSet" = weakref.WeakSet()
_exit_hook = False


def _close_all():
    for o in list(_live_objects):
        o.close()
    for h in list(_live_handles):
        h.close()


def _register(obj, handle: bool = False):
    global _exit_hook
    if not _exit_hook:
        atexit.register(_close_all)
        _exit_hook = True
    (_live_handles if handle else _live_objects).add(obj)


def _stream_ptr(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Handle:
    """An itn_handle on one device (device=-1: host-only, planning and
    validation only)."""

    def __init__(self, device: int = 0):
        self.lib = L.load()
        h = C.c_void_p()
        st = self.lib.itn_create(C.byref(h), int(device))
        if st != L.ITN_OK:
            raise ItnError(st, "itn_create(device=%d) failed" % device)
        self.h = h
        self.device = device
        _register(self, handle=True)

    def close(self):
        """Free the handle (its workspace, tables and solver state).  Objects
        made from it (plans, MPS, MPO) should be closed first."""
        if getattr(self, "h", None):
            self.lib.itn_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != L.ITN_OK:
            msg = self.lib.itn_last_error(self.h)
            raise ItnError(st, msg.decode() if msg else "")

    def _sp(self, stream):
        if self.device < 0:
            return C.c_void_p(None)
        return _stream_ptr(stream)

    def last_error(self) -> str:
        return self.lib.itn_last_error(self.h).decode()

    def sync(self, stream=None):
        self._check(self.lib.itn_sync(self.h, self._sp(stream)))

    def profile(self, on: bool = True):
        self._check(self.lib.itn_profile_enable(self.h, 1 if on else 0))

    def profile_report(self):
        """{kernel name: (total ms, launches)} since the last report."""
        mx = 64
        names = C.create_string_buffer(32 * mx)
        tot = (C.c_double * mx)()
        cnt = (C.c_int64 * mx)()
        n = C.c_int32()
        self._check(self.lib.itn_profile_report(self.h, mx, names, tot, cnt, C.byref(n)))
        out = {}
        for i in range(min(n.value, mx)):
            nm = names.raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (tot[i], cnt[i])
        return out

    # ---------------------------------------------------------------- calls
    def cast(self, src, dst, stream=None):
        k = _Keep()
        ts, td = _dense(k, src), _dense(k, dst)
        self._check(self.lib.itn_cast(self.h, C.byref(ts), C.byref(td), self._sp(stream)))
        return dst

    def contract(self, A, la, B, lb, Cout, lc, prec: str = "f64", stream=None):
        k = _Keep()
        ta, tb, tc = _dense(k, A, la), _dense(k, B, lb), _dense(k, Cout, lc)
        self._check(self.lib.itn_contract(self.h, C.byref(ta), C.byref(tb), C.byref(tc),
                                          PREC[prec], self._sp(stream)))
        return Cout

    def _check_vectors(self, psi, out, n1: int, nv: int):
        """psi and out must each hold exactly nv vectors of n1 elements, be
        contiguous tensors on this handle's device (any tensor on a host-only
        handle, which validates and then refuses the work), and not overlap
        (the library sees only their base pointers)."""
        if nv < 1:
            raise ValueError("nv must be >= 1")
        for name, t in (("psi", psi), ("out", out)):
            if isinstance(t, np.ndarray) or not hasattr(t, "data_ptr"):
                raise TypeError("%s must be a device tensor" % name)
            if self.device >= 0 and (t.device.type != "cuda" or (t.device.index or 0) != self.device):
                raise ValueError("%s must live on cuda:%d" % (name, self.device))
            if not t.is_contiguous():
                raise ValueError("%s must be contiguous" % name)
            if t.numel() != nv * n1:
                raise ValueError("%s holds %d elements, expected nv * chi_l*d*d*chi_r = %d"
                                 % (name, t.numel(), nv * n1))
        pa, pb = psi.data_ptr(), out.data_ptr()
        na, nb = psi.numel() * psi.element_size(), out.numel() * out.element_size()
        if pa < pb + nb and pb < pa + na:
            raise ValueError("out must not overlap psi")

    def heff_apply(self, Lenv, W1: np.ndarray, W2: np.ndarray, Renv, psi, out, nv: int = 1,
                   prec: str = "f64", stream=None):
        """psi/out: contiguous device tensors holding nv vectors
        [chi_l, d, d, chi_r] back to back (any leading shape)."""
        cl, cr = Lenv.shape[0], Renv.shape[0]
        d = W1.shape[2]
        shp = (cl, d, d, cr)
        self._check_vectors(psi, out, cl * d * d * cr, int(nv))
        k = _Keep()
        tl, tr = _dense(k, Lenv), _dense(k, Renv)
        W1c = np.ascontiguousarray(W1, np.float64)
        W2c = np.ascontiguousarray(W2, np.float64)
        k.items += [W1c, W2c]
        t1, t2 = _dense(k, W1c), _dense(k, W2c)
        tp, to = _dense(k, psi, shape=shp), _dense(k, out, shape=shp)
        self._check(self.lib.itn_heff_apply(self.h, C.byref(tl), C.byref(t1), C.byref(t2),
                                            C.byref(tr), C.byref(tp), int(nv), C.byref(to),
                                            PREC[prec], self._sp(stream)))
        return out

    def heff_apply_noalloc(self, Lenv, W1: np.ndarray, W2: np.ndarray, Renv, psi, out,
                           nv: int = 1, prec: str = "f64", stream=None):
        """heff_apply whose scratch is the library's fixed device array
        (itn_heff_apply_noalloc: no device allocation; calls overlapping on
        one device race)."""
        cl, cr = Lenv.shape[0], Renv.shape[0]
        d = W1.shape[2]
        shp = (cl, d, d, cr)
        self._check_vectors(psi, out, cl * d * d * cr, int(nv))
        k = _Keep()
        tl, tr = _dense(k, Lenv), _dense(k, Renv)
        W1c = np.ascontiguousarray(W1, np.float64)
        W2c = np.ascontiguousarray(W2, np.float64)
        k.items += [W1c, W2c]
        t1, t2 = _dense(k, W1c), _dense(k, W2c)
        tp, to = _dense(k, psi, shape=shp), _dense(k, out, shape=shp)
        self._check(self.lib.itn_heff_apply_noalloc(self.h, C.byref(tl), C.byref(t1), C.byref(t2),
                                                    C.byref(tr), C.byref(tp), int(nv), C.byref(to),
                                                    PREC[prec], self._sp(stream)))
        return out

    def heff_noalloc_max_bytes(self) -> int:
        b = C.c_size_t()
        self._check(self.lib.itn_heff_noalloc_max_bytes(C.byref(b)))
        return b.value

    def heff_apply_sum(self, terms, psi, out, nv: int = 1, prec: str = "f64", stream=None):
        """out = sum of H_eff,k psi over terms [(Lenv, W1, W2, Renv), ...]."""
        cl, cr = terms[0][0].shape[0], terms[0][3].shape[0]
        d = terms[0][1].shape[2]
        shp = (cl, d, d, cr)
        self._check_vectors(psi, out, cl * d * d * cr, int(nv))
        k = _Keep()
        n = len(terms)
        arrs = {x: (L.itn_tensor * n)() for x in "LABR"}
        for i, (Le, W1, W2, Re) in enumerate(terms):
            W1c = np.ascontiguousarray(W1, np.float64)
            W2c = np.ascontiguousarray(W2, np.float64)
            k.items += [W1c, W2c]
            arrs["L"][i], arrs["A"][i] = _dense(k, Le), _dense(k, W1c)
            arrs["B"][i], arrs["R"][i] = _dense(k, W2c), _dense(k, Re)
        ptrs = {x: (C.c_void_p * n)(*[C.addressof(arrs[x][i]) for i in range(n)]) for x in arrs}
        k.items += [arrs, ptrs]
        tp, to = _dense(k, psi, shape=shp), _dense(k, out, shape=shp)
        self._check(self.lib.itn_heff_apply_sum(self.h, n, ptrs["L"], ptrs["A"], ptrs["B"], ptrs["R"],
                                                C.byref(tp), int(nv), C.byref(to), PREC[prec],
                                                self._sp(stream)))
        return out

    def workspace_size(self, op: str, *args, nv: int = 1, direction: str = "left",
                       prec: str = "f64") -> int:
        """Workspace bytes one call would use (itn_workspace_size):
        op "contract": (A, la, B, lb, C, lc), dense tensors or QN descriptors;
        op "heff": (L, W1, W2, R, psi) with nv; op "env": (E, A, W, E_out)
        with direction.  Validates like the call (same errors)."""
        k = _Keep()
        if op == "contract":
            A, la, B, lb, Cc, lc = args
            ts = [_qn(k, dict(x, labels=list(l))) if isinstance(x, dict) else _dense(k, x, l)
                  for x, l in ((A, la), (B, lb), (Cc, lc))]
            code, dr = L.ITN_OP_CONTRACT, 0
        elif op == "heff":
            Lenv, W1, W2, Renv, psi = args
            cl, cr, d = Lenv.shape[0], Renv.shape[0], W1.shape[2]
            W1c = np.ascontiguousarray(W1, np.float64)
            W2c = np.ascontiguousarray(W2, np.float64)
            k.items += [W1c, W2c]
            ts = [_dense(k, Lenv), _dense(k, W1c), _dense(k, W2c), _dense(k, Renv),
                  _dense(k, psi, shape=(cl, d, d, cr))]
            code, dr = L.ITN_OP_HEFF, 0
        elif op == "env":
            E, A, W, out = args
            Wc = np.ascontiguousarray(W, np.float64)
            k.items.append(Wc)
            ts = [_dense(k, E), _dense(k, A), _dense(k, Wc), _dense(k, out)]
            code, dr = L.ITN_OP_ENV_UPDATE, (L.ITN_LEFT if direction == "left" else L.ITN_RIGHT)
        else:
            raise ValueError("op must be contract, heff or env")
        arr = (C.POINTER(L.itn_tensor) * len(ts))(*[C.pointer(t) for t in ts])
        b = C.c_size_t()
        self._check(self.lib.itn_workspace_size(self.h, code, len(ts), arr, int(nv), dr, PREC[prec],
                                                C.byref(b)))
        return b.value

    def set_workspace(self, buf=None):
        """Use a caller-owned device buffer (a torch tensor, 256-byte aligned)
        as the workspace; None returns to library-owned workspace.  The
        handle keeps a reference to the buffer while it is in use."""
        if buf is None:
            self._check(self.lib.itn_set_workspace(self.h, None, 0))
            self._ws_buf = None
            return
        nbytes = buf.numel() * buf.element_size()
        self._check(self.lib.itn_set_workspace(self.h, C.c_void_p(buf.data_ptr()), nbytes))
        self._ws_buf = buf

    def heff_workspace_size(self, chi_l, chi_r, d, w, nv=1, prec="f64") -> int:
        b = C.c_size_t()
        self._check(self.lib.itn_heff_workspace_size(self.h, chi_l, chi_r, d, w, nv, PREC[prec],
                                                     C.byref(b)))
        return b.value

    def env_update(self, E, A, W: np.ndarray, direction: str, out, prec: str = "f64",
                   stream=None):
        k = _Keep()
        Wc = np.ascontiguousarray(W, np.float64)
        k.items.append(Wc)
        te, ta, tw, to = _dense(k, E), _dense(k, A), _dense(k, Wc), _dense(k, out)
        dr = L.ITN_LEFT if direction == "left" else L.ITN_RIGHT
        self._check(self.lib.itn_env_update(self.h, C.byref(te), C.byref(ta), C.byref(tw), dr,
                                            C.byref(to), PREC[prec], self._sp(stream)))
        return out

    # ------------------------------------------------------------- sweeps
    def mpo(self, Ws):
        """Upload an MPO given as a list of N host arrays [w, w, d, d]."""
        W = np.ascontiguousarray(np.stack([np.asarray(x, np.float64) for x in Ws]))
        N, w, _, d, _ = W.shape
        out = C.c_void_p()
        self._check(self.lib.itn_mpo_create(self.h, N, w, d,
                                            W.ctypes.data_as(C.POINTER(C.c_double)),
                                            C.byref(out)))
        return _Owned(self, self.lib.itn_mpo_destroy, out, N=N, w=w, d=d)

    def mps(self, As):
        """Upload an MPS given as a list of N host arrays [bond_l, d, bond_r]
        (right-canonical, norm on site 0)."""
        N = len(As)
        d = As[0].shape[1]
        bond = [As[0].shape[0]] + [A.shape[2] for A in As]
        flat = np.ascontiguousarray(np.concatenate([np.asarray(A, np.float64).ravel() for A in As]))
        bd = (C.c_int32 * (N + 1))(*bond)
        out = C.c_void_p()
        self._check(self.lib.itn_mps_create(self.h, N, d, bd,
                                            flat.ctypes.data_as(C.POINTER(C.c_double)),
                                            C.byref(out)))
        return _Owned(self, self.lib.itn_mps_destroy, out, N=N, d=d)

    def mps_bonds(self, mps):
        b = (C.c_int32 * (mps.N + 1))()
        self._check(self.lib.itn_mps_bonds(mps.ptr, b))
        return list(b)

    def mps_sites(self, mps):
        bond = self.mps_bonds(mps)
        out = []
        for i in range(mps.N):
            a = np.zeros((bond[i], mps.d, bond[i + 1]))
            self._check(self.lib.itn_mps_get_site(self.h, mps.ptr, i,
                                                  a.ctypes.data_as(C.POINTER(C.c_double))))
            out.append(a)
        return out

    def _sweep_call(self, fn, sweeps, prec, mindim, krylovdim, maxiter, eig_tol, refine, energy_tol,
                    allow_unconverged, timing, ortho, weight, block):
        ns = len(sweeps)
        md = (C.c_int32 * max(1, ns))(*[int(m) for m, _ in sweeps])
        co = (C.c_double * max(1, ns))(*[float(c) for _, c in sweeps])
        prm = L.itn_sweep_params(ns, md, co, int(mindim), int(krylovdim), int(maxiter),
                                 float(eig_tol), PREC[prec], 1 if refine else 0, float(energy_tol),
                                 1 if timing else 0)
        optrs = (C.c_void_p * max(1, len(ortho)))(
            *[o.ptr.value if isinstance(o.ptr, C.c_void_p) else o.ptr for o in ortho])
        prm.northo = len(ortho)
        prm.ortho = C.cast(optrs, C.POINTER(C.c_void_p)) if ortho else None
        prm.weight = float(weight)
        prm.block = int(block)
        fields = [("energy", C.c_double), ("max_trunc", C.c_double), ("max_bond", C.c_int32),
                  ("seconds", C.c_double), ("matvecs", C.c_int64), ("residual", C.c_double),
                  ("matvecs_f64", C.c_int64)]
        if timing:
            fields += [(k, C.c_double) for k in ("t_matvec", "t_solver", "t_split", "t_env")]
        arrs = {k: (t * max(1, ns))() for k, t in fields}
        res = L.itn_sweep_result(0, *[arrs[k] for k, _ in fields[:6]])
        res.matvecs_f64 = arrs["matvecs_f64"]
        if timing:
            res.t_matvec, res.t_solver, res.t_split, res.t_env = (arrs[k] for k in
                                                                   ("t_matvec", "t_solver", "t_split", "t_env"))
        st = fn(C.byref(prm), C.byref(res))
        if not (allow_unconverged and st == 9):
            self._check(st)
        return [{k: arrs[k][i] for k in arrs} for i in range(res.sweeps_done)]

    def dmrg_sweep(self, mps, mpo, sweeps, prec="f64", mindim=1, krylovdim=8, maxiter=100,
                   eig_tol=1e-10, refine=True, energy_tol=0.0, allow_unconverged=False,
                   timing=False, ortho=(), weight=0.0, block=1):
        """Run a schedule [(maxdim, cutoff), ...]; returns per-sweep records
        (with per-phase seconds t_matvec/t_solver/t_split/t_env if timing).
        ortho: previously found MPS whose projectors, times `weight`, are
        added to H (excited states).  block: Davidson vectors per batched
        matvec."""
        return self._sweep_call(
            lambda prm, res: self.lib.itn_dmrg_sweep(self.h, mps.ptr, mpo.ptr, prm, res), sweeps, prec,
            mindim, krylovdim, maxiter, eig_tol, refine, energy_tol, allow_unconverged, timing, ortho,
            weight, block)

    # ------------------------------------------------- block-sparse sweeps
    def qn_mps(self, site_qn, state, mod=None):
        """Block-sparse MPS, the product state `state` (basis index per site);
        site_qn: QN tuple of each basis state."""
        sq = [tuple(int(x) for x in (q if isinstance(q, (tuple, list)) else (q,))) for q in site_qn]
        d, nq, N = len(sq), len(sq[0]), len(state)
        qarr = (C.c_int32 * (d * nq))(*[x for q in sq for x in q])
        marr = (C.c_int32 * nq)(*[int(m) for m in mod]) if mod else None
        st = (C.c_int32 * N)(*[int(s) for s in state])
        out = C.c_void_p()
        self._check(self.lib.itn_qn_mps_create(self.h, N, d, nq, qarr, marr, st, C.byref(out)))
        return _Owned(self, self.lib.itn_qn_mps_destroy, out, N=N, d=d, nq=nq)

    def qn_mps_bonds(self, mps):
        b = (C.c_int32 * (mps.N + 1))()
        self._check(self.lib.itn_qn_mps_bonds(mps.ptr, b))
        return list(b)

    def qn_mps_link(self, mps, k):
        """[(QN tuple, dim)] of link k."""
        n = C.c_int32(0)
        self._check(self.lib.itn_qn_mps_link(mps.ptr, int(k), C.byref(n), None, None))
        q = (C.c_int32 * max(1, n.value * mps.nq))()
        dm = (C.c_int32 * max(1, n.value))()
        self._check(self.lib.itn_qn_mps_link(mps.ptr, int(k), C.byref(n), q, dm))
        return [(tuple(q[s * mps.nq:(s + 1) * mps.nq]), dm[s]) for s in range(n.value)]

    def qn_mps_sites(self, mps):
        bond = self.qn_mps_bonds(mps)
        out = []
        for i in range(mps.N):
            a = np.zeros((bond[i], mps.d, bond[i + 1]))
            self._check(self.lib.itn_qn_mps_get_site(self.h, mps.ptr, i,
                                                     a.ctypes.data_as(C.POINTER(C.c_double))))
            out.append(a)
        return out

    def qn_dmrg_sweep(self, mps, mpo, link_qn, sweeps, prec="f64", mindim=1, krylovdim=8,
                      maxiter=100, eig_tol=1e-10, refine=True, energy_tol=0.0,
                      allow_unconverged=False, timing=False, block=1):
        """Two-site sweeps on a block-sparse MPS; link_qn: QN tuple of each MPO
        channel.  block: Davidson vectors per batched matvec."""
        lq = [tuple(int(x) for x in (q if isinstance(q, (tuple, list)) else (q,))) for q in link_qn]
        larr = (C.c_int32 * (len(lq) * len(lq[0])))(*[x for q in lq for x in q])
        return self._sweep_call(
            lambda prm, res: self.lib.itn_qn_dmrg_sweep(self.h, mps.ptr, mpo.ptr, larr, prm, res), sweeps,
            prec, mindim, krylovdim, maxiter, eig_tol, refine, energy_tol, allow_unconverged, timing, (),
            0.0, block)


def _qn(keep: _Keep, desc) -> L.itn_tensor:
    """itn_tensor for a QN tensor described as a dict:
      spaces : [(qns, dims, arrow), ...]  qns = list of QN tuples per sector
      blocks : [sector tuple, ...] sorted (absent for a dense host MPO tensor)
      offsets: [element offset per block]
      data   : device torch tensor (flat) / host numpy array / None (planning)
    """
    spaces = desc["spaces"]
    rank = len(spaces)
    sp = (L.itn_space * rank)()
    for i, spc in enumerate(spaces):
        qns, dims, arrow = spc[:3]
        mod = spc[3] if len(spc) > 3 else None
        qns = [tuple(int(x) for x in (q if isinstance(q, (tuple, list)) else (q,))) for q in qns]
        nq = len(qns[0])
        sp[i].nsec = len(dims)
        sp[i].nq = nq
        sp[i].qn = keep.arr(C.c_int32, [x for q in qns for x in q])
        sp[i].dim = keep.arr(C.c_int32, [int(x) for x in dims])
        sp[i].arrow = int(arrow)
        if mod:
            sp[i].mod = keep.arr(C.c_int32, [int(m) for m in mod])
    keep.items.append(sp)
    tt = L.itn_tensor()
    tt.rank = rank
    totals = [int(sum(spc[1])) for spc in spaces]
    tt.dims = keep.arr(C.c_int64, totals)
    tt.space = C.cast(sp, C.POINTER(L.itn_space))
    data = desc.get("data")
    if data is None:
        tt.dtype = desc.get("dtype", L.ITN_F64)
        tt.data = C.c_void_p(None)
    else:
        if isinstance(data, np.ndarray):
            data = np.ascontiguousarray(data)
            keep.items.append(data)
            tt.data = C.c_void_p(data.ctypes.data)
        else:
            tt.data = C.c_void_p(data.data_ptr())
        tt.dtype = _dtype_code(data)
    blocks = desc.get("blocks")
    if blocks is not None:
        tt.nblocks = len(blocks)
        tt.block_sec = keep.arr(C.c_int32, [int(x) for b in blocks for x in b])
        tt.block_off = keep.arr(C.c_int64, [int(x) for x in desc["offsets"]])
        nq = len(spaces[0][0][0]) if spaces and isinstance(spaces[0][0][0], (tuple, list)) else 1
        flux = desc.get("flux")
        tt.flux = keep.arr(C.c_int32, [int(x) for x in flux] if flux is not None else [0] * nq)
    labels = desc.get("labels")
    if labels is not None:
        tt.label = keep.arr(C.c_int32, [int(x) for x in labels])
    return tt


def _qn_handle_methods():
    def qn_plan(self, Ld, W1d, W2d, Rd, Pd, nv: int = 1, prec: str = "f64"):
        k = _Keep()
        ts = [_qn(k, x) for x in (Ld, W1d, W2d, Rd, Pd)]
        out = C.c_void_p()
        self._check(self.lib.itn_qn_heff_plan(self.h, *[C.byref(t) for t in ts], int(nv),
                                              PREC[prec], C.byref(out)))
        return Plan(self, out)

    def qn_heff_diag(self, Ld, W1d, W2d, Rd, Od, stream=None):
        """Diagonal of the block-sparse two-site H_eff into Od's data (psi's
        block layout, F64); descriptors as for qn_plan, L/R/out with data."""
        k = _Keep()
        ts = [_qn(k, x) for x in (Ld, W1d, W2d, Rd, Od)]
        self._check(self.lib.itn_qn_heff_diag(self.h, *[C.byref(t) for t in ts], self._sp(stream)))

    def contract_blocks(self, Ad, la, Bd, lb, Cd, lc, prec: str = "f64", stream=None):
        """Block-sparse C = A * B over labels (itn_contract with QN
        operands).  Ad, Bd, Cd: QN descriptors (spaces, blocks, offsets,
        flux, data); C's block list must hold every block a contributing
        pair reaches, its other blocks are zeroed."""
        k = _Keep()
        ts = [_qn(k, dict(d, labels=list(l))) for d, l in ((Ad, la), (Bd, lb), (Cd, lc))]
        self._check(self.lib.itn_contract(self.h, *[C.byref(t) for t in ts], PREC[prec],
                                          self._sp(stream)))
        return Cd

    def qn_allowed_blocks(self, spaces, flux=None):
        """(blocks, offsets, total) of the zero-flux (or `flux`) blocks."""
        k = _Keep()
        t = _qn(k, {"spaces": spaces})
        if flux is not None:
            t.flux = k.arr(C.c_int32, list(flux))
        n, tot = C.c_int64(0), C.c_int64(0)
        self._check(self.lib.itn_qn_allowed_blocks(self.h, C.byref(t), C.byref(n), None, None,
                                                   C.byref(tot)))
        sec = (C.c_int32 * max(1, n.value * len(spaces)))()
        off = (C.c_int64 * max(1, n.value))()
        self._check(self.lib.itn_qn_allowed_blocks(self.h, C.byref(t), C.byref(n), sec, off,
                                                   C.byref(tot)))
        r = len(spaces)
        return ([tuple(sec[b * r:(b + 1) * r]) for b in range(n.value)], list(off[:n.value]),
                tot.value)

    def qn_apply(self, plan, Ld, Rd, Pd, Od, stream=None):
        """H_eff*psi into Od.  Ld = Rd = None uses the environments of the
        plan's last prepare_env (or of its last apply that passed them)."""
        k = _Keep()
        refs = [None if x is None else C.byref(_qn(k, x)) for x in (Ld, Rd, Pd, Od)]
        self._check(self.lib.itn_qn_heff_apply(self.h, plan.ptr, *refs, self._sp(stream)))
    return qn_plan, qn_allowed_blocks, qn_apply, contract_blocks, qn_heff_diag


class Plan:
    """A QN H_eff plan (owned by the library)."""

    def __init__(self, handle, ptr):
        self.handle = handle
        self.lib = handle.lib
        self.ptr = ptr
        _register(self)

    def info(self):
        i = L.itn_plan_info()
        self.handle._check(self.lib.itn_plan_query(self.ptr, C.byref(i)))
        return {f: getattr(i, f) for f, _ in L.itn_plan_info._fields_}

    def out_blocks(self):
        n = self.info()["out_nblocks"]
        sec = (C.c_int32 * (4 * max(1, n)))()
        off = (C.c_int64 * max(1, n))()
        self.handle._check(self.lib.itn_plan_out_blocks(self.ptr, sec, off))
        return [tuple(sec[4 * b:4 * b + 4]) for b in range(n)], list(off[:n])

    def prepare_env(self, Ld, Rd, stream=None):
        """Repack the environments once for applies with Ld = Rd = None
        (the environments must stay unchanged while those run)."""
        k = _Keep()
        refs = [C.byref(_qn(k, x)) for x in (Ld, Rd)]
        self.handle._check(self.lib.itn_qn_prepare_env(self.handle.h, self.ptr, *refs,
                                                       self.handle._sp(stream)))
        self._env_keep = (k, Ld, Rd)

    def bind(self, Ld, Rd, Pd, Od, stream=None):
        """A callable applying the plan to these operands: the descriptors
        are marshalled once (the tensors' current storage is used on every
        call), so a loop of applies costs one library call each.  Ld = Rd =
        None binds to the prepared environments (prepare_env)."""
        k = _Keep()
        ts = [None if x is None else _qn(k, x) for x in (Ld, Rd, Pd, Od)]
        refs = [None if t is None else C.byref(t) for t in ts]
        sp = self.handle._sp(stream)
        lib, h, ptr, check = self.lib, self.handle.h, self.ptr, self.handle._check

        def apply():
            check(lib.itn_qn_heff_apply(h, ptr, *refs, sp))
        apply.keep = (k, ts, Ld, Rd, Pd, Od)
        return apply

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.itn_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass


(Handle.qn_plan, Handle.qn_allowed_blocks, Handle.qn_apply,
 Handle.contract_blocks, Handle.qn_heff_diag) = _qn_handle_methods()


class _Owned:
    """An opaque library object (MPS, MPO) freed with its destroy call; it
    keeps the handle it was made on alive."""

    def __init__(self, handle, destroy, ptr, **info):
        self.handle = handle
        self._destroy = destroy
        self.ptr = ptr
        for k, v in info.items():
            setattr(self, k, v)
        _register(self)

    def close(self):
        if getattr(self, "ptr", None):
            self._destroy(self.ptr)
            self.ptr = None

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass
