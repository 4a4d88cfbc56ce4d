"""Python binding of libdmrg: argument marshalling around the C ABI.

A superblock description is plain data (numpy arrays):

    {"S": {"q": int64[nsec], "dim": int[nsec]},  "E": {...},
     "q_target": int,
     "terms": [{"c": float, "A": op | None, "B": op | None, "group": int}, ...]}
    op = {"delta": int, "blocks": [(row_sec, col_sec, float64 2-D array), ...]}

Device vectors are torch float64 CUDA tensors of length D in the library's
psi layout.  Every computation runs in libdmrg; this module only converts
arguments and owns handles.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import PREC, check, lib


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """A libdmrg context on a CUDA (HIP) device, queueing on a torch stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        h = C.c_void_p()
        check(lib().dmrg_ctx_create(self.device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.handle = h

    def set_stream(self, stream):
        self._stream = stream
        check(lib().dmrg_ctx_set_stream(self.handle, C.c_void_p(stream.cuda_stream)))

    def set_mem_cap(self, nbytes):
        """dmrg_ctx_set_mem_cap: cap the device memory the library holds on
        this context's device (0: no cap)."""
        check(lib().dmrg_ctx_set_mem_cap(self.handle, int(nbytes)))

    def mem(self):
        """dmrg_ctx_mem: (bytes the library holds on the device, cap)."""
        u = C.c_int64()
        c = C.c_int64()
        check(lib().dmrg_ctx_mem(self.handle, C.byref(u), C.byref(c)))
        return u.value, c.value

    def set_timing(self, every=1):
        """Time every `every`-th product launch with HIP events (0 or False:
        off); all product launches are counted while it is on."""
        check(lib().dmrg_ctx_set_timing(self.handle, int(every)))

    def timing(self, prec, reset=True, products=False):
        """(summed event ms, timed launches) of the product kernels of one
        precision; with products=True also the number of all launches."""
        ms = C.c_double()
        n = C.c_int64()
        tot = C.c_int64()
        check(lib().dmrg_ctx_timing(self.handle, PREC[prec], C.byref(ms), C.byref(n), C.byref(tot),
                                    int(bool(reset))))
        if products:
            return ms.value, n.value, tot.value
        return ms.value, n.value

    def transform_blocks(self, blocks, O, W, out):
        """dmrg_transform_blocks: out_b = Wr_b^T O_b Wc_b for every block.

        ``blocks`` is a list of dicts with o_off, rows, cols, wr_off, kr,
        wc_off, kc, out_off (element offsets into the float64 CUDA tensors
        O, W, out)."""
        n = len(blocks)
        arr = (_lib.dmrg_tblock * max(1, n))()
        for i, b in enumerate(blocks):
            arr[i] = _lib.dmrg_tblock(int(b["o_off"]), int(b["rows"]), int(b["cols"]),
                                      int(b["wr_off"]), int(b["kr"]), int(b["wc_off"]),
                                      int(b["kc"]), int(b["out_off"]), int(b.get("o_ld", 0)),
                                      int(b.get("out_ld", 0)))
        check(lib().dmrg_transform_blocks(self.handle, n, arr, _ptr(O), _ptr(W), _ptr(out)))
        return out

    def close(self):
        if getattr(self, "handle", None) and _lib.alive():
            lib().dmrg_ctx_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Marshal:
    """Keeps the ctypes views of a description alive during a build call."""

    def __init__(self, sb):
        self.keep = []
        self.S = self._basis(sb["S"])
        self.E = self._basis(sb["E"])
        terms = sb["terms"]
        self.nterms = len(terms)
        arr = (_lib.dmrg_term * max(1, self.nterms))()
        for k, t in enumerate(terms):
            arr[k].c = float(t["c"])
            arr[k].group = int(t.get("group", 0))
            arr[k].A = self._op(t["A"])
            arr[k].B = self._op(t["B"])
        self.terms = arr

    def _basis(self, b):
        q = np.ascontiguousarray(b["q"], dtype=np.int64)
        d = np.ascontiguousarray(b["dim"], dtype=np.int32)
        self.keep += [q, d]
        return _lib.dmrg_basis(len(q), q.ctypes.data_as(C.POINTER(C.c_int64)),
                               d.ctypes.data_as(C.POINTER(C.c_int32)))

    def _op(self, op):
        if op is None:
            return C.POINTER(_lib.dmrg_op)()
        blocks = op["blocks"]
        n = len(blocks)
        rows = np.ascontiguousarray([b[0] for b in blocks], dtype=np.int32)
        cols = np.ascontiguousarray([b[1] for b in blocks], dtype=np.int32)
        data = [np.ascontiguousarray(b[2], dtype=np.float64) for b in blocks]
        ptrs = (C.POINTER(C.c_double) * max(1, n))(*[d.ctypes.data_as(C.POINTER(C.c_double)) for d in data])
        o = _lib.dmrg_op(int(op["delta"]), n, rows.ctypes.data_as(C.POINTER(C.c_int32)),
                         cols.ctypes.data_as(C.POINTER(C.c_int32)), ptrs)
        self.keep += [rows, cols, data, ptrs, o]
        return C.pointer(o)


class Superblock:
    """A superblock built in libdmrg (dmrg_build_superblock).

    ``ctx=None`` builds the host plan only (layout and statistics).
    """

    def __init__(self, desc, prec="fp32", ctx=None, q_in=None):
        """q_in: build the operator from the q_in sector to desc["q_target"]
        (dmrg_build_operator) instead of a Hamiltonian superblock."""
        self.ctx = ctx
        self.prec = prec
        self.nterms = len(desc["terms"])
        m = _Marshal(desc)
        h = C.c_void_p()
        dev = ctx.handle if ctx is not None else None
        if q_in is None:
            check(lib().dmrg_build_superblock(dev, C.byref(m.S), C.byref(m.E), int(desc["q_target"]),
                                              m.nterms, m.terms, PREC[prec], C.byref(h)))
        else:
            check(lib().dmrg_build_operator(dev, C.byref(m.S), C.byref(m.E), int(q_in),
                                            int(desc["q_target"]), m.nterms, m.terms, PREC[prec],
                                            C.byref(h)))
        self.handle = h
        di, do = C.c_int64(), C.c_int64()
        check(lib().dmrg_sb_dims(h, C.byref(di), C.byref(do)))
        self.D_in = int(di.value)
        self._dims = (np.asarray(desc["S"]["dim"]), np.asarray(desc["E"]["dim"]))
        D = C.c_int64()
        npairs = C.c_int32()
        off = C.POINTER(C.c_int64)()
        ss = C.POINTER(C.c_int32)()
        es = C.POINTER(C.c_int32)()
        check(lib().dmrg_sb_layout(h, C.byref(D), C.byref(npairs), C.byref(off), C.byref(ss),
                                   C.byref(es)))
        self.D = int(D.value)
        n = npairs.value
        self.offsets = np.array([off[i] for i in range(n)], dtype=np.int64)
        self.s_sec = np.array([ss[i] for i in range(n)], dtype=np.int32)
        self.e_sec = np.array([es[i] for i in range(n)], dtype=np.int32)

    # -- queries -------------------------------------------------------------
    def stats(self):
        fa, fe, ba = C.c_double(), C.c_double(), C.c_double()
        nt = C.c_int32()
        check(lib().dmrg_sb_stats(self.handle, C.byref(fa), C.byref(fe), C.byref(ba), C.byref(nt)))
        return dict(flops_alg=fa.value, flops_exec=fe.value, bytes_alg=ba.value, ntiles=nt.value)

    def set_coeffs(self, c):
        c = np.ascontiguousarray(c, dtype=np.float64)
        if c.shape != (self.nterms,):
            raise ValueError("need one coefficient per term")
        check(lib().dmrg_sb_set_coeffs(self.handle, c.ctypes.data_as(C.POINTER(C.c_double))))

    def autotune(self, reps=20):
        """dmrg_sb_autotune: time the fused kernel's variants for the current
        precision and keep the fastest; returns the chosen variant."""
        v = C.c_int32()
        check(lib().dmrg_sb_autotune(self.handle, int(reps), C.byref(v)))
        return v.value

    def set_variant(self, variant):
        """dmrg_sb_set_variant: pin the fused kernel's variant."""
        check(lib().dmrg_sb_set_variant(self.handle, int(variant)))

    def set_reorth(self, mode):
        """dmrg_sb_set_reorth: 0 = Gram-Schmidt pass on every other Lanczos
        step after the local recurrence (default), 1 = classical
        Gram-Schmidt twice at every step."""
        check(lib().dmrg_sb_set_reorth(self.handle, int(mode)))

    def set_graphs(self, enable):
        """dmrg_sb_set_graphs: replay the Lanczos steps between two host
        checks from captured HIP graphs (True) or launch them one by one."""
        check(lib().dmrg_sb_set_graphs(self.handle, int(bool(enable))))

    def graph_stats(self):
        """dmrg_sb_graph_stats: (captures, graph launches) so far."""
        c = C.c_int64()
        r = C.c_int64()
        check(lib().dmrg_sb_graph_stats(self.handle, C.byref(c), C.byref(r)))
        return c.value, r.value

    def set_prec(self, prec):
        check(lib().dmrg_sb_set_prec(self.handle, PREC[prec]))
        self.prec = prec

    # -- device work -----------------------------------------------------------
    def _vec(self, t, name, n=None):
        import torch
        n = self.D if n is None else n
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of length {n}")
        return t

    def lanczos_tridiag(self, v0, nsteps):
        """dmrg_lanczos_tridiag: (alpha, beta, ||v0||) of the recursion from v0."""
        self._vec(v0, "v0")
        a = np.zeros(nsteps)
        b = np.zeros(nsteps)
        steps = C.c_int32()
        nrm = C.c_double()
        check(lib().dmrg_lanczos_tridiag(self.handle, _ptr(v0), int(nsteps),
                                         a.ctypes.data_as(C.POINTER(C.c_double)),
                                         b.ctypes.data_as(C.POINTER(C.c_double)), C.byref(steps),
                                         C.byref(nrm)))
        k = steps.value
        return a[:k], b[:k], nrm.value

    def hpsi(self, psi, y=None, alpha=1.0, beta=0.0):
        import torch
        self._vec(psi, "psi", self.D_in)
        if y is None:
            y = torch.empty(self.D, dtype=psi.dtype, device=psi.device)
            beta = 0.0
        self._vec(y, "y")
        check(lib().dmrg_hpsi(self.handle, _ptr(psi), _ptr(y), float(alpha), float(beta)))
        return y

    def adjoint(self, psi, g, want_psi=True, want_c=True):
        import torch
        self._vec(psi, "psi")
        self._vec(g, "g")
        gpsi = torch.empty_like(psi) if want_psi else None
        gc = np.zeros(max(1, self.nterms)) if want_c else None
        check(lib().dmrg_hpsi_adjoint(self.handle, _ptr(psi), _ptr(g),
                                      _ptr(gpsi) if want_psi else None,
                                      gc.ctypes.data_as(C.POINTER(C.c_double)) if want_c else None))
        return gpsi, (gc[:self.nterms] if want_c else None)

    def lanczos(self, psi0, max_iter=300, tol=1e-10, out=None, raise_noconv=True):
        import torch
        self._vec(psi0, "psi0")
        if out is None:
            out = torch.empty_like(psi0)
        E = C.c_double()
        it = C.c_int32()
        res = C.c_double()
        st = lib().dmrg_lanczos_ground(self.handle, _ptr(psi0), int(max_iter), float(tol),
                                       C.byref(E), _ptr(out), C.byref(it), C.byref(res))
        if st != _lib.DMRG_OK and (raise_noconv or st != 6):
            check(st)
        return dict(energy=E.value, psi=out, iters=it.value, resid=res.value, converged=st == 0)

    def rho_truncate(self, psi, side, m, no_split=False):
        self._vec(psi, "psi")
        tr = _lib.dmrg_trunc()
        check(lib().dmrg_rho_truncate(self.handle, _ptr(psi), int(side), int(m), int(bool(no_split)),
                                      C.byref(tr)))
        kept = tr.kept

        def arr(ptr, n, dtype):   # copy of a library-owned array (ctypes indexing is slow)
            if n == 0:
                return np.zeros(0, dtype=dtype)
            return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)

        kps = arr(tr.kept_per_sec, tr.nsec, np.int64)
        # one copy of all kept vectors; each sector's block is a view into it
        wall = arr(tr.W_all, int(tr.W_total), np.float64)
        W = {}
        off = 0
        for s in np.flatnonzero(kps):
            k = int(kps[s])
            d = self._dim(side, int(s))
            W[int(s)] = wall[off:off + d * k].reshape(d, k)
            off += d * k
        return dict(eps=tr.trunc_err, kept=kept, straddle=bool(tr.straddle),
                    lam=arr(tr.lambda_, kept, np.float64),
                    lam_sec=arr(tr.lambda_sec, kept, np.int64),
                    kept_per_sec=kps, W=W)

    def _dim(self, side, s):
        return int(self._dims[side][s])

    def close(self):
        if getattr(self, "handle", None) and _lib.alive():
            lib().dmrg_sb_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_superblock(desc, prec="fp32", ctx=None):
    return Superblock(desc, prec=prec, ctx=ctx)


def ldos(alpha, beta, weight, e0, omega, eta):
    """dmrg_host_ldos: the Eq. (5) density of states on the grid omega."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    w = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.zeros(len(w))
    check(lib().dmrg_host_ldos(len(a), a.ctypes.data_as(C.POINTER(C.c_double)),
                               b.ctypes.data_as(C.POINTER(C.c_double)), float(weight), float(e0),
                               len(w), w.ctypes.data_as(C.POINTER(C.c_double)), float(eta),
                               out.ctypes.data_as(C.POINTER(C.c_double))))
    return out
