"""Python front end of libbse: torch tensors in, torch tensors out.

Only argument marshalling happens here.  Every step of the solve runs in the
HIP kernels behind the C ABI; torch provides device memory and the stream.
Matrices cross the boundary column-major, so a logical (rows x cols) matrix
is held in a contiguous torch tensor of shape (cols, rows) and passed by
pointer.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib

_P = ctypes.c_void_p


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def to_colmajor(M: torch.Tensor, device) -> torch.Tensor:
    """Column-major device copy of a logical matrix M: a contiguous tensor
    holding M^T row-major (same bytes as M column-major)."""
    return M.to(device).transpose(0, 1).contiguous()


def from_colmajor(buf: torch.Tensor) -> torch.Tensor:
    """Logical matrix from a column-major buffer created by to_colmajor."""
    return buf.transpose(0, 1)


class Context:
    """A bse_ctx bound to a CUDA/HIP device and the current torch stream."""

    def __init__(self, device: int | torch.device = 0, stream: torch.cuda.Stream | None = None,
                 arena: torch.Tensor | None = None, apply_tuning: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("libbse needs a GPU; none is visible")
        self.lib = _lib.load()
        self.device = torch.device("cuda", device if isinstance(device, int) else device.index or 0)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._arena = arena
        h = _P()
        arena_ptr = _ptr(arena)
        arena_bytes = 0 if arena is None else arena.numel() * arena.element_size()
        _lib.check(self.lib.bse_ctx_create(ctypes.byref(h), self.device.index, arena_ptr, arena_bytes,
                                           _P(self.stream.cuda_stream)), "bse_ctx_create")
        self.h = h
        if apply_tuning:
            self.apply_tuning()

    def apply_tuning(self, path: str | None = None) -> bool:
        """Apply the autotuner's tile table (tuning.json next to this file,
        written by paper_1501_03830_amd.autotune) if there is one."""
        import json
        import os
        path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
        if not os.path.exists(path):
            return False
        table = json.load(open(path))["table"]
        arr = (ctypes.c_int * 18)(*(list(table[0]) + list(table[1])))
        _lib.check(self.lib.bse_set_tile_table(self.h, arr), "bse_set_tile_table")
        return True

    def set_graphs(self, enable: bool):
        """Graph replay of the chain after the Cholesky (FP64 calls)."""
        _lib.check(self.lib.bse_ctx_set_graphs(self.h, 1 if enable else 0), "bse_ctx_set_graphs")

    def set_timing(self, enable: bool):
        """Per-launch hipEvent timing of the dominant skew matvec kernel."""
        _lib.check(self.lib.bse_ctx_set_timing(self.h, 1 if enable else 0), "bse_ctx_set_timing")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.bse_ctx_destroy(self.h)
            self.h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ solve
    def solve(self, A: torch.Tensor, B: torch.Tensor, d_r: torch.Tensor | None = None,
              d_l: torch.Tensor | None = None, vectors: bool = True, report: bool = False,
              prec: int = _lib.BSE_PREC_FP64, extra_flags: int = 0):
        """Full eigensolve.  A, B: complex128 (n, n) logical matrices (lower
        triangles used).  Returns dict with lam (n,), X (2n, n) or None,
        w (n,) or None, info, report."""
        n = A.shape[0]
        dev = self.device
        Ac = to_colmajor(A.to(torch.complex128), dev)
        Bc = to_colmajor(B.to(torch.complex128), dev)
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        flags = 0
        Xbuf = None
        w = None
        drb = dlb = None
        if vectors:
            flags |= _lib.BSE_WANT_VECTORS
            Xbuf = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
        if d_r is not None:
            flags |= _lib.BSE_WANT_WEIGHTS | _lib.BSE_WANT_VECTORS
            if Xbuf is None:
                Xbuf = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
            drb = d_r.to(dev, torch.complex128).contiguous()
            dlb = None if d_l is None else d_l.to(dev, torch.complex128).contiguous()
            w = torch.empty(n, dtype=torch.complex128, device=dev)
        flags |= extra_flags
        rep = _lib.BseReport() if report else None
        info = _lib.check(self.lib.bse_solve(
            self.h, n, _ptr(Ac), n, _ptr(Bc), n, prec, flags, _ptr(lam),
            _ptr(Xbuf), 2 * n, _ptr(drb), _ptr(dlb), _ptr(w),
            ctypes.byref(rep) if rep is not None else None), "bse_solve")
        return {
            "info": info,
            "lam": lam,
            "X": None if Xbuf is None else from_colmajor(Xbuf),
            "w": w,
            "report": rep.as_dict() if rep is not None else None,
        }

    def solve_real(self, A: torch.Tensor, B: torch.Tensor, d_r: torch.Tensor | None = None, vectors: bool = True,
                   report: bool = False, prec: int = _lib.BSE_PREC_FP64, extra_flags: int = 0):
        """Real problem (Algorithm 2): A, B real (n, n) (lower triangles
        used).  Returns dict with lam (n,), X real (2n, n) or None, w (n,)
        complex or None, info, report."""
        n = A.shape[0]
        dev = self.device
        Ac = to_colmajor(A.real.to(torch.float64), dev)
        Bc = to_colmajor(B.real.to(torch.float64), dev)
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        flags = 0
        Xbuf = w = drb = None
        if vectors or d_r is not None:
            flags |= _lib.BSE_WANT_VECTORS
            Xbuf = torch.empty((n, 2 * n), dtype=torch.float64, device=dev)
        if d_r is not None:
            flags |= _lib.BSE_WANT_WEIGHTS
            drb = d_r.to(dev, torch.complex128).contiguous()
            w = torch.empty(n, dtype=torch.complex128, device=dev)
        flags |= extra_flags
        rep = _lib.BseReport() if report else None
        info = _lib.check(self.lib.bse_solve_real(
            self.h, n, _ptr(Ac), n, _ptr(Bc), n, prec, flags, _ptr(lam), _ptr(Xbuf), 2 * n, _ptr(drb), None,
            _ptr(w), ctypes.byref(rep) if rep is not None else None), "bse_solve_real")
        return {"info": info, "lam": lam, "X": None if Xbuf is None else from_colmajor(Xbuf), "w": w,
                "report": rep.as_dict() if rep is not None else None}

    def solve_tda(self, A: torch.Tensor, d_r: torch.Tensor | None = None, vectors: bool = True,
                  report: bool = False, prec: int = _lib.BSE_PREC_FP64, extra_flags: int = 0):
        """Tamm-Dancoff solve (B = 0): eigenvalues of A ascending, x_j =
        [v_j; 0], TDA weights.  Same return layout as solve()."""
        n = A.shape[0]
        dev = self.device
        Ac = to_colmajor(A.to(torch.complex128), dev)
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        flags = 0
        Xbuf = w = drb = None
        if vectors or d_r is not None:
            flags |= _lib.BSE_WANT_VECTORS
            Xbuf = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
        if d_r is not None:
            flags |= _lib.BSE_WANT_WEIGHTS
            drb = d_r.to(dev, torch.complex128).contiguous()
            w = torch.empty(n, dtype=torch.complex128, device=dev)
        flags |= extra_flags
        rep = _lib.BseReport() if report else None
        info = _lib.check(self.lib.bse_solve_tda(
            self.h, n, _ptr(Ac), n, prec, flags, _ptr(lam), _ptr(Xbuf), 2 * n, _ptr(drb), None, _ptr(w),
            ctypes.byref(rep) if rep is not None else None), "bse_solve_tda")
        return {"info": info, "lam": lam, "X": None if Xbuf is None else from_colmajor(Xbuf), "w": w,
                "report": rep.as_dict() if rep is not None else None}

    def spectra(self, lam: torch.Tensor, w: torch.Tensor | None, omega0: float, domega: float, npts: int,
                sigma: float, dos: bool = True):
        """Broadened density of states and absorption spectrum on the grid
        omega0 + k domega (device tensors in, device tensors out)."""
        n = lam.shape[0]
        dev = self.device
        lam = lam.to(dev, torch.float64).contiguous()
        wc = None if w is None else w.to(dev, torch.complex128).contiguous()
        d = torch.empty(npts, dtype=torch.float64, device=dev) if dos else None
        e = torch.empty(npts, dtype=torch.complex128, device=dev) if wc is not None else None
        _lib.check(self.lib.bse_spectra(self.h, n, _ptr(lam), _ptr(wc), npts, omega0, domega, sigma,
                                        _ptr(d), _ptr(e)), "bse_spectra")
        return d, e

    def solve_noalloc(self, A: torch.Tensor, B: torch.Tensor, d_r: torch.Tensor | None = None,
                      vectors: bool = True, prec: int = _lib.BSE_PREC_FP64, extra_flags: int = 0):
        """bse_solve_noalloc: the solve on the library's fixed workspace array
        (no device or pinned allocation inside the call).  The tensors made
        here for inputs and outputs are the caller's side.  Returns dict with
        lam, X, w, info."""
        n = A.shape[0]
        dev = self.device
        Ac = to_colmajor(A.to(torch.complex128), dev)
        Bc = to_colmajor(B.to(torch.complex128), dev)
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        flags = 0
        Xbuf = w = drb = None
        if vectors or d_r is not None:
            flags |= _lib.BSE_WANT_VECTORS
            Xbuf = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev)
        if d_r is not None:
            flags |= _lib.BSE_WANT_WEIGHTS
            drb = d_r.to(dev, torch.complex128).contiguous()
            w = torch.empty(n, dtype=torch.complex128, device=dev)
        flags |= extra_flags
        torch.cuda.synchronize(dev)
        info = _lib.check(self.lib.bse_solve_noalloc(
            self.h, n, _ptr(Ac), n, _ptr(Bc), n, prec, flags, _ptr(lam),
            _ptr(Xbuf), 2 * n, _ptr(drb), None, _ptr(w)), "bse_solve_noalloc")
        return {"info": info, "lam": lam, "X": None if Xbuf is None else from_colmajor(Xbuf), "w": w}

    def solve_raw(self, n: int, Ac: torch.Tensor, Bc: torch.Tensor, lam: torch.Tensor,
                  Xbuf: torch.Tensor | None, drb: torch.Tensor | None = None, dlb: torch.Tensor | None = None,
                  w: torch.Tensor | None = None, report: bool = False, prec: int = _lib.BSE_PREC_FP64,
                  extra_flags: int = 0):
        """bse_solve on buffers that are already column-major on the device
        (as made by to_colmajor); nothing is copied.  Returns (info, report)."""
        flags = 0
        if Xbuf is not None:
            flags |= _lib.BSE_WANT_VECTORS
        if drb is not None:
            flags |= _lib.BSE_WANT_WEIGHTS
        flags |= extra_flags
        rep = _lib.BseReport() if report else None
        info = _lib.check(self.lib.bse_solve(
            self.h, n, _ptr(Ac), n, _ptr(Bc), n, prec, flags, _ptr(lam),
            _ptr(Xbuf), 2 * n, _ptr(drb), _ptr(dlb), _ptr(w),
            ctypes.byref(rep) if rep is not None else None), "bse_solve")
        return info, (rep.as_dict() if rep is not None else None)

    def solve_batched_raw(self, ns, Acs, Bcs, lams, Xbufs=None, ds=None, ws=None, report: bool = False,
                          prec: int = _lib.BSE_PREC_FP64, extra_flags: int = 0):
        """bse_solve_batched on column-major device buffers (as made by
        to_colmajor), one entry per problem; nothing is copied.  Returns
        (info list, report)."""
        count = len(ns)
        flags = extra_flags
        if Xbufs is not None:
            flags |= _lib.BSE_WANT_VECTORS
        if ds is not None:
            flags |= _lib.BSE_WANT_WEIGHTS
        IA = ctypes.c_int * count
        PA = _P * count
        n_arr = IA(*ns)
        A_arr = PA(*[t.data_ptr() for t in Acs])
        B_arr = PA(*[t.data_ptr() for t in Bcs])
        ld_arr = IA(*ns)
        lam_arr = PA(*[t.data_ptr() for t in lams])
        X_arr = PA(*[t.data_ptr() for t in Xbufs]) if Xbufs is not None else None
        ldx_arr = IA(*[2 * k for k in ns]) if Xbufs is not None else None
        d_arr = PA(*[t.data_ptr() for t in ds]) if ds is not None else None
        w_arr = PA(*[t.data_ptr() for t in ws]) if ws is not None else None
        info = IA()
        rep = _lib.BseReport() if report else None
        _lib.check(self.lib.bse_solve_batched(
            self.h, count, n_arr, A_arr, ld_arr, B_arr, ld_arr, prec, flags, lam_arr,
            X_arr, ldx_arr, d_arr, w_arr, info, ctypes.byref(rep) if rep is not None else None),
            "bse_solve_batched")
        return list(info), (rep.as_dict() if rep is not None else None)

    def solve_batched(self, As, Bs, ds=None, vectors: bool = True, report: bool = False,
                      prec: int = _lib.BSE_PREC_FP64, extra_flags: int = 0):
        """Batched eigensolve of independent problems (lists of complex128
        (n_i, n_i) logical matrices; ds: optional list of complex 2n_i dipole
        vectors used as d_r = d_l).  Returns a list of per-problem dicts like
        solve() and the batch report."""
        dev = self.device
        ns = [int(A.shape[0]) for A in As]
        Acs = [to_colmajor(A.to(torch.complex128), dev) for A in As]
        Bcs = [to_colmajor(B.to(torch.complex128), dev) for B in Bs]
        lams = [torch.empty(k, dtype=torch.float64, device=dev) for k in ns]
        want_x = vectors or ds is not None
        Xbufs = [torch.empty((k, 2 * k), dtype=torch.complex128, device=dev) for k in ns] if want_x else None
        dbs = [d.to(dev, torch.complex128).contiguous() for d in ds] if ds is not None else None
        ws = [torch.empty(k, dtype=torch.complex128, device=dev) for k in ns] if ds is not None else None
        info, rep = self.solve_batched_raw(ns, Acs, Bcs, lams, Xbufs, dbs, ws, report, prec, extra_flags)
        out = []
        for i in range(len(ns)):
            out.append({
                "info": info[i],
                "lam": lams[i],
                "X": None if Xbufs is None else from_colmajor(Xbufs[i]),
                "w": None if ws is None else ws[i],
            })
        return out, rep

    # ---------------------------------------------------------------- serving
    def serve_config(self, pool_bytes: int = 0, slots: int = 0, max_batch: int = 0):
        """Configure the request server before the first submit."""
        _lib.check(self.lib.bse_serve_config(self.h, pool_bytes, slots, max_batch), "bse_serve_config")

    def submit_raw(self, n: int, Ac: torch.Tensor, Bc: torch.Tensor, lam: torch.Tensor,
                   Xbuf: torch.Tensor | None = None, drb: torch.Tensor | None = None,
                   dlb: torch.Tensor | None = None, w: torch.Tensor | None = None,
                   prec: int = _lib.BSE_PREC_FP64) -> int:
        """bse_submit on column-major device buffers; returns the ticket.  The
        buffers are kept referenced here until the ticket is released."""
        flags = 0
        if Xbuf is not None:
            flags |= _lib.BSE_WANT_VECTORS
        if drb is not None:
            flags |= _lib.BSE_WANT_WEIGHTS
        req = _lib.BseRequest(n, Ac.data_ptr(), n, Bc.data_ptr(), n, prec, flags, lam.data_ptr(),
                              None if Xbuf is None else Xbuf.data_ptr(), 2 * n,
                              None if drb is None else drb.data_ptr(), None if dlb is None else dlb.data_ptr(),
                              None if w is None else w.data_ptr())
        t = ctypes.c_uint64()
        _lib.check(self.lib.bse_submit(self.h, ctypes.byref(req), ctypes.byref(t)), "bse_submit")
        if not hasattr(self, "_keep"):
            self._keep = {}
        self._keep[t.value] = (Ac, Bc, lam, Xbuf, drb, dlb, w)
        return t.value

    def submit(self, A: torch.Tensor, B: torch.Tensor, d_r: torch.Tensor | None = None, vectors: bool = True,
               prec: int = _lib.BSE_PREC_FP64):
        """Queue a solve of logical complex matrices; returns (ticket, outputs)
        where outputs = {lam, X, w} are filled once the ticket is done."""
        n = A.shape[0]
        dev = self.device
        Ac = to_colmajor(A.to(torch.complex128), dev)
        Bc = to_colmajor(B.to(torch.complex128), dev)
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        want_x = vectors or d_r is not None
        Xbuf = torch.empty((n, 2 * n), dtype=torch.complex128, device=dev) if want_x else None
        drb = d_r.to(dev, torch.complex128).contiguous() if d_r is not None else None
        w = torch.empty(n, dtype=torch.complex128, device=dev) if d_r is not None else None
        t = self.submit_raw(n, Ac, Bc, lam, Xbuf, drb, None, w, prec=prec)
        return t, {"lam": lam, "X": None if Xbuf is None else from_colmajor(Xbuf), "w": w}

    def poll(self, ticket: int):
        """(state, info) of a ticket; raises for unknown tickets."""
        st, info = ctypes.c_int(), ctypes.c_int()
        _lib.check(self.lib.bse_poll(self.h, ticket, ctypes.byref(st), ctypes.byref(info)), "bse_poll")
        return st.value, info.value

    def release(self, ticket: int) -> int:
        """bse_release; returns its code (0, or BSE_EBUSY while running)."""
        rc = self.lib.bse_release(self.h, ticket)
        if rc == 0 and getattr(self, "_keep", None) is not None:
            self._keep.pop(ticket, None)
        elif rc not in (0, _lib.BSE_EBUSY):
            _lib.check(rc, "bse_release")
        return rc

    def ticket_times(self, ticket: int):
        """(submit, start, done) server timestamps in microseconds."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(self.lib.bse_ticket_times(self.h, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                   "bse_ticket_times")
        return a.value, b.value, c.value

    def serve_stats(self) -> dict:
        st = _lib.BseServeCounters()
        _lib.check(self.lib.bse_serve_stats(self.h, ctypes.byref(st)), "bse_serve_stats")
        return st.as_dict()

    # ----------------------------------------------------------------- stages
    def build_M(self, A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
        n = A.shape[0]
        Ac = to_colmajor(A.to(torch.complex128), self.device)
        Bc = to_colmajor(B.to(torch.complex128), self.device)
        Mb = torch.empty((2 * n, 2 * n), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.bse_build_M(self.h, n, _ptr(Ac), n, _ptr(Bc), n, _ptr(Mb), 2 * n), "bse_build_M")
        return from_colmajor(Mb)

    def potrf(self, M: torch.Tensor):
        N = M.shape[0]
        Mb = to_colmajor(M.to(torch.float64), self.device)
        info = _lib.check(self.lib.bse_potrf(self.h, N, _ptr(Mb), N), "bse_potrf")
        return from_colmajor(Mb), info

    def form_W(self, L: torch.Tensor) -> torch.Tensor:
        N = L.shape[0]
        Lb = to_colmajor(L.to(torch.float64), self.device)
        Wb = torch.empty((N, N), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.bse_form_W(self.h, N, _ptr(Lb), N, _ptr(Wb), N), "bse_form_W")
        return from_colmajor(Wb)

    def sktrd(self, W: torch.Tensor):
        N = W.shape[0]
        Wb = to_colmajor(W.to(torch.float64), self.device)
        alpha = torch.empty(N - 1, dtype=torch.float64, device=self.device)
        tau = torch.empty(N - 1, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.bse_sktrd(self.h, N, _ptr(Wb), N, _ptr(alpha), _ptr(tau)), "bse_sktrd")
        return from_colmajor(Wb), alpha, tau

    def sktrd2(self, W: torch.Tensor):
        """Two-stage reduction of a full skew W; returns alpha (N-1,)."""
        N = W.shape[0]
        Wb = to_colmajor(W.to(torch.float64), self.device)
        alpha = torch.empty(N - 1, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.bse_sktrd2(self.h, N, _ptr(Wb), N, _ptr(alpha)), "bse_sktrd2")
        return alpha

    def tridiag_eig(self, alpha: torch.Tensor, vectors: bool = True, flags: int = 0):
        N = alpha.shape[0] + 1
        a = alpha.to(self.device, torch.float64).contiguous()
        lam = torch.empty(N // 2, dtype=torch.float64, device=self.device)
        Vb = torch.empty((N // 2, N), dtype=torch.float64, device=self.device) if vectors else None
        _lib.check(self.lib.bse_tridiag_eig_flags(self.h, N, _ptr(a), _ptr(lam), _ptr(Vb), N, flags),
                   "bse_tridiag_eig_flags")
        return lam, (None if Vb is None else from_colmajor(Vb))


def footprint_bytes(n: int, prec: int = _lib.BSE_PREC_FP64, flags: int = 0) -> int:
    """Device workspace of one bse_solve of order n."""
    return int(_lib.load().bse_footprint_bytes(n, prec, flags))


def footprint_batched_bytes(ns, prec: int = _lib.BSE_PREC_FP64, flags: int = 0) -> int:
    arr = (ctypes.c_int * len(ns))(*ns)
    return int(_lib.load().bse_footprint_batched_bytes(len(ns), arr, prec, flags))
