"""Python binding of ``libhsrq.so`` (batched robust shifted Hessenberg solves).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the library.  PyTorch provides device memory and the stream.  The raw C-ABI
functions are available under their C names (``hsrq_create``, ``hsrq_dhsrq3``,
...); ``Solver`` wraps them for torch tensors.

There is no CPU fallback: importing works without a GPU (so that the library
can be inspected), but any solve raises if the library or a GPU is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsrq.so")

HSRQ_OK = 0
INFO_OK, INFO_NOT_CONVERGED, INFO_SINGULAR, INFO_NONFINITE, INFO_REDUCED = 0, 1, 2, 3, 4

EXPORTED = [
    "hsrq_create", "hsrq_destroy", "hsrq_set_stream", "hsrq_workspace_size", "hsrq_dhsrq3",
    "hsrq_workspace_size_batched", "hsrq_dhsrq3_batched", "hsrq_debug_view",
    "hsrq_profile_enable", "hsrq_profile_read", "hsrq_autotune", "hsrq_fallback_count",
    "hsrq_server_create", "hsrq_server_submit", "hsrq_server_poll", "hsrq_server_clock", "hsrq_server_destroy",
    "hsrq_dhsrq3_noalloc", "hsrq_hsrq3in_workspace_size", "hsrq_hsrq3in",
    "hsrq_autotune_save", "hsrq_autotune_load",
    "hsrq_gehrd_workspace_size", "hsrq_gehrd", "hsrq_ormhr_workspace_size", "hsrq_ormhr",
]
HSRQ_ERR_TOO_LARGE = -1006
NOALLOC_SCRATCH_BYTES = 64 << 20
KERNEL_KINDS = ["prep", "init", "crit", "far", "final", "output", "resid"]


class HsrqOpts(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("cols_per_block", ctypes.c_int), ("precision", ctypes.c_int),
                ("residual", ctypes.c_int), ("graph", ctypes.c_int), ("rotations", ctypes.c_int),
                ("share_min_far", ctypes.c_int), ("reserved", ctypes.c_int)]


class HsrqCompletion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("fallback", ctypes.c_int),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class HsrqProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("H", ctypes.c_void_p), ("ldh", ctypes.c_int), ("m", ctypes.c_int),
                ("wr", ctypes.c_void_p), ("wi", ctypes.c_void_p), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int),
                ("scale_exp", ctypes.c_void_p), ("scale_mant", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("resid", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhsrq.so and declare the C signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER
    lib.hsrq_create.argtypes = [P(vp), i]
    lib.hsrq_destroy.argtypes = [vp]
    lib.hsrq_set_stream.argtypes = [vp, vp]
    lib.hsrq_workspace_size.argtypes = [vp, i, i, vp, P(HsrqOpts), P(sz)]
    lib.hsrq_dhsrq3.argtypes = [vp, i, vp, i, i, vp, vp, vp, i, vp, vp, vp, vp, vp, sz, P(HsrqOpts)]
    lib.hsrq_workspace_size_batched.argtypes = [vp, i, P(HsrqProblem), P(HsrqOpts), P(sz)]
    lib.hsrq_dhsrq3_batched.argtypes = [vp, i, P(HsrqProblem), vp, sz, P(HsrqOpts)]
    lib.hsrq_debug_view.argtypes = [vp, i, i, vp, P(HsrqOpts), vp, P(vp), P(vp), P(vp), P(vp), P(i), P(i), vp]
    lib.hsrq_profile_enable.argtypes = [vp, i]
    lib.hsrq_profile_read.argtypes = [vp, i, vp, vp]
    lib.hsrq_autotune.argtypes = [vp, i, P(HsrqProblem), vp, sz, P(HsrqOpts), P(i), P(i), vp]
    lib.hsrq_fallback_count.argtypes = [vp, P(ctypes.c_int64)]
    lib.hsrq_server_create.argtypes = [P(vp), i, sz, P(HsrqOpts)]
    lib.hsrq_server_submit.argtypes = [vp, P(HsrqProblem), ctypes.c_uint64, vp]
    lib.hsrq_server_poll.argtypes = [vp, P(HsrqCompletion), i, P(i), i]
    lib.hsrq_server_clock.argtypes = [vp, P(ctypes.c_double)]
    lib.hsrq_server_destroy.argtypes = [vp]
    lib.hsrq_dhsrq3_noalloc.argtypes = [vp, i, vp, i, i, vp, vp, vp, i, vp, vp, vp, vp, P(HsrqOpts)]
    lib.hsrq_gehrd_workspace_size.argtypes = [vp, i, P(sz)]
    lib.hsrq_gehrd.argtypes = [vp, i, vp, i, vp, vp, sz]
    lib.hsrq_ormhr_workspace_size.argtypes = [vp, i, i, P(sz)]
    lib.hsrq_ormhr.argtypes = [vp, i, vp, i, vp, i, vp, i, vp, sz]
    lib.hsrq_autotune_save.argtypes = [vp, ctypes.c_char_p]
    lib.hsrq_autotune_load.argtypes = [vp, ctypes.c_char_p]
    lib.hsrq_hsrq3in_workspace_size.argtypes = [vp, i, i, vp, P(HsrqOpts), P(sz)]
    lib.hsrq_hsrq3in.argtypes = [vp, i, vp, i, i, vp, vp, vp, i, i, vp, i, vp, vp, vp, vp, vp, vp, sz,
                                 P(HsrqOpts)]
    for f in EXPORTED:
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def __getattr__(name):
    if name in EXPORTED:
        return getattr(load_library(), name)
    raise AttributeError(name)


def _check(st, what):
    if st != HSRQ_OK:
        raise RuntimeError(f"{what} failed with status {st}")


def _opts(nb=0, precision=0, residual=False, graph=0, rotations=0, share_min_far=0, cols_per_block=0):
    o = HsrqOpts()
    o.nb = int(nb or 0)
    o.cols_per_block = int(cols_per_block)
    o.precision = int(precision)
    o.residual = 1 if residual else 0
    o.graph = int(graph)
    o.rotations = int(rotations)
    o.share_min_far = int(share_min_far)
    return o


def ncols_of(wi) -> int:
    wi = np.asarray(wi)
    return int(np.sum(np.where(wi != 0.0, 2, 1)))


def colmajor(t):
    """A column-major view/copy of a 2-D torch tensor: returns (tensor, ld)."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    r, c = t.shape
    if (t.stride(0) == 1 or r == 1) and (t.stride(1) >= max(1, r) or c == 1):
        return t, max(1, r) if c == 1 else t.stride(1)
    tc = t.t().contiguous().t()
    return tc, max(1, r)


class Batch:
    """A problem set marshalled for hsrq_dhsrq3_batched (see Solver.prepare):
    the descriptor array, the arrays it points to, and the per-problem output
    views (E, mu, info, resid), which every call with this Batch overwrites."""

    def __init__(self, arr, keep, outs, count, residual):
        self.arr, self.keep, self.outs, self.count, self.residual = arr, keep, outs, count, residual
        self.need = {}

    def set_x(self, xs):
        """New starting-vector arrays (same shapes and layout as before)."""
        if len(xs) != self.count:
            raise ValueError("one X per problem")
        for p, X in enumerate(xs):
            a = self.arr[p]
            ld = X.stride(1) if X.shape[1] > 1 else a.n
            if X.shape[0] != a.n or ld != a.ldx:
                raise ValueError(f"X of problem {p} does not match the prepared layout")
            a.X = X.data_ptr()
        self.xs = list(xs)


class Solver:
    """Handle + workspace management on one device, for torch tensors."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP library has no CPU fallback")
        self.torch = torch
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        _check(self.lib.hsrq_create(ctypes.byref(h), device), "hsrq_create")
        self.h = h
        self._ws = None

    def close(self):
        if self.h:
            self.lib.hsrq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, stream=None):
        s = stream if stream is not None else self.torch.cuda.current_stream(self.device)
        _check(self.lib.hsrq_set_stream(self.h, ctypes.c_void_p(s.cuda_stream)), "hsrq_set_stream")

    def workspace(self, nbytes):
        torch = self.torch
        if self._ws is None or self._ws.numel() < nbytes + 256:
            self._ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        return aligned, self._ws.numel() - (aligned - base)

    def workspace_size(self, n, wi, nb=0, precision=0, rotations=0):
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        o = _opts(nb, precision, rotations=rotations)
        out = ctypes.c_size_t()
        _check(self.lib.hsrq_workspace_size(self.h, n, wi.shape[0], wi.ctypes.data_as(ctypes.c_void_p),
                                            ctypes.byref(o), ctypes.byref(out)), "hsrq_workspace_size")
        return out.value

    def dhsrq3(self, H, wr, wi, X, nb=0, precision=0, residual=False, graph=0, stream=None, rotations=0,
               share_min_far=0, cols_per_block=0):
        """Solve in place: X (device, n x ncols) holds the starting vectors and
        receives the unit vectors.  Returns (scale_exp, scale_mant, info,
        resid) device tensors of length m.  rotations=1 applies the
        off-diagonal rotations of a tile column as one product on the matrix
        cores (default 0: one at a time, bit-identical to Alg. 1's order).
        share_min_far, cols_per_block: see hsrq_opts_t (0 = library default)."""
        torch = self.torch
        n = H.shape[0]
        wr = np.ascontiguousarray(wr, dtype=np.float64)
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        m = wr.shape[0]
        Hc, ldh = colmajor(H)
        if X.shape[0] > 1 and X.stride(0) != 1:
            raise ValueError("X must be column-major (X.stride(0) == 1), e.g. B.t().contiguous().t()")
        ldx = X.stride(1) if X.shape[1] > 1 else n
        ldx = max(ldx, n)
        dev = H.device
        E = torch.empty(m, dtype=torch.int32, device=dev)
        mu = torch.empty(m, dtype=torch.float64, device=dev)
        info = torch.empty(m, dtype=torch.int32, device=dev)
        res = torch.empty(m, dtype=torch.float64, device=dev) if residual else None
        o = _opts(nb, precision, residual, graph, rotations, share_min_far, cols_per_block)
        need = self.workspace_size(n, wi, nb, precision, rotations)
        wp, wb = self.workspace(need)
        self._stream(stream)
        st = self.lib.hsrq_dhsrq3(self.h, n, Hc.data_ptr(), ldh, m, wr.ctypes.data_as(ctypes.c_void_p),
                                  wi.ctypes.data_as(ctypes.c_void_p), X.data_ptr(), ldx, E.data_ptr(),
                                  mu.data_ptr(), info.data_ptr(), res.data_ptr() if res is not None else None,
                                  ctypes.c_void_p(wp), wb, ctypes.byref(o))
        _check(st, "hsrq_dhsrq3")
        self._keep = (Hc,)  # keep a temporary column-major copy alive until the stream runs
        return E, mu, info, res

    def dhsrq3_noalloc(self, H, wr, wi, X, nb=0, residual=False, stream=None, rotations=0, share_min_far=0):
        """As dhsrq3 (precision 0, kernel by kernel) with the library's fixed
        device scratch array as the workspace: the library allocates nothing.
        Returns (status, scale_exp, scale_mant, info, resid); status is
        HSRQ_ERR_TOO_LARGE when the problem does not fit the array.  Calls on
        one device must not overlap (they share the array)."""
        torch = self.torch
        n = H.shape[0]
        wr = np.ascontiguousarray(wr, dtype=np.float64)
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        m = wr.shape[0]
        Hc, ldh = colmajor(H)
        if X.shape[0] > 1 and X.stride(0) != 1:
            raise ValueError("X must be column-major (X.stride(0) == 1)")
        ldx = max(X.stride(1) if X.shape[1] > 1 else n, n)
        dev = H.device
        E = torch.empty(m, dtype=torch.int32, device=dev)
        mu = torch.empty(m, dtype=torch.float64, device=dev)
        info = torch.empty(m, dtype=torch.int32, device=dev)
        res = torch.empty(m, dtype=torch.float64, device=dev) if residual else None
        o = _opts(nb, 0, residual, -1, rotations, share_min_far)
        self._stream(stream)
        st = self.lib.hsrq_dhsrq3_noalloc(self.h, n, Hc.data_ptr(), ldh, m, wr.ctypes.data_as(ctypes.c_void_p),
                                          wi.ctypes.data_as(ctypes.c_void_p), X.data_ptr(), ldx, E.data_ptr(),
                                          mu.data_ptr(), info.data_ptr(),
                                          res.data_ptr() if res is not None else None, ctypes.byref(o))
        self._keep = (Hc,)
        return st, E, mu, info, res

    def hsrq3in(self, H, wr, wi, S, nb=0, residual=False, stream=None, rotations=0, work_bytes=None):
        """Inverse iteration with restarts (hsrq_hsrq3in): S (device, n x
        ntries, column-major) holds the starting vectors of the successive
        tries.  Returns (X, scale_exp, scale_mant, info, tries, resid) with X
        column-major in the caller's column layout.  work_bytes bounds the
        workspace (the library then solves the shifts in groups); default:
        enough for one group."""
        torch = self.torch
        n = H.shape[0]
        wr = np.ascontiguousarray(wr, dtype=np.float64)
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        m = wr.shape[0]
        Hc, ldh = colmajor(H)
        Sc, lds = colmajor(S)
        dev = H.device
        X = torch.empty((ncols_of(wi), n), dtype=torch.float64, device=dev).t()
        E = torch.empty(m, dtype=torch.int32, device=dev)
        mu = torch.empty(m, dtype=torch.float64, device=dev)
        info = torch.empty(m, dtype=torch.int32, device=dev)
        tries = torch.empty(m, dtype=torch.int32, device=dev)
        res = torch.empty(m, dtype=torch.float64, device=dev) if residual else None
        o = _opts(nb, 0, residual, 0, rotations)
        if work_bytes is None:
            need = ctypes.c_size_t()
            _check(self.lib.hsrq_hsrq3in_workspace_size(self.h, n, m, wi.ctypes.data_as(ctypes.c_void_p),
                                                        ctypes.byref(o), ctypes.byref(need)),
                   "hsrq_hsrq3in_workspace_size")
            work_bytes = need.value
        wp, wb = self.workspace(work_bytes)
        self._stream(stream)
        _check(self.lib.hsrq_hsrq3in(self.h, n, Hc.data_ptr(), ldh, m, wr.ctypes.data_as(ctypes.c_void_p),
                                     wi.ctypes.data_as(ctypes.c_void_p), Sc.data_ptr(), lds, Sc.shape[1],
                                     X.data_ptr(), n, E.data_ptr(), mu.data_ptr(), info.data_ptr(),
                                     tries.data_ptr(), res.data_ptr() if res is not None else None,
                                     ctypes.c_void_p(wp), min(wb, int(work_bytes)), ctypes.byref(o)),
               "hsrq_hsrq3in")
        self._keep = (Hc, Sc)
        return X, E, mu, info, tries, res

    def solve(self, H, wr, wi, B, **kw):
        """Out-of-place: returns (Y, E, mu, info, resid) with Y column-major."""
        Y = B.t().contiguous().t().clone()
        E, mu, info, res = self.dhsrq3(H, wr, wi, Y, **kw)
        return Y, E, mu, info, res

    def _problem_array(self, problems, residual):
        torch = self.torch
        count = len(problems)
        arr = (HsrqProblem * max(count, 1))()
        keep = []
        ms = [int(np.asarray(pr["wr"]).shape[0]) for pr in problems]
        sizes = [max(m, 1) for m in ms]
        tot = max(sum(sizes), 1)
        dev = problems[0]["H"].device if count else torch.device("cuda", self.device)
        # one allocation per output kind, split into per-problem views
        E_all = torch.empty(tot, dtype=torch.int32, device=dev)
        mu_all = torch.empty(tot, dtype=torch.float64, device=dev)
        info_all = torch.empty(tot, dtype=torch.int32, device=dev)
        res_all = torch.empty(tot, dtype=torch.float64, device=dev) if residual else None
        keep += [E_all, mu_all, info_all, res_all]
        Es = torch.split(E_all, sizes) if count else ()
        mus = torch.split(mu_all, sizes) if count else ()
        infos = torch.split(info_all, sizes) if count else ()
        ress = torch.split(res_all, sizes) if (count and residual) else [None] * count
        outs = []
        off = 0
        for p, pr in enumerate(problems):
            Hc, ldh = colmajor(pr["H"])
            wr = np.ascontiguousarray(pr["wr"], dtype=np.float64)
            wi = np.ascontiguousarray(pr["wi"], dtype=np.float64)
            X = pr["X"]
            m = ms[p]
            keep += [Hc, wr, wi]
            res = ress[p]
            outs.append((Es[p][:m], mus[p][:m], infos[p][:m], res[:m] if res is not None else None))
            a = arr[p]
            a.n, a.H, a.ldh, a.m = Hc.shape[0], Hc.data_ptr(), ldh, m
            a.wr, a.wi = wr.ctypes.data, wi.ctypes.data
            a.X, a.ldx = X.data_ptr(), (X.stride(1) if X.shape[1] > 1 else Hc.shape[0])
            a.scale_exp = E_all.data_ptr() + 4 * off
            a.scale_mant = mu_all.data_ptr() + 8 * off
            a.info = info_all.data_ptr() + 4 * off
            a.resid = res_all.data_ptr() + 8 * off if residual else None
            off += sizes[p]
        return arr, keep, outs

    def prepare(self, problems, residual=False):
        """Marshals a problem set once (the C array of problem descriptors and
        one output buffer per kind) for repeated calls of batched(): pass the
        returned Batch in place of the list.  Its X pointers can be replaced
        with Batch.set_x; every other input must stay where it is."""
        arr, keep, outs = self._problem_array(problems, residual)
        return Batch(arr, keep, outs, len(problems), residual)

    def batched(self, problems, nb=0, precision=0, residual=False, graph=0, stream=None, rotations=0,
                share_min_far=0, cols_per_block=0):
        """problems: list of dict(H, wr, wi, X) with device H and X (column-major,
        solved in place), or a Batch from prepare().  Returns a list of (E, mu,
        info, resid).  graph: 1 replay as a HIP graph, -1 launch kernel by
        kernel, 0 library default (graph)."""
        if isinstance(problems, Batch):
            b = problems
            if residual and not b.residual:
                raise ValueError("this Batch was prepared without residual buffers")
            residual = b.residual
        else:
            b = self.prepare(problems, residual)
        count, arr = b.count, b.arr
        o = _opts(nb, precision, residual, graph, rotations, share_min_far, cols_per_block)
        key = (nb, precision, residual, rotations, cols_per_block)
        need = b.need.get(key)
        if need is None:
            nv = ctypes.c_size_t()
            _check(self.lib.hsrq_workspace_size_batched(self.h, count, arr, ctypes.byref(o), ctypes.byref(nv)),
                   "hsrq_workspace_size_batched")
            need = b.need[key] = nv.value
        wp, wb = self.workspace(need)
        self._stream(stream)
        _check(self.lib.hsrq_dhsrq3_batched(self.h, count, arr, ctypes.c_void_p(wp), wb, ctypes.byref(o)),
               "hsrq_dhsrq3_batched")
        self._keep = b.keep
        return b.outs

    def autotune(self, problems, precision=0, stream=None, rotations=0):
        """Times each (tile size, far-block width) on this problem set and
        records the fastest in the handle (used by later calls with nb=0 and
        cols_per_block=0).  Returns (best_nb, best_cb, {(nb, cb): ms}) with
        ms 0 for a pair not run.  The problems' X are not modified."""
        count = len(problems)
        arr, keep, outs = self._problem_array(problems, False)
        o = _opts(0, precision, rotations=rotations)
        need = ctypes.c_size_t()
        _check(self.lib.hsrq_workspace_size_batched(self.h, count, arr, ctypes.byref(o), ctypes.byref(need)),
               "hsrq_workspace_size_batched")
        wp, wb = self.workspace(need.value)
        self._stream(stream)
        best, best_cb = ctypes.c_int(), ctypes.c_int()
        ms = np.zeros(4)
        _check(self.lib.hsrq_autotune(self.h, count, arr, ctypes.c_void_p(wp), wb, ctypes.byref(o),
                                      ctypes.byref(best), ctypes.byref(best_cb),
                                      ms.ctypes.data_as(ctypes.c_void_p)), "hsrq_autotune")
        grid = {(nb, cb): float(ms[2 * (nb == 128) + (cb == 64)]) for nb in (64, 128) for cb in (32, 64)}
        return best.value, best_cb.value, grid

    def gehrd(self, A, stream=None):
        """Reduce A (device, n x n, column-major, modified in place) to upper
        Hessenberg form H = Q0^T A Q0 (hsrq_gehrd).  Returns tau (device,
        n - 1); A then holds H and the reflectors below its subdiagonal."""
        torch = self.torch
        n = A.shape[0]
        if A.shape[0] != A.shape[1] or (n > 1 and A.stride(0) != 1):
            raise ValueError("A must be square and column-major")
        lda = max(A.stride(1), n) if n > 1 else 1
        tau = torch.zeros(max(n - 1, 1), dtype=torch.float64, device=A.device)
        need = ctypes.c_size_t()
        _check(self.lib.hsrq_gehrd_workspace_size(self.h, n, ctypes.byref(need)), "hsrq_gehrd_workspace_size")
        wp, wb = self.workspace(need.value)
        self._stream(stream)
        _check(self.lib.hsrq_gehrd(self.h, n, A.data_ptr(), lda, tau.data_ptr(), ctypes.c_void_p(wp), wb),
               "hsrq_gehrd")
        return tau

    def ormhr(self, A, tau, Z, stream=None):
        """Z <- Q0 Z in place (hsrq_ormhr), A and tau as gehrd left them."""
        n = A.shape[0]
        if Z.shape[0] > 1 and Z.stride(0) != 1:
            raise ValueError("Z must be column-major")
        lda = max(A.stride(1), n) if n > 1 else 1
        ldz = max(Z.stride(1) if Z.shape[1] > 1 else n, n)
        need = ctypes.c_size_t()
        _check(self.lib.hsrq_ormhr_workspace_size(self.h, n, Z.shape[1], ctypes.byref(need)),
               "hsrq_ormhr_workspace_size")
        wp, wb = self.workspace(need.value)
        self._stream(stream)
        _check(self.lib.hsrq_ormhr(self.h, n, A.data_ptr(), lda, tau.data_ptr(), Z.shape[1], Z.data_ptr(), ldz,
                                   ctypes.c_void_p(wp), wb), "hsrq_ormhr")
        return Z

    def autotune_save(self, path):
        """Write the handle's tuned choices to a text file (hsrq_autotune_save)."""
        _check(self.lib.hsrq_autotune_save(self.h, os.fsencode(path)), "hsrq_autotune_save")

    def autotune_load(self, path):
        """Merge a file written by autotune_save into the handle."""
        _check(self.lib.hsrq_autotune_load(self.h, os.fsencode(path)), "hsrq_autotune_load")

    def fallback_count(self):
        """Shifts re-solved in FP64 by the last mixed-precision call."""
        n = ctypes.c_int64()
        _check(self.lib.hsrq_fallback_count(self.h, ctypes.byref(n)), "hsrq_fallback_count")
        return n.value

    def profile(self, on=True):
        _check(self.lib.hsrq_profile_enable(self.h, 1 if on else 0), "hsrq_profile_enable")

    def profile_read(self):
        """{kind: (ms, launches)} accumulated since the last read."""
        k = len(KERNEL_KINDS)
        ms = np.zeros(k)
        ln = np.zeros(k, dtype=np.int64)
        _check(self.lib.hsrq_profile_read(self.h, k, ms.ctypes.data_as(ctypes.c_void_p),
                                          ln.ctypes.data_as(ctypes.c_void_p)), "hsrq_profile_read")
        return {name: (float(ms[i]), int(ln[i])) for i, name in enumerate(KERNEL_KINDS)}

    def debug_view(self, n, wi, nb=0):
        """After a single-problem call: device pointers of the recorded
        rotations C, S, the diagonal PHI of R and the working columns V
        (row-major n x ld, internal column order) as torch tensors, plus the
        internal column of every shift."""
        torch = self.torch
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        m = wi.shape[0]
        o = _opts(nb)
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        ld, nbo = ctypes.c_int(), ctypes.c_int()
        col_of = np.zeros(max(m, 1), dtype=np.int32)
        wp = (self._ws.data_ptr() + 255) & ~255
        _check(self.lib.hsrq_debug_view(self.h, n, m, wi.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o),
                                        ctypes.c_void_p(wp), *[ctypes.byref(p) for p in ptrs],
                                        ctypes.byref(ld), ctypes.byref(nbo),
                                        col_of.ctypes.data_as(ctypes.c_void_p)), "hsrq_debug_view")
        base = self._ws.data_ptr()
        out = []
        for p in ptrs:
            off = p.value - base
            assert off % 8 == 0
            out.append(self._ws[off:off + 8 * n * ld.value].view(torch.float64).view(n, ld.value))
        return dict(C=out[0], S=out[1], PHI=out[2], V=out[3], ld=ld.value, nb=nbo.value, col_of=col_of[:m])


class Server:
    """The library's serving loop (continuous batching under an HBM budget)
    for torch tensors.  submit() takes device H and X (X column-major, solved
    in place) and returns the device output tensors; they are valid once
    poll() has returned the request's tag."""

    def __init__(self, device: int = 0, budget_bytes: int = 200 * 10 ** 9, nb: int = 0, precision: int = 0,
                 residual: bool = False, rotations: int = 0, cols_per_block: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP library has no CPU fallback")
        self.torch = torch
        self.lib = load_library()
        self.residual = residual
        h = ctypes.c_void_p()
        o = _opts(nb, precision, residual, rotations=rotations, cols_per_block=cols_per_block)
        _check(self.lib.hsrq_server_create(ctypes.byref(h), device, int(budget_bytes), ctypes.byref(o)),
               "hsrq_server_create")
        self.h = h
        self._pending = {}

    def submit(self, H, wr, wi, X, tag, stream=None):
        """Queue one request; returns (E, mu, info, resid) device tensors.
        Raises on an invalid request; returns None if it can never fit.  The
        server's kernels for the request wait for the work enqueued so far on
        `stream` (default: torch's current stream), which produced H and X."""
        torch = self.torch
        Hc, ldh = colmajor(H)
        wr = np.ascontiguousarray(wr, dtype=np.float64)
        wi = np.ascontiguousarray(wi, dtype=np.float64)
        m = wr.shape[0]
        dev = Hc.device
        E = torch.empty(m, dtype=torch.int32, device=dev)
        mu = torch.empty(m, dtype=torch.float64, device=dev)
        info = torch.empty(m, dtype=torch.int32, device=dev)
        res = torch.empty(m, dtype=torch.float64, device=dev) if self.residual else None
        a = HsrqProblem()
        a.n, a.H, a.ldh, a.m = Hc.shape[0], Hc.data_ptr(), ldh, m
        a.wr, a.wi = wr.ctypes.data, wi.ctypes.data
        a.X, a.ldx = X.data_ptr(), (X.stride(1) if X.shape[1] > 1 else Hc.shape[0])
        a.scale_exp, a.scale_mant, a.info = E.data_ptr(), mu.data_ptr(), info.data_ptr()
        a.resid = res.data_ptr() if res is not None else None
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        st = self.lib.hsrq_server_submit(self.h, ctypes.byref(a), int(tag), ctypes.c_void_p(s.cuda_stream))
        if st == -1005:
            return None
        _check(st, "hsrq_server_submit")
        out = (E, mu, info, res)
        self._pending[int(tag)] = (Hc, X, out)
        return out

    def poll(self, max_count=1024, wait_ms=0):
        """Completion records (dicts) of finished requests."""
        buf = (HsrqCompletion * max(1, max_count))()
        n = ctypes.c_int()
        _check(self.lib.hsrq_server_poll(self.h, buf, max_count, ctypes.byref(n), int(wait_ms)), "hsrq_server_poll")
        out = []
        for k in range(n.value):
            c = buf[k]
            self._pending.pop(int(c.tag), None)
            out.append(dict(tag=int(c.tag), status=c.status, fallback=c.fallback, t_submit=c.t_submit,
                            t_start=c.t_start, t_done=c.t_done))
        return out

    def clock(self):
        t = ctypes.c_double()
        _check(self.lib.hsrq_server_clock(self.h, ctypes.byref(t)), "hsrq_server_clock")
        return t.value

    def close(self):
        if self.h:
            self.lib.hsrq_server_destroy(self.h)
            self.h = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
