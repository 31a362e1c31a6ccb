"""ctypes binding of libppcg (argument marshalling only).

Every step of the solver runs in the HIP library; this module only converts
torch tensors to device pointers, passes the current torch stream and turns
status codes into exceptions.  It raises if libppcg.so is missing: there is
no CPU fallback.

Layout: a block is column-major n x ncols; in torch it is a (ncols, n)
contiguous CUDA tensor, float64 for a real operator and complex128 for a
complex one (nonzero Bloch vector ``kpt``).  ``solve`` accepts the start
block as an (n, K) tensor (any strides) and returns X as an (n, k) view of
such a buffer.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import CFUNCTYPE, POINTER, byref, c_char_p, c_double, c_int32, c_int64, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppcg.so")

PPCG_FP64, PPCG_MIXED = 0, 1
PPCG_NO_GRAPHS, PPCG_AUTOTUNE, PPCG_RETURN_BUFFERS = 1, 2, 4
STATUS = {0: "PPCG_OK", 1: "PPCG_EINVAL", 2: "PPCG_ENOTHPD", 3: "PPCG_ERANK", 4: "PPCG_ENOCONV",
          5: "PPCG_ENOSTATE", 6: "PPCG_EHIP", 7: "PPCG_ENOMEM"}
STATUS_CODE = {v: k for k, v in STATUS.items()}


class PPCGError(RuntimeError):
    def __init__(self, code, msg, info=None):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))
        self.info = info


class IterLog(ctypes.Structure):
    _fields_ = [("iter", c_int32), ("n_locked", c_int32), ("n_active", c_int32), ("kind", c_int32),
                ("rho", c_double), ("time_s", c_double), ("orth_err", c_double), ("trace", c_double)]


LOG_FN = CFUNCTYPE(None, POINTER(IterLog), c_void_p)
ITER_KIND = {0: "start", 1: "cholqr", 2: "rr", 3: "final_rr_failed"}


class Options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("nbuf", c_int32), ("max_iter", c_int32), ("profile", c_int32),
                ("flags", c_int32), ("singular_tol", c_double), ("seed", c_uint64), ("tune_table", c_char_p),
                ("log_cb", LOG_FN), ("log_user", c_void_p), ("orth", c_int32), ("stop", c_int32),
                ("rr_max", c_int32), ("orth_skip", c_double), ("orth_taylor", c_double)]


ORTH = {"cholqr": 0, "skip": 1, "taylor": 2, "none": 3}
STOP = {"residual": 0, "trace": 1}


class Operator(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("h", c_double), ("order", c_int32), ("kpt", c_double * 3),
                ("V", c_void_p), ("precond", c_int32), ("B", c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("n_rr", c_int32), ("n_locked", c_int32), ("n_backtrack", c_int32),
                ("resid_final", c_double), ("orth_err", c_double), ("time_s", c_double),
                ("stage_ms", c_double * 6), ("n_dropped", c_int32), ("n_unlock", c_int32),
                ("n_cholqr", c_int32), ("n_taylor", c_int32), ("n_orth_skip", c_int32),
                ("roofline_ms", c_double)]

    def as_dict(self):
        return {f: (list(getattr(self, f)) if f == "stage_ms" else getattr(self, f)) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libppcg.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1407_7506_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.ppcg_create.argtypes = [POINTER(c_void_p), POINTER(Options), c_void_p]
    L.ppcg_create.restype = c_int32
    L.ppcg_solve.argtypes = [c_void_p, POINTER(Operator), c_int32, c_int32, c_double, c_int32,
                             c_void_p, c_void_p, c_void_p, POINTER(Info)]
    L.ppcg_solve.restype = c_int32
    L.ppcg_solve_batched.argtypes = [c_void_p, c_int32, POINTER(Operator), POINTER(c_int32), c_int32, c_double,
                                     c_int32, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                     POINTER(Info), POINTER(c_int32)]
    L.ppcg_solve_batched.restype = c_int32
    L.ppcg_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32, POINTER(c_int32),
                            POINTER(c_double)]
    L.ppcg_grad.restype = c_int32
    L.ppcg_density.argtypes = [c_void_p, c_void_p]
    L.ppcg_density.restype = c_int32
    L.ppcg_columns.argtypes = [c_void_p, c_int32, c_int32]
    L.ppcg_columns.restype = c_int32
    L.ppcg_apply_h.argtypes = [c_void_p, POINTER(Operator), c_int32, c_void_p, c_void_p]
    L.ppcg_apply_h.restype = c_int32
    L.ppcg_start_block.argtypes = [c_void_p, c_int64, c_int32, c_int32, c_uint64, c_void_p]
    L.ppcg_start_block.restype = c_int32
    L.ppcg_block_pencils.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_double,
                                     c_void_p, c_void_p]
    L.ppcg_block_pencils.restype = c_int32
    L.ppcg_block_pencils_noalloc.argtypes = L.ppcg_block_pencils.argtypes
    L.ppcg_block_pencils_noalloc.restype = c_int32
    L.ppcg_kernel_times.argtypes = [c_void_p, POINTER(c_char_p), POINTER(c_double), POINTER(c_int64), c_int32]
    L.ppcg_kernel_times.restype = c_int32
    L.ppcg_kernel_stats.argtypes = [c_void_p, POINTER(c_char_p), POINTER(c_double), POINTER(c_int64),
                                    POINTER(c_double), POINTER(c_double), c_int32]
    L.ppcg_kernel_stats.restype = c_int32
    L.ppcg_reset_kernel_times.argtypes = [c_void_p]
    L.ppcg_reset_kernel_times.restype = None
    L.ppcg_destroy.argtypes = [c_void_p]
    L.ppcg_destroy.restype = None
    L.ppcg_tune_report.argtypes = [c_void_p, c_char_p, c_int32]
    L.ppcg_tune_report.restype = c_int32
    L.ppcg_last_error.argtypes = [c_void_p]
    L.ppcg_last_error.restype = c_char_p
    _lib = L
    return L


_PRECONDS = {"none": 0, "jacobi": 1}  # ppcg_precond


def _is_complex_kpt(kpt) -> bool:
    return any(float(c) != 0.0 for c in kpt)


def _check_tensor(t, name, numel=None, cplx=False):
    import torch
    want = torch.complex128 if cplx else torch.float64
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != want:
        raise TypeError(f"{name} must be a CUDA {str(want).replace('torch.', '')} tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


class Handle:
    """One libppcg handle bound to the current device and torch stream."""

    def __init__(self, precision: str = "fp64", nbuf: int = -1, max_iter: int = 0, profile: bool = False,
                 stream=None, graphs: bool = True, autotune: bool = False, singular_tol: float = 0.0,
                 seed: int = 0, tune_table: str | None = None, log=None, orth: str = "cholqr",
                 orth_skip: float = 0.0, orth_taylor: float = 0.0, rr_max: int = 0, stop: str = "residual",
                 return_buffers: bool = False):
        """log: optional callable receiving one dict per PPCG iteration (iter,
        n_locked, n_active, kind, rho, time_s, orth_err, trace).  orth:
        "cholqr", "skip", "taylor" or "none"; stop: "residual" or "trace".
        return_buffers: solve returns all K columns and Ritz values."""
        import torch
        self._L = lib()
        flags = (0 if graphs else PPCG_NO_GRAPHS) | (PPCG_AUTOTUNE if autotune else 0) | \
            (PPCG_RETURN_BUFFERS if return_buffers else 0)
        self.return_buffers = return_buffers
        self._log_fn = LOG_FN(0)
        if log is not None:
            def _cb(rec, _user):
                r = rec.contents
                log({"iter": r.iter, "n_locked": r.n_locked, "n_active": r.n_active,
                     "kind": ITER_KIND.get(r.kind, r.kind), "rho": r.rho, "time_s": r.time_s,
                     "orth_err": r.orth_err, "trace": r.trace})
            self._log_fn = LOG_FN(_cb)
        opt = Options(PPCG_MIXED if precision == "mixed" else PPCG_FP64, nbuf, max_iter, 1 if profile else 0, flags,
                      float(singular_tol), int(seed), tune_table.encode() if tune_table else None, self._log_fn, None,
                      ORTH[orth], STOP[stop], int(rr_max), float(orth_skip), float(orth_taylor))
        st = stream if stream is not None else torch.cuda.current_stream()
        self.stream = st
        h = c_void_p()
        code = self._L.ppcg_create(byref(h), byref(opt), c_void_p(st.cuda_stream))
        if code != 0:
            raise PPCGError(code, "ppcg_create failed")
        self._h = h
        self.precision = precision
        self._last_n = None

    def close(self):
        if getattr(self, "_h", None):
            self._L.ppcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return self._L.ppcg_last_error(self._h).decode()

    @staticmethod
    def operator(V, N, h=0.5, order=2, kpt=(0.0, 0.0, 0.0), B=None, precond="jacobi"):
        _check_tensor(V, "V", N ** 3)
        if B is not None:
            _check_tensor(B, "B", N ** 3)
        code = _PRECONDS.get(precond, precond)  # a name, or a raw ppcg_precond value passed through
        return Operator(int(N), float(h), int(order), (c_double * 3)(*kpt), c_void_p(V.data_ptr()), int(code),
                        c_void_p(B.data_ptr()) if B is not None else None)

    def columns(self, k, sbsize):
        """K = k + nbuf columns the start block must have."""
        K = self._L.ppcg_columns(self._h, int(k), int(sbsize))
        if K < 0:
            raise ValueError("bad k or sbsize")
        return K

    def apply_h(self, V, N, X, h=0.5, order=2, kpt=(0.0, 0.0, 0.0)):
        """Y = H X for a (ncols, n) column-major block X (complex128 when kpt != 0)."""
        import torch
        _check_tensor(X, "X", cplx=_is_complex_kpt(kpt))
        X = X.contiguous()
        if X.numel() % (N ** 3):
            raise ValueError("X must hold whole columns of length N^3")
        ncols = X.numel() // (N ** 3)
        Y = torch.empty_like(X)
        op = self.operator(V, N, h, order, kpt)
        code = self._L.ppcg_apply_h(self._h, byref(op), ncols, c_void_p(X.data_ptr()), c_void_p(Y.data_ptr()))
        if code != 0:
            raise PPCGError(code, self.error())
        return Y

    def start_block(self, n, ncols, seed, cplx=False):
        """The start block a solve draws on the device when X0 is None, for a
        given seed: a (ncols, n) column-major CUDA tensor, float64 N(0,1) or
        complex128 with N(0,1/2) parts."""
        import torch
        X = torch.empty((int(ncols), int(n)), dtype=torch.complex128 if cplx else torch.float64, device="cuda")
        code = self._L.ppcg_start_block(self._h, int(n), int(ncols), 1 if cplx else 0, int(seed),
                                        c_void_p(X.data_ptr()) if X.numel() else None)
        if code != 0:
            raise PPCGError(code, self.error())
        return X

    def solve(self, V, N, k, sbsize, tol, rr_period, X0, h=0.5, order=2, check=True, kpt=(0.0, 0.0, 0.0), B=None,
              precond="jacobi"):
        """Lowest k eigenpairs.  X0: (n, K) start block (torch CUDA float64, or
        complex128 for a nonzero Bloch vector kpt), or None for a start block
        drawn on the device from the handle's seed.  B: optional diagonal of the
        generalized problem H x = lambda B x (CUDA float64, n).  precond:
        "jacobi" (T = diag(H)^-1) or "none" (T = I).
        Returns (lam (k,), X (n, k), info dict)."""
        import torch
        n = N ** 3
        cplx = _is_complex_kpt(kpt)
        K = self.columns(k, sbsize)
        if X0 is not None:
            _check_tensor(X0, "X0", cplx=cplx)
            if X0.dim() != 2 or X0.shape[0] != n or X0.shape[1] != K:
                raise ValueError(f"X0 must have shape (n, K) = ({n}, {K})")
            X0cm = X0.t().contiguous()
        else:
            X0cm = None
        dt = torch.complex128 if cplx else torch.float64
        kout = K if self.return_buffers else k
        Xout = torch.empty((kout, n), dtype=dt, device=V.device)
        lam = torch.empty(kout, dtype=torch.float64, device=V.device)
        op = self.operator(V, N, h, order, kpt, B, precond)
        info = Info()
        code = self._L.ppcg_solve(self._h, byref(op), int(k), int(sbsize), float(tol), int(rr_period),
                                  c_void_p(X0cm.data_ptr()) if X0cm is not None else None,
                                  c_void_p(Xout.data_ptr()), c_void_p(lam.data_ptr()), byref(info))
        self._last_n = n if code == 0 else None
        if code != 0 and check:
            raise PPCGError(code, self.error(), info.as_dict())
        d = info.as_dict()
        d["status"] = STATUS.get(code, code)
        return lam, Xout.t(), d

    def solve_batched(self, problems, sbsize, tol, rr_period, check=True):
        """Solve many independent problems in lockstep.  problems: list of
        dicts with V (CUDA float64, N^3), N, k, X0 ((n, K) CUDA float64, or
        complex128 with kpt; None or absent: drawn on the device from the
        handle's seed + problem index), and optional h, order, kpt.  All problems are
        real or all complex.  Returns a list of (lam, X (n, k), info, status)."""
        import torch
        nb = len(problems)
        ops = (Operator * nb)()
        ks = (c_int32 * nb)()
        x0p = (c_void_p * nb)()
        xop = (c_void_p * nb)()
        lop = (c_void_p * nb)()
        infos = (Info * nb)()
        sts = (c_int32 * nb)()
        keep = []
        outs = []
        for b, p in enumerate(problems):
            N, k = int(p["N"]), int(p["k"])
            n = N ** 3
            K = self.columns(k, sbsize)
            X0 = p.get("X0")
            kpt = p.get("kpt", (0.0, 0.0, 0.0))
            cplx = _is_complex_kpt(kpt)
            if X0 is not None:
                _check_tensor(X0, "X0", cplx=cplx)
                if X0.dim() != 2 or X0.shape[0] != n or X0.shape[1] != K:
                    raise ValueError(f"problem {b}: X0 must have shape ({n}, {K})")
                X0cm = X0.t().contiguous()
                keep.append(X0cm)
            dt = torch.complex128 if cplx else torch.float64
            kout = K if self.return_buffers else k
            Xo = torch.empty((kout, n), dtype=dt, device=p["V"].device)
            lo = torch.empty(kout, dtype=torch.float64, device=p["V"].device)
            ops[b] = self.operator(p["V"], N, p.get("h", 0.5), p.get("order", 2), kpt)
            ks[b] = k
            x0p[b] = X0cm.data_ptr() if X0 is not None else None
            xop[b] = Xo.data_ptr()
            lop[b] = lo.data_ptr()
            keep.append(p["V"])
            outs.append((lo, Xo))
        code = self._L.ppcg_solve_batched(self._h, nb, ops, ks, int(sbsize), float(tol), int(rr_period), x0p, xop,
                                          lop, infos, sts)
        self._last_n = None
        if code != 0 and check:
            raise PPCGError(code, self.error())
        return [(outs[b][0], outs[b][1].t(), infos[b].as_dict(), STATUS.get(sts[b], sts[b])) for b in range(nb)]

    def grad(self, g_lambda, w=None, tol=1e-10, max_iter=0):
        """dL/dV for L = g_lambda . lambda + w . rho of the last solve (torch CUDA
        float64 tensors); returns (dL/dV (n,), CG iterations)."""
        import torch
        _check_tensor(g_lambda, "g_lambda")
        if w is not None:
            _check_tensor(w, "w")
        n = self._last_n
        if n is None:
            raise PPCGError(5, "no successful solve on this handle")
        out = torch.empty(n, dtype=torch.float64, device=g_lambda.device)
        it = c_int32(0)
        res = c_double(0.0)
        code = self._L.ppcg_grad(self._h, c_void_p(g_lambda.contiguous().data_ptr()),
                                 c_void_p(w.contiguous().data_ptr()) if w is not None else None,
                                 c_void_p(out.data_ptr()), float(tol), int(max_iter), byref(it), byref(res))
        self.grad_iters, self.grad_resid = it.value, res.value
        if code != 0:
            raise PPCGError(code, self.error(), {"iters": it.value, "resid": res.value})
        return out, it.value

    def block_pencils(self, A, B, q, has_p, tol=1e-9, noalloc=False):
        """The sub-block projected problems alone: A, B (nblocks, nS, nS)
        CUDA float64 / complex128 tensors (row-major view of column-major
        matrices: element [j, c, r] is row r, column c of block j), nS = 3q
        with P or 2q.  Returns (C (nblocks, q, 3q): C[j, t, i] is row i of
        eigenvector t, flags (nblocks,) int32).  noalloc=True calls
        ppcg_block_pencils_noalloc (library scratch in a static device array;
        the call only enqueues, so the handle's stream is synchronised here)."""
        import torch
        cplx = A.dtype == torch.complex128
        _check_tensor(A, "A", cplx=cplx)
        _check_tensor(B, "B", cplx=cplx)
        nb, nS = A.shape[0], A.shape[1]
        if A.shape != (nb, nS, nS) or B.shape != A.shape or nS != (3 if has_p else 2) * q:
            raise ValueError("A, B must be (nblocks, nS, nS) with nS = 3q (has_p) or 2q")
        A = A.contiguous()
        B = B.contiguous()
        C = torch.zeros((nb, q, 3 * q), dtype=A.dtype, device=A.device)
        flags = torch.zeros(nb, dtype=torch.int32, device=A.device)
        fn = self._L.ppcg_block_pencils_noalloc if noalloc else self._L.ppcg_block_pencils
        code = fn(self._h, int(nb), int(q), 1 if has_p else 0, 1 if cplx else 0, c_void_p(A.data_ptr()),
                  c_void_p(B.data_ptr()), float(tol), c_void_p(C.data_ptr()), c_void_p(flags.data_ptr()))
        if code != 0:
            raise PPCGError(code, self.error())
        if noalloc:
            self.stream.synchronize()
        return C, flags

    def density(self):
        """rho = sum_i x_i^2 of the last solve (torch CUDA float64, (n,))."""
        import torch
        if self._last_n is None:
            raise PPCGError(5, "no successful solve on this handle")
        rho = torch.empty(self._last_n, dtype=torch.float64, device="cuda")
        code = self._L.ppcg_density(self._h, c_void_p(rho.data_ptr()))
        if code != 0:
            raise PPCGError(code, self.error())
        return rho

    def tune_report(self) -> str:
        """The autotuner's decisions (one line per shape class); empty without
        autotune=True."""
        n = self._L.ppcg_tune_report(self._h, None, 0)
        if n <= 0:
            return ""
        buf = ctypes.create_string_buffer(n + 1)
        self._L.ppcg_tune_report(self._h, buf, n + 1)
        return buf.value.decode()

    def kernel_times(self):
        """{kernel kind: (total ms, launches, algorithmic flops, compulsory bytes)}"""
        cap = 64
        names = (c_char_p * cap)()
        ms = (c_double * cap)()
        cnt = (c_int64 * cap)()
        fl = (c_double * cap)()
        by = (c_double * cap)()
        w = self._L.ppcg_kernel_stats(self._h, names, ms, cnt, fl, by, cap)
        return {names[i].decode(): (ms[i], cnt[i], fl[i], by[i]) for i in range(w)}

    def reset_kernel_times(self):
        self._L.ppcg_reset_kernel_times(self._h)


def solve(V, N, k, sbsize, tol, rr_period, X0, precision="fp64", **kw):
    """Convenience wrapper: one-shot handle on the current stream."""
    h = Handle(precision=precision, nbuf=kw.pop("nbuf", -1), max_iter=kw.pop("max_iter", 0))
    try:
        return h.solve(V, N, k, sbsize, tol, rr_period, X0, **kw)
    finally:
        h.close()
