"""Thin Python binding of libairga (C ABI in include/airga.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every computation runs in the library's HIP kernels.  There is no
CPU fallback: if ``libairga.so`` is missing or cannot be loaded, every call
raises.

Names follow the C ABI: ``Context.set_pencil`` wraps ``airga_set_pencil``,
``Context.spai_build`` wraps ``airga_spai_build`` and so on.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libairga.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SYS_CONVERGED, SYS_MAXIT, SYS_BREAKDOWN, SYS_NONFINITE = 0, 1, 2, 3
MODE_FP64, MODE_MIXED = 0, 1
BETA_FLEXIBLE, BETA_CLASSICAL = 0, 1
STATUS_NAMES = {SYS_CONVERGED: "converged", SYS_MAXIT: "maxit", SYS_BREAKDOWN: "breakdown",
                SYS_NONFINITE: "nonfinite"}


class AirgaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"airga status {status}: {msg}")
        self.status = status


class PencilInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("max_row_len", ctypes.c_int32),
                ("bandwidth", ctypes.c_int32), ("slice_rows", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("nnz_stored", ctypes.c_int64),
                ("gram_mm", ctypes.c_double), ("gram_mk", ctypes.c_double),
                ("gram_kk", ctypes.c_double), ("trace_m", ctypes.c_double),
                ("trace_k", ctypes.c_double)]


class SpaiOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("equilibrate", ctypes.c_int32),
                ("symmetrize", ctypes.c_int32), ("general_only", ctypes.c_int32),
                ("mr_iters", ctypes.c_int32), ("lfil", ctypes.c_int32)]


class PrecInfo(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_double), ("alpha", ctypes.c_double),
                ("chain_len", ctypes.c_int32), ("scalar_only", ctypes.c_int32),
                ("skipped_cols", ctypes.c_int64), ("shift_im", ctypes.c_double),
                ("alpha_im", ctypes.c_double), ("is_complex", ctypes.c_int32)]


class PcgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("max_sweeps", ctypes.c_int32), ("poll_every", ctypes.c_int32),
                ("x0_given", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_sys", ctypes.c_int32), ("general_only", ctypes.c_int32),
                ("beta_form", ctypes.c_int32), ("inner_max", ctypes.c_int32)]


class SysStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("finished_fp64", ctypes.c_int32),
                ("relres", ctypes.c_double)]


class ReduceOpts(ctypes.Structure):
    _fields_ = [("r_max", ctypes.c_int32), ("tol_inner", ctypes.c_double),
                ("tol_outer", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("update_from", ctypes.c_int32), ("spai", SpaiOpts), ("pcg", PcgOpts)]


class ReduceResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("r", ctypes.c_int32), ("change", ctypes.c_double),
                ("mhat", ctypes.c_void_p), ("khat", ctypes.c_void_p), ("fhat", ctypes.c_void_p),
                ("cphat", ctypes.c_void_p), ("cvhat", ctypes.c_void_p),
                ("next_shifts", ctypes.c_void_p)]


class ReduceIter(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int32), ("moment_steps", ctypes.c_int32),
                ("updated", ctypes.c_int32), ("chain_len_max", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("all_converged", ctypes.c_int32),
                ("change", ctypes.c_double), ("last_inner_change", ctypes.c_double)]


class ReducedModel(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("m", ctypes.c_int32), ("p", ctypes.c_int32),
                ("mhat", ctypes.c_void_p), ("khat", ctypes.c_void_p), ("fhat", ctypes.c_void_p),
                ("cphat", ctypes.c_void_p), ("cvhat", ctypes.c_void_p)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_P = ctypes.c_void_p
_SIGS = [
    ("airga_create", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    ("airga_destroy", None, [_P]),
    ("airga_last_error", ctypes.c_char_p, []),
    ("airga_version", ctypes.c_char_p, []),
    ("airga_set_pencil", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P,
                                        ctypes.c_double, ctypes.c_double]),
    ("airga_get_pencil_info", ctypes.c_int, [_P, ctypes.POINTER(PencilInfo)]),
    ("airga_assemble_shift", ctypes.c_int, [_P, ctypes.c_double, _P]),
    ("airga_apply_shift", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32, _P, ctypes.c_int64,
                                         _P, ctypes.c_int64]),
    ("airga_shift_diagnostics", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double,
                                               ctypes.POINTER(ctypes.c_double)]),
    ("airga_spai_opts_default", None, [ctypes.POINTER(SpaiOpts)]),
    ("airga_spai_build", ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(SpaiOpts),
                                        ctypes.POINTER(_P)]),
    ("airga_spai_update", ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.POINTER(SpaiOpts),
                                         ctypes.POINTER(_P)]),
    ("airga_spai_update_many", ctypes.c_int, [_P, ctypes.c_int32, _P, _P,
                                              ctypes.POINTER(SpaiOpts), _P]),
    ("airga_spai_build_many", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.POINTER(SpaiOpts),
                                             _P]),
    ("airga_get_prec_info", ctypes.c_int, [_P, ctypes.POINTER(PrecInfo)]),
    ("airga_prec_export", ctypes.c_int, [_P, _P, _P]),
    ("airga_prec_skip_flags", ctypes.c_int, [_P, _P]),
    ("airga_prec_apply", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, _P,
                                        ctypes.c_int64]),
    ("airga_prec_release", None, [_P]),
    ("airga_pcg_opts_default", None, [ctypes.POINTER(PcgOpts)]),
    ("airga_pcg_solve", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.c_int64,
                                       _P, ctypes.c_int64, ctypes.POINTER(PcgOpts),
                                       ctypes.POINTER(SysStats)]),
    ("airga_kernel_count", ctypes.c_int32, []),
    ("airga_kernel_name", ctypes.c_char_p, [ctypes.c_int32]),
    ("airga_get_kernel_times", ctypes.c_int, [_P, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(ctypes.c_double)]),
    ("airga_get_tile_config", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32)]),
    ("airga_get_kernel_work", ctypes.c_int, [_P, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int64)]),
    ("airga_assemble_shift_complex", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, _P]),
    ("airga_spai_build_complex", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double,
                                                ctypes.POINTER(SpaiOpts), ctypes.POINTER(_P)]),
    ("airga_spai_update_complex", ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double,
                                                 ctypes.POINTER(SpaiOpts), ctypes.POINTER(_P)]),
    ("airga_spai_build_complex_many", ctypes.c_int, [_P, ctypes.c_int32,
                                                     ctypes.POINTER(ctypes.c_double),
                                                     ctypes.POINTER(SpaiOpts),
                                                     ctypes.POINTER(_P)]),
    ("airga_spai_update_complex_many", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(_P),
                                                      ctypes.POINTER(ctypes.c_double),
                                                      ctypes.POINTER(SpaiOpts),
                                                      ctypes.POINTER(_P)]),
    ("airga_prec_export_complex", ctypes.c_int, [_P, _P, _P]),
    ("airga_cocg_solve", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.c_int64,
                                        _P, ctypes.c_int64, ctypes.POINTER(PcgOpts),
                                        ctypes.POINTER(SysStats)]),
    ("airga_pencil_apply", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                          _P, ctypes.c_int64, _P, ctypes.c_int64]),
    ("airga_gram", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int32, _P,
                                  ctypes.c_int64, _P]),
    ("airga_gram_noalloc", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int32,
                                          _P, ctypes.c_int64, _P]),
    ("airga_global_orth", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int64,
                                         ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    ("airga_block_qr", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_double)]),
    ("airga_project", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    ("airga_reduce_opts_default", None, [ctypes.POINTER(ReduceOpts)]),
    ("airga_reduce", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int32, _P, _P,
                                    ctypes.c_int64, ctypes.c_int32, _P,
                                    ctypes.POINTER(ReduceOpts), _P, ctypes.c_int64,
                                    ctypes.POINTER(ReduceResult), _P, _P, _P]),
    ("airga_qep_poles", ctypes.c_int, [ctypes.c_int32, _P, _P, ctypes.c_double, ctypes.c_double,
                                       _P, _P]),
    ("airga_next_shifts", ctypes.c_int, [ctypes.c_int32, _P, _P, ctypes.c_int32, _P]),
    ("airga_h2_distance", ctypes.c_int, [ctypes.POINTER(ReducedModel),
                                         ctypes.POINTER(ReducedModel), ctypes.c_double,
                                         ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
]

EXPORTED = [s[0] for s in _SIGS]


def lib():
    """Load libairga.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _check(status: int):
    if status != OK:
        msg = lib().airga_last_error().decode(errors="replace")
        raise AirgaError(status, msg)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, device) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor on {device}, got "
                         f"{t.dtype} on {t.device}")
    return t


# ---- decisions of the outer iteration (host computations, no GPU) --------

def _host(a):
    """Column-major float64 copy of a host matrix, and its address."""
    import numpy as np
    arr = np.asfortranarray(np.asarray(a, dtype=np.float64))
    return arr, ctypes.c_void_p(arr.ctypes.data)


def qep_poles(mh, kh, alpha: float, beta: float):
    """The 2r poles of lambda^2 Mh + lambda (alpha Mh + beta Kh) + Kh
    (complex numpy array, two per mode, modes in ascending frequency)."""
    import numpy as np
    r = int(np.shape(mh)[0])
    m_arr, m_p = _host(mh)
    k_arr, k_p = _host(kh)
    re = np.zeros(2 * r)
    im = np.zeros(2 * r)
    _check(lib().airga_qep_poles(r, m_p, k_p, float(alpha), float(beta),
                                 ctypes.c_void_p(re.ctypes.data),
                                 ctypes.c_void_p(im.ctypes.data)))
    return re + 1j * im


def next_shifts(poles, l: int):
    """The next l expansion points from the poles (ascending numpy array)."""
    import numpy as np
    poles = np.asarray(poles, dtype=complex)
    re = np.ascontiguousarray(poles.real, dtype=np.float64)
    im = np.ascontiguousarray(poles.imag, dtype=np.float64)
    out = np.zeros(max(int(l), 1))
    _check(lib().airga_next_shifts(poles.size, ctypes.c_void_p(re.ctypes.data),
                                   ctypes.c_void_p(im.ctypes.data), int(l),
                                   ctypes.c_void_p(out.ctypes.data)))
    return out[:l]


def _model(mod, keep):
    """ReducedModel for (mh, kh, fh, cph, cvh or None); keep holds the arrays."""
    mh, kh, fh, cph, cvh = mod
    arrs = [_host(x) for x in (mh, kh, fh, cph)]
    cv = _host(cvh) if cvh is not None else (None, None)
    keep.extend(a for a, _ in arrs)
    keep.append(cv[0])
    r, m = arrs[2][0].shape
    p = arrs[3][0].shape[0]
    return ReducedModel(r, m, p, arrs[0][1], arrs[1][1], arrs[2][1], arrs[3][1], cv[1])


def h2_distance(a, b, alpha: float, beta: float) -> float:
    """||H_a - H_b||_H2 (b None: ||H_a||_H2); a, b = (mh, kh, fh, cph, cvh or None)."""
    keep = []
    ma = _model(a, keep)
    mb = _model(b, keep) if b is not None else None
    out = ctypes.c_double()
    _check(lib().airga_h2_distance(ctypes.byref(ma), ctypes.byref(mb) if mb is not None else None,
                                   float(alpha), float(beta), ctypes.byref(out)))
    return out.value


class Context:
    """airga_ctx on one GPU; all work is ordered on ``self.stream``, which is
    joined with torch's current stream around every call."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        _check(lib().airga_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream)))
        self._h = h
        self.n = None
        self.nnz = None
        self._precs = weakref.WeakSet()

    # stream joins
    def _enter(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _leave(self):
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def close(self):
        if getattr(self, "_h", None):
            # handles must go before their context
            for p in list(self._precs):
                p.release()
            lib().airga_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- pencil
    def set_pencil(self, row_ptr, col_idx, m_val, k_val, alpha: float, beta: float):
        n = row_ptr.numel() - 1
        _dev(row_ptr, torch.int32, self.device)
        _dev(col_idx, torch.int32, self.device)
        _dev(m_val, torch.float64, self.device)
        _dev(k_val, torch.float64, self.device)
        self._enter()
        _check(lib().airga_set_pencil(self._h, n, col_idx.numel(), _ptr(row_ptr), _ptr(col_idx),
                                      _ptr(m_val), _ptr(k_val), float(alpha), float(beta)))
        self._leave()
        self.n, self.nnz = n, col_idx.numel()

    def pencil_info(self) -> PencilInfo:
        info = PencilInfo()
        _check(lib().airga_get_pencil_info(self._h, ctypes.byref(info)))
        return info

    def assemble_shift(self, s: float, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        _dev(out, torch.float64, self.device)
        self._enter()
        _check(lib().airga_assemble_shift(self._h, float(s), _ptr(out)))
        self._leave()
        return out

    def apply_shift(self, s: float, x: torch.Tensor) -> torch.Tensor:
        """y = K(s) x for x of shape (count, n) (float64, contiguous)."""
        _dev(x, torch.float64, self.device)
        x2 = x.reshape(-1, self.n)
        y = torch.empty_like(x2)
        self._enter()
        _check(lib().airga_apply_shift(self._h, float(s), x2.shape[0], _ptr(x2), self.n, _ptr(y),
                                       self.n))
        self._leave()
        return y.reshape(x.shape)

    # ------------------------------------------------ moment sequence blocks
    #
    # Blocks of k vectors are (k, n) tensors: vector c is row c (the C ABI's
    # column-major n x k with leading dimension n).

    def _block(self, t: torch.Tensor) -> torch.Tensor:
        _dev(t, torch.float64, self.device)
        if t.dim() != 2 or t.shape[1] != self.n:
            raise ValueError(f"expected a (k, {self.n}) block")
        return t

    def pencil_apply(self, a: float, b: float, x: torch.Tensor) -> torch.Tensor:
        """(a M + b K) x for the rows of x (k, n)."""
        x = self._block(x)
        y = torch.empty_like(x)
        self._enter()
        _check(lib().airga_pencil_apply(self._h, float(a), float(b), x.shape[0], _ptr(x), self.n,
                                        _ptr(y), self.n))
        self._leave()
        return y

    def gram(self, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        """(k, l) device tensor of the products a_i . b_j over the n rows."""
        a, b = self._block(a), self._block(b)
        g = torch.empty((b.shape[0], a.shape[0]), dtype=torch.float64, device=self.device)
        self._enter()
        _check(lib().airga_gram(self._h, a.shape[0], _ptr(a), self.n, b.shape[0], _ptr(b), self.n,
                                _ptr(g)))
        self._leave()
        return g.t()

    def gram_noalloc(self, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """airga_gram_noalloc into out, an (l, k) float64 device tensor (the
        column-major k x l result); returns out.t(), the (k, l) products."""
        a, b = self._block(a), self._block(b)
        _dev(out, torch.float64, self.device)
        if tuple(out.shape) != (b.shape[0], a.shape[0]):
            raise ValueError("out must be (l, k)")
        self._enter()
        _check(lib().airga_gram_noalloc(self._h, a.shape[0], _ptr(a), self.n, b.shape[0], _ptr(b),
                                        self.n, _ptr(out)))
        self._leave()
        return out.t()

    def global_orth(self, v: torch.Tensor | None, x: torch.Tensor, m: int,
                    normalize: bool = False):
        """Orthogonalise the n x m blocks of x (rows x m .. x m + m - 1) in
        place against those of v in the trace inner product; returns gamma
        (nx, nb) and the Frobenius norms (nx,) as numpy arrays."""
        import numpy as np
        x = self._block(x)
        nb = 0 if v is None else self._block(v).shape[0] // m
        nx = x.shape[0] // m
        if x.shape[0] != nx * m or (v is not None and v.shape[0] != nb * m):
            raise ValueError("block rows must be a multiple of m")
        gam = (ctypes.c_double * max(1, nx * nb))()
        fro = (ctypes.c_double * max(1, nx))()
        self._enter()
        _check(lib().airga_global_orth(self._h, int(m), nb, _ptr(v), self.n, nx, _ptr(x), self.n,
                                       1 if normalize else 0, gam, fro))
        self._leave()
        return (np.array(gam[:nx * nb], dtype=float).reshape(nx, nb),
                np.array(fro[:nx], dtype=float))

    def block_qr(self, w: torch.Tensor):
        """Thin QR of the k columns (rows of w): w becomes Q; returns R
        (k, k) as a numpy array, w_in = R^T Q in the (k, n) layout."""
        import numpy as np
        w = self._block(w)
        k = w.shape[0]
        r = (ctypes.c_double * max(1, k * k))()
        self._enter()
        _check(lib().airga_block_qr(self._h, k, _ptr(w), self.n, r))
        self._leave()
        return np.array(r[:k * k], dtype=float).reshape(k, k).T

    def project(self, w: torch.Tensor):
        """(W^T M W, W^T K W) as numpy arrays for the k columns of w."""
        import numpy as np
        w = self._block(w)
        k = w.shape[0]
        mh = (ctypes.c_double * max(1, k * k))()
        kh = (ctypes.c_double * max(1, k * k))()
        self._enter()
        _check(lib().airga_project(self._h, k, _ptr(w), self.n, mh, kh))
        self._leave()
        return (np.array(mh[:k * k], dtype=float).reshape(k, k).T,
                np.array(kh[:k * k], dtype=float).reshape(k, k).T)

    def shift_diagnostics(self, s_old: float, s_new: float):
        out = (ctypes.c_double * 4)()
        _check(lib().airga_shift_diagnostics(self._h, float(s_old), float(s_new), out))
        return tuple(out)

    # ------------------------------------------------------- preconditioners
    @staticmethod
    def _spai_opts(tol, equilibrate, symmetrize, general_only=False, mr_iters=0, lfil=0):
        o = SpaiOpts()
        lib().airga_spai_opts_default(ctypes.byref(o))
        if tol is not None:
            o.tol = float(tol)
        o.equilibrate = int(bool(equilibrate))
        o.symmetrize = int(bool(symmetrize))
        o.general_only = int(bool(general_only))
        o.mr_iters = int(mr_iters)
        o.lfil = int(lfil)
        return o

    def spai_build(self, s: float, *, equilibrate=True, symmetrize=True,
                   general_only=False, mr_iters=0, tol=None, lfil=0) -> "Prec":
        """SPAI of K(s); mr_iters > 0 selects the paper's minimal-residual
        column loop (stopping tolerance tol, default 0.01) instead of the exact
        column solves, lfil > 0 its pattern control (at most lfil entries per
        column)."""
        o = self._spai_opts(tol, equilibrate, symmetrize, general_only, mr_iters, lfil)
        h = ctypes.c_void_p()
        self._enter()
        _check(lib().airga_spai_build(self._h, float(s), ctypes.byref(o), ctypes.byref(h)))
        self._leave()
        return Prec(self, h)

    def spai_build_many(self, shifts, *, equilibrate=True, symmetrize=True, general_only=False,
                        mr_iters=0, tol=None, lfil=0) -> list:
        """[SPAI of K(s) for s in shifts], each block's rows staged once per batch."""
        k = len(shifts)
        o = self._spai_opts(tol, equilibrate, symmetrize, general_only, mr_iters, lfil)
        c_s = (ctypes.c_double * max(k, 1))(*[float(v) for v in shifts])
        c_out = (ctypes.c_void_p * max(k, 1))()
        self._enter()
        _check(lib().airga_spai_build_many(self._h, k, c_s, ctypes.byref(o), c_out))
        self._leave()
        return [Prec(self, ctypes.c_void_p(c_out[i])) for i in range(k)]

    def spai_update(self, old: "Prec", s_new: float, *, tol=0.01, equilibrate=True,
                    general_only=False, mr_iters=0, lfil=0) -> "Prec":
        o = self._spai_opts(tol, equilibrate, False, general_only, mr_iters, lfil)
        h = ctypes.c_void_p()
        self._enter()
        _check(lib().airga_spai_update(self._h, old._h, float(s_new), ctypes.byref(o),
                                       ctypes.byref(h)))
        self._leave()
        return Prec(self, h)

    def spai_update_many(self, olds, s_new, *, tol=0.01, equilibrate=True,
                         general_only=False, mr_iters=0, lfil=0) -> list:
        """[update of olds[i] to s_new[i]], the pencil read once per batch."""
        k = len(olds)
        if len(s_new) != k:
            raise ValueError("one new shift per preconditioner")
        o = self._spai_opts(tol, equilibrate, False, general_only, mr_iters, lfil)
        c_old = (ctypes.c_void_p * max(k, 1))(*[p._h.value for p in olds])
        c_s = (ctypes.c_double * max(k, 1))(*[float(v) for v in s_new])
        c_out = (ctypes.c_void_p * max(k, 1))()
        self._enter()
        _check(lib().airga_spai_update_many(self._h, k, c_old, c_s, ctypes.byref(o), c_out))
        self._leave()
        return [Prec(self, ctypes.c_void_p(c_out[i])) for i in range(k)]

    # ---------------------------------------------------------------- solves
    def pcg_solve(self, shifts, precs, F: torch.Tensor, X: torch.Tensor | None = None, *,
                  tol=1e-10, max_iter=20000, mode=MODE_FP64, inner_tol=None, max_sweeps=12,
                  poll_every=8, x0_given=False, use_graph=True, profile=False, tile=None,
                  general_only=False, beta_form=0, inner_max=None):
        """Solve K(s_k) X[k, c] = F[c] for all shifts k and columns c.

        F: (m, n) float64 on the device; X: (nshift, m, n) float64 (allocated
        when None).  precs: list of Prec or None per shift.  Returns
        (X, stats) with stats a list of dicts in (k, c) order.  tile: None (the
        autotuner picks) or (matrix rows per wavefront, systems per group).
        inner_tol / inner_max: None for the library defaults.
        """
        _dev(F, torch.float64, self.device)
        m = F.shape[0]
        shifts = [float(s) for s in shifts]
        nshift = len(shifts)
        if X is None:
            X = torch.empty((nshift, m, self.n), dtype=torch.float64, device=self.device)
        _dev(X, torch.float64, self.device)
        if tuple(X.shape) != (nshift, m, self.n) or tuple(F.shape) != (m, self.n):
            raise ValueError("F must be (m, n) and X (nshift, m, n)")
        if precs is None:
            precs = [None] * nshift
        if len(precs) != nshift:
            raise ValueError("one preconditioner (or None) per shift")
        c_shifts = (ctypes.c_double * nshift)(*shifts)
        c_precs = (ctypes.c_void_p * nshift)(*[p._h.value if p is not None else None for p in precs])
        o = PcgOpts()
        lib().airga_pcg_opts_default(ctypes.byref(o))
        o.tol, o.max_iter, o.mode = float(tol), int(max_iter), int(mode)
        if inner_tol is not None:
            o.inner_tol = float(inner_tol)
        if inner_max is not None:
            o.inner_max = int(inner_max)
        o.max_sweeps, o.poll_every = int(max_sweeps), int(poll_every)
        o.x0_given, o.use_graph, o.profile = int(bool(x0_given)), int(bool(use_graph)), int(bool(profile))
        o.general_only = int(bool(general_only))
        o.beta_form = int(beta_form)
        if tile is not None:
            o.tile_rows, o.tile_sys = int(tile[0]), int(tile[1])
        stats = (SysStats * (nshift * m))()
        self._enter()
        _check(lib().airga_pcg_solve(self._h, nshift, c_shifts, c_precs, m, _ptr(F), self.n,
                                     _ptr(X), self.n, ctypes.byref(o), stats))
        self._leave()
        out = [dict(status=s.status, iters=s.iters, sweeps=s.sweeps, relres=s.relres,
                    finished_fp64=s.finished_fp64) for s in stats]
        return X, out

    def reduce(self, F: torch.Tensor, cp: torch.Tensor, shifts0, *, cv: torch.Tensor | None = None,
               r_max=24, tol_inner=1e-6, tol_outer=1e-6, max_outer=10, update_from=0,
               symmetrize=True, spai_tol=None, mode=MODE_FP64, tol=1e-10, max_iter=20000,
               poll_every=8):
        """AIRGA's outer loop (airga_reduce).  F: (m, n), cp / cv: (p, n)
        float64 device tensors.  Returns a dict: V (r, n) device tensor (the
        basis, row c = column c), the reduced matrices (numpy), the history
        (expansion points, sigmas and per-iteration records) and the final
        change."""
        import numpy as np
        _dev(F, torch.float64, self.device)
        _dev(cp, torch.float64, self.device)
        if cv is not None:
            _dev(cv, torch.float64, self.device)
        m, p, l = F.shape[0], cp.shape[0], len(shifts0)
        o = ReduceOpts()
        lib().airga_reduce_opts_default(ctypes.byref(o))
        o.r_max, o.tol_inner, o.tol_outer = int(r_max), float(tol_inner), float(tol_outer)
        o.max_outer, o.update_from = int(max_outer), int(update_from)
        o.spai.symmetrize = int(bool(symmetrize))
        if spai_tol is not None:
            o.spai.tol = float(spai_tol)
        o.pcg.mode, o.pcg.tol, o.pcg.max_iter = int(mode), float(tol), int(max_iter)
        o.pcg.poll_every = int(poll_every)
        jmax = max(int(r_max) // m, 1)
        V = torch.zeros((max(int(r_max), 1), self.n), dtype=torch.float64, device=self.device)
        rm = max(int(r_max), 1)
        outs = {k: np.zeros(sz) for k, sz in (("mhat", rm * rm), ("khat", rm * rm),
                                               ("fhat", rm * m), ("cphat", p * rm),
                                               ("cvhat", p * rm), ("next_shifts", l))}
        res = ReduceResult()
        for k, arr in outs.items():
            setattr(res, k, ctypes.c_void_p(arr.ctypes.data))
        if cv is None:
            res.cvhat = None
        sh_hist = np.zeros(int(max_outer) * l)
        sg_hist = np.zeros(int(max_outer) * jmax, dtype=np.int32)
        it_hist = (ReduceIter * int(max_outer))()
        c_sh = (ctypes.c_double * l)(*[float(v) for v in shifts0])
        self._enter()
        _check(lib().airga_reduce(self._h, m, _ptr(F), self.n, p, _ptr(cp), _ptr(cv), self.n, l,
                                  c_sh, ctypes.byref(o), _ptr(V), self.n, ctypes.byref(res),
                                  ctypes.c_void_p(sh_hist.ctypes.data),
                                  ctypes.c_void_p(sg_hist.ctypes.data), it_hist))
        self._leave()
        r, z = res.r, res.iterations
        mat = lambda a, rows, cols: a[:rows * cols].reshape(cols, rows).T.copy()  # noqa: E731
        hist = []
        for i in range(z):
            h = it_hist[i]
            sig = [int(v) for v in sg_hist[i * jmax:(i + 1) * jmax] if v >= 0]
            hist.append(dict(shifts=sh_hist[i * l:(i + 1) * l].copy(), sigmas=sig, J=h.blocks,
                             moment_steps=h.moment_steps, updated=bool(h.updated),
                             chain_len_max=h.chain_len_max, max_iters=h.max_iters,
                             all_converged=bool(h.all_converged),
                             change=None if np.isnan(h.change) else h.change,
                             last_inner_change=None if np.isnan(h.last_inner_change)
                             else h.last_inner_change))
        return dict(V=V[:r], r=r, iterations=z, converged=bool(res.converged),
                    change=None if np.isnan(res.change) else res.change,
                    mhat=mat(outs["mhat"], r, r), khat=mat(outs["khat"], r, r),
                    fhat=mat(outs["fhat"], r, m), cphat=mat(outs["cphat"], p, r),
                    cvhat=mat(outs["cvhat"], p, r) if cv is not None else None,
                    next_shifts=outs["next_shifts"].copy(), history=hist)

    # ---------------------------------------------------- complex shifts
    def assemble_shift_complex(self, s: complex) -> torch.Tensor:
        """K(s) entries in CSR order as a complex128 device tensor."""
        out = torch.empty(self.nnz, dtype=torch.complex128, device=self.device)
        s = complex(s)
        self._enter()
        _check(lib().airga_assemble_shift_complex(self._h, s.real, s.imag, _ptr(out)))
        self._leave()
        return out

    def spai_build_complex(self, s: complex, *, equilibrate=True, symmetrize=True,
                           general_only=False) -> "Prec":
        """SPAI of K(s) for a complex expansion point s (general_only: the
        Givens column kernel even where the normal-equation kernel applies)."""
        o = self._spai_opts(None, equilibrate, symmetrize, general_only)
        h = ctypes.c_void_p()
        s = complex(s)
        self._enter()
        _check(lib().airga_spai_build_complex(self._h, s.real, s.imag, ctypes.byref(o),
                                              ctypes.byref(h)))
        self._leave()
        return Prec(self, h)

    def spai_build_complex_many(self, shifts, *, equilibrate=True, symmetrize=True,
                                general_only=False) -> list:
        """spai_build_complex for several complex points in one call."""
        o = self._spai_opts(None, equilibrate, symmetrize, general_only)
        shifts = [complex(z) for z in shifts]
        k = len(shifts)
        c_s = (ctypes.c_double * max(2 * k, 1))(*[v for z in shifts for v in (z.real, z.imag)])
        hs = (ctypes.c_void_p * max(k, 1))()
        self._enter()
        _check(lib().airga_spai_build_complex_many(self._h, k, c_s, ctypes.byref(o), hs))
        self._leave()
        return [Prec(self, ctypes.c_void_p(hs[i])) for i in range(k)]

    def spai_update_complex_many(self, olds, shifts, *, tol=0.01, equilibrate=True,
                                 general_only=False) -> list:
        """spai_update_complex for several (old factor, new point) pairs in one
        call (one synchronisation for all)."""
        o = self._spai_opts(tol, equilibrate, False, general_only)
        shifts = [complex(z) for z in shifts]
        k = len(shifts)
        if len(olds) != k:
            raise ValueError("one old factor per point")
        c_s = (ctypes.c_double * max(2 * k, 1))(*[v for z in shifts for v in (z.real, z.imag)])
        c_o = (ctypes.c_void_p * max(k, 1))(*[p._h.value for p in olds])
        hs = (ctypes.c_void_p * max(k, 1))()
        self._enter()
        _check(lib().airga_spai_update_complex_many(self._h, k, c_o, c_s, ctypes.byref(o), hs))
        self._leave()
        return [Prec(self, ctypes.c_void_p(hs[i])) for i in range(k)]

    def spai_update_complex(self, old: "Prec", s_new: complex, *, tol=0.01,
                            equilibrate=True, general_only=False) -> "Prec":
        """Update of the complex factor old to the complex point s_new
        (general_only: the Givens column kernel only)."""
        o = self._spai_opts(tol, equilibrate, False, general_only)
        h = ctypes.c_void_p()
        s_new = complex(s_new)
        self._enter()
        _check(lib().airga_spai_update_complex(self._h, old._h, s_new.real, s_new.imag,
                                               ctypes.byref(o), ctypes.byref(h)))
        self._leave()
        return Prec(self, h)

    def cocg_solve(self, shifts, precs, F: torch.Tensor, X: torch.Tensor | None = None, *,
                   tol=1e-10, max_iter=20000, poll_every=8, beta_form=0, mode=MODE_FP64,
                   inner_tol=1e-5, inner_max=0, max_sweeps=12):
        """Solve K(s_k) X[k, c] = F[c] for complex shifts s_k by COCG.
        F: (m, n) float64 device tensor; X: (nshift, m, n) complex128
        (allocated when None).  mode MODE_MIXED: float32 inner solves inside
        float64 refinement (inner_tol per sweep, inner_max float32
        iterations per sweep, 0 = the library's default, max_sweeps).
        Returns (X, stats)."""
        _dev(F, torch.float64, self.device)
        m = F.shape[0]
        shifts = [complex(s) for s in shifts]
        nshift = len(shifts)
        if X is None:
            X = torch.empty((nshift, m, self.n), dtype=torch.complex128, device=self.device)
        _dev(X, torch.complex128, self.device)
        if tuple(X.shape) != (nshift, m, self.n) or tuple(F.shape) != (m, self.n):
            raise ValueError("F must be (m, n) and X (nshift, m, n)")
        if precs is None:
            precs = [None] * nshift
        if len(precs) != nshift:
            raise ValueError("one preconditioner (or None) per shift")
        c_shifts = (ctypes.c_double * (2 * nshift))(*[v for s in shifts for v in (s.real, s.imag)])
        c_precs = (ctypes.c_void_p * nshift)(*[p._h.value if p is not None else None for p in precs])
        o = PcgOpts()
        lib().airga_pcg_opts_default(ctypes.byref(o))
        o.tol, o.max_iter, o.poll_every, o.beta_form = float(tol), int(max_iter), int(poll_every), int(beta_form)
        o.mode, o.inner_tol, o.inner_max, o.max_sweeps = int(mode), float(inner_tol), int(inner_max), int(max_sweeps)
        stats = (SysStats * (nshift * m))()
        self._enter()
        _check(lib().airga_cocg_solve(self._h, nshift, c_shifts, c_precs, m, _ptr(F), self.n,
                                      _ptr(X), self.n, ctypes.byref(o), stats))
        self._leave()
        out = [dict(status=s.status, iters=s.iters, relres=s.relres, sweeps=s.sweeps) for s in stats]
        return X, out

    def kernel_times(self) -> dict:
        """{kernel: (launches, total ms)} of the last profiled solve."""
        k = lib().airga_kernel_count()
        launches = (ctypes.c_int64 * k)()
        ms = (ctypes.c_double * k)()
        _check(lib().airga_get_kernel_times(self._h, k, launches, ms))
        return {lib().airga_kernel_name(i).decode(): (launches[i], ms[i]) for i in range(k)}

    def tile_config(self) -> tuple:
        """(matrix rows per wavefront, systems per group) of the last solve."""
        r, u = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().airga_get_tile_config(self._h, ctypes.byref(r), ctypes.byref(u)))
        return r.value, u.value

    def kernel_work(self) -> dict:
        """{kernel: (system passes, shift passes)} of the last profiled solve."""
        k = lib().airga_kernel_count()
        sysp = (ctypes.c_int64 * k)()
        shp = (ctypes.c_int64 * k)()
        _check(lib().airga_get_kernel_work(self._h, k, sysp, shp))
        return {lib().airga_kernel_name(i).decode(): (sysp[i], shp[i]) for i in range(k)}


class Prec:
    """airga_prec handle (released on garbage collection)."""

    def __init__(self, ctx: Context, h: ctypes.c_void_p):
        self.ctx = ctx
        self._h = h
        ctx._precs.add(self)

    def info(self) -> PrecInfo:
        i = PrecInfo()
        _check(lib().airga_get_prec_info(self._h, ctypes.byref(i)))
        return i

    def export_complex(self):
        """(values in CSR order (nnz,) complex128, per-column objective (n,))."""
        c = self.ctx
        vals = torch.empty(c.nnz, dtype=torch.complex128, device=c.device)
        obj = torch.empty(c.n, dtype=torch.float64, device=c.device)
        c._enter()
        _check(lib().airga_prec_export_complex(self._h, _ptr(vals), _ptr(obj)))
        c._leave()
        return vals, obj

    def export(self):
        """(values in CSR order (nnz,), per-column objective (n,)), float64."""
        c = self.ctx
        vals = torch.empty(c.nnz, dtype=torch.float64, device=c.device)
        obj = torch.empty(c.n, dtype=torch.float64, device=c.device)
        c._enter()
        _check(lib().airga_prec_export(self._h, _ptr(vals), _ptr(obj)))
        c._leave()
        return vals, obj

    def skip_flags(self) -> torch.Tensor:
        """(n,) uint8 device tensor: 1 where the update kept column j at
        alpha e_j, 0 where it solved the column (all 0 for a build)."""
        c = self.ctx
        out = torch.empty(c.n, dtype=torch.uint8, device=c.device)
        c._enter()
        _check(lib().airga_prec_skip_flags(self._h, _ptr(out)))
        c._leave()
        return out

    def apply(self, r: torch.Tensor) -> torch.Tensor:
        c = self.ctx
        _dev(r, torch.float64, c.device)
        r2 = r.reshape(-1, c.n)
        z = torch.empty_like(r2)
        c._enter()
        _check(lib().airga_prec_apply(self._h, r2.shape[0], _ptr(r2), c.n, _ptr(z), c.n))
        c._leave()
        return z.reshape(r.shape)

    def release(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().airga_prec_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
