"""Thin ctypes binding of libnep (include/nep.h).

Argument marshalling only: every step of the moment path runs in the HIP
library.  PyTorch provides device memory (tensor data pointers) and streams.
If the library is missing the import of this module fails loudly; there is
no CPU fallback.
"""
import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnep.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nep.h")

NEP_OK = 0
ERRORS = {-1: "NEP_ERR_ARG", -2: "NEP_ERR_OOM", -3: "NEP_ERR_SINGULAR",
          -4: "NEP_ERR_NOT_HOLOMORPHIC", -5: "NEP_ERR_REFINE", -6: "NEP_ERR_RANK",
          -7: "NEP_ERR_DEVICE", -8: "NEP_ERR_BUSY"}
globals().update({v: k for k, v in ERRORS.items()})  # NEP_ERR_ARG = -1, ...
FN_TYPES = {"rational": 0, "exp": 1, "log": 2, "sqrt": 3, "invsqrt": 4, "phi": 5, "combine": 6}
PREC = {"fp64": 0, "mixed": 1}


class NepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class nep_fn(C.Structure):
    pass


nep_fn._fields_ = [("type", C.c_int), ("alpha", C.c_double * 2), ("beta", C.c_double * 2),
                   ("nnum", C.c_int), ("nden", C.c_int),
                   ("num", C.POINTER(C.c_double)), ("den", C.POINTER(C.c_double)),
                   ("phi_k", C.c_int), ("comb_op", C.c_int),
                   ("comb_a", C.POINTER(nep_fn)), ("comb_b", C.POINTER(nep_fn))]


class nep_mat(C.Structure):
    _fields_ = [("type", C.c_int), ("data", C.c_void_p), ("ld", C.c_longlong), ("on_device", C.c_int)]


class nep_contour(C.Structure):
    _fields_ = [("kind", C.c_int), ("c", C.c_double * 2), ("rho", C.c_double), ("v", C.c_double)]


class nep_ciss_opts(C.Structure):
    _fields_ = [("N", C.c_int), ("L", C.c_int), ("K", C.c_int), ("prec", C.c_int),
                ("max_refine", C.c_int), ("fp64_fallback", C.c_int), ("refine_tol", C.c_double),
                ("stream", C.c_void_p)]


class nep_ciss_stats(C.Structure):
    _fields_ = [("N", C.c_int), ("refine_sweeps", C.c_int), ("n_fallback", C.c_int),
                ("n_unconverged", C.c_int), ("singular_node", C.c_int), ("bad_node", C.c_int),
                ("max_rel_residual", C.c_double), ("ms_total", C.c_float), ("ms_lu", C.c_float),
                ("min_abs_pivot", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class nep_extract_opts(C.Structure):
    _fields_ = [("rank_tol", C.c_double), ("eta_tol", C.c_double), ("max_eigs", C.c_int), ("polish_its", C.c_int)]


class nep_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_longlong), ("max_inflight", C.c_int), ("nstreams", C.c_int)]


class nep_query_info(C.Structure):
    _fields_ = [("status", C.c_int), ("m", C.c_int), ("n_inside", C.c_int), ("reused", C.c_int),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double), ("L_used", C.c_int)]


class nep_tune_cand(C.Structure):
    _fields_ = [("lg", C.c_int), ("paired", C.c_int), ("small_min", C.c_int), ("early_fork", C.c_int),
                ("jb", C.c_int), ("ms", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class nep_nleigs_opts(C.Structure):
    _fields_ = [("sigma", C.c_double * 2), ("k", C.c_int), ("dmax", C.c_int), ("npts", C.c_int),
                ("tol", C.c_double), ("nxi", C.c_int), ("xi", C.POINTER(C.c_double)),
                ("eta_tol", C.c_double), ("max_eigs", C.c_int)]


class nep_nleigs_info(C.Structure):
    _fields_ = [("d", C.c_int), ("met", C.c_int), ("k_done", C.c_int), ("basis", C.c_int),
                ("h_last", C.c_double), ("ms_lu", C.c_float), ("ms_krylov", C.c_float),
                ("ms_total", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def declared_symbols():
    """Function names declared in include/nep.h."""
    with open(HEADER) as fh:
        txt = fh.read()
    return sorted(set(re.findall(r"\b(nep_[a-z0-9_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libnep.so not built ({LIB_PATH}); run paper_1910_11712_amd/build.py")
        # torch first: its HIP runtime must be the one loaded when libnep.so
        # resolves libamdhip64 (tensors handed to the library come from torch)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, ip = C.c_void_p, C.c_int
        L.nep_last_error.restype = C.c_char_p
        L.nep_version.restype = C.c_char_p
        L.nep_split_create.argtypes = [ip, ip, C.POINTER(nep_mat), C.POINTER(nep_fn), vp, C.POINTER(vp)]
        L.nep_split_destroy.argtypes = [C.POINTER(vp)]
        L.nep_split_info.argtypes = [vp, C.POINTER(ip), C.POINTER(ip)]
        L.nep_ciss_moments.argtypes = [vp, C.POINTER(nep_contour), C.POINTER(nep_ciss_opts), vp, vp,
                                       C.POINTER(nep_ciss_stats)]
        L.nep_ciss_wait.argtypes = [vp, C.POINTER(nep_ciss_stats)]
        L.nep_ciss_moments_more.argtypes = [vp, vp, vp, C.c_longlong, C.POINTER(nep_ciss_stats)]
        L.nep_ciss_count.argtypes = [vp, C.POINTER(ip), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.nep_count_eigs.argtypes = [vp, C.POINTER(nep_contour), ip, ip, C.POINTER(ip), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.nep_eigs.argtypes = [vp, C.POINTER(nep_contour), C.POINTER(nep_ciss_opts), C.POINTER(nep_extract_opts), vp,
                               ip, C.POINTER(ip), C.POINTER(C.c_double), vp, C.POINTER(C.c_double), C.POINTER(ip),
                               C.POINTER(C.c_double), C.POINTER(ip), C.POINTER(nep_ciss_stats)]
        L.nep_extract.argtypes = [vp, C.POINTER(nep_contour), C.POINTER(nep_ciss_opts), vp,
                                  C.POINTER(nep_extract_opts), C.POINTER(ip), C.POINTER(C.c_double), vp,
                                  C.POINTER(C.c_double), C.POINTER(ip), C.POINTER(C.c_double)]
        L.nep_backward_error.argtypes = [vp, ip, C.POINTER(C.c_double), vp, C.POINTER(C.c_double)]
        L.nep_backward_error_noalloc.argtypes = [vp, ip, C.POINTER(C.c_double), vp, C.POINTER(C.c_double)]
        L.nep_rii_polish.argtypes = [vp, ip, C.POINTER(C.c_double), vp, C.POINTER(C.c_double), C.c_double, ip,
                                     C.POINTER(ip)]
        L.nep_split_adjoint.argtypes = [vp, C.POINTER(vp)]
        L.nep_left_eigenvectors.argtypes = [vp, ip, C.POINTER(C.c_double), vp, C.POINTER(C.c_double), ip]
        L.nep_apply_resolvent.argtypes = [vp, ip, C.POINTER(C.c_double), vp, vp, C.POINTER(C.c_double), ip, vp, vp]
        L.nep_solve_at.argtypes = [vp, ip, C.POINTER(C.c_double), ip, vp, ip, vp, C.POINTER(nep_ciss_stats)]
        L.nep_fn_eval.argtypes = [vp, ip, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.nep_fn_eval_derivative.argtypes = [vp, ip, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.nep_batch_create.argtypes = [ip, C.POINTER(vp), C.POINTER(nep_contour), C.POINTER(nep_ciss_opts),
                                       C.POINTER(vp), C.POINTER(vp), ip, vp, C.POINTER(vp)]
        L.nep_batch_run.argtypes = [vp, C.POINTER(nep_ciss_stats)]
        L.nep_batch_destroy.argtypes = [C.POINTER(vp)]
        L.nep_batch_wait.argtypes = [vp, C.POINTER(nep_ciss_stats)]
        L.nep_ciss_moments_batch.argtypes = [ip, C.POINTER(vp), C.POINTER(nep_contour), C.POINTER(nep_ciss_opts),
                                             C.POINTER(vp), C.POINTER(vp), C.POINTER(nep_ciss_stats)]
        L.nep_prof_enable.argtypes = [ip]
        L.nep_tune_set.argtypes = [ip, ip]
        L.nep_tune_report.argtypes = [ip, C.POINTER(nep_tune_cand), C.POINTER(ip), C.POINTER(ip), C.POINTER(ip)]
        L.nep_tune_clear.argtypes = []
        L.nep_prof_read.argtypes = [ip, C.POINTER(ip), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.nep_server_create.argtypes = [C.POINTER(nep_server_opts), C.POINTER(vp)]
        L.nep_server_submit.argtypes = [vp, vp, C.POINTER(nep_contour), C.POINTER(nep_ciss_opts),
                                        C.POINTER(nep_extract_opts), vp, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(ip), vp, C.POINTER(C.c_longlong)]
        L.nep_server_submit_pool.argtypes = [vp, vp, C.POINTER(nep_contour), C.POINTER(nep_ciss_opts),
                                             C.POINTER(nep_extract_opts), vp, C.c_int, C.POINTER(C.c_double),
                                             C.POINTER(C.c_double), C.POINTER(ip), vp, C.POINTER(C.c_longlong)]
        L.nep_server_poll.argtypes = [vp, C.c_longlong, C.POINTER(ip), C.POINTER(nep_query_info)]
        L.nep_server_wait.argtypes = [vp, C.c_longlong, C.POINTER(nep_query_info)]
        L.nep_server_clock.argtypes = [vp]
        L.nep_server_clock.restype = C.c_double
        L.nep_server_destroy.argtypes = [C.POINTER(vp)]
        dp = C.POINTER(C.c_double)
        L.nep_nleigs_interp.argtypes = [vp, C.POINTER(nep_contour), C.POINTER(nep_nleigs_opts), C.POINTER(ip),
                                        C.POINTER(ip), dp, dp, dp, dp]
        L.nep_nleigs.argtypes = [vp, C.POINTER(nep_contour), C.POINTER(nep_nleigs_opts), vp, C.POINTER(ip), dp,
                                 vp, dp, dp, C.POINTER(nep_nleigs_info)]
        L.nep_nleigs_batch.argtypes = [ip, C.POINTER(vp), C.POINTER(nep_contour), C.POINTER(nep_nleigs_opts),
                                       C.POINTER(vp), C.POINTER(ip), dp, C.POINTER(vp), dp,
                                       C.POINTER(nep_nleigs_info)]
        _lib = L
    return _lib


def check(code):
    if code != NEP_OK:
        raise NepError(code, lib().nep_last_error().decode())
    return code


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _cplx_array(vals):
    a = np.zeros(2 * max(1, len(vals)), dtype=np.float64)
    for i, v in enumerate(vals):
        a[2 * i], a[2 * i + 1] = complex(v).real, complex(v).imag
    return a


def make_fn(desc, keep):
    """workloads FN descriptor (dict) -> nep_fn; `keep` holds the buffers."""
    f = nep_fn()
    f.type = FN_TYPES[desc["type"]]
    a, b = complex(desc.get("alpha", 1.0)), complex(desc.get("beta", 1.0))
    f.alpha[0], f.alpha[1] = a.real, a.imag
    f.beta[0], f.beta[1] = b.real, b.imag
    if desc["type"] == "rational":
        num, den = _cplx_array(desc["num"]), _cplx_array(desc["den"])
        keep += [num, den]
        f.nnum, f.nden = len(desc["num"]), len(desc["den"])
        f.num = num.ctypes.data_as(C.POINTER(C.c_double))
        f.den = den.ctypes.data_as(C.POINTER(C.c_double))
    elif desc["type"] == "phi":
        f.phi_k = int(desc["k"])
    elif desc["type"] == "combine":
        f.comb_op = int(desc["op"])
        fa, fb = make_fn(desc["a"], keep), make_fn(desc["b"], keep)
        keep += [fa, fb]
        f.comb_a = C.pointer(fa)
        f.comb_b = C.pointer(fb)
    return f


def contour_struct(con):
    g = nep_contour()
    g.kind = int(con.kind)
    g.c[0], g.c[1] = complex(con.c).real, complex(con.c).imag
    g.rho = float(con.rho)
    g.v = float(con.v)
    return g


def opts_struct(N, L, K, prec="mixed", max_refine=None, fallback=True, tol=0.0, stream=None):
    o = nep_ciss_opts()
    o.N, o.L, o.K = int(N), int(L), int(K)
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    if max_refine is None:
        max_refine = 5 if o.prec == PREC["mixed"] else 0
    o.max_refine = int(max_refine)
    o.fp64_fallback = 1 if fallback else 0
    o.refine_tol = float(tol)
    o.stream = stream
    return o


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


# ---------------------------------------------------------------------------
# C-ABI names
# ---------------------------------------------------------------------------

def nep_split_create(mats, fns, stream=None):
    """mats: list of numpy (n x n, float64 or complex128); fns: FN dicts."""
    n = int(mats[0].shape[0])
    ell = len(mats)
    keep = []
    marr = (nep_mat * ell)()
    for i, A in enumerate(mats):
        if np.iscomplexobj(A):
            A = np.asfortranarray(A, dtype=np.complex128)
            marr[i].type = 1
        else:
            A = np.asfortranarray(A, dtype=np.float64)
            marr[i].type = 0
        keep.append(A)
        marr[i].data = A.ctypes.data
        marr[i].ld = n
        marr[i].on_device = 0
    farr = (nep_fn * ell)()
    for i, d in enumerate(fns):
        farr[i] = make_fn(d, keep)
    h = C.c_void_p()
    check(lib().nep_split_create(n, ell, marr, farr, _stream_ptr(stream), C.byref(h)))
    return h


def nep_split_destroy(h):
    hh = C.c_void_p(h.value if isinstance(h, C.c_void_p) else h)
    check(lib().nep_split_destroy(C.byref(hh)))


def nep_ciss_moments(h, contour, opts, V, S, sync=True):
    """V, S: CUDA complex128 tensors (n x L and 2K x L x n views of
    column-major storage, see Split.moments)."""
    st = nep_ciss_stats() if sync else None
    code = lib().nep_ciss_moments(h, C.byref(contour_struct(contour)), C.byref(opts), C.c_void_p(V.data_ptr()),
                                  C.c_void_p(S.data_ptr()), C.byref(st) if st is not None else None)
    check(code)
    return st.as_dict() if st is not None else None


def nep_ciss_moments_more(h, V, S, s_stride=0, offset=0):
    """Moments of the probes V (device (L, n) tensor) on the resident
    factors, written into S's storage from element `offset` with moment
    blocks s_stride elements apart (0: n*L).  Synchronous; returns stats."""
    st = nep_ciss_stats()
    ptr = S.data_ptr() + 16 * int(offset)
    check(lib().nep_ciss_moments_more(h, C.c_void_p(V.data_ptr()), C.c_void_p(ptr), int(s_stride), C.byref(st)))
    return st.as_dict()


def nep_ciss_count(h):
    """(count, max_step, winding) from the resident factors."""
    c, ms, w = C.c_int(0), C.c_double(0), C.c_double(0)
    check(lib().nep_ciss_count(h, C.byref(c), C.byref(ms), C.byref(w)))
    return c.value, ms.value, w.value


def nep_count_eigs(h, contour, N, prec="mixed"):
    c, ms, w = C.c_int(0), C.c_double(0), C.c_double(0)
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    check(lib().nep_count_eigs(h, C.byref(contour_struct(contour)), int(N), p, C.byref(c), C.byref(ms), C.byref(w)))
    return c.value, ms.value, w.value


def nep_eigs(h, contour, opts, V, Lmax, X, max_eigs=64, rank_tol=0.0, eta_tol=0.0, polish_its=0):
    """End to end with probe augmentation.  V: device (Lmax, n) tensor."""
    e = nep_extract_opts()
    e.rank_tol, e.eta_tol, e.max_eigs, e.polish_its = float(rank_tol), float(eta_tol), int(max_eigs), int(polish_its)
    m, lu = C.c_int(0), C.c_int(0)
    lam = np.zeros(2 * max_eigs)
    eta = np.zeros(max_eigs)
    ins = np.zeros(max_eigs, dtype=np.int32)
    sig = np.zeros(opts.K * Lmax)
    st = nep_ciss_stats()
    code = lib().nep_eigs(h, C.byref(contour_struct(contour)), C.byref(opts), C.byref(e), C.c_void_p(V.data_ptr()),
                          int(Lmax), C.byref(m), lam.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(X.data_ptr()),
                          eta.ctypes.data_as(C.POINTER(C.c_double)), ins.ctypes.data_as(C.POINTER(C.c_int)),
                          sig.ctypes.data_as(C.POINTER(C.c_double)), C.byref(lu), C.byref(st))
    k = m.value
    if code != NEP_OK:
        err = NepError(code, lib().nep_last_error().decode())
        err.m, err.L_used = k, lu.value
        raise err
    return {"m": k, "lam": lam[0:2 * k:2] + 1j * lam[1:2 * k:2], "eta": eta[:k].copy(), "inside": ins[:k] == 1,
            "unconverged": ins[:k] == 2, "sigma": sig, "L_used": lu.value, "stats": st.as_dict()}


def nep_ciss_wait(h):
    st = nep_ciss_stats()
    check(lib().nep_ciss_wait(h, C.byref(st)))
    return st.as_dict()


def nep_extract(h, contour, opts, S, X, max_eigs=64, rank_tol=0.0, eta_tol=0.0, polish_its=0):
    """Returns m, lam, eta, inside (inside the contour and converged),
    unconverged (inside with eta > eta_tol) and the singular values."""
    e = nep_extract_opts()
    e.rank_tol, e.eta_tol, e.max_eigs, e.polish_its = float(rank_tol), float(eta_tol), int(max_eigs), int(polish_its)
    m = C.c_int(0)
    lam = np.zeros(2 * max_eigs)
    eta = np.zeros(max_eigs)
    ins = np.zeros(max_eigs, dtype=np.int32)
    sig = np.zeros(opts.K * opts.L)
    code = lib().nep_extract(h, C.byref(contour_struct(contour)), C.byref(opts), C.c_void_p(S.data_ptr()),
                             C.byref(e), C.byref(m), lam.ctypes.data_as(C.POINTER(C.c_double)),
                             C.c_void_p(X.data_ptr()), eta.ctypes.data_as(C.POINTER(C.c_double)),
                             ins.ctypes.data_as(C.POINTER(C.c_int)), sig.ctypes.data_as(C.POINTER(C.c_double)))
    k = m.value
    if code != NEP_OK:
        err = NepError(code, lib().nep_last_error().decode())
        err.m = k
        err.sigma = sig
        raise err
    lam_c = lam[0:2 * k:2] + 1j * lam[1:2 * k:2]
    return {"m": k, "lam": lam_c, "eta": eta[:k].copy(), "inside": ins[:k] == 1, "unconverged": ins[:k] == 2,
            "sigma": sig}


def nep_backward_error(h, lam, X):
    lam = np.asarray(lam, dtype=np.complex128)
    m = len(lam)
    la = np.zeros(2 * m)
    la[0::2], la[1::2] = lam.real, lam.imag
    eta = np.zeros(m)
    check(lib().nep_backward_error(h, m, la.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(X.data_ptr()),
                                   eta.ctypes.data_as(C.POINTER(C.c_double))))
    return eta


def nep_rii_polish(h, lam, X, tol=0.0, max_it=10):
    """Polishes the pairs (lam, columns of the device tensor X (m, n)) in
    place on the device; returns (lam, eta, iters)."""
    lam = np.asarray(lam, dtype=np.complex128)
    m = len(lam)
    la = np.zeros(2 * m)
    la[0::2], la[1::2] = lam.real, lam.imag
    eta = np.zeros(m)
    its = np.zeros(m, dtype=np.int32)
    check(lib().nep_rii_polish(h, m, la.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(X.data_ptr()),
                               eta.ctypes.data_as(C.POINTER(C.c_double)), float(tol), int(max_it),
                               its.ctypes.data_as(C.POINTER(C.c_int))))
    return la[0::2] + 1j * la[1::2], eta, its


def _cplx_host(vals):
    vals = np.asarray(vals, dtype=np.complex128).ravel()
    a = np.zeros(2 * len(vals))
    a[0::2], a[1::2] = vals.real, vals.imag
    return a


def nep_split_adjoint(h):
    out = C.c_void_p()
    check(lib().nep_split_adjoint(h, C.byref(out)))
    return out


def nep_left_eigenvectors(h, lam, Y, max_it=10):
    """Y: device tensor (m, n) of start vectors, overwritten with the left
    eigenvectors; returns (lam, eta)."""
    la = _cplx_host(lam)
    m = len(la) // 2
    eta = np.zeros(m)
    check(lib().nep_left_eigenvectors(h, m, la.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(Y.data_ptr()),
                                      eta.ctypes.data_as(C.POINTER(C.c_double)), int(max_it)))
    return la[0::2] + 1j * la[1::2], eta


def nep_apply_resolvent(h, lam, X, Y, z, V, W):
    """X, Y: device (m, n); V, W: device (L, n) tensors."""
    la = _cplx_host(lam)
    zz = _cplx_host([z])
    L = V.shape[0]
    check(lib().nep_apply_resolvent(h, len(la) // 2, la.ctypes.data_as(C.POINTER(C.c_double)),
                                    C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                    zz.ctypes.data_as(C.POINTER(C.c_double)), int(L), C.c_void_p(V.data_ptr()),
                                    C.c_void_p(W.data_ptr())))


def nep_solve_at(h, z, V, Y, prec="fp64"):
    """V: device (L, n); Y: device (m, L, n) tensor; returns stats."""
    zz = _cplx_host(z)
    st = nep_ciss_stats()
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    check(lib().nep_solve_at(h, len(zz) // 2, zz.ctypes.data_as(C.POINTER(C.c_double)), int(V.shape[0]),
                             C.c_void_p(V.data_ptr()), p, C.c_void_p(Y.data_ptr()), C.byref(st)))
    return st.as_dict()


def nep_backward_error_noalloc(h, lam, X):
    """As nep_backward_error, with the library's fixed device scratch."""
    lam = np.asarray(lam, dtype=np.complex128)
    m = len(lam)
    la = np.zeros(2 * m)
    la[0::2], la[1::2] = lam.real, lam.imag
    eta = np.zeros(m)
    check(lib().nep_backward_error_noalloc(h, m, la.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(X.data_ptr()),
                                           eta.ctypes.data_as(C.POINTER(C.c_double))))
    return eta


def nep_fn_eval(h, ell, z):
    z = np.asarray(z, dtype=np.complex128).ravel()
    m = len(z)
    zi = np.zeros(2 * m)
    zi[0::2], zi[1::2] = z.real, z.imag
    out = np.zeros(2 * m * ell)
    check(lib().nep_fn_eval(h, m, zi.ctypes.data_as(C.POINTER(C.c_double)),
                            out.ctypes.data_as(C.POINTER(C.c_double))))
    return (out[0::2] + 1j * out[1::2]).reshape(ell, m)


def nep_fn_eval_derivative(h, ell, z):
    z = np.asarray(z, dtype=np.complex128).ravel()
    m = len(z)
    zi = np.zeros(2 * m)
    zi[0::2], zi[1::2] = z.real, z.imag
    out = np.zeros(2 * m * ell)
    check(lib().nep_fn_eval_derivative(h, m, zi.ctypes.data_as(C.POINTER(C.c_double)),
                                       out.ctypes.data_as(C.POINTER(C.c_double))))
    return (out[0::2] + 1j * out[1::2]).reshape(ell, m)


def nep_tune_set(on, reps=3):
    check(lib().nep_tune_set(1 if on else 0, int(reps)))


def nep_tune_report(max_cand=32):
    """The last plan's tuning: {"candidates": [dict], "chosen": i, "cached": bool}."""
    arr = (nep_tune_cand * max_cand)()
    n, chosen, cached = C.c_int(), C.c_int(), C.c_int()
    check(lib().nep_tune_report(max_cand, arr, C.byref(n), C.byref(chosen), C.byref(cached)))
    return {"candidates": [arr[i].as_dict() for i in range(min(n.value, max_cand))],
            "chosen": chosen.value, "cached": bool(cached.value)}


def nep_tune_clear():
    check(lib().nep_tune_clear())


def nep_prof_enable(on):
    check(lib().nep_prof_enable(1 if on else 0))


def nep_prof_read(kind):
    """(launches, ms, flops) of the LU trailing-update GEMM launches."""
    n, ms, fl = C.c_int(0), C.c_double(0), C.c_double(0)
    check(lib().nep_prof_read(int(kind), C.byref(n), C.byref(ms), C.byref(fl)))
    return n.value, ms.value, fl.value


# --------------------------------------------------------------------------
# Serving

def nep_server_create(hbm_budget, max_inflight=64, nstreams=4):
    o = nep_server_opts()
    o.hbm_budget, o.max_inflight, o.nstreams = int(hbm_budget), int(max_inflight), int(nstreams)
    s = C.c_void_p()
    check(lib().nep_server_create(C.byref(o), C.byref(s)))
    return s


def nep_server_submit(s, h, contour, opts, V, max_eigs=64, rank_tol=0.0, want_X=False, eta_tol=0.0, polish_its=0):
    """Queues a query.  V: host complex (n, L), or (n, Lmax) with Lmax a
    multiple of L: a probe pool whose further blocks of L columns are used
    when the moment rank saturates (nep_server_submit_pool).  Returns (ticket,
    out) where out holds the host result arrays the server fills; keep it
    until the query is collected."""
    e = nep_extract_opts()
    e.rank_tol, e.eta_tol, e.max_eigs, e.polish_its = float(rank_tol), float(eta_tol), int(max_eigs), int(polish_its)
    Vf = np.asfortranarray(np.asarray(V, dtype=np.complex128))
    n = Vf.shape[0]
    out = {"V": Vf, "lam": np.zeros(2 * max_eigs), "eta": np.zeros(max_eigs),
           "inside": np.zeros(max_eigs, dtype=np.int32),
           "X": np.zeros((n, max_eigs), dtype=np.complex128, order="F") if want_X else None,
           "opts": opts, "eopts": e, "contour": contour_struct(contour)}
    t = C.c_longlong(0)
    xp = C.c_void_p(out["X"].ctypes.data) if want_X else None
    res = (out["lam"].ctypes.data_as(C.POINTER(C.c_double)), out["eta"].ctypes.data_as(C.POINTER(C.c_double)),
           out["inside"].ctypes.data_as(C.POINTER(C.c_int)), xp, C.byref(t))
    if Vf.shape[1] == opts.L:
        check(lib().nep_server_submit(s, h, C.byref(out["contour"]), C.byref(opts), C.byref(e),
                                      C.c_void_p(Vf.ctypes.data), *res))
    else:
        check(lib().nep_server_submit_pool(s, h, C.byref(out["contour"]), C.byref(opts), C.byref(e),
                                           C.c_void_p(Vf.ctypes.data), int(Vf.shape[1]), *res))
    return t.value, out


def _query_result(info, out):
    k = info.m
    lam = out["lam"]
    r = {"status": info.status, "m": k, "n_inside": info.n_inside, "reused": bool(info.reused), "L_used": info.L_used,
         "t_submit": info.t_submit, "t_start": info.t_start, "t_done": info.t_done,
         "lam": lam[0:2 * k:2] + 1j * lam[1:2 * k:2], "eta": out["eta"][:k].copy(),
         "inside": out["inside"][:k] == 1, "unconverged": out["inside"][:k] == 2}
    if out["X"] is not None:
        r["X"] = out["X"][:, :k].copy()
    return r


def nep_server_poll(s, ticket, out):
    done = C.c_int(0)
    info = nep_query_info()
    check(lib().nep_server_poll(s, int(ticket), C.byref(done), C.byref(info)))
    return _query_result(info, out) if done.value else None


def nep_server_wait(s, ticket, out):
    info = nep_query_info()
    check(lib().nep_server_wait(s, int(ticket), C.byref(info)))
    return _query_result(info, out)


def nep_server_clock(s):
    return lib().nep_server_clock(s)


def nep_server_destroy(s):
    check(lib().nep_server_destroy(C.byref(s)))


# --------------------------------------------------------------------------
# Batched moments

def nep_batch_create(handles, contours, opts, Vs, Ss, use_graph=True, stream=None):
    """handles: list of nep_split; contours: list; Vs/Ss: device tensors
    (L, n) and (2K, L, n) complex128.  Returns the batch handle."""
    n = len(handles)
    harr = (C.c_void_p * n)(*[h.value for h in handles])
    garr = (nep_contour * n)(*[contour_struct(c) for c in contours])
    varr = (C.c_void_p * n)(*[v.data_ptr() for v in Vs])
    sarr = (C.c_void_p * n)(*[s.data_ptr() for s in Ss])
    b = C.c_void_p()
    check(lib().nep_batch_create(n, harr, garr, C.byref(opts), varr, sarr, 1 if use_graph else 0,
                                 _stream_ptr(stream), C.byref(b)))
    return b


def nep_batch_run(b, nprob=None):
    """Runs the plan; with nprob the call is synchronous and returns the
    per-problem stats."""
    if nprob is None:
        check(lib().nep_batch_run(b, None))
        return None
    st = (nep_ciss_stats * nprob)()
    check(lib().nep_batch_run(b, st))
    return [s.as_dict() for s in st]


def nep_batch_wait(b, nprob=None):
    """Waits for the last run; with nprob returns the per-problem stats."""
    if nprob is None:
        check(lib().nep_batch_wait(b, None))
        return None
    st = (nep_ciss_stats * nprob)()
    check(lib().nep_batch_wait(b, st))
    return [s.as_dict() for s in st]


def nep_batch_destroy(b):
    check(lib().nep_batch_destroy(C.byref(b)))


def _nleigs_opts(sigma, k, dmax, npts, tol, xi, eta_tol, max_eigs):
    xa = _cplx_host(xi) if xi is not None and len(xi) else None
    o = nep_nleigs_opts()
    o.sigma[0], o.sigma[1] = complex(sigma).real, complex(sigma).imag
    o.k, o.dmax, o.npts, o.tol = int(k), int(dmax), int(npts), float(tol)
    o.nxi = 0 if xa is None else len(xa) // 2
    o.xi = None if xa is None else xa.ctypes.data_as(C.POINTER(C.c_double))
    o.eta_tol, o.max_eigs = float(eta_tol), int(max_eigs)
    return o, xa


def nep_nleigs_interp(h, contour, dmax=50, npts=1024, tol=0.0, xi=()):
    """The NLEIGS interpolant: dict with d, met, sigma, xi, beta (d+1 each)
    and dd (ell x (d+1))."""
    o, xa = _nleigs_opts(0.0, 1, dmax, npts, tol, xi, 0.0, 1)
    D = dmax if dmax > 0 else 50
    n_, ell = C.c_int(), C.c_int()
    check(lib().nep_split_info(h, C.byref(n_), C.byref(ell)))
    sig = np.zeros(2 * (D + 1))
    xo = np.zeros(2 * (D + 1))
    beta = np.zeros(D + 1)
    dd = np.zeros(2 * ell.value * (D + 1))
    d, met = C.c_int(), C.c_int()
    dp = C.POINTER(C.c_double)
    check(lib().nep_nleigs_interp(h, C.byref(contour_struct(contour)), C.byref(o), C.byref(d), C.byref(met),
                                  sig.ctypes.data_as(dp), xo.ctypes.data_as(dp), beta.ctypes.data_as(dp),
                                  dd.ctypes.data_as(dp)))
    del xa
    n = d.value + 1
    ddc = (dd[0::2] + 1j * dd[1::2]).reshape(ell.value, D + 1)[:, :n]
    return {"d": d.value, "met": met.value, "sigma": (sig[0::2] + 1j * sig[1::2])[:n],
            "xi": (xo[0::2] + 1j * xo[1::2])[:n], "beta": beta[:n], "dd": ddc}


def nep_nleigs(h, contour, W0, X, sigma, k, dmax=50, npts=1024, tol=0.0, xi=(), eta_tol=0.0, max_eigs=64,
               want_H=False):
    """NLEIGS eigenpairs.  W0: device tensor (dmax, n) complex128 (row q =
    part w^q of the starting vector); X: device tensor (max_eigs, n) for the
    eigenvectors.  Returns (lam, eta, info dict[, H])."""
    o, xa = _nleigs_opts(sigma, k, dmax, npts, tol, xi, eta_tol, max_eigs)
    m = C.c_int()
    lam = np.zeros(2 * max_eigs)
    eta = np.zeros(max_eigs)
    H = np.zeros(2 * (k + 1) * k) if want_H else None
    info = nep_nleigs_info()
    dp = C.POINTER(C.c_double)
    check(lib().nep_nleigs(h, C.byref(contour_struct(contour)), C.byref(o), C.c_void_p(W0.data_ptr()),
                           C.byref(m), lam.ctypes.data_as(dp), C.c_void_p(X.data_ptr()),
                           eta.ctypes.data_as(dp), None if H is None else H.ctypes.data_as(dp), C.byref(info)))
    del xa
    q = m.value
    out = ((lam[0::2] + 1j * lam[1::2])[:q], eta[:q], info.as_dict())
    if want_H:
        out = out + ((H[0::2] + 1j * H[1::2]).reshape(k, k + 1).T,)
    return out


def nep_nleigs_batch(hs, contours, W0s, Xs, sigmas, k, dmax=50, npts=1024, tol=0.0, xis=None, eta_tol=0.0,
                     max_eigs=16):
    """NLEIGS over many problems in one call.  hs: handles; contours, sigmas,
    xis (singularity points per problem, or None), W0s (device tensors
    (dmax, n_p)) and Xs (device tensors (max_eigs, n_p)) per problem.
    Returns a list of (lam, eta, info dict) per problem."""
    P = len(hs)
    xis = xis if xis is not None else [()] * P
    opts = (nep_nleigs_opts * P)()
    keep = []
    for p in range(P):
        o, xa = _nleigs_opts(sigmas[p], k, dmax, npts, tol, xis[p], eta_tol, max_eigs)
        opts[p] = o
        keep.append(xa)
    harr = (C.c_void_p * P)(*[hh.value if isinstance(hh, C.c_void_p) else hh for hh in hs])
    garr = (nep_contour * P)(*[contour_struct(c) for c in contours])
    warr = (C.c_void_p * P)(*[w.data_ptr() for w in W0s])
    xarr = (C.c_void_p * P)(*[x.data_ptr() for x in Xs])
    m = (C.c_int * P)()
    lam = np.zeros(2 * P * max_eigs)
    eta = np.zeros(P * max_eigs)
    info = (nep_nleigs_info * P)()
    dp = C.POINTER(C.c_double)
    check(lib().nep_nleigs_batch(P, harr, garr, opts, warr, m, lam.ctypes.data_as(dp), xarr,
                                 eta.ctypes.data_as(dp), info))
    del keep
    out = []
    for p in range(P):
        q = m[p]
        lp = lam[2 * p * max_eigs:2 * (p + 1) * max_eigs]
        out.append(((lp[0::2] + 1j * lp[1::2])[:q], eta[p * max_eigs:p * max_eigs + q].copy(), info[p].as_dict()))
    return out
