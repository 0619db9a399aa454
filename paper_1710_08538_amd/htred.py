"""Thin ctypes binding of libhtred.so (C ABI declared in include/htred.h).

Argument marshalling only: every step of the reduction runs in the HIP
library.  Matrices are torch FP64 CUDA(HIP) tensors in column-major layout
(stride(0) == 1), e.g. ``torch.from_numpy(np.asfortranarray(M)).cuda()``
or ``colmajor_empty(n)``.  The library must be built (``build.py``); if it
is missing or cannot be loaded every call raises -- there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhtred.so")

HT_QZ_IDENTITY, HT_QZ_ACCUMULATE, HT_QZ_NONE = 0, 1, 2
HT_PREC_FP64, HT_PREC_SPLIT_BF16, HT_PREC_SPLIT_FP8 = 0, 1, 2
HT_FLAG_CHECK_FINITE = 1
# return codes (include/htred.h); negative values name an invalid argument
(HT_OK, HT_ERR_HIP, HT_ERR_WORKSPACE, HT_ERR_NONFINITE, HT_ERR_UNSUPPORTED, HT_ERR_NOLIB,
 HT_ERR_TOO_LARGE) = range(7)
HT_NOALLOC_SCRATCH_BYTES = 64 << 20
HT_FLAG_PROFILE = 2
HT_FLAG_SOLVE_SOLO = 4
PROF_CLASSES = ("wy", "trsv", "trmv", "ygemv", "chain", "sweep")


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("max_ir", ctypes.c_int32), ("qmode", ctypes.c_int32),
                ("zmode", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("n_slices", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("ir_tol_factor", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("batch_block", ctypes.c_int32), ("batch_wg_per_cu", ctypes.c_int32),
                ("ilo", ctypes.c_int32), ("ell", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("columns", ctypes.c_int64), ("cols_extra_ir", ctypes.c_int64),
                ("ir_steps", ctypes.c_int64), ("ir_failures", ctypes.c_int64),
                ("absorptions", ctypes.c_int64), ("scaled_solves", ctypes.c_int64),
                ("flops", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("prof_ms", ctypes.c_double * 8), ("prof_work", ctypes.c_double * 8),
                ("prof_launches", ctypes.c_int64 * 8)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name.startswith("prof_") else v
        return d


class HTError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libhtred.so (after torch has initialised its HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HTError("libhtred.so not built: run `python -m paper_1710_08538_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
        L.ht_default_options.argtypes = [ctypes.POINTER(Options)]
        L.ht_default_options.restype = ctypes.c_int
        L.ht_workspace_size.argtypes = [i64, ctypes.POINTER(Options)]
        L.ht_workspace_size.restype = ctypes.c_size_t
        L.ht_reduce.argtypes = [vp, vp, vp, vp, i64, i64, i64, i64, i64,
                                ctypes.POINTER(Options), ctypes.POINTER(Stats), vp,
                                ctypes.c_size_t, vp]
        L.ht_reduce.restype = ctypes.c_int
        L.ht_reduce_noalloc.argtypes = [vp, vp, vp, vp, i64, i64, i64, i64, i64,
                                        ctypes.POINTER(Options), ctypes.POINTER(Stats), vp]
        L.ht_reduce_noalloc.restype = ctypes.c_int
        L.ht_triangularize_b.argtypes = [vp, vp, vp, i64, i64, i64, i64, ctypes.POINTER(Options),
                                         vp, ctypes.c_size_t, vp]
        L.ht_triangularize_b.restype = ctypes.c_int
        L.ht_preprocess.argtypes = [vp, vp, vp, vp, i64, i64, i64, i64, i64,
                                    ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_int32), vp,
                                    ctypes.c_size_t, vp]
        L.ht_preprocess.restype = ctypes.c_int
        L.ht_batched_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(Options)]
        L.ht_batched_workspace_size.restype = ctypes.c_size_t
        L.ht_reduce_batched.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                        ctypes.c_int32, ctypes.POINTER(Options), vp,
                                        ctypes.c_size_t, vp]
        L.ht_reduce_batched.restype = ctypes.c_int
        L.ht_batched_pencil_stats.argtypes = [vp, ctypes.c_int32, vp, vp]
        L.ht_batched_pencil_stats.restype = ctypes.c_int
        L.ht_check.argtypes = [vp, vp, vp, vp, vp, vp, i64, i64, vp, vp]
        L.ht_check.restype = ctypes.c_int
        L.ht_wy_gemm.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 i64, i64, i64, ctypes.c_double, vp, i64, vp, i64,
                                 ctypes.c_double, vp, i64, vp]
        L.ht_wy_gemm.restype = ctypes.c_int
        L.ht_strerror.argtypes = [ctypes.c_int]
        L.ht_strerror.restype = ctypes.c_char_p
        L.ht_version.argtypes = []
        L.ht_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def options(**kw):
    o = Options()
    lib().ht_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    return o


def colmajor_empty(n, m=None, device="cuda"):
    """Uninitialised n x m FP64 tensor with column-major strides (1, n)."""
    m = n if m is None else m
    return torch.empty((m, n), dtype=torch.float64, device=device).t()


def to_device_colmajor(M, device="cuda"):
    """Copy a numpy/torch matrix to a column-major FP64 device tensor."""
    t = torch.as_tensor(M, dtype=torch.float64)
    out = colmajor_empty(t.shape[0], t.shape[1], device=device)
    out.copy_(t)
    return out


def _ld(t, n, name):
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a float64 GPU tensor" % name)
    if tuple(t.shape) != (n, n):
        raise ValueError("%s must be %dx%d" % (name, n, n))
    if n > 0 and t.stride(0) != 1:
        raise ValueError("%s must be column-major (stride(0) == 1)" % name)
    return max(t.stride(1), max(n, 1))


def _check(rc):
    if rc != 0:
        msg = lib().ht_strerror(rc).decode()
        raise HTError("ht_reduce failed: %d (%s)" % (rc, msg))


def _qz(X, mode, n, like, name):
    """Output matrix for qmode/zmode: None (not computed) for HT_QZ_NONE,
    else the caller's tensor (required for HT_QZ_ACCUMULATE) or a new one."""
    if mode == HT_QZ_NONE:
        return None, n if n > 0 else 1
    if X is None:
        if mode == HT_QZ_ACCUMULATE:
            raise ValueError("%s_in is required with HT_QZ_ACCUMULATE" % name)
        X = colmajor_empty(n, device=like.device)
    return X, _ld(X, n, name)


def _reduce_args(A, B, Q, Z, nb, max_ir, ir_tol_factor, seed, prec, n_slices, check_finite,
                 profile, solve_solo, qmode, zmode, ilo=0, ell=2):
    n = A.shape[0]
    lda, ldb = _ld(A, n, "A"), _ld(B, n, "B")
    Q, ldq = _qz(Q, qmode, n, A, "Q")
    Z, ldz = _qz(Z, zmode, n, A, "Z")
    if nb == 0:
        from paper_1710_08538_amd import autotune
        nb = autotune.pick_nb(n)
    o = options(nb=nb, max_ir=max_ir, ir_tol_factor=ir_tol_factor, seed=seed, prec=prec,
                n_slices=n_slices, qmode=qmode, zmode=zmode, ilo=ilo, ell=ell,
                flags=(HT_FLAG_CHECK_FINITE if check_finite else 0)
                | (HT_FLAG_PROFILE if profile else 0)
                | (HT_FLAG_SOLVE_SOLO if solve_solo else 0))
    ptrs = (A.data_ptr(), B.data_ptr(), Q.data_ptr() if Q is not None else None,
            Z.data_ptr() if Z is not None else None, n, lda, ldb, ldq, ldz)
    return Q, Z, o, ptrs


def reduce(A, B, Q=None, Z=None, nb=64, max_ir=10, ir_tol_factor=2.0, seed=0x5EED,
           prec=HT_PREC_FP64, n_slices=0, stats=False, workspace=None, stream=None,
           check_finite=False, profile=False, solve_solo=False, qmode=HT_QZ_IDENTITY,
           zmode=HT_QZ_IDENTITY, ilo=0, ell=2):
    """In-place HouseHT reduction: A -> H, B -> T; returns (Q, Z[, stats]).

    A, B: n x n column-major float64 GPU tensors (B upper triangular).
    Q, Z: optional preallocated outputs (allocated when None); with
        qmode/zmode = HT_QZ_ACCUMULATE they hold Q_in, Z_in and receive
        Q_in Q, Z_in Z; with HT_QZ_NONE they are not computed (None).
    workspace: optional uint8 GPU tensor of >= workspace_size(n) bytes.
    nb: panel width 1..128; 0 takes it from the autotuner's table
        (``autotune.py``) for the nearest order, else the library default.
    solve_solo: run every triangular solve on one workgroup (testing).
    ilo: first column to reduce (columns before it already final, e.g. after
        preprocess()).
    ell: blocks per absorption window; 2 = the basic scheme, >= 3 the
        accelerated absorption with block upper triangular B ((ell-1) nb <= 128).
    """
    Q, Z, o, ptrs = _reduce_args(A, B, Q, Z, nb, max_ir, ir_tol_factor, seed, prec, n_slices,
                                 check_finite, profile, solve_solo, qmode, zmode, ilo, ell)
    st = Stats()
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    rc = lib().ht_reduce(*ptrs, ctypes.byref(o), ctypes.byref(st) if stats else None,
                         ws_ptr, ws_bytes, s.cuda_stream)
    _check(rc)
    if stats:
        return Q, Z, st.as_dict()
    return Q, Z


def reduce_noalloc(A, B, Q=None, Z=None, nb=64, max_ir=10, ir_tol_factor=2.0, seed=0x5EED,
                   prec=HT_PREC_FP64, n_slices=0, stats=False, stream=None,
                   check_finite=False, solve_solo=False, qmode=HT_QZ_IDENTITY,
                   zmode=HT_QZ_IDENTITY, ilo=0, ell=2):
    """ht_reduce_noalloc: as reduce(), with the library's fixed device
    scratch in place of a workspace (no allocation inside the call; pass Q
    and Z to keep this wrapper from allocating them)."""
    Q, Z, o, ptrs = _reduce_args(A, B, Q, Z, nb, max_ir, ir_tol_factor, seed, prec, n_slices,
                                 check_finite, False, solve_solo, qmode, zmode, ilo, ell)
    st = Stats()
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    rc = lib().ht_reduce_noalloc(*ptrs, ctypes.byref(o), ctypes.byref(st) if stats else None,
                                 s.cuda_stream)
    _check(rc)
    if stats:
        return Q, Z, st.as_dict()
    return Q, Z


def triangularize_b(A, B, Q=None, nb=64, qmode=HT_QZ_IDENTITY, workspace=None, stream=None):
    """ht_triangularize_b: B <- R = Q0^T B (upper triangular), A <- Q0^T A;
    returns Q (Q0, or Q_in Q0 with HT_QZ_ACCUMULATE; None with HT_QZ_NONE)."""
    n = A.shape[0]
    lda, ldb = _ld(A, n, "A"), _ld(B, n, "B")
    Q, ldq = _qz(Q, qmode, n, A, "Q")
    o = options(nb=nb, qmode=qmode)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    _check(lib().ht_triangularize_b(A.data_ptr(), B.data_ptr(),
                                    Q.data_ptr() if Q is not None else None, n, lda, ldb, ldq,
                                    ctypes.byref(o), ws_ptr, ws_bytes, s.cuda_stream))
    return Q


def preprocess(A, B, Q=None, Z=None, nb=64, qmode=HT_QZ_IDENTITY, zmode=HT_QZ_IDENTITY,
               workspace=None, stream=None):
    """ht_preprocess (zero columns of B moved to the front, Sec. 3.5); returns
    (Q, Z, ilo).  Follow with reduce(A, B, Q, Z, ilo=ilo,
    qmode=HT_QZ_ACCUMULATE, zmode=HT_QZ_ACCUMULATE)."""
    n = A.shape[0]
    lda, ldb = _ld(A, n, "A"), _ld(B, n, "B")
    Q, ldq = _qz(Q, qmode, n, A, "Q")
    Z, ldz = _qz(Z, zmode, n, A, "Z")
    o = options(nb=nb, qmode=qmode, zmode=zmode)
    ilo = ctypes.c_int32(0)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    _check(lib().ht_preprocess(A.data_ptr(), B.data_ptr(), Q.data_ptr() if Q is not None else None,
                               Z.data_ptr() if Z is not None else None, n, lda, ldb, ldq, ldz,
                               ctypes.byref(o), ctypes.byref(ilo), ws_ptr, ws_bytes,
                               s.cuda_stream))
    return Q, Z, ilo.value


class BatchedPlan:
    """Device-side argument arrays and workspace for ht_reduce_batched over a
    fixed list of column-major pencils (A_i, B_i, Q_i, Z_i share ld_i).  The
    arrays stay alive with the plan, so `run` may be captured in a hipGraph."""

    def __init__(self, As, Bs, Qs, Zs, max_ir=10, ir_tol_factor=2.0, seed=0x5EED, nb=None,
                 block=None, wg_per_cu=None):
        dev = As[0].device if As else torch.device("cuda")
        self.batch = len(As)
        ns, lds = [], []
        for A, B, Q, Z in zip(As, Bs, Qs, Zs):
            n = A.shape[0]
            ld = _ld(A, n, "A")
            for M, name in ((B, "B"), (Q, "Q"), (Z, "Z")):
                if M.shape[0] != n or _ld(M, n, name) != ld:
                    raise ValueError("pencil matrices must share order and leading dimension")
            ns.append(n)
            lds.append(ld)
        self.nmax = max(ns) if ns else 0
        i32 = dict(dtype=torch.int32, device=dev)
        i64 = dict(dtype=torch.int64, device=dev)
        self.n = torch.tensor(ns, **i32)
        self.ld = torch.tensor(lds, **i32)
        self.pA = torch.tensor([t.data_ptr() for t in As], **i64)
        self.pB = torch.tensor([t.data_ptr() for t in Bs], **i64)
        self.pQ = torch.tensor([t.data_ptr() for t in Qs], **i64)
        self.pZ = torch.tensor([t.data_ptr() for t in Zs], **i64)
        self.info = torch.zeros(max(self.batch, 1), **i32)
        # nb: panel width of every pencil's reduction (0: one panel per pencil);
        # block: reflectors per block of B's re-triangularisation; wg_per_cu:
        # resident workgroups per compute unit.  None: the autotuned value
        # (autotune.py), else the library default.
        from paper_1710_08538_amd import autotune
        tuned = autotune.pick_batched()
        self.nb = tuned["nb"] if nb is None else nb
        self.block = tuned["block"] if block is None else block
        self.wg_per_cu = tuned["wg_per_cu"] if wg_per_cu is None else wg_per_cu
        self.opt = options(max_ir=max_ir, ir_tol_factor=ir_tol_factor, seed=seed, nb=self.nb,
                           batch_block=self.block, batch_wg_per_cu=self.wg_per_cu)
        nbytes = lib().ht_batched_workspace_size(self.batch, self.nmax, ctypes.byref(self.opt))
        if nbytes == 0:
            raise HTError("invalid batched sizes or options (orders must be <= 512)")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.keep = (As, Bs, Qs, Zs)

    def run(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        rc = lib().ht_reduce_batched(self.batch, self.n.data_ptr(), self.pA.data_ptr(),
                                     self.pB.data_ptr(), self.pQ.data_ptr(), self.pZ.data_ptr(),
                                     self.ld.data_ptr(), self.info.data_ptr(), self.nmax,
                                     ctypes.byref(self.opt), self.ws.data_ptr(),
                                     self.ws.numel(), s.cuda_stream)
        _check(rc)

    def pencil_stats(self, stream=None):
        """Per-pencil record of the last run as a host int64 tensor of shape
        (batch, 8): start_ns, end_ns, panels, ir_steps, solve_ns, residual_ns,
        absorb_ns, retriangularise_ns.  Waits for the stream."""
        s = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        out = torch.zeros((max(self.batch, 1), 8), dtype=torch.int64)
        _check(lib().ht_batched_pencil_stats(self.ws.data_ptr(), self.batch, out.data_ptr(),
                                             s.cuda_stream))
        return out[:self.batch]


def reduce_batched(As, Bs, Qs=None, Zs=None, **kw):
    """Batched HouseHT of small pencils (orders <= 512) in one persistent launch:
    A_i -> H_i, B_i -> T_i in place; returns (Qs, Zs, info)."""
    if Qs is None:
        Qs = [colmajor_empty(A.shape[0], device=A.device) for A in As]
    if Zs is None:
        Zs = [colmajor_empty(A.shape[0], device=A.device) for A in As]
    plan = BatchedPlan(As, Bs, Qs, Zs, **kw)
    plan.run()
    return Qs, Zs, plan.info[:len(As)].clone()


def _colmajor_ld(t, rows, cols, name):
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a float64 GPU tensor" % name)
    if tuple(t.shape) != (rows, cols):
        raise ValueError("%s must be %dx%d" % (name, rows, cols))
    if rows > 0 and cols > 0 and t.stride(0) != 1:
        raise ValueError("%s must be column-major (stride(0) == 1)" % name)
    return max(t.stride(1) if cols > 1 else rows, rows, 1)


def wy_gemm(A, B, C=None, transA=False, transB=False, alpha=1.0, beta=0.0, prec=HT_PREC_FP64,
            n_slices=0, stream=None):
    """One WY-update product as ht_reduce forms it for `prec`:
    C = alpha op(A) op(B) + beta C on column-major float64 GPU tensors.
    Returns C (allocated when None)."""
    ra, ca = A.shape
    rb, cb = B.shape
    m, k = (ca, ra) if transA else (ra, ca)
    k2, n = (cb, rb) if transB else (rb, cb)
    if k != k2:
        raise ValueError("inner dimensions differ: %d vs %d" % (k, k2))
    lda = _colmajor_ld(A, ra, ca, "A")
    ldb = _colmajor_ld(B, rb, cb, "B")
    if C is None:
        C = colmajor_empty(m, n, device=A.device)
        beta = 0.0
    ldc = _colmajor_ld(C, m, n, "C")
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    _check(lib().ht_wy_gemm(prec, n_slices, int(transA), int(transB), m, n, k, alpha,
                            A.data_ptr(), lda, B.data_ptr(), ldb, beta, C.data_ptr(), ldc,
                            s.cuda_stream))
    return C


def check(A0, B0, H, T, Q, Z, stream=None):
    """Backward errors and orthogonality of a reduction, computed on the
    device (ht_check): dict with bwd_A, bwd_B, orth_Q, orth_Z.  All six
    matrices n x n column-major float64 GPU tensors with one leading
    dimension."""
    n = A0.shape[0]
    ld = _ld(A0, n, "A0")
    for M, name in ((B0, "B0"), (H, "H"), (T, "T"), (Q, "Q"), (Z, "Z")):
        if _ld(M, n, name) != ld:
            raise ValueError("all matrices must share the leading dimension")
    out = (ctypes.c_double * 4)()
    s = stream if stream is not None else torch.cuda.current_stream(A0.device)
    _check(lib().ht_check(A0.data_ptr(), B0.data_ptr(), H.data_ptr(), T.data_ptr(),
                          Q.data_ptr(), Z.data_ptr(), n, ld, out, s.cuda_stream))
    return {"bwd_A": out[0], "bwd_B": out[1], "orth_Q": out[2], "orth_Z": out[3]}


def workspace_size(n, nb=64, ell=2):
    return lib().ht_workspace_size(n, ctypes.byref(options(nb=nb, ell=ell)))


def version():
    return lib().ht_version().decode()
