"""CPU-side checks of the C ABI: the library loads, exports every function
include/htred.h declares, and its host-only entry points (defaults,
workspace query, argument validation that needs no device, error strings)
behave as documented.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "htred.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ht_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    import torch  # noqa: F401  (initialise the HIP runtime the same way users do)
    from paper_1710_08538_amd import htred
    if not os.path.exists(htred.LIB_PATH):
        pytest.fail("libhtred.so is not built (run __graft_entry__.build())")
    return htred.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert {"ht_reduce", "ht_reduce_batched", "ht_workspace_size", "ht_default_options",
            "ht_strerror", "ht_version", "ht_batched_workspace_size", "ht_check",
            "ht_wy_gemm", "ht_batched_pencil_stats"} <= set(names)
    for name in names:
        assert hasattr(L, name), name


def test_defaults_and_struct_size(L):
    from paper_1710_08538_amd import htred
    o = htred.Options()
    assert L.ht_default_options(ctypes.byref(o)) == 0
    assert o.struct_size == ctypes.sizeof(htred.Options)
    assert o.nb == 64 and o.max_ir == 10 and o.ir_tol_factor == 2.0
    assert o.batch_block == 32 and o.batch_wg_per_cu == 3


def test_workspace_size_grows_with_n(L):
    from paper_1710_08538_amd import htred
    o = htred.options(nb=64)
    s1 = L.ht_workspace_size(1000, ctypes.byref(o))
    s2 = L.ht_workspace_size(4000, ctypes.byref(o))
    assert 0 < s1 < s2
    bad = htred.options(nb=500)
    assert L.ht_workspace_size(1000, ctypes.byref(bad)) == 0


def test_ell_option(L):
    """l-block absorption (Sec. 3.5): 0 and 2 are the basic scheme; l >= 3
    needs (l - 1) nb <= 128 and adds the diagonal-block LU area (n x (l-1) nb
    doubles and n pivots) to the workspace."""
    from paper_1710_08538_amd import htred
    o = htred.Options()
    L.ht_default_options(ctypes.byref(o))
    assert o.ell == 2
    n = 1000
    base = L.ht_workspace_size(n, ctypes.byref(htred.options(nb=64)))
    assert L.ht_workspace_size(n, ctypes.byref(htred.options(nb=64, ell=0))) == base
    e3 = L.ht_workspace_size(n, ctypes.byref(htred.options(nb=64, ell=3)))
    assert e3 >= base + 8 * n * 128 + 4 * n
    assert L.ht_workspace_size(n, ctypes.byref(htred.options(nb=32, ell=5))) > 0
    for bad in (dict(nb=128, ell=3), dict(nb=64, ell=4), dict(nb=32, ell=6), dict(ell=1),
                dict(ell=-1)):
        assert L.ht_workspace_size(n, ctypes.byref(htred.options(**bad))) == 0, bad


def test_argument_validation_without_device(L):
    from paper_1710_08538_amd import htred
    o = htred.options()
    # negative n, bad leading dimensions, bad struct size: rejected before any device work
    assert L.ht_reduce(None, None, None, None, -1, 1, 1, 1, 1, ctypes.byref(o), None, None, 0, None) == -5
    assert L.ht_reduce(None, None, None, None, 10, 5, 10, 10, 10, ctypes.byref(o), None, None, 0, None) == -6
    assert L.ht_reduce(None, None, None, None, 10, 10, 9, 10, 10, ctypes.byref(o), None, None, 0, None) == -7
    bad = htred.options()
    bad.struct_size = 3
    assert L.ht_reduce(None, None, None, None, 10, 10, 10, 10, 10, ctypes.byref(bad), None, None, 0, None) == -10
    assert L.ht_reduce(None, None, None, None, 10, 10, 10, 10, 10, ctypes.byref(o), None, None, 0, None) == -1
    # n == 0 is a valid no-op
    assert L.ht_reduce(None, None, None, None, 0, 1, 1, 1, 1, ctypes.byref(o), None, None, 0, None) == 0
    # leading dimensions are 32-bit inside the kernels: larger ones are rejected
    big = 1 << 31
    for pos, lds in ((-6, (big, 10, 10, 10)), (-7, (10, big, 10, 10)), (-8, (10, 10, big, 10)),
                     (-9, (10, 10, 10, big))):
        assert L.ht_reduce(None, None, None, None, 10, *lds, ctypes.byref(o), None, None, 0,
                           None) == pos, pos
    # Q, Z not computed: their leading dimensions and pointers are ignored
    none = htred.options(qmode=htred.HT_QZ_NONE, zmode=htred.HT_QZ_NONE)
    assert L.ht_reduce(None, None, None, None, 10, 10, 10, 0, 0, ctypes.byref(none), None, None, 0,
                       None) == -1
    # accumulation needs Q_in / Z_in
    acc = htred.options(qmode=htred.HT_QZ_ACCUMULATE)
    p = ctypes.c_void_p(64)
    assert L.ht_reduce(p, p, None, p, 10, 10, 10, 10, 10, ctypes.byref(acc), None, None, 0,
                       None) == -3


def test_noalloc_argument_validation_without_device(L):
    """ht_reduce_noalloc: the same argument checks as ht_reduce, and orders
    whose workspace exceeds the fixed scratch are refused with
    HT_ERR_TOO_LARGE before any device work."""
    from paper_1710_08538_amd import htred
    o = htred.options(nb=128)
    lim = htred.HT_NOALLOC_SCRATCH_BYTES
    # the largest orders the header states: 2248 (nb 128), 4984 (64), 9958 (32)
    for nb, nmax in ((128, 2248), (64, 4984), (32, 9958)):
        ob = htred.options(nb=nb)
        assert L.ht_workspace_size(nmax, ctypes.byref(ob)) <= lim
        assert L.ht_workspace_size(nmax + 1, ctypes.byref(ob)) > lim
    assert L.ht_reduce_noalloc(None, None, None, None, 2249, 2249, 2249, 2249, 2249,
                               ctypes.byref(o), None, None) == htred.HT_ERR_TOO_LARGE
    assert L.ht_reduce_noalloc(None, None, None, None, -1, 1, 1, 1, 1, ctypes.byref(o), None,
                               None) == -5
    assert L.ht_reduce_noalloc(None, None, None, None, 0, 1, 1, 1, 1, ctypes.byref(o), None,
                               None) == 0
    bad = htred.options()
    bad.struct_size = 3
    assert L.ht_reduce_noalloc(None, None, None, None, 10, 10, 10, 10, 10, ctypes.byref(bad), None,
                               None) == -10
    assert b"scratch" in L.ht_strerror(htred.HT_ERR_TOO_LARGE)


def test_front_end_argument_validation_without_device(L):
    """ht_triangularize_b and ht_preprocess: argument checks before any
    device work; n = 0 is a no-op; split precisions are refused."""
    from paper_1710_08538_amd import htred
    o = htred.options()
    ilo = ctypes.c_int32(7)
    T, P = L.ht_triangularize_b, L.ht_preprocess
    assert T(None, None, None, -1, 1, 1, 1, ctypes.byref(o), None, 0, None) == -5
    assert T(None, None, None, 10, 9, 10, 10, ctypes.byref(o), None, 0, None) == -6
    assert T(None, None, None, 10, 10, 9, 10, ctypes.byref(o), None, 0, None) == -7
    assert T(None, None, None, 10, 10, 10, 9, ctypes.byref(o), None, 0, None) == -8
    assert T(None, None, None, 10, 10, 10, 10, ctypes.byref(o), None, 0, None) == -1
    assert T(None, None, None, 0, 1, 1, 1, ctypes.byref(o), None, 0, None) == 0
    split = htred.options(prec=htred.HT_PREC_SPLIT_BF16)
    assert T(None, None, None, 10, 10, 10, 10, ctypes.byref(split), None, 0, None) == \
        htred.HT_ERR_UNSUPPORTED
    assert P(None, None, None, None, 10, 10, 10, 10, 9, ctypes.byref(o), ctypes.byref(ilo), None,
             0, None) == -9
    p = ctypes.c_void_p(64)
    assert P(p, p, p, None, 10, 10, 10, 10, 10, ctypes.byref(o), ctypes.byref(ilo), None, 0,
             None) == -4
    assert P(p, p, p, p, 10, 10, 10, 10, 10, ctypes.byref(o), None, None, 0, None) == -11
    assert P(None, None, None, None, 0, 1, 1, 1, 1, ctypes.byref(o), ctypes.byref(ilo), None, 0,
             None) == 0 and ilo.value == 0


def test_strerror(L):
    assert L.ht_strerror(0) == b"success"
    assert b"argument" in L.ht_strerror(-3)
    assert L.ht_version().startswith(b"htred")


def test_batched_argument_validation(L):
    from paper_1710_08538_amd import htred
    o = htred.options()
    assert L.ht_batched_workspace_size(4, 513, ctypes.byref(o)) == 0
    assert L.ht_batched_workspace_size(4, 64, ctypes.byref(o)) > 0
    assert L.ht_reduce_batched(-1, None, None, None, None, None, None, None, 64,
                               ctypes.byref(o), None, 0, None) == -1
    assert L.ht_reduce_batched(0, None, None, None, None, None, None, None, 64,
                               ctypes.byref(o), None, 0, None) == 0
    assert L.ht_reduce_batched(3, None, None, None, None, None, None, None, 64,
                               ctypes.byref(o), None, 0, None) == -2
    # batched shape options: 0 = default, out of range rejected; the
    # workspace holds one scratch area per resident workgroup
    for kw in ({"batch_block": 65}, {"batch_block": -1}, {"batch_wg_per_cu": 4},
               {"batch_wg_per_cu": -1}):
        assert L.ht_batched_workspace_size(4, 64, ctypes.byref(htred.options(**kw))) == 0, kw
    zero = htred.options(batch_block=0, batch_wg_per_cu=0)
    assert L.ht_batched_workspace_size(4, 64, ctypes.byref(zero)) == \
        L.ht_batched_workspace_size(4, 64, ctypes.byref(o))
    big = [L.ht_batched_workspace_size(4096, 512, ctypes.byref(htred.options(batch_wg_per_cu=w)))
           for w in (1, 2, 3)]
    assert 0 < big[0] < big[1] < big[2]
    few = [L.ht_batched_workspace_size(3, 512, ctypes.byref(htred.options(batch_wg_per_cu=w)))
           for w in (1, 3)]
    assert few[0] == few[1]  # never more workgroups than pencils


def test_wy_gemm_argument_validation(L):
    z = ctypes.c_void_p(0)
    args = lambda prec=0, ns=0, m=4, n=4, k=4, lda=4, ldb=4, ldc=4, ta=0, tb=0: (
        prec, ns, ta, tb, m, n, k, 1.0, z, lda, z, ldb, 0.0, z, ldc, z)
    assert L.ht_wy_gemm(*args(prec=3)) == -1
    assert L.ht_wy_gemm(*args(prec=1, ns=9)) == -2
    assert L.ht_wy_gemm(*args(prec=2, ns=15)) == -2
    assert L.ht_wy_gemm(*args(prec=1, ns=-1)) == -2
    assert L.ht_wy_gemm(*args(m=-1)) == -5
    assert L.ht_wy_gemm(*args(n=-1)) == -6
    assert L.ht_wy_gemm(*args(k=-1)) == -7
    assert L.ht_wy_gemm(*args(lda=3)) == -10
    assert L.ht_wy_gemm(*args(ta=1, m=8, lda=4, ldc=8)) == -9  # A^T is k x m: lda 4 suffices
    assert L.ht_wy_gemm(*args(ta=1, k=8, lda=4)) == -10
    assert L.ht_wy_gemm(*args(ldb=3)) == -12
    assert L.ht_wy_gemm(*args(tb=1, n=8, ldb=4)) == -12
    assert L.ht_wy_gemm(*args(ldc=3)) == -15
    assert L.ht_wy_gemm(*args(m=0)) == 0  # empty: no pointer needed
    assert L.ht_wy_gemm(*args()) == -9    # NULL A with a non-empty product


def test_split_precision_options(L):
    from paper_1710_08538_amd import htred
    for prec, ok, bad in ((htred.HT_PREC_SPLIT_BF16, (0, 1, 8), (9, -1)),
                          (htred.HT_PREC_SPLIT_FP8, (0, 1, 14), (15,))):
        for ns in ok:
            o = htred.options(prec=prec, n_slices=ns)
            assert L.ht_workspace_size(100, ctypes.byref(o)) > 0
        for ns in bad:
            o = htred.options(prec=prec, n_slices=ns)
            assert L.ht_workspace_size(100, ctypes.byref(o)) == 0
    o = htred.options(prec=3)
    assert L.ht_workspace_size(100, ctypes.byref(o)) == 0
    # the batched form is FP64 only
    o = htred.options(prec=htred.HT_PREC_SPLIT_BF16)
    one = (ctypes.c_int32 * 1)(8)
    ptr = (ctypes.c_void_p * 1)(8)
    info = (ctypes.c_int32 * 1)(0)
    assert L.ht_reduce_batched(1, one, ptr, ptr, ptr, ptr, one, info, 8, ctypes.byref(o),
                               None, 0, None) == htred_unsupported(L)


def htred_unsupported(L):
    for code in range(1, 10):
        if b"unsupported" in L.ht_strerror(code):
            return code
    raise AssertionError("no unsupported-option code")


def test_check_argument_validation(L):
    out = (ctypes.c_double * 4)()
    z = ctypes.c_void_p(0)
    assert L.ht_check(z, z, z, z, z, z, -1, 4, out, z) == -7
    assert L.ht_check(z, z, z, z, z, z, 4, 3, out, z) == -8
    assert L.ht_check(z, z, z, z, z, z, 4, 4, None, z) == -9
    assert L.ht_check(z, z, z, z, z, z, 4, 4, out, z) == -1
    assert L.ht_check(z, z, z, z, z, z, 0, 1, out, z) == 0 and list(out) == [0.0] * 4


def _gpu_count():
    import torch
    return torch.cuda.device_count()  # counts devices without initialising HIP


@pytest.mark.skipif(_gpu_count() > 0, reason="the calls use placeholder pointers: only "
                    "meaningful (and only safe) where no GPU is visible")
def test_compute_calls_fail_without_a_gpu():
    """No CPU fallback: with no device, the compute entry points fail with
    HT_ERR_HIP instead of computing anything on the host.  Run in a child
    process with every GPU hidden as well."""
    import subprocess
    import sys
    code = (
        "import ctypes, sys\n"
        "sys.path.insert(0, %r)\n"
        "from paper_1710_08538_amd import htred\n"
        "L = htred.lib()\n"
        "p = [ctypes.c_void_p(64 * (i + 1)) for i in range(4)]\n"
        "print(L.ht_reduce(p[0], p[1], p[2], p[3], 4, 4, 4, 4, 4, None, None, None, 0, None))\n"
        "print(L.ht_wy_gemm(0, 0, 0, 0, 4, 4, 4, 1.0, p[0], 4, p[1], 4, 0.0, p[2], 4, None))\n"
        "print(L.ht_reduce_noalloc(p[0], p[1], p[2], p[3], 4, 4, 4, 4, 4, None, None, None))\n"
    ) % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", CUDA_VISIBLE_DEVICES="-1",
               ROCR_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    from paper_1710_08538_amd import htred
    assert [int(x) for x in r.stdout.split()] == [htred.HT_ERR_HIP] * 3


def test_return_codes_match_the_header():
    from paper_1710_08538_amd import htred
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "include", "htred.h")).read()
    codes = dict(re.findall(r"#define (HT_(?:OK|ERR_[A-Z_]+))\s+(\d+)", hdr))
    assert len(codes) == 7
    for name, val in codes.items():
        assert getattr(htred, name) == int(val), name


def test_every_declaration_is_documented_and_cited():
    """Each entry point in include/htred.h has its own comment block; those
    that compute something cite the passage of the paper they follow, the
    utilities say that they have none."""
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "include", "htred.h")).read()
    cite = re.compile(r"(Sec\. [0-9]|Algorithm [0-9]|Theorem [A-Z0-9]|Remark [0-9]|Lemma [0-9])")
    names = []
    for m in re.finditer(r"^(?:int|size_t|const char \*)\s*(ht_\w+)\(", hdr, re.M):
        name = m.group(1)
        names.append(name)
        before = hdr[:m.start()]
        end = before.rfind("*/")
        assert end >= 0 and len(before) - end < 400, name  # a comment right above
        block = before[before.rfind("/*", 0, end):end]
        if name in ("ht_strerror", "ht_version"):
            assert "no passage of the paper" in block, name
        elif name == "ht_reduce_noalloc":
            # in place of a citation: the callers it is for
            assert "cannot allocate" in block, name
        else:
            assert cite.search(block), name
    assert len(names) == 13
