"""The C-ABI library loads on a machine without a GPU and exports every
function that include/iblb.h declares.  Only host-side argument validation
is exercised here (no device call is made)."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iblb.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(iblb_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2503_20605_amd import _lib
    return _lib.load()


def test_header_declarations_match_binding():
    from paper_2503_20605_amd import _lib
    assert declared_functions() == sorted(_lib.EXPORTED)


def test_every_declared_symbol_is_exported(lib):
    so = os.path.join(ROOT, "paper_2503_20605_amd", "libiblb.so")
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (iblb_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None
    # nothing else leaks out of the library under an iblb_ name
    assert exported == set(declared_functions())


def test_struct_layouts():
    from paper_2503_20605_amd._lib import iblb_diag, iblb_params
    # int dim, nx, ny, nz, bc[3] (28 bytes) + pad to 8, 4 doubles, 3 ints + pad
    assert ctypes.sizeof(iblb_params) == 32 + 32 + 16
    assert iblb_params.tau.offset == 32
    assert ctypes.sizeof(iblb_diag) % 8 == 0


def _params(**kw):
    from paper_2503_20605_amd import make_params
    return make_params(**kw)


def test_workspace_size_and_validation_on_host(lib):
    from paper_2503_20605_amd._lib import IBLB_EINVAL, iblb_params
    P = (iblb_params * 1)(_params(dim=2, nx=128, ny=64))
    NN = (ctypes.c_int * 1)(128)
    nbytes = lib.iblb_workspace_bytes(1, P, NN, None, 0)
    # two fp32 population copies dominate: 2 * 9 * 128 * 64 * 4 bytes
    assert nbytes >= 2 * 9 * 128 * 64 * 4
    assert lib.iblb_workspace_bytes(1, P, NN, None, 1) < nbytes   # fp16 storage
    bad = (iblb_params * 1)(_params(dim=2, nx=128, ny=64, tau=0.5))
    assert lib.iblb_workspace_bytes(1, bad, NN, None, 0) == 0
    ctx = ctypes.c_void_p()
    rc = lib.iblb_create(1, bad, NN, None, 0, ctypes.c_void_p(256), ctypes.c_size_t(1 << 30),
                         None, ctypes.byref(ctx))
    assert rc == IBLB_EINVAL and not ctx.value
    assert b"tau" in lib.iblb_last_error(None)
    two = (ctypes.c_int * 1)(2)
    assert lib.iblb_workspace_bytes(1, P, two, None, 0) == 0        # < 3 nodes
    p3 = (iblb_params * 1)(_params(dim=3, nx=8, ny=8, nz=8))
    n3 = (ctypes.c_int * 1)(12)
    t3 = (ctypes.c_int * 1)(2)
    assert lib.iblb_workspace_bytes(1, p3, n3, t3, 0) == 0          # < 4 triangles
    assert lib.iblb_workspace_bytes(1, p3, n3, None, 3) == 0        # bad storage
    pinf = (iblb_params * 1)(_params(dim=2, nx=4, ny=4, tau=math.inf))
    z = (ctypes.c_int * 1)(0)
    assert lib.iblb_workspace_bytes(1, pinf, z, None, 0) > 0       # pure streaming is legal


@pytest.mark.parametrize("case,words", [
    ("no droplets", b"n_droplets"),
    ("empty box", b"sizes"),
    ("dim 4", b"dim"),
    ("mixed dims", b"dim"),
    ("too many cells", b"2^31"),
    ("negative node count", b"nodes"),
    ("bad boundary code", b"boundary"),
    ("wetting without xi", b"xi"),
])
def test_degenerate_inputs_rejected_on_host(lib, case, words):
    """Sizing refuses degenerate batches and says why (iblb_last_error(NULL))."""
    from paper_2503_20605_amd._lib import iblb_params
    n, ps, nn = 1, [_params(dim=2, nx=64, ny=32)], [0]
    if case == "no droplets":
        n, ps, nn = 0, [_params(dim=2, nx=64, ny=32)], [0]
    elif case == "empty box":
        ps = [_params(dim=2, nx=0, ny=32)]
    elif case == "dim 4":
        ps = [_params(dim=2, nx=64, ny=32)]
        ps[0].dim = 4
    elif case == "mixed dims":
        n, ps, nn = 2, [_params(dim=2, nx=64, ny=32), _params(dim=3, nx=8, ny=8, nz=8)], [0, 0]
    elif case == "too many cells":
        ps = [_params(dim=2, nx=65536, ny=8192)]          # 9 * 2^29 elements
    elif case == "negative node count":
        nn = [-5]
    elif case == "bad boundary code":
        ps = [_params(dim=2, nx=64, ny=32)]
        ps[0].bc[0] = 7
    elif case == "wetting without xi":
        ps, nn = [_params(dim=2, nx=64, ny=32, xi=0.0)], [40]
    P = (iblb_params * len(ps))(*ps)
    NN = (ctypes.c_int * len(nn))(*nn)
    assert lib.iblb_workspace_bytes(n, P, NN, None, 0) == 0
    assert words in lib.iblb_last_error(None), lib.iblb_last_error(None)

