"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/smg.h, and rejects invalid arguments on the host."""
import ctypes as C
import os
import re

import pytest

from paper_1212_6680_amd import smg as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = S.lib()
    names = _declared()
    assert {"smg_setup", "smg_apply", "pcg_solve", "fpcg_solve", "psd_solve"} <= names
    for n in names:
        assert hasattr(lib, n), n


def _ws(grid, opts, nrhs=1):
    n = C.c_size_t(0)
    rc = S.lib().smg_workspace_bytes(C.byref(grid), C.byref(opts), nrhs, C.byref(n))
    return rc, n.value


def test_workspace_query_and_invalid_arguments():
    g = S.smg_grid(32, 32, 32, 1.0, 1.0, 1.0)
    o = S.smg_opts(1, 0, -1, -1, 0, 0, 0)
    rc, n = _ws(g, o)
    assert rc == 0 and n > 5 * 32 ** 3 * 8
    rc2, n2 = _ws(g, o, 4)
    assert rc2 == 0 and n2 > n
    # FP32 and BF16 hierarchies need less than FP64 for a big batch
    rc3, n3 = _ws(g, S.smg_opts(1, 0, -1, -1, 0, 1, 0), 16)
    rc4, n4 = _ws(g, S.smg_opts(1, 0, -1, -1, 0, 2, 0), 16)
    rc5, n5 = _ws(g, o, 16)
    assert rc3 == rc4 == rc5 == 0 and n4 < n3 < n5
    for bad in [S.smg_grid(0, 4, 4, 1, 1, 1), S.smg_grid(4, -1, 4, 1, 1, 1), S.smg_grid(513, 4, 4, 1, 1, 1),
                S.smg_grid(4, 4, 4, 0.0, 1, 1), S.smg_grid(4, 4, 4, 1, float("nan"), 1)]:
        assert _ws(bad, o)[0] == -1
    for bado in [S.smg_opts(-1, 0, -1, -1, 0, 0, 0), S.smg_opts(1, 9, -1, -1, 0, 0, 0),
                 S.smg_opts(1, 0, -2, -1, 0, 0, 0), S.smg_opts(1, 0, -1, -1, 2, 0, 0),
                 S.smg_opts(1, 0, -1, -1, 0, 3, 0), S.smg_opts(1, 0, -1, -1, 0, 0, 3),
                 S.smg_opts(1, 0, -1, -1, 0, 0, -1)]:
        assert _ws(g, bado)[0] == -1
    assert _ws(g, o, 0)[0] == -1


def test_setup_rejects_small_workspace_before_touching_the_device():
    g = S.smg_grid(16, 16, 16, 1.0, 1.0, 1.0)
    o = S.smg_opts(1, 1, -1, -1, 0, 0, 0)
    rc, n = _ws(g, o)
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)   # never dereferenced: the size check comes first
    assert S.lib().smg_setup(C.byref(g), C.byref(o), 1, fake, n - 1, None, C.byref(h)) == -2
    assert not h.value
    assert S.lib().smg_setup(C.byref(g), C.byref(o), 1, None, n, None, C.byref(h)) == -1


def test_strerror():
    assert S.strerror(0) == "ok"
    assert "workspace" in S.strerror(-2)
    assert S.strerror(12345) == "unknown status"


def test_net_workspace_query_and_invalid_arguments():
    L = S.lib()
    n = C.c_size_t(0)
    assert L.net_workspace_bytes(32 ** 3, 0, 0, C.byref(n)) == 0
    infer = n.value
    assert infer >= 32 ** 3 * (8 + 8 + 2 * 16 * 2)
    assert L.net_workspace_bytes(32 ** 3, 0, 1, C.byref(n)) == 0 and n.value > infer
    assert L.net_workspace_bytes(32 ** 3, 1, 0, C.byref(n)) == 0 and n.value > infer
    for args in [(0, 0, 0), (32, 2, 0), (32, 0, 2), (-5, 1, 1)]:
        assert L.net_workspace_bytes(*args, C.byref(n)) == -1
    h = C.c_void_p()
    buf = (C.c_uint8 * 64)()
    assert L.net_setup(32 ** 3, 0, 0, C.cast(buf, C.c_void_p), 64, None, C.byref(h)) == -2
    assert not h.value
    assert L.net_setup(32 ** 3, 0, 0, None, 1 << 30, None, C.byref(h)) == -1


def _bare_smg(n=1000, max_nrhs=2):
    """An SMG binding object without a device handle: the operand checks run
    before anything reaches the library, so they can be exercised on the CPU."""
    G = object.__new__(S.SMG)
    G.n, G.max_nrhs, G.h = n, max_nrhs, None
    return G


def test_binding_rejects_wrong_operand_sizes_before_any_launch():
    import torch
    G = _bare_smg()
    f64 = torch.float64
    for bad in (torch.zeros(999, dtype=f64), torch.zeros(1001, dtype=f64), torch.zeros(2, 999, dtype=f64),
                torch.zeros(3, 1000, dtype=f64), torch.zeros(1000, 1, dtype=f64), torch.zeros(2, 2, 1000, dtype=f64),
                torch.zeros(2, 1500, dtype=f64)[:, ::2][:, :1000]):
        with pytest.raises(S.SMGError):
            G.apply(bad)
    with pytest.raises(S.SMGError, match="max_nrhs"):
        G.apply(torch.zeros(3, 1000, dtype=f64))
    with pytest.raises(S.SMGError):
        G.matvec(torch.zeros(1001, dtype=f64))
    # outputs must match the input's shape and strides
    r = torch.zeros(2, 1200, dtype=f64)[:, :1000]
    with pytest.raises(S.SMGError, match="differ"):
        G.apply(r, torch.zeros(2, 1000, dtype=f64))
    with pytest.raises(S.SMGError, match="differ"):
        G.matvec(torch.zeros(1000, dtype=f64), torch.zeros(999, dtype=f64))
    # right shapes on a CPU tensor: rejected for the device, after the shape checks
    with pytest.raises(S.SMGError, match="CUDA"):
        G.apply(torch.zeros(1000, dtype=f64))
    # solver vectors must have exactly n entries
    for b in (torch.zeros(999, dtype=f64), torch.zeros(1001, dtype=f64)):
        with pytest.raises(S.SMGError, match="elements"):
            G.fpcg(b)
    with pytest.raises(S.SMGError, match="elements"):
        G.fpcg(torch.zeros(1000, dtype=f64), torch.zeros(1002, dtype=f64))
    # LOBPCG's initial block must be (m + guard, n)
    for X0 in (torch.zeros(4, 999, dtype=f64), torch.zeros(1000, dtype=f64), torch.zeros(1000, 4, dtype=f64)):
        with pytest.raises(S.SMGError, match="X0"):
            G.lobpcg(X0)
    with pytest.raises(S.SMGError, match="max_nrhs"):
        G.lobpcg(torch.zeros(3, 1000, dtype=f64))
    with pytest.raises(S.SMGError, match="wanted"):
        G.lobpcg(torch.zeros(2, 1000, dtype=f64), guard=2)


def test_padded_block_layout_is_accepted():
    import torch
    G = _bare_smg()
    X = torch.zeros(2, 1300, dtype=torch.float64)[:, :1000]
    assert S._block(X, 1000) == (2, 1300)
    assert S._block(torch.zeros(1000, dtype=torch.float64).view(1, 1000), 1000) == (1, 1000)
    Y = S._like(X)
    assert Y.shape == X.shape and Y.stride() == X.stride()
    S._same_layout(X, Y)
