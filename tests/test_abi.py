"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and its host logic (sizing, argument checks) behaves.
No call here launches GPU work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fv():
    import paper_2510_19301_amd as m
    m.lib()
    return m


def _declared():
    src = open(os.path.join(ROOT, "include", "flashviterbi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fv_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(fv):
    names = _declared()
    assert len(names) >= 10
    h = C.CDLL(fv._lib.LIB_PATH)
    for n in names:
        assert hasattr(h, n), n
    assert set(names) <= set(fv._lib.SIGNATURES), set(names) - set(fv._lib.SIGNATURES)


def test_status_strings(fv):
    l = fv.lib()
    for s in (0, -1, -2, -3, -4, -5, 1):
        assert l.fv_status_str(s)
    assert l.fv_abi_version() == 1


def test_workspace_size_properties(fv):
    d = fv
    K = 1024
    v_short = d.workspace_bytes("vanilla", K, [500])
    v_long = d.workspace_bytes("vanilla", K, [8000])
    f_long = d.workspace_bytes("flash", K, [8000], P=16)
    # vanilla keeps a K x T pointer table; FLASH keeps O(P K) per sequence
    assert v_long - v_short >= (8000 - 500) * K * 2
    big = [8000] * 64
    assert d.workspace_bytes("flash", K, big, P=16) < d.workspace_bytes("vanilla", K, big)
    assert f_long > 0
    # with the slot pool at its cap for both, P only changes the per-sequence division copies
    assert d.workspace_bytes("flash", K, big, P=64) > d.workspace_bytes("flash", K, big, P=2)
    # below the cap the pool follows the leaf-cut task tree: one root and 16
    # leaves of 32 steps for T = 512, P = 16, so FLASH stays near vanilla's size
    f_small = d.workspace_bytes("flash", 512, [512], P=16)
    v_small = d.workspace_bytes("vanilla", 512, [512])
    assert f_small < 2 * v_small
    assert d.workspace_bytes("flash", 512, [512], P=16) < d.workspace_bytes("flash", 512, [512], P=2)


def test_workspace_size_rejects_bad_args(fv):
    d = fv
    with pytest.raises(fv.FvError):
        d.workspace_bytes("vanilla", 0, [10])
    with pytest.raises(fv.FvError):
        d.workspace_bytes("vanilla", 8, [-1])
    with pytest.raises(fv.FvError):
        d.workspace_bytes("vanilla", 70000, [10])


def test_decode_argument_errors_are_synchronous(fv):
    """Invalid arguments are reported before any device work is queued."""
    l = fv.lib()
    m = fv._lib.FvTrans(0, 8, 1, None, None, None, 0)
    fake = 4096
    assert l.fv_decode_vanilla(C.byref(m), None, fake, 8, 0, fake, fake, None, 0, fake, 1 << 20, None) == -1
    assert l.fv_decode_vanilla(C.byref(m), None, fake, 4, 5, fake, fake, None, 0, fake, 1 << 20, None) == -1
    assert l.fv_decode_vanilla(C.byref(m), None, None, 8, 5, fake, fake, None, 0, fake, 1 << 20, None) == -1
    assert l.fv_decode_flash(C.byref(m), None, fake, 8, 0, 4, fake, fake, None, 0, fake, 1 << 20, None) == -1
    # workspace too small is caught on the host
    assert l.fv_decode_vanilla(C.byref(m), None, fake, 8, 5, fake, fake, None, 0, fake, 16, None) == -3
    # malformed CSR descriptors and flags that do not apply to them
    for bad in (fv._lib.FvTrans(1, 8, None, fake, fake, fake, -1),     # nnz < 0
                fv._lib.FvTrans(1, 8, None, None, fake, fake, 3),      # no row_ptr
                fv._lib.FvTrans(1, 8, None, fake, None, fake, 3),      # no col
                fv._lib.FvTrans(7, 8, None, fake, fake, fake, 3)):     # unknown kind
        assert l.fv_decode_vanilla(C.byref(bad), None, fake, 8, 5, fake, fake, None, 0, fake, 1 << 20, None) == -1
    csr = fv._lib.FvTrans(1, 8, None, fake, fake, fake, 3)
    assert l.fv_decode_flash(C.byref(csr), None, fake, 8, 5, 4, fake, fake, None, fv._lib.FV_FLAG_WIDE_ROWS,
                             fake, 1 << 20, None) == -1
    assert l.fv_decode_vanilla(C.byref(csr), None, fake, 8, 5, fake, fake, None, 0, fake, 16, None) == -3
    # the paper's displayed subtask start is offered for dense models only
    rel = fv._lib.FV_FLAG_RELATIVE_INIT
    assert l.fv_decode_flash(C.byref(csr), None, fake, 8, 5, 4, fake, fake, None, rel, fake, 1 << 20, None) == -2
    assert l.fv_decode_flash(C.byref(m), None, fake, 8, 5, 4, fake, fake, None, 1 << 9, fake, 1 << 20, None) == -1
    assert l.fv_last_error()


def test_flash_memory_below_vanilla_at_large_k(fv):
    """FLASH keeps O(P'K) state instead of the K x T backpointer table
    (Sec. V-B): with w-way subtasks (dense K above the leaf limit) its slot
    pool is capped below vanilla's table, so a long sequence needs less
    memory than vanilla's decode."""
    for T in (2000, 10000):
        f = fv.workspace_bytes("flash", 16384, [T], 16, 0)
        v = fv.workspace_bytes("vanilla", 16384, [T], 1, 0)
        assert f < v, (T, f, v)


def test_sparse_workspace_size(fv):
    d = fv
    fake = 4096
    K, nnz = 100000, 900000
    m = fv._lib.FvTrans(1, K, None, fake, fake, fake, nnz)
    lens = [2000] * 4
    v = d.workspace_bytes("vanilla", m, lens)
    f = d.workspace_bytes("flash", m, lens, P=16)
    b = d.workspace_bytes("beam", m, lens, P=16, B=128)
    # the in-edge transpose (pointers + sources + scores + scratch) is part of every sparse plan
    assert f >= (K + 1) * 4 + 3 * nnz * 4
    # vanilla keeps a uint16 in-edge slot per state and step
    assert v >= sum(lens) * K * 2
    assert f < v and b < v
    # no dense beam limit on K for sparse models; B is bounded
    assert d.workspace_bytes("beam", fv._lib.FvTrans(1, 1 << 20, None, fake, fake, fake, 9 << 20), [50],
                             P=4, B=64) > 0
    with pytest.raises(fv.FvError):
        d.workspace_bytes("beam", fv._lib.FvTrans(1, 10000, None, fake, fake, fake, 30), [50], P=4, B=4096)


def test_backward_workspace_size(fv):
    # K*K float totals + K start totals + per-sequence cell lists
    b = fv.backward_workspace_bytes(256, 512, 512)
    assert b >= 256 * 256 * 4 + 512 * 512 * 8
    assert fv.backward_workspace_bytes(256, 0, 0) >= 256 * 256 * 4
    assert fv.backward_workspace_bytes(256, 512, 1024) > b
    for args in ((0, 1, 1), (65536, 1, 1), (4, -1, 1), (4, 1, -1)):
        with pytest.raises(fv.FvError):
            fv.backward_workspace_bytes(*args)
    with pytest.raises(fv.FvError):
        fv.backward_workspace_bytes(4, 1, 16386)   # beyond the per-sequence sort capacity


def test_backward_argument_errors_are_synchronous(fv):
    l = fv.lib()
    fake = C.c_void_p(256)   # never dereferenced: every call below fails on the host
    ws = C.c_void_p(4096)
    # K out of range
    assert l.fv_viterbi_backward(0, 1, 4, fake, fake, fake, None, fake, None, 0, ws, 1 << 30, None) == -1
    # missing inputs with n > 0
    assert l.fv_viterbi_backward(8, 2, 4, None, fake, fake, None, fake, None, 0, ws, 1 << 30, None) == -1
    assert l.fv_viterbi_backward(8, 2, 4, fake, None, fake, fake, None, None, 0, None, 0, None) == -1
    # shared-parameter gradients need the workspace
    assert l.fv_viterbi_backward(8, 2, 4, fake, fake, fake, None, fake, None, 0, None, 0, None) == -3
    assert l.fv_viterbi_backward(8, 2, 4, fake, fake, fake, None, None, fake, 0, ws, 16, None) == -3
    # misaligned workspace
    assert l.fv_viterbi_backward(8, 2, 4, fake, fake, fake, None, fake, None, 0, C.c_void_p(4100), 1 << 30,
                                 None) == -1
    assert l.fv_last_error()


def test_multimodel_workspace_size(fv):
    d = fv
    fake = 4096
    models = (fv._lib.FvTrans * 3)(fv._lib.FvTrans(0, 64, fake, None, None, None, 0),
                                    fv._lib.FvTrans(0, 1024, fake, None, None, None, 0),
                                    fv._lib.FvTrans(1, 5000, None, fake, fake, fake, 45000))
    lens = np.array([100, 2000, 300, 50], np.int32)
    mh = np.array([0, 1, 2, 1], np.int32)
    both = d.workspace_bytes_models("flash", models, 3, lens, mh, 16, 0)
    parts = [d.workspace_bytes_models("flash", (fv._lib.FvTrans * 1)(models[m]), 1, lens[mh == m],
                                              np.zeros((mh == m).sum(), np.int32), 16, 0) for m in range(3)]
    # one region per model (plus the engine's argument table and alignment)
    assert sum(parts) - 3 * 4096 <= both <= sum(parts) + 4096
    # a model without sequences costs nothing
    mh2 = np.array([0, 1, 1, 1], np.int32)
    parts2 = [d.workspace_bytes_models("flash", (fv._lib.FvTrans * 1)(models[m]), 1, lens[mh2 == m],
                                       np.zeros((mh2 == m).sum(), np.int32), 16, 0) for m in range(2)]
    both2 = d.workspace_bytes_models("flash", models, 3, lens, mh2, 16, 0)
    assert sum(parts2) - 2 * 4096 <= both2 <= sum(parts2) + 4096
    l = fv.lib()
    out = C.c_size_t(0)
    # several models need the per-sequence model indices, and they must be in range
    assert l.fv_workspace_size(1, models, 3, lens.ctypes.data, None, 4, 16, 0, C.byref(out)) == -1
    bad = np.array([0, 3, 0, 0], np.int32)
    assert l.fv_workspace_size(1, models, 3, lens.ctypes.data, bad.ctypes.data, 4, 16, 0, C.byref(out)) == -1
    assert l.fv_workspace_size(1, models, 0, lens.ctypes.data, mh.ctypes.data, 4, 16, 0, C.byref(out)) == -1


def test_auto_parallelism_rule(fv):
    """P <= 0 picks the largest power of two in [2, 512] with P <= T/16 for
    the median length: the plan equals the explicit P's plan."""
    d = fv
    for lens, P in (([4000] * 3, 128), ([4250, 100, 9000], 256), ([20], 2), ([31, 64, 64], 4),
                    ([10 ** 6], 512), ([0, 0, 700], 32)):
        assert d.workspace_bytes("flash", 1024, lens, 0) == d.workspace_bytes("flash", 1024, lens, P), (lens, P)
