"""The C-ABI library: loads on a CPU-only host, exports every declared symbol,
and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qds.h")
LIB = os.path.join(ROOT, "paper_2609_03550_amd", "libqds.so")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(qds_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libqds.so not built (run __graft_entry__.build())")
    from paper_2609_03550_amd import qds
    return qds.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("qds_init", "qds_step", "qds_destroy", "qds_last_error", "qds_state_bytes",
              "qds_plane_offset", "qds_add_pulse"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_constants_match_the_header():
    """Every option key, tile slot and the tile count the Python binding
    passes equal the header's enum values."""
    from paper_2609_03550_amd import qds
    txt = open(HEADER).read()
    enum = {k: int(v) for k, v in re.findall(r"\b(QDS_(?:OPT|TILE)_\w+|QDS_NTILES)\s*=\s*(\d+)", txt)}
    names = [k for k in dir(qds) if k.startswith(("OPT_", "TILE_")) or k == "NTILES"]
    assert len(names) >= 20
    for k in names:
        assert "QDS_" + k in enum, k
        assert getattr(qds, k) == enum["QDS_" + k], k
    for k in enum:
        assert hasattr(qds, k[4:]), k


def test_init_rejects_bad_arguments(lib):
    from paper_2609_03550_amd import qds
    h = ctypes.c_void_p()
    g = qds.Grid(64, 16, qds.F64, 0, 0, 0, 1.0)
    # c dt != dx
    assert lib.qds_init(ctypes.byref(g), 2, 0.25, 0.3, ctypes.byref(h)) == qds.QDS_ECFL
    assert b"dt" in lib.qds_last_error(None)
    # radial stability bound (dr far too small for the step)
    g2 = qds.Grid(64, 16, qds.F64, 0, 0, 0, 0.05)
    assert lib.qds_init(ctypes.byref(g2), 3, 0.25, 0.25, ctypes.byref(h)) == qds.QDS_ECFL
    # too many modes, tiny grid, regenerated fields without the axion
    assert lib.qds_init(ctypes.byref(g), 9, 0.25, 0.25, ctypes.byref(h)) == qds.QDS_EUNSUPPORTED
    g3 = qds.Grid(4, 16, qds.F64, 0, 0, 0, 1.0)
    assert lib.qds_init(ctypes.byref(g3), 2, 0.25, 0.25, ctypes.byref(h)) == qds.QDS_EINVAL
    g4 = qds.Grid(64, 16, qds.F64, 0, 0, qds.HAS_AREM, 1.0)
    assert lib.qds_init(ctypes.byref(g4), 2, 0.25, 0.25, ctypes.byref(h)) == qds.QDS_EINVAL


def test_layout_queries_on_cpu(lib):
    """Handles without the regenerated set allocate nothing on the device, so
    the layout can be queried on a CPU-only host."""
    from paper_2609_03550_amd import qds
    h = ctypes.c_void_p()
    g = qds.Grid(100, 16, qds.F64, 0, 0, qds.HAS_PLASMA | qds.HAS_AXION, 1.0)
    assert lib.qds_init(ctypes.byref(g), 3, 0.25, 0.25, ctypes.byref(h)) == qds.QDS_OK
    ld = lib.qds_row_pitch(h)
    assert ld % 32 == 0 and ld >= 100
    plane = 3 * 17 * ld * 16
    assert lib.qds_state_bytes(h) == 12 * plane
    assert lib.qds_plane_offset(h, qds.P_TRP) == 0
    assert lib.qds_plane_offset(h, qds.P_JT) == 8 * plane
    assert lib.qds_plane_offset(h, qds.P_SET1) == -1
    assert lib.qds_plane_offset(h, qds.P_PHI) == 9 * plane
    assert lib.qds_step(h, None, None, None, 1, None) == qds.QDS_EINVAL
    st = qds.State()
    assert lib.qds_step(h, ctypes.byref(st), None, None, 1, None) == qds.QDS_ESTATE
    assert lib.qds_destroy(h) == qds.QDS_OK


def test_path_selection_at_the_limits(lib):
    """The fused kernels address a plane with 32-bit byte offsets and run up
    to 8 modes (every mode count qds_init accepts): a plane of exactly 4 GiB
    selects the staged kernels, one row pitch less the fused ones, at 1, 4, 5
    and 8 modes alike.  The largest
    grid qds_init accepts (nx < 2^20, nr < 4096) and the smallest (nx = 8,
    nr = 4) create handles; one beyond either is rejected.  (No device memory
    is needed without the regenerated set.)"""
    from paper_2609_03550_amd import qds

    def handle(nx, nr, modes, dr=8.0):
        h = ctypes.c_void_p()
        g = qds.Grid(nx, nr, qds.F64, 0, 0, 0, dr)
        st = lib.qds_init(ctypes.byref(g), modes, 0.25, 0.25, ctypes.byref(h))
        return st, h

    cases = [((65536, 4095, 1), 0),      # 4096 rows x 65536 x 16 B = 2^32 B
             ((65504, 4095, 1), 1),      # one 32-column pitch less
             ((1000, 50, 5), 1),
             ((1000, 50, 8), 1),
             ((1000, 50, 4), 1),
             ((8, 4, 1), 1)]
    for (nx, nr, m), fused in cases:
        st, h = handle(nx, nr, m)
        assert st == qds.QDS_OK, (nx, nr, m)
        assert lib.qds_row_pitch(h) == (nx + 31) // 32 * 32
        assert lib.qds_uses_fused(h) == fused, (nx, nr, m)
        assert lib.qds_destroy(h) == qds.QDS_OK
    st, h = handle((1 << 20) - 1, 4095, 1)
    assert st == qds.QDS_OK
    assert lib.qds_uses_fused(h) == 0
    assert lib.qds_destroy(h) == qds.QDS_OK
    for nx, nr in ((1 << 20, 100), (100, 4096), (7, 10), (100, 3)):
        st, h = handle(nx, nr, 1)
        assert st == qds.QDS_EINVAL, (nx, nr)


def test_noalloc_loss_rejects_beyond_its_scratch_on_cpu(lib):
    """The allocation-free loss refuses a loss window of more than 65536
    64 x 4 tiles before touching a device (a handle without the regenerated
    set needs no device memory, and the buffer is never dereferenced)."""
    from paper_2609_03550_amd import qds
    h = ctypes.c_void_p()
    g = qds.Grid((1 << 20) - 1, 4095, qds.F64, 0, 0, 0, 8.0)
    assert lib.qds_init(ctypes.byref(g), 1, 0.25, 0.25, ctypes.byref(h)) == qds.QDS_OK
    out = ctypes.c_double()
    lo = qds.Loss(0, 0, 0, (1 << 20) - 1)
    st = lib.qds_loss_eval_noalloc(h, ctypes.c_void_p(64), ctypes.byref(lo), ctypes.byref(out), None)
    assert st == qds.QDS_EINVAL
    assert b"65536" in lib.qds_last_error(h)
    lo = qds.Loss(0, 0, 0, 8)
    lo.mode = 1
    assert lib.qds_loss_eval_noalloc(h, ctypes.c_void_p(64), ctypes.byref(lo), ctypes.byref(out), None) == qds.QDS_EINVAL
    assert lib.qds_destroy(h) == qds.QDS_OK


def test_step_refuses_drive_noise_counter_overflow(lib):
    """The drive noise is keyed on step << 32 | lab column << 12 | row: with
    the moving window, a call whose last lab column would reach 2^20 is
    refused before anything runs (checked on the CPU; the buffers are never
    dereferenced)."""
    from paper_2609_03550_amd import qds
    h = ctypes.c_void_p()
    g = qds.Grid(4096, 16, qds.F64, qds.X_BC["window"], 0, 0, 8.0)
    assert lib.qds_init(ctypes.byref(g), 1, 0.25, 0.25, ctypes.byref(h)) == qds.QDS_OK
    st = qds.State()
    st.buf[0], st.buf[1] = 64, 128
    st.window = (1 << 20) - 4096 - 5
    J = qds.Current()
    J.kind = qds.J_RING
    J.sx = J.sr = 1.0
    # last lab column = 4095 + window + 6 = 2^20
    assert lib.qds_step(h, ctypes.byref(st), ctypes.byref(J), None, 6, None) == qds.QDS_ESTATE
    assert b"2^20" in lib.qds_last_error(h)
    assert lib.qds_destroy(h) == qds.QDS_OK
