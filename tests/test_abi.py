"""The C-ABI library loads, exports what include/qless.h declares, and
rejects bad arguments on the host before launching anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2603_20889_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    decl = declared_functions()
    for name in ("qless_tsqr_r", "cholqr2_r", "shifted_cholqr3_r", "svqb", "qless_workspace_bytes",
                 "qless_lstsq_finish"):
        assert name in decl


def test_library_exports_every_declared_symbol():
    lib = q.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(q.EXPORTED) <= set(declared_functions())


def test_status_strings_and_version():
    assert q.version().startswith("qless")
    for st in (0, -1, -2, -3, -4):
        assert q.status_string(st).startswith("QLESS_")


NULL = ctypes.c_void_p(0)
FAKE = ctypes.c_void_p(0x100000)   # never dereferenced: every case fails validation first


@pytest.mark.parametrize("m,n,ldx,R,ldr,expect", [
    (100, 0, 8, FAKE, 8, q.QLESS_ERR_ARG),
    (-1, 4, 4, FAKE, 4, q.QLESS_ERR_ARG),
    (100, 65, 65, FAKE, 65, q.QLESS_ERR_UNSUPPORTED),
    (100, 8, 7, FAKE, 8, q.QLESS_ERR_ARG),
    (100, 8, 8, NULL, 8, q.QLESS_ERR_ARG),
    (100, 8, 8, FAKE, 7, q.QLESS_ERR_ARG),
])
def test_tsqr_argument_errors(m, n, ldx, R, ldr, expect):
    st = q.load().qless_tsqr_r(FAKE, m, n, ldx, R, ldr, NULL, 0, NULL)
    assert st == expect


def test_tsqr_null_x_with_rows_is_an_error():
    assert q.load().qless_tsqr_r(NULL, 10, 4, 4, FAKE, 4, NULL, 0, NULL) == q.QLESS_ERR_ARG


def test_tsqr_workspace_errors():
    lib = q.load()
    need = q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, 10_000_000, 8)
    assert need > 0
    assert lib.qless_tsqr_r(FAKE, 10_000_000, 8, 8, FAKE, 8, NULL, need, NULL) == q.QLESS_ERR_WORKSPACE
    assert lib.qless_tsqr_r(FAKE, 10_000_000, 8, 8, FAKE, 8, FAKE, need - 1, NULL) == q.QLESS_ERR_WORKSPACE
    mis = ctypes.c_void_p(0x100008)
    assert lib.qless_tsqr_r(FAKE, 10_000_000, 8, 8, FAKE, 8, mis, need, NULL) == q.QLESS_ERR_WORKSPACE


def test_workspace_query_rejects_bad_sizes():
    assert q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, 100, 0) == 0
    assert q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, 100, 65) == 0
    assert q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, -5, 4) == 0
    assert q.qless_workspace_bytes(99, 100, 4) == 0


def test_lstsq_argument_errors():
    lib = q.load()
    assert lib.qless_lstsq_finish(NULL, 3, 4, FAKE, NULL, NULL, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_lstsq_finish(FAKE, 3, 3, FAKE, NULL, NULL, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_lstsq_finish(FAKE, 0, 4, FAKE, NULL, NULL, NULL) == q.QLESS_ERR_ARG


def test_timing_read_rejects_unknown_kernel():
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    assert q.load().qless_timing_read(b"nope", ctypes.byref(ms), ctypes.byref(cnt)) == q.QLESS_ERR_ARG


def test_small_problems_plan_one_wavefront():
    """An n x n (or few-panel) TSQR needs no tree, so no workspace beyond the
    minimum -- the SVQB R mode relies on this for its n x n Z, and its own
    workspace also reserves the TSQR slice."""
    for n in (1, 8, 16, 24, 32, 48, 56, 64):
        assert q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, n, n) == 256
    assert (q.qless_workspace_bytes(q.QLESS_METHOD_SVQB, 10_000, 64)
            >= q.qless_workspace_bytes(q.QLESS_METHOD_CHOLQR2, 10_000, 64))
    assert (q.qless_workspace_bytes(q.QLESS_METHOD_SHIFTED_CHOLQR3, 10_000, 64)
            == q.qless_workspace_bytes(q.QLESS_METHOD_CHOLQR2, 10_000, 64) > 0)


def test_update_argument_and_workspace_errors():
    lib = q.load()
    # R is read and written, so it is always required; the update always needs a workspace
    assert lib.qless_tsqr_r_update(FAKE, 100, 4, 4, NULL, 4, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_tsqr_r_update(FAKE, 100, 65, 65, FAKE, 65, FAKE, 1 << 20, NULL) == q.QLESS_ERR_UNSUPPORTED
    need = q.qless_workspace_bytes(q.QLESS_METHOD_TSQR_UPDATE, 0, 8)
    assert need >= 2 * 8 * 8 * 8 * 8 > q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, 0, 8)
    assert lib.qless_tsqr_r_update(NULL, 0, 8, 8, FAKE, 8, NULL, need, NULL) == q.QLESS_ERR_WORKSPACE
    assert lib.qless_tsqr_r_update(FAKE, 10_000, 8, 8, FAKE, 8, FAKE, need - 1, NULL) == q.QLESS_ERR_WORKSPACE


def test_two_phase_argument_errors_on_host():
    lib = q.load()
    # p + n above the kernel limit, negative sizes, missing outputs
    assert lib.qless_two_phase_r(FAKE, 40, 40, FAKE, 100, 30, 30, FAKE, 30, FAKE, 30, FAKE, 1 << 20, NULL) == \
        q.QLESS_ERR_UNSUPPORTED
    assert lib.qless_two_phase_r(FAKE, -1, 4, FAKE, 100, 3, 3, FAKE, 3, FAKE, 3, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_two_phase_r(FAKE, 4, 4, FAKE, 100, 3, 3, NULL, 3, FAKE, 3, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_two_phase_r(FAKE, 4, 3, FAKE, 100, 3, 3, FAKE, 3, FAKE, 3, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_two_phase_r(FAKE, 4, 4, FAKE, 100, 3, 3, FAKE, 3, NULL, 3, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    need = lib.qless_two_phase_workspace_bytes(10_000_000, 4, 3)
    assert need > 0 and lib.qless_two_phase_workspace_bytes(100, 40, 30) == 0
    assert lib.qless_two_phase_r(FAKE, 4, 4, FAKE, 10_000_000, 3, 3, FAKE, 3, FAKE, 3, FAKE, need - 1, NULL) == \
        q.QLESS_ERR_WORKSPACE
    # a leading dimension whose panel would not fit 32-bit byte offsets (width 7:
    # 256-row panels, so ld 2^20 spans 2 GiB), before any launch
    for ldy, ldx in ((1 << 20, 3), (4, 1 << 20)):
        assert lib.qless_two_phase_r(FAKE, 4, ldy, FAKE, 10_000_000, 3, ldx, FAKE, 3, FAKE, 3, FAKE, need,
                                     NULL) == q.QLESS_ERR_UNSUPPORTED


def test_q_from_r_argument_errors_on_host():
    lib = q.load()
    assert lib.qless_q_from_r(FAKE, 100, 4, 4, FAKE, 4, NULL, 4, NULL, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_q_from_r(FAKE, 100, 4, 4, FAKE, 4, FAKE, 3, NULL, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_q_from_r(FAKE, 100, 65, 65, FAKE, 65, FAKE, 65, NULL, FAKE, 1 << 20, NULL) == \
        q.QLESS_ERR_UNSUPPORTED
    need = q.qless_workspace_bytes(q.QLESS_METHOD_Q_FROM_R, 100, 4)
    assert need > 0
    assert lib.qless_q_from_r(FAKE, 100, 4, 4, FAKE, 4, FAKE, 4, NULL, NULL, need, NULL) == q.QLESS_ERR_WORKSPACE
    assert lib.svqb_q(FAKE, 100, 4, 4, NULL, 4, FAKE, 4, NULL, 0.0, NULL, FAKE, 1 << 30, NULL) == q.QLESS_ERR_ARG


def test_running_state_argument_errors_on_host():
    lib = q.load()
    assert lib.qless_tsqr_state_bytes(100, 0) == 0 and lib.qless_tsqr_state_bytes(-1, 4) == 0
    assert lib.qless_tsqr_state_bytes(100, 65) == 0
    need = lib.qless_tsqr_state_bytes(10_000_000, 8)
    assert need >= 8 * 8 * 8
    assert lib.qless_tsqr_state_init(FAKE, need - 1, 10_000_000, 8, NULL) == q.QLESS_ERR_WORKSPACE
    assert lib.qless_tsqr_state_init(NULL, need, 10_000_000, 8, NULL) == q.QLESS_ERR_WORKSPACE
    assert lib.qless_tsqr_state_init(FAKE, need, 10_000_000, 65, NULL) == q.QLESS_ERR_UNSUPPORTED
    assert lib.qless_tsqr_state_fold(NULL, 10, 8, FAKE, need, 10_000_000, 8, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_tsqr_state_fold(FAKE, 10, 7, FAKE, need, 10_000_000, 8, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_tsqr_state_fold(FAKE, 0, 8, FAKE, need, 10_000_000, 8, NULL) == q.QLESS_OK   # nothing to do
    assert lib.qless_tsqr_state_finish(FAKE, need, 10_000_000, 8, NULL, 8, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_tsqr_state_finish(FAKE, need, 10_000_000, 8, FAKE, 7, NULL) == q.QLESS_ERR_ARG


def test_wide_argument_errors_on_host():
    lib = q.load()
    assert lib.qless_wide_workspace_bytes(100, 200, 64) == 0          # m < n
    assert lib.qless_wide_workspace_bytes(1000, 200, 65) == 0
    need = lib.qless_wide_workspace_bytes(1000, 200, 64)
    assert need > 0
    assert lib.qless_wide_r(FAKE, 100, 200, 200, FAKE, 200, FAKE, 200, 64, NULL, FAKE, need, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_wide_r(FAKE, 1000, 200, 200, FAKE, 200, FAKE, 200, 65, NULL, FAKE, need, NULL) == \
        q.QLESS_ERR_UNSUPPORTED
    assert lib.qless_wide_r(FAKE, 1000, 200, 200, FAKE, 200, NULL, 200, 64, NULL, FAKE, need, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_wide_r(FAKE, 1000, 200, 200, FAKE, 200, FAKE, 200, 64, NULL, FAKE, need - 1, NULL) == \
        q.QLESS_ERR_WORKSPACE


def test_gram_entry_points_argument_errors_on_host():
    lib = q.load()
    assert lib.qless_gram(FAKE, 100, 0, 4, FAKE, 4, NULL, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_gram(FAKE, 100, 4, 4, FAKE, 3, NULL, FAKE, 1 << 20, NULL) == q.QLESS_ERR_ARG
    assert lib.qless_gram(FAKE, 100, 65, 65, FAKE, 65, NULL, FAKE, 1 << 20, NULL) == q.QLESS_ERR_UNSUPPORTED
    need = q.qless_workspace_bytes(q.QLESS_METHOD_GRAM, 10_000_000, 8)
    assert need > 0
    assert lib.qless_gram(FAKE, 10_000_000, 8, 8, FAKE, 8, NULL, FAKE, need - 1, NULL) == q.QLESS_ERR_WORKSPACE
    need = q.qless_workspace_bytes(q.QLESS_METHOD_CHOLQR2_DD, 10_000_000, 8)
    assert need > q.qless_workspace_bytes(q.QLESS_METHOD_CHOLQR2, 10_000_000, 8) // 4
    assert lib.cholqr2_dd_r(FAKE, 10_000_000, 8, 8, FAKE, 8, NULL, FAKE, need - 1, NULL) == q.QLESS_ERR_WORKSPACE
    assert lib.cholqr2_dd_r(FAKE, 100, 8, 7, FAKE, 8, NULL, FAKE, need, NULL) == q.QLESS_ERR_ARG


def test_workspace_outdated_by_tuning_is_refused():
    """A workspace sized under one set of launch parameters that is too small
    for the plan under new ones is refused before any launch."""
    lib = q.load()
    m, n = 50_000_000, 8
    old = lib.qless_workspace_bytes(q.QLESS_METHOD_TSQR, m, n)
    try:
        q.qless_tune_set(n, 16, 0, 0)      # twice the stage-1 blocks: more stacked triangles
        assert lib.qless_workspace_bytes(q.QLESS_METHOD_TSQR, m, n) > old
        assert lib.qless_tsqr_r(FAKE, m, n, n, FAKE, n, FAKE, old, NULL) == q.QLESS_ERR_WORKSPACE
    finally:
        q.qless_tune_set(n, 0, 0, 0)
