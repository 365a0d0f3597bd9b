"""CPU checks of the C ABI: the library loads and exports every function
include/ebic.h declares (no compute call; no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(ebic_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_entry_points():
    names = _declared()
    for n in ("ebic_matrix_prepare", "ebic_evaluate", "ebic_support_rows", "ebic_version",
              "ebic_last_error", "ebic_population_upload", "ebic_matrix_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2105_01196_amd import ebic
    L = ebic.lib()
    missing = [n for n in sorted(_declared()) if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2105_01196_amd import ebic
    assert _declared() <= set(ebic._SIGNATURES), _declared() - set(ebic._SIGNATURES)


def test_host_only_calls():
    from paper_2105_01196_amd import ebic
    assert ebic.ebic_version() == 200
    assert ebic.ebic_matrix_bytes(100, 20) == 20 * 128 * 2
    assert ebic.ebic_matrix_bytes(0, 20) == 0
    # pair rows: 64-bit row words rounded up to 16 (128-byte lines)
    assert [ebic.ebic_pairs_words(r) for r in (0, 1, 64, 1024, 1025, 10000)] == \
        [0, 16, 16, 16, 32, 160]
    assert ebic.ebic_pairs_bytes(10000, 500) == 500 * 499 // 2 * 160 * 8
    assert ebic.ebic_pairs_bytes(100, 1) == 0


def test_population_validation_rejects_on_host():
    """Host-side validation runs before any device call."""
    import numpy as np
    from paper_2105_01196_amd import ebic
    L = ebic.lib()
    for off, cols in (([0, 1], [3]), ([0, 2], [3, 3]), ([0, 2], [3, 20]), ([1, 3], [0, 1])):
        o = np.array(off, np.int32)
        c = np.array(cols, np.uint16)
        rc = L.ebic_population_upload(o.ctypes.data, c.ctypes.data, 1, 10, 0x1000, 0x1000, None)
        assert rc == ebic.EBIC_ERR_INVALID_ARG
        assert L.ebic_last_error()


def test_evaluate_rejects_bad_arguments_on_host():
    from paper_2105_01196_amd import ebic
    L = ebic.lib()
    m = ebic.ebic_matrix(0x1000, 100, 20, 128, None)
    pop = ebic.ebic_population(0, 0, None, None)
    out = ebic.ebic_eval_out(None, None, None, None)
    arch = ebic.ebic_archive(65, 0, 0x1000, 0x1000, 0x1000)
    p = ebic.make_params()
    assert L.ebic_evaluate(ctypes.byref(m), ctypes.byref(pop), ctypes.byref(arch),
                           ctypes.byref(p), ctypes.byref(out), None) == ebic.EBIC_ERR_INVALID_ARG
    bad_m = ebic.ebic_matrix(0x1000, 100, 20, 100, None)  # rows_pad not a multiple of 64
    arch0 = ebic.ebic_archive(0, 0, None, None, None)
    assert L.ebic_evaluate(ctypes.byref(bad_m), ctypes.byref(pop), ctypes.byref(arch0),
                           ctypes.byref(p), ctypes.byref(out), None) == ebic.EBIC_ERR_INVALID_ARG
    bad_p = ebic.make_params(approx_permille=1001)
    assert L.ebic_evaluate(ctypes.byref(m), ctypes.byref(pop), ctypes.byref(arch0),
                           ctypes.byref(bad_p), ctypes.byref(out), None) == ebic.EBIC_ERR_INVALID_ARG


def test_run_rejects_bad_parameters_on_host():
    import numpy as np
    from paper_2105_01196_amd import ebic
    L = ebic.lib()
    X = np.zeros((10, 5), np.float32)
    res = ctypes.POINTER(ebic.ebic_result)()
    for bad in (dict(k_min=1), dict(k_max=6), dict(k_min=4, k_max=3), dict(population=0),
                dict(archive_size=65), dict(tournament=0), dict(max_tabu_hits=0),
                dict(generations=0), dict(approx_permille=-1),
                dict(op_permille=[200, 200, 200, 200, 199]), dict(op_permille=[-1, 201, 200, 200, 400]),
                dict(op_permille=[1001, 0, 0, 0, -1])):
        p = ebic.make_params(**{**dict(k_min=2, k_max=4), **bad})
        rc = L.ebic_run(X.ctypes.data, 10, 5, ctypes.byref(p), 1, None, None, ctypes.byref(res))
        assert rc == ebic.EBIC_ERR_INVALID_ARG, bad


def test_batch_set_tuning_rejects_null_batch_on_host():
    from paper_2105_01196_amd import ebic
    L = ebic.lib()
    assert L.ebic_batch_set_tuning(None, 1, 2, 1) == ebic.EBIC_ERR_INVALID_ARG
    assert L.ebic_last_error()


def test_session_restore_rejects_malformed_checkpoints_on_host():
    """A checkpoint is checked (magic, version, shape, matrix hash, length)
    before any device work, so these fail on a machine without a GPU."""
    import numpy as np
    from paper_2105_01196_amd import ebic
    L = ebic.lib()
    X = np.zeros((10, 5), np.float32)
    h = ctypes.c_void_p()
    for blob in (b"", b"EBICCKP1", b"NOTACKPT" + bytes(200), bytes(300)):
        buf = ctypes.create_string_buffer(blob, max(len(blob), 1))
        rc = L.ebic_session_restore(X.ctypes.data, 10, 5, buf, len(blob), None, None,
                                    ctypes.byref(h))
        assert rc == ebic.EBIC_ERR_INVALID_ARG, blob[:8]
        assert L.ebic_last_error()
    assert L.ebic_session_step(None, 1, None) == ebic.EBIC_ERR_INVALID_ARG
    n = ctypes.c_size_t(0)
    assert L.ebic_session_checkpoint(None, None, ctypes.byref(n)) == ebic.EBIC_ERR_INVALID_ARG
    res = ctypes.POINTER(ebic.ebic_result)()
    assert L.ebic_session_result(None, ctypes.byref(res)) == ebic.EBIC_ERR_INVALID_ARG
    L.ebic_session_free(None)
