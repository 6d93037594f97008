"""The C-ABI library on the host: it loads, exports what include/fcm.h declares,
and rejects invalid arguments before any HIP call (no GPU needed)."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_1601_00072_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcm.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1601_00072_amd import build
        build.build()
    return L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(fcm_\w+)\s*\(", text))


def test_header_matches_binding_table():
    assert declared_functions() == set(L.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fcm_\w+)", out))
    assert declared_functions() <= exported
    for name in declared_functions():
        assert getattr(lib, name) is not None


def test_version_and_strerror(lib):
    assert lib.fcm_version() == 10100
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        assert lib.fcm_strerror(code) != b"unknown status"
    assert lib.fcm_strerror(12345) == b"unknown status"


def _params(**kw):
    d = dict(n_clusters=4, m=2.0, eps=1e-5, max_iter=300, init=L.FCM_INIT_LINSPACE,
             init_centroids=None, flags=0)
    d.update(kw)
    return L.FcmParams(**d)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first


@pytest.mark.parametrize("kw", [
    dict(n_clusters=1), dict(n_clusters=9), dict(n_clusters=-3),
    dict(m=1.0), dict(m=0.5), dict(m=math.nan), dict(m=math.inf),
    dict(eps=0.0), dict(eps=-1.0), dict(eps=math.nan), dict(eps=math.inf),
    dict(max_iter=0), dict(max_iter=-5),
    dict(init=7), dict(init=L.FCM_INIT_GIVEN),
    dict(flags=1 << 9),
])
def test_init_rejects_invalid_params(lib, kw):
    h = ctypes.c_void_p()
    p = _params(**kw)
    assert lib.fcm_init(ctypes.byref(h), FAKE, 100, ctypes.byref(p), None) == L.FCM_EINVAL
    assert not h.value


def test_init_rejects_nonfinite_given_centroids(lib):
    buf = (ctypes.c_double * 4)(1.0, math.nan, 3.0, 4.0)
    p = _params(init=L.FCM_INIT_GIVEN, init_centroids=ctypes.cast(buf, ctypes.POINTER(ctypes.c_double)))
    h = ctypes.c_void_p()
    assert lib.fcm_init(ctypes.byref(h), FAKE, 100, ctypes.byref(p), None) == L.FCM_EINVAL


def test_init_rejects_bad_pointers_and_sizes(lib):
    h = ctypes.c_void_p()
    p = _params()
    assert lib.fcm_init(ctypes.byref(h), None, 100, ctypes.byref(p), None) == L.FCM_EINVAL
    assert lib.fcm_init(ctypes.byref(h), FAKE, 0, ctypes.byref(p), None) == L.FCM_EINVAL
    assert lib.fcm_init(ctypes.byref(h), FAKE, -4, ctypes.byref(p), None) == L.FCM_EINVAL
    assert lib.fcm_init(None, FAKE, 100, ctypes.byref(p), None) == L.FCM_EINVAL
    assert lib.fcm_init(ctypes.byref(h), FAKE, 100, None, None) == L.FCM_EINVAL


def test_null_handle_calls(lib):
    r = L.FcmResult()
    t = L.FcmTuning(block=256, grid=0, unroll=1, driver=1, graph_k=8, exchange=0, launch=0)
    buf = (ctypes.c_double * 8)()
    assert lib.fcm_iterate(None, 1, ctypes.byref(r)) == L.FCM_EINVAL
    assert lib.fcm_solve(None, ctypes.byref(r)) == L.FCM_EINVAL
    assert lib.fcm_labels(None, FAKE) == L.FCM_EINVAL
    assert lib.fcm_centroids(None, buf) == L.FCM_EINVAL
    assert lib.fcm_trajectory(None, 0, buf, None, None) == L.FCM_EINVAL
    assert lib.fcm_set_tuning(None, ctypes.byref(t)) == L.FCM_EINVAL
    assert lib.fcm_get_tuning(None, ctypes.byref(t)) == L.FCM_EINVAL
    assert lib.fcm_solve_async(None, None) == L.FCM_EINVAL
    assert lib.fcm_solve_wait(None, ctypes.byref(r), None) == L.FCM_EINVAL
    lib.fcm_destroy(None)


def test_batch_init_validation(lib):
    b = ctypes.c_void_p()
    recs = (L.FcmParams * 2)(_params(), _params())
    off = (ctypes.c_int64 * 3)(0, 100, 250)
    assert lib.fcm_batch_init(ctypes.byref(b), None, off, 2, recs, None) == L.FCM_EINVAL
    assert lib.fcm_batch_init(ctypes.byref(b), FAKE, off, 0, recs, None) == L.FCM_EINVAL
    bad_off = (ctypes.c_int64 * 3)(1, 100, 250)
    assert lib.fcm_batch_init(ctypes.byref(b), FAKE, bad_off, 2, recs, None) == L.FCM_EINVAL
    empty = (ctypes.c_int64 * 3)(0, 100, 100)
    assert lib.fcm_batch_init(ctypes.byref(b), FAKE, empty, 2, recs, None) == L.FCM_EINVAL
    bad = (L.FcmParams * 2)(_params(), _params(n_clusters=9))
    assert lib.fcm_batch_init(ctypes.byref(b), FAKE, off, 2, bad, None) == L.FCM_EINVAL
    r = (L.FcmResult * 2)()
    assert lib.fcm_batch_solve(None, r) == L.FCM_EINVAL
    assert lib.fcm_batch_labels(None, FAKE) == L.FCM_EINVAL
    assert lib.fcm_batch_set_tiling(None, 4, 0) == L.FCM_EINVAL
    assert lib.fcm_batch_trajectory(None, 0, 0, None, None, None) == L.FCM_EINVAL
    lib.fcm_batch_destroy(None)


def test_learned_start_validation(lib):
    """Argument checks of the warm-start entry points (before any HIP call)."""
    assert lib.fcm_mlp_param_count(4) == 256 * 128 + 128 + 128 * 64 + 64 + 64 * 4 + 4 == 41412
    assert lib.fcm_mlp_param_count(8) == 41412 + 4 * 64 + 4
    assert lib.fcm_mlp_param_count(1) == L.FCM_EINVAL
    assert lib.fcm_mlp_param_count(9) == L.FCM_EINVAL
    h = ctypes.c_void_p()
    assert lib.fcm_mlp_create(None, 4, 0, None) == L.FCM_EINVAL
    assert lib.fcm_mlp_create(ctypes.byref(h), 1, 0, None) == L.FCM_EINVAL
    assert lib.fcm_mlp_create(ctypes.byref(h), 9, 0, None) == L.FCM_EINVAL
    buf = (ctypes.c_float * 8)()
    assert lib.fcm_mlp_get_params(None, buf) == L.FCM_EINVAL
    assert lib.fcm_mlp_set_params(None, buf) == L.FCM_EINVAL
    assert lib.fcm_mlp_forward(None, FAKE, 1, FAKE, 0) == L.FCM_EINVAL
    loss = ctypes.c_double()
    assert lib.fcm_mlp_loss_grad(None, FAKE, FAKE, 1, ctypes.byref(loss), buf) == L.FCM_EINVAL
    cfg = L.FcmTrainCfg(epochs=1, batch=16, lr=1e-3, pad=0, seed=0)
    assert lib.fcm_mlp_train(None, FAKE, FAKE, 10, ctypes.byref(cfg), None) == L.FCM_EINVAL
    lib.fcm_mlp_destroy(None)
    off = (ctypes.c_int64 * 3)(0, 10, 10)  # second instance empty
    assert lib.fcm_histogram(FAKE, off, 2, FAKE, None) == L.FCM_EINVAL
    off = (ctypes.c_int64 * 2)(1, 10)      # does not start at 0
    assert lib.fcm_histogram(FAKE, off, 1, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_histogram(None, off, 1, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_histogram_noalloc(None, off, 1, FAKE, None) == L.FCM_EINVAL
    off2 = (ctypes.c_int64 * 3)(0, 10, 10)
    assert lib.fcm_histogram_noalloc(FAKE, off2, 2, FAKE, None) == L.FCM_EINVAL
    big = (ctypes.c_int64 * 1026)(*range(1026))
    assert lib.fcm_histogram_noalloc(FAKE, big, 1025, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_warm_centroids(None, FAKE, 1, FAKE, None) == L.FCM_EINVAL
    r = L.FcmResult()
    assert lib.fcm_solve_warm(None, None, 0, ctypes.byref(r), None, None) == L.FCM_EINVAL
    assert lib.fcm_batch_set_start(None, None, None) == L.FCM_EINVAL
    assert lib.fcm_mlp_save(None, b"/tmp/x.fcmmlp") == L.FCM_EINVAL
    assert lib.fcm_mlp_load(None, b"/tmp/x.fcmmlp") == L.FCM_EINVAL
    assert lib.fcm_mlp_save(FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_mlp_load(FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_mlp_save(FAKE, b"") == L.FCM_EINVAL
    out = (L.FcmResult * 2)()
    used = (ctypes.c_uint8 * 2)()
    assert lib.fcm_batch_solve_warm(None, FAKE, 1, out, None, used) == L.FCM_EINVAL
    assert lib.fcm_batch_solve_warm(FAKE, None, 1, out, None, used) == L.FCM_EINVAL
    assert lib.fcm_batch_solve_warm(FAKE, FAKE, 1, None, None, used) == L.FCM_EINVAL
    assert lib.fcm_batch_targets(None, 4, FAKE) == L.FCM_EINVAL
    assert lib.fcm_batch_targets(FAKE, 4, None) == L.FCM_EINVAL
    assert lib.fcm_batch_targets(FAKE, 1, FAKE) == L.FCM_EINVAL
    assert lib.fcm_batch_targets(FAKE, 9, FAKE) == L.FCM_EINVAL
    assert lib.fcm_set_wait_limit(None, 1.0, None) == L.FCM_EINVAL
    assert lib.fcm_batch_timeline(None, 0, None, 0, None) == L.FCM_EINVAL
    assert lib.fcm_batch_set_tail_tiling(None, 48, 1) == L.FCM_EINVAL
    assert lib.fcm_batch_set_tail_tiling(FAKE, -1, 1) == L.FCM_EINVAL
    assert lib.fcm_batch_set_tail_tiling(FAKE, 48, 0) == L.FCM_EINVAL
    assert lib.fcm_batch_set_tail_tiling(FAKE, 48, 65) == L.FCM_EINVAL


def test_autotune_validation(lib):
    t = L.FcmTuning()
    ms = ctypes.c_double()
    assert lib.fcm_autotune(None, None, 3, ctypes.byref(t), ctypes.byref(ms)) == L.FCM_EINVAL
    assert lib.fcm_batch_autotune(None, None, 2, None, None, None, None) == L.FCM_EINVAL
    assert lib.fcm_batch_set_block(None, 512) == L.FCM_EINVAL
    assert lib.fcm_batch_set_block(FAKE, 64) == L.FCM_EINVAL


def test_quality_validation(lib):
    """Argument checks of the Eq.5 entry points return before any device call."""
    i32 = ctypes.c_int32
    assert lib.fcm_confusion(FAKE, FAKE, 10, 0, 4, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_confusion(FAKE, FAKE, 10, 4, 17, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_confusion(FAKE, FAKE, -1, 4, 4, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_confusion(None, FAKE, 10, 4, 4, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_confusion(FAKE, FAKE, 10, 4, 4, None, None) == L.FCM_EINVAL
    assert lib.fcm_dice(None, 4, 4, None, FAKE, None) == L.FCM_EINVAL
    assert lib.fcm_dice(FAKE, 4, 4, None, None, None) == L.FCM_EINVAL
    assert lib.fcm_dice(FAKE, 17, 4, None, FAKE, None) == L.FCM_EINVAL
    bad = (i32 * 4)(0, 1, 4, 2)
    assert lib.fcm_dice(FAKE, 4, 4, bad, FAKE, None) == L.FCM_EINVAL
    bad = (i32 * 4)(0, -2, 1, 2)
    assert lib.fcm_dice(FAKE, 4, 4, bad, FAKE, None) == L.FCM_EINVAL


def test_random_start_is_single_handle_only(lib):
    recs = (L.FcmParams * 2)(_params(), _params(init=L.FCM_INIT_RANDOM_U, seed=5))
    off = (ctypes.c_int64 * 3)(0, 100, 250)
    b = ctypes.c_void_p()
    assert lib.fcm_batch_init(ctypes.byref(b), FAKE, off, 2, recs, None) == L.FCM_EINVAL


def test_paper_baseline_validation(lib):
    r = L.FcmResult()
    p = _params()
    assert lib.fcm_paper_solve(None, 100, ctypes.byref(p), None, ctypes.byref(r), None, None, None, None) == L.FCM_EINVAL
    assert lib.fcm_paper_solve(FAKE, 0, ctypes.byref(p), None, ctypes.byref(r), None, None, None, None) == L.FCM_EINVAL
    assert lib.fcm_paper_solve(FAKE, 100, None, None, ctypes.byref(r), None, None, None, None) == L.FCM_EINVAL
    assert lib.fcm_paper_solve(FAKE, 100, ctypes.byref(p), None, None, None, None, None, None) == L.FCM_EINVAL
    for kw in (dict(init=L.FCM_INIT_DEVICE), dict(n_clusters=9), dict(m=1.0), dict(eps=0.0), dict(max_iter=0),
               dict(init=L.FCM_INIT_GIVEN)):
        q = _params(**kw)
        assert lib.fcm_paper_solve(FAKE, 100, ctypes.byref(q), None, ctypes.byref(r), None, None, None,
                                   None) == L.FCM_EINVAL, kw
