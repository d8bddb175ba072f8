"""The C-ABI library loads and exports every entry point include/svmhip.h declares; host-side
argument checks run without a GPU.  CPU only (no kernel launches)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svmhip.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def S():
    from paper_1406_5161_amd import svmhip
    if not os.path.exists(svmhip.LIB_PATH):
        pytest.fail("libsvmhip.so not built (run __graft_entry__.build())")
    svmhip.lib()
    return svmhip


def test_every_declared_symbol_is_exported(S):
    names = declared_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(S.lib(), n)]
    assert not missing, missing
    assert set(names) == set(S.EXPORTS)


def test_strerror_and_version(S):
    assert S.strerror(S.SVM_OK) == "ok"
    assert "one class" in S.strerror(S.SVM_EONECLASS)
    assert S.lib().svm_version() >= 100


def test_host_side_argument_checks(S):
    p = S.svm_problem_t(0, 4, S.SVM_DENSE_ROW_MAJOR, 0, None, 4, None, None, None, None)
    q = S.make_params(1.0, 0.5)
    res = S.svm_result_t()
    L = S.lib()
    assert L.svm_train(C.byref(p), C.byref(q), None, None, C.byref(res), None, 0, None) == S.SVM_EINVAL
    fake = C.c_void_p(0x1000)
    p = S.svm_problem_t(10, 4, S.SVM_DENSE_ROW_MAJOR, 0, fake, 4, None, None, None, fake)
    for bad in [S.make_params(0.0, 0.5), S.make_params(1.0, -1.0), S.make_params(1.0, 0.5, eps=0.0),
                S.make_params(1.0, 0.5, shrink_mode=2, shrink_param=0.0), S.make_params(1.0, 0.5, max_iter=0),
                S.make_params(1.0, 0.5, lanes_per_row=3), S.make_params(1.0, 0.5, kernel_precision=7)]:
        assert L.svm_train(C.byref(p), C.byref(bad), fake, None, C.byref(res), None, 0, None) == S.SVM_EINVAL
    p2 = S.svm_problem_t(10, 4, S.SVM_DENSE_ROW_MAJOR, 0, fake, 2, None, None, None, fake)   # ldx < d
    assert L.svm_train(C.byref(p2), C.byref(q), fake, None, C.byref(res), None, 0, None) == S.SVM_EINVAL
    assert L.svm_train_workspace_size(C.byref(p), C.byref(q)) > 10 * 8


def test_workspace_size_grows_with_n(S):
    q = S.make_params(1.0, 0.5)
    fake = C.c_void_p(0x1000)
    sizes = []
    for n in (100, 1000, 10000):
        p = S.svm_problem_t(n, 8, S.SVM_DENSE_ROW_MAJOR, 0, fake, 8, None, None, None, fake)
        sizes.append(S.lib().svm_train_workspace_size(C.byref(p), C.byref(q)))
    assert sizes[0] < sizes[1] < sizes[2]
