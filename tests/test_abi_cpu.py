"""The C-ABI library loads, exports every symbol include/hmm.h declares, and its
host-side checks behave (CPU only: no kernel is launched by any call here)."""
import ctypes
import os
import re

import pytest

from paper_1310_3322_amd import hmm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hmm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hmm.LIB_PATH):
        import paper_1310_3322_amd.build as b
        b.build()
    return hmm.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert set(names) == set(hmm.EXPORTS), names
    for n in names:
        assert hasattr(lib, n), n


def _bank(K=4, N=16, M=32):
    return hmm.Bank(K, N, M, 0x1000, 0x2000, 0x3000)


def _batch(S=100, max_len=50, total=5000, models=False):
    return hmm.Batch(S, 0x4000, 0x5000, 0x6000, 0x7000 if models else None, max_len, total)


def test_workspace_size_rules(lib):
    b = _bank()
    q = _batch()
    for op in (0, 1, 2, 3):
        assert lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), op) > 0
    assert lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 7) == 0
    bad = hmm.Bank(0, 16, 32, 0x1000, 0x2000, 0x3000)
    assert lib.hmm_workspace_size(ctypes.byref(bad), ctypes.byref(q), 0) == 0
    bad = hmm.Bank(4, 300, 32, 0x1000, 0x2000, 0x3000)
    assert lib.hmm_workspace_size(ctypes.byref(bad), ctypes.byref(q), 0) == 0
    # monotone in S and max_len (past the few-pairs range where the time-parallel forward is chosen)
    prev = 0
    for S in (100, 1000, 10000):
        n = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(_batch(S=S)), 1)
        assert n >= prev
        prev = n
    # few pairs: the time-parallel forward reserves one 16x16 product per chunk of 64 steps and pair
    few = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(_batch(S=2, max_len=1000)), 0)
    assert few >= 2 * 16 * 1024
    prev = 0
    for ml in (0, 10, 1000):
        n = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(_batch(max_len=ml, models=True)), 2)
        assert n >= prev
        prev = n


def test_host_side_errors_enqueue_nothing(lib):
    b = _bank()
    q = _batch()
    out = ctypes.c_void_p(0x8000)
    ws_al = ctypes.c_void_p(0x100000)
    # null bank / batch
    assert lib.hmm_forward_loglik(None, ctypes.byref(q), out, ws_al, 1 << 30, None) == -1
    # bad shape
    bad = hmm.Bank(4, 0, 32, 0x1000, 0x2000, 0x3000)
    assert lib.hmm_forward_loglik(ctypes.byref(bad), ctypes.byref(q), out, ws_al, 1 << 30, None) == -2
    # null parameter pointer
    nb = hmm.Bank(4, 16, 32, 0x1000, None, 0x3000)
    assert lib.hmm_forward_loglik(ctypes.byref(nb), ctypes.byref(q), out, ws_al, 1 << 30, None) == -1
    # null output
    assert lib.hmm_forward_loglik(ctypes.byref(b), ctypes.byref(q), None, ws_al, 1 << 30, None) == -1
    # workspace too small, null or misaligned
    need = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 0)
    assert lib.hmm_forward_loglik(ctypes.byref(b), ctypes.byref(q), out, ws_al, need - 1, None) == -3
    assert lib.hmm_forward_loglik(ctypes.byref(b), ctypes.byref(q), out, None, need, None) == -3
    assert lib.hmm_forward_loglik(ctypes.byref(b), ctypes.byref(q), out, ctypes.c_void_p(0x100004), need, None) == -3
    # classify needs labels
    assert lib.hmm_classify(ctypes.byref(b), ctypes.byref(q), None, None, ws_al, 1 << 30, None) == -1
    # gradient: model_of_seq required, counts required for phases 0 and 2, phase range
    args = (ctypes.byref(b), ctypes.byref(q), None, out, out, out, out)
    assert lib.hmm_forward_backward_grad(*args, 0, ws_al, 1 << 40, None) == -1
    qm = _batch(models=True)
    assert lib.hmm_forward_backward_grad(ctypes.byref(b), ctypes.byref(qm), None, out, None, out, out, 0, ws_al,
                                         1 << 40, None) == -1
    assert lib.hmm_forward_backward_grad(ctypes.byref(b), ctypes.byref(qm), None, out, out, out, out, 3, ws_al,
                                         1 << 40, None) == -6
    # a gradient whose length-sorting plan would exceed its bin limit (models x (max_len + 1))
    # is reported, not attempted
    big = hmm.Bank(64, 16, 32, 0x1000, 0x2000, 0x3000)
    ql = hmm.Batch(100, 0x4000, 0x5000, 0x6000, 0x7000, 1 << 20, 5000)
    need = lib.hmm_workspace_size(ctypes.byref(big), ctypes.byref(ql), 2)
    assert lib.hmm_forward_backward_grad(ctypes.byref(big), ctypes.byref(ql), None, out, out, out, out, 0, ws_al,
                                         need, None) == -4
    # Viterbi: model_of_seq, score and path required; more than 64 states reported, not attempted
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(q), out, out, ws_al, 1 << 40, None) == -1
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(qm), None, out, ws_al, 1 << 40, None) == -1
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(qm), out, None, ws_al, 1 << 40, None) == -1
    need = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(qm), 3)
    assert need >= 5000 * 16  # one back-pointer byte per padded state and symbol
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(qm), out, out, ws_al, need - 1, None) == -3
    wide = hmm.Bank(4, 65, 32, 0x1000, 0x2000, 0x3000)
    need = lib.hmm_workspace_size(ctypes.byref(wide), ctypes.byref(qm), 3)
    assert lib.hmm_viterbi(ctypes.byref(wide), ctypes.byref(qm), out, out, ws_al, need, None) == -4
    assert lib.hmm_reestimate_rows(out, out, out, -1, 4, None) == -2
    assert lib.hmm_reestimate_rows(None, out, out, 3, 4, None) == -1
    # softmax / logit-grad shape checks
    assert lib.hmm_softmax_rows(out, out, -1, 4, None) == -2
    assert lib.hmm_logit_grad(out, out, out, 4, 0, None) == -2
    assert lib.hmm_workspace_error(None, None, None) == -1


def test_kernel_selector(lib):
    assert lib.hmm_select_kernel(7) == -6
    assert lib.hmm_select_kernel(-1) == -6
    for k in (1, 2, 3, 4, 5, 6, 0):
        assert lib.hmm_select_kernel(k) == 0


def test_status_strings(lib):
    for code, name in hmm.STATUS.items():
        assert lib.hmm_status_string(code).decode() == name
