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
    # Viterbi: model_of_seq, score and path required; a plan beyond the bin limit reported, not attempted
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(q), out, out, ws_al, 1 << 40, None) == -1
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(qm), None, out, ws_al, 1 << 40, None) == -1
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(qm), out, None, ws_al, 1 << 40, None) == -1
    # the default workspace holds every delta row here (5000 symbols x 16 padded states);
    # anything down to two halves that each hold the longest sequence (2 x max_len = 100) is accepted
    need = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(qm), 3)
    assert need >= 5000 * 16 * 4
    vws = lambda bank, batch, rows: lib.hmm_viterbi_workspace_size(ctypes.byref(bank), ctypes.byref(batch),
                                                                   ctypes.c_int64(rows))
    least = vws(b, qm, 100)
    assert 0 < least < need
    assert vws(b, qm, 99) == 0
    assert vws(b, qm, 5000) == need == vws(b, qm, 10 ** 12)
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(qm), out, out, ws_al, least - 1, None) == -3
    assert lib.hmm_viterbi(ctypes.byref(b), ctypes.byref(qm), out, out, None, need, None) == -3
    # every state count up to HMM_MAX_STATES decodes: the workspace holds the delta rows
    # (states padded to 128 / 256) and ln A transposed
    for n, np_ in ((65, 128), (256, 256)):
        wide = hmm.Bank(4, n, 32, 0x1000, 0x2000, 0x3000)
        assert lib.hmm_workspace_size(ctypes.byref(wide), ctypes.byref(qm), 3) >= 5000 * np_ * 4 + 4 * n * np_ * 4
    assert lib.hmm_reestimate_rows(out, out, out, -1, 4, None) == -2
    assert lib.hmm_reestimate_rows(None, out, out, 3, 4, None) == -1
    # softmax / logit-grad shape checks
    assert lib.hmm_softmax_rows(out, out, -1, 4, None) == -2
    assert lib.hmm_logit_grad(out, out, out, 4, 0, None) == -2
    assert lib.hmm_workspace_error(None, None, None) == -1


def test_viterbi_workspace_is_bounded(lib):
    """Viterbi's default workspace stays under 2 GB for 16 models of 256 states and 16,384
    sequences of up to 4096 steps (36 GB of delta rows, decoded in rounds), and grows with
    the rows a round may keep, up to every row."""
    b = hmm.Bank(16, 256, 1024, 0x1000, 0x2000, 0x3000)
    total = 16384 * 2176
    q = hmm.Batch(16384, 0x4000, 0x5000, 0x6000, 0x7000, 4096, total)
    vws = lambda rows: lib.hmm_viterbi_workspace_size(ctypes.byref(b), ctypes.byref(q), ctypes.c_int64(rows))
    dflt = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 3)
    assert 0 < dflt <= 2_000_000_000
    assert vws(total) >= total * 256 * 4 > dflt
    prev = 0
    for rows in (8192, 100_000, 1 << 21, total):
        n = vws(rows)
        assert n > prev and n >= rows * 1024
        prev = n
    assert vws(8191) == 0


def test_grad_workspace_storage(lib):
    """The gradient's workspace: checkpoints only at rows = 0; each stored step adds a
    row of NP floats and an exponent; requests clamp at S max_len; negative rows are
    refused.  The default stores every step when that takes at most 4 GiB (the c4 shape)
    and keeps checkpoints only above (the c5 shape: 36 GB of rows); below 49 states the
    gradient keeps checkpoints whatever the request."""
    gws = lambda b, q, rows: lib.hmm_grad_workspace_size(ctypes.byref(b), ctypes.byref(q), ctypes.c_int64(rows))
    dflt = lambda b, q: lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 2)
    b4 = hmm.Bank(8, 64, 512, 0x1000, 0x2000, 0x3000)
    tot4 = 8192 * 550
    q4 = hmm.Batch(8192, 0x4000, 0x5000, 0x6000, 0x7000, 1000, tot4)
    base = gws(b4, q4, 0)
    assert base > 0 and gws(b4, q4, -1) == 0
    assert gws(b4, q4, tot4) >= base + tot4 * (64 * 4 + 4)
    assert dflt(b4, q4) == gws(b4, q4, tot4)
    assert gws(b4, q4, 8192 * 1000) == gws(b4, q4, 1 << 40) > gws(b4, q4, tot4)
    prev = base
    for rows in (1, 1000, 1 << 20, tot4):
        n = gws(b4, q4, rows)
        assert n > prev
        prev = n
    b5 = hmm.Bank(16, 256, 1024, 0x1000, 0x2000, 0x3000)
    tot5 = 16384 * 2176
    q5 = hmm.Batch(16384, 0x4000, 0x5000, 0x6000, 0x7000, 4096, tot5)
    assert dflt(b5, q5) == gws(b5, q5, 0) < 2_000_000_000
    assert gws(b5, q5, tot5) >= tot5 * (256 * 4 + 4)
    b2 = hmm.Bank(4, 40, 64, 0x1000, 0x2000, 0x3000)
    q2 = hmm.Batch(100, 0x4000, 0x5000, 0x6000, 0x7000, 50, 2500)
    assert gws(b2, q2, 0) == gws(b2, q2, 2500) == gws(b2, q2, 1 << 30) == dflt(b2, q2) > 0


def test_kernel_selector(lib):
    assert lib.hmm_select_kernel(7) == -6
    assert lib.hmm_select_kernel(-1) == -6
    for k in (1, 2, 3, 4, 5, 6, 0):
        assert lib.hmm_select_kernel(k) == 0


def test_status_strings(lib):
    for code, name in hmm.STATUS.items():
        assert lib.hmm_status_string(code).decode() == name


def _key(op=0, all_pairs=1, K=4, N=16, M=32, sb=7, lb=6):
    return hmm.TuneKey(op, all_pairs, K, N, M, sb, lb)


def test_tune_key_buckets(lib):
    k = hmm.tune_key(_bank(), _batch(S=100, max_len=50), hmm.OP_FORWARD)
    assert k.as_dict() == {"op": 0, "all_pairs": 1, "K": 4, "N": 16, "M": 32, "s_bucket": 7, "len_bucket": 6}
    k = hmm.tune_key(_bank(), _batch(S=128, max_len=64, models=True), hmm.OP_FORWARD)
    assert (k.all_pairs, k.s_bucket, k.len_bucket) == (0, 8, 7)
    k = hmm.tune_key(_bank(), _batch(S=0, max_len=0, models=True), hmm.OP_CLASSIFY)
    assert (k.all_pairs, k.s_bucket, k.len_bucket) == (1, 0, 0)
    k = hmm.tune_key(_bank(), _batch(models=True), hmm.OP_GRAD)
    assert k.all_pairs == 0
    with pytest.raises(hmm.HMMError):
        hmm.tune_key(_bank(), _batch(), 9)
    with pytest.raises(hmm.HMMError):
        hmm.tune_key(hmm.Bank(0, 16, 32, 0x1000, 0x2000, 0x3000), _batch(), 0)


def test_tune_table_set_get_remove(lib):
    hmm.tune_clear()
    k = _key()
    assert hmm.tune_get(k) is None
    hmm.tune_set(k, hmm.KERNEL_TILE32, 2, hmm.TUNE_XCD_OFF | hmm.TUNE_BT_LDS)
    assert hmm.tune_get(k) == (hmm.KERNEL_TILE32, 2, hmm.TUNE_XCD_OFF | hmm.TUNE_BT_LDS)
    hmm.tune_set(k, hmm.KERNEL_COOP, 0)  # replaces
    assert hmm.tune_get(k) == (hmm.KERNEL_COOP, 0, 0)
    other = _key(sb=8)
    assert hmm.tune_get(other) is None
    hmm.tune_set(k, None)
    assert hmm.tune_get(k) is None
    hmm.tune_set(k, None)  # removing an absent entry is fine
    # invalid keys and choices
    bad = [(_key(op=4), hmm.KERNEL_AUTO, 0), (_key(all_pairs=2), hmm.KERNEL_AUTO, 0), (_key(K=0), hmm.KERNEL_AUTO, 0),
           (_key(N=257), hmm.KERNEL_AUTO, 0), (_key(sb=32), hmm.KERNEL_AUTO, 0), (_key(), 7, 0),
           (_key(), hmm.KERNEL_AUTO, -1), (_key(), hmm.KERNEL_AUTO, hmm.TUNE_MAX_WG + 1),
           (_key(op=hmm.OP_GRAD, all_pairs=0), hmm.KERNEL_TILE16, 0),
           (_key(op=hmm.OP_VITERBI, all_pairs=0), hmm.KERNEL_SCAN, 0)]
    for key, kind, cap in bad:
        with pytest.raises(hmm.HMMError) as e:
            hmm.tune_set(key, kind, cap)
        assert e.value.status == -6
    for flags in (8, -1, hmm.TUNE_BT_GLOBAL | hmm.TUNE_BT_LDS):  # unknown bits, both table placements
        with pytest.raises(hmm.HMMError) as e:
            hmm.tune_set(_key(), hmm.KERNEL_TILE32, 0, flags)
        assert e.value.status == -6
    hmm.tune_set(_key(op=hmm.OP_GRAD, all_pairs=0), hmm.KERNEL_BATCHED, 4)
    assert lib.hmm_tune_set(None, None) == -1
    assert lib.hmm_tune_get(ctypes.byref(k), None, None) == -1
    hmm.tune_clear()
    assert hmm.tune_get(_key(op=hmm.OP_GRAD, all_pairs=0)) is None


def test_tune_table_capacity(lib):
    hmm.tune_clear()
    for i in range(hmm.TUNE_MAX):
        hmm.tune_set(_key(K=i + 1), hmm.KERNEL_TILE16, 1)
    with pytest.raises(hmm.HMMError) as e:
        hmm.tune_set(_key(K=hmm.TUNE_MAX + 1), hmm.KERNEL_TILE16, 1)
    assert e.value.status == -4
    hmm.tune_set(_key(K=5), hmm.KERNEL_TILE32, 2)  # replacing still works when full
    assert hmm.tune_get(_key(K=5)) == (hmm.KERNEL_TILE32, 2, 0)
    hmm.tune_set(_key(K=7), None)
    hmm.tune_set(_key(K=hmm.TUNE_MAX + 1), hmm.KERNEL_TILE16, 1)  # a freed slot is reused
    assert hmm.tune_get(_key(K=hmm.TUNE_MAX + 1)) == (hmm.KERNEL_TILE16, 1, 0)
    assert hmm.tune_get(_key(K=7)) is None
    hmm.tune_clear()


def test_tune_entry_sizes_workspace(lib):
    """A tuned family applies to hmm_workspace_size too: the time-parallel forward
    reserves its chunk products only when it is the call's choice, and a forced
    selector overrides the table."""
    hmm.tune_clear()
    hmm.select_kernel(hmm.KERNEL_AUTO)
    b, q = _bank(), _batch(S=1000, max_len=1000)
    plain = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 0)
    key = hmm.tune_key(b, q, hmm.OP_FORWARD)
    try:
        hmm.tune_set(key, hmm.KERNEL_SCAN, 0)
        scan = lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 0)
        assert scan >= plain + 1000 * 4 * 16 * 1024  # 4 000 pairs x 16 chunks x (16x16 floats)
        # another shape bucket is unaffected
        assert lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(_batch(S=3000, max_len=1000)), 0) < scan
        # a workspace sized before the entry was installed is refused before anything is enqueued
        out = ctypes.c_void_p(0x8000)
        assert lib.hmm_forward_loglik(ctypes.byref(b), ctypes.byref(q), out, ctypes.c_void_p(0x100000), plain,
                                      None) == -3
        hmm.select_kernel(hmm.KERNEL_TILE16)
        assert lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 0) == plain
    finally:
        hmm.select_kernel(hmm.KERNEL_AUTO)
        hmm.tune_clear()
    assert lib.hmm_workspace_size(ctypes.byref(b), ctypes.byref(q), 0) == plain


def test_tune_cache_roundtrip(lib, tmp_path):
    from paper_1310_3322_amd import tune
    hmm.tune_clear()
    path = str(tmp_path / "tune.json")
    r1 = {"key": _key().as_dict(), "choice": {"kernel": "tile32", "wg_per_cu": 2}, "ms": 1.5}
    r2 = {"key": _key(op=hmm.OP_VITERBI, all_pairs=0).as_dict(), "choice": {"kernel": "batched", "wg_per_cu": 1},
          "ms": 0.5}
    tune.save_cache(path, [r1], arch="gfx950")
    tune.save_cache(path, [r2], arch="gfx950")          # merged
    tune.save_cache(path, [dict(r1, choice={"kernel": "coop", "wg_per_cu": 0})], arch="gfx942")  # other arch
    tune.save_cache(path, [dict(r1, choice={"kernel": "tile16", "wg_per_cu": 4, "flags": hmm.TUNE_BT_GLOBAL})],
                    arch="gfx950")  # replaces r1
    assert tune.load_cache(path, arch="gfx950") == 2
    assert hmm.tune_get(_key()) == (hmm.KERNEL_TILE16, 4, hmm.TUNE_BT_GLOBAL)
    assert hmm.tune_get(_key(op=hmm.OP_VITERBI, all_pairs=0)) == (hmm.KERNEL_BATCHED, 1, 0)  # no flags: 0
    hmm.tune_clear()
    assert tune.load_cache(path, arch="gfx90a") == 0
    assert hmm.tune_get(_key()) is None


def test_call_kernel_resolution(lib):
    """Which family a call would run: heuristics, then table, then a forced selector
    (host only; the device count of compute units defaults to 256 without a GPU)."""
    hmm.tune_clear()
    hmm.select_kernel(hmm.KERNEL_AUTO)
    try:
        c3b, c3q = hmm.Bank(64, 32, 256, 1, 2, 3), hmm.Batch(65536, 4, 5, 6, None, 2048, 1 << 25)
        assert hmm.call_kernel(c3b, c3q, hmm.OP_CLASSIFY) == hmm.KERNEL_TILE32
        big = hmm.Bank(16, 256, 1024, 1, 2, 3)
        own = hmm.Batch(16384, 4, 5, 6, 7, 4096, 1 << 26)
        assert hmm.call_kernel(big, own, hmm.OP_FORWARD) == hmm.KERNEL_COOP
        assert hmm.call_kernel(big, own, hmm.OP_GRAD) == hmm.KERNEL_COOP
        one = hmm.Batch(1, 4, 5, 6, 7, 64, 64)
        assert hmm.call_kernel(hmm.Bank(1, 8, 16, 1, 2, 3), one, hmm.OP_FORWARD) == hmm.KERNEL_SCAN
        assert hmm.call_kernel(hmm.Bank(8, 32, 64, 1, 2, 3), hmm.Batch(9000, 4, 5, 6, 7, 100, 1 << 20),
                               hmm.OP_GRAD) == hmm.KERNEL_TILE16
        assert hmm.call_kernel(hmm.Bank(8, 32, 64, 1, 2, 3), one, hmm.OP_VITERBI) == hmm.KERNEL_BATCHED
        # above 64 states the workgroup decoder (the batched family as well)
        assert hmm.call_kernel(hmm.Bank(8, 100, 64, 1, 2, 3), one, hmm.OP_VITERBI) == hmm.KERNEL_BATCHED
        # one work list for all models: every max_len up to HMM_MAX_LEN fits the planner's bins
        assert hmm.call_kernel(hmm.Bank(64, 100, 64, 1, 2, 3), hmm.Batch(100, 4, 5, 6, 7, 1 << 20, 5000),
                               hmm.OP_VITERBI) == hmm.KERNEL_BATCHED
        # the table
        hmm.tune_set(hmm.tune_key(c3b, c3q, hmm.OP_CLASSIFY), hmm.KERNEL_TILE16, 2)
        assert hmm.call_kernel(c3b, c3q, hmm.OP_CLASSIFY) == hmm.KERNEL_TILE16
        hmm.tune_set(hmm.tune_key(big, own, hmm.OP_FORWARD), hmm.KERNEL_TILE32, 0)
        with pytest.raises(hmm.HMMError) as e:
            hmm.call_kernel(big, own, hmm.OP_FORWARD)
        assert e.value.status == -4
        # a forced selector ignores the table
        hmm.select_kernel(hmm.KERNEL_PLAIN)
        assert hmm.call_kernel(c3b, c3q, hmm.OP_CLASSIFY) == hmm.KERNEL_PLAIN
        hmm.select_kernel(hmm.KERNEL_BATCHED)
        assert hmm.call_kernel(c3b, c3q, hmm.OP_CLASSIFY) == hmm.KERNEL_TILE32
        assert hmm.call_kernel(big, own, hmm.OP_FORWARD) == hmm.KERNEL_COOP
    finally:
        hmm.select_kernel(hmm.KERNEL_AUTO)
        hmm.tune_clear()


def test_debug_flags_in_the_normal_build(lib):
    """The normal build compiles no bounds checks: hmm_debug_flags reports unsupported."""
    v = ctypes.c_uint32(7)
    assert lib.hmm_debug_flags(None) == -1
    assert lib.hmm_debug_flags(ctypes.byref(v)) == -4 and v.value == 0


def test_debug_build_exports_the_same_symbols():
    """The bounds-checked copy of the library exports every declared entry point."""
    if not os.path.exists(hmm.LIB_DEBUG_PATH):
        import paper_1310_3322_amd.build as b
        b.build(debug=True)
    dbg = ctypes.CDLL(hmm.LIB_DEBUG_PATH)
    for n in declared_functions():
        assert hasattr(dbg, n), n
