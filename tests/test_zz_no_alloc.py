"""hmm_classify_noalloc (the library's static scratch array, no caller workspace)
against hmm_classify with a caller workspace, through the C ABI (MI355X only).

Three calls in a row, each on a smaller batch than the one before (the array keeps
the previous call's contents, so a stale histogram, queue head or plan entry would
show here): labels bit-exact, log-likelihoods within the path's tolerance
|l - l_ref| / max(|l_ref|, 1) <= 1e-5 (both calls run the same kernels, so they are
expected to be identical).  A batch whose workspace exceeds the array is refused
with HMM_ERR_WORKSPACE and nothing is written.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1310_3322_amd import hmm, workloads

pytestmark = pytest.mark.gpu

LL_TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def problem(w):
    return hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(w.symbols), dev(w.offsets), dev(w.lengths), None,
                       max_len=w.max_len, total_symbols=w.total_symbols)


def compare(w, with_loglik):
    p = problem(w)
    need = p.workspace_size(hmm.OP_CLASSIFY, p.batch_without_models())
    assert 0 < need <= hmm.STATIC_SCRATCH_BYTES, need
    ref_ll = torch.empty((p.S, p.K), dtype=torch.float32, device="cuda")
    ref_labels = hmm.classify(p, loglik=ref_ll)
    labels = torch.full((p.S,), -7, dtype=torch.int32, device="cuda")
    ll = torch.full((p.S, p.K), float("nan"), dtype=torch.float32, device="cuda") if with_loglik else None
    hmm.classify_noalloc(p, labels, ll)
    torch.cuda.synchronize()
    assert torch.equal(labels, ref_labels), w.name
    if with_loglik:
        a = ll.cpu().numpy().astype(np.float64)
        r = ref_ll.cpu().numpy().astype(np.float64)
        assert np.array_equal(np.isfinite(a), np.isfinite(r)), w.name
        fin = np.isfinite(r)
        err = float(np.max(np.abs(a[fin] - r[fin]) / np.maximum(np.abs(r[fin]), 1.0))) if fin.any() else 0.0
        assert err <= LL_TOL, (w.name, err)
        print(f"[case] noalloc {w.name}: S={p.S} K={p.K} ws={need} B, labels equal, loglik err {err:.1e}, "
              f"bit-identical {bool(torch.equal(ll, ref_ll))}", flush=True)
    else:
        print(f"[case] noalloc {w.name}: S={p.S} K={p.K} ws={need} B, labels equal (no loglik)", flush=True)


def test_noalloc_matches_classify_on_shrinking_batches():
    # the full recognition batch (64 models x 65,536 sequences up to 2048 steps, 19 MB of
    # scratch), 3277 of its sequences, 12 models x 1024 sequences up to 400 steps (with and
    # without log-likelihoods), then one model and one sequence of 64 steps (the
    # time-parallel family)
    for cfg, scale, with_ll in (("c3", 1.0, True), ("c3", 0.05, True), ("c2", 0.25, True), ("c2", 0.05, False),
                                ("c1", 1.0, True)):
        compare(workloads.make_workload(cfg, scale=scale), with_ll)


def test_noalloc_refuses_batches_beyond_the_array():
    lib = hmm.load_library()
    # 64 models x 200,000 sequences: the [S][K] log-likelihoods alone take 51 MB
    bank = hmm.Bank(64, 32, 256, 0x1000, 0x2000, 0x3000)
    batch = hmm.Batch(200_000, 0x4000, 0x5000, 0x6000, None, 2048, 200_000 * 1000)
    assert lib.hmm_workspace_size(ctypes.byref(bank), ctypes.byref(batch), hmm.OP_CLASSIFY) > hmm.STATIC_SCRATCH_BYTES
    rc = lib.hmm_classify_noalloc(ctypes.byref(bank), ctypes.byref(batch), ctypes.c_void_p(0x8000), None, None)
    assert rc == -3, rc
    # after the refusal the array still serves a batch that fits
    compare(workloads.make_workload("paper"), True)
