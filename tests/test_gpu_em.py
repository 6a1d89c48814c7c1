"""Baum-Welch EM on the GPU vs the FP64 oracle's EM, through the C ABI (MI355X only).

Per iteration: parameters ||theta_gpu - theta_oracle||_2 / ||theta_oracle||_2 <= 1e-4 per
array and model, sequence log-likelihoods within 1e-5 relative; the GPU's total
log-likelihood never decreases beyond FP32 rounding (the EM theorem).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1310_3322_amd import hmm, workloads

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(g, r):
    worst = 0.0
    for k in range(r.shape[0]):
        worst = max(worst, np.linalg.norm(g[k] - r[k]) / np.linalg.norm(r[k]))
    return worst


@pytest.mark.parametrize("cfg,scale", [("c2", 0.05), ("c4", 0.01), ("paper", 1.0)])
def test_em_iterations_match_oracle(cfg, scale):
    print(f"[case] em {cfg} scale={scale}", flush=True)
    hmm.load_library()
    w = workloads.make_workload(cfg, scale=scale)
    p = hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(w.symbols), dev(w.offsets), dev(w.lengths), dev(w.owner),
                    max_len=w.max_len, total_symbols=w.total_symbols)
    iters = 5
    hist, lls = O.baum_welch(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner, iters=iters)
    totals = []
    for it in range(iters):
        ll = hmm.baum_welch(p, 1)[0].cpu().numpy().astype(np.float64)
        totals.append(ll.sum())
        assert abs(ll.sum() - lls[it]) <= 1e-5 * abs(lls[it]), it
        for got, ref in zip((p.pi, p.A, p.B), hist[it]):
            assert rel(got.cpu().numpy().astype(np.float64), ref) <= 1e-4, it
    assert all(b >= a - 1e-6 * abs(a) for a, b in zip(totals, totals[1:])), totals


def test_reestimate_rows_kernel():
    hmm.load_library()
    n = torch.tensor([[1.0, 3.0, 0.0], [0.0, 0.0, 0.0], [2.0, 2.0, 4.0]], device="cuda")
    old = torch.tensor([[0.2, 0.3, 0.5], [0.1, 0.6, 0.3], [1.0, 0.0, 0.0]], device="cuda")
    out = hmm.reestimate_rows(n, old).cpu().numpy()
    assert np.allclose(out, [[0.25, 0.75, 0.0], [0.1, 0.6, 0.3], [0.25, 0.25, 0.5]], rtol=1e-7)
    hmm.reestimate_rows(n, old, out=old)  # in place over the old rows
    assert np.allclose(old.cpu().numpy(), out)
