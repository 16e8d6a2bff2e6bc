"""Batched solves (rpca_svd_batched) on the GPU.

  * in streams mode, every problem of a mixed batch (dense of uneven shapes,
    centered or not, symmetric PSD, sparse) gives bit for bit what the single
    call gives: the same kernels run on the same inputs, only on other streams;
  * sampled problems match the FP64 oracle (singular values within 1e-4);
  * the batch captured into a HIP graph (through torch.cuda.graph) and replayed
    several times, with unrelated eager work and synchronizations between the
    replays, reproduces the eager outputs exactly on every replay (the dense
    problems go to the persistent launch, the sparse one to a stream).
"""

import numpy as np
import pytest
import torch

from oracle import nystrom, philox, rsvd
from synth import dense, sparse

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _batch(gpu_lib, seed=5000, count=20):
    rng = np.random.default_rng(seed)
    probs, host = [], []
    for p in range(count):
        if p % 4 == 3:  # symmetric PSD
            n = int(rng.integers(128, 700))
            k = int(rng.integers(5, 30))
            A = dense.psd(n, np.exp(-np.arange(1, n + 1) / 10.0), seed=10000 + p)
            probs.append(dict(A=_dev(A), k=k, l=k + 5, its=2, seed=20000 + p, kind="psd"))
        elif p == 5:  # sparse
            m, n = 3000, 2500
            rp, ci, va = sparse.random_rows(m, n, 10, seed=10000 + p)
            cp, ri, vt = sparse.transpose(m, n, rp, ci, va)
            S = gpu_lib.csr(m, n, _dev(rp), _dev(ci), _dev(va), _dev(cp), _dev(ri), _dev(vt))
            A = sparse.to_scipy(m, n, rp, ci, va)
            probs.append(dict(A=S, k=10, l=15, its=2, seed=20000 + p))
        else:
            m = int(np.exp(rng.uniform(np.log(256), np.log(4096))))
            n = int(np.exp(rng.uniform(np.log(64), np.log(1024))))
            k = int(rng.integers(5, min(40, min(m, n) - 5)))
            A = dense.dense(m, n, np.arange(1, min(m, n) + 1, dtype=np.float64) ** -1.5,
                            seed=10000 + p)
            probs.append(dict(A=_dev(A), k=k, l=k + 5, its=2, seed=20000 + p, center=(p % 2 == 0)))
        host.append(A)
    return probs, host


def _single(ctx, pr):
    if pr.get("kind") == "psd":
        return ctx.eig_psd(pr["A"], pr["k"], pr["l"], pr["its"], pr["seed"], sync=True)
    return ctx.svd(pr["A"], pr["k"], pr["l"], pr["its"], pr["seed"], center=pr.get("center", False),
                   sync=True)


def test_batched_equals_single_calls(ctx, gpu_lib):
    # streams mode: the single-problem kernels, so bit-identical results
    probs, host = _batch(gpu_lib)
    ctx.set_batch_mode(1)
    try:
        outs = ctx.svd_batched(probs, sync=True)
    finally:
        ctx.set_batch_mode(0)
    for pr, got in zip(probs, outs):
        want = _single(ctx, pr)
        for g, w in zip(got, want):
            assert torch.equal(g, w)
    # sampled oracle parity
    for i in (0, 3, 5):
        pr, A = probs[i], host[i]
        n = A.shape[1]
        om = philox.omega(pr["seed"], n, pr["l"])
        if pr.get("kind") == "psd":
            _, S0, _, _ = nystrom.eig_psd(A, pr["k"], pr["l"], pr["its"], om, u_A=2.0 ** -16)
        else:
            _, S0, _ = rsvd.rsvd(A, pr["k"], pr["l"], pr["its"], om, center=pr.get("center", False))
        np.testing.assert_allclose(outs[i][1].cpu().numpy(), S0, rtol=1e-4)


def test_batched_graph_replay(ctx, gpu_lib):
    probs, _ = _batch(gpu_lib, seed=5001, count=12)
    s = torch.cuda.Stream()
    ctx.set_stream(s)
    try:
        with torch.cuda.stream(s):
            eager = ctx.svd_batched(probs)       # also sizes the per-stream workspaces
            s.synchronize()
            eager = [[t.clone() for t in o] for o in eager]
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                outs = ctx.svd_batched(probs)
        junk = torch.zeros(1 << 20, device="cuda")
        for rep in range(3):
            for o in outs:
                for t in o:
                    t.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                for t, te in zip(o, e):
                    assert torch.equal(t, te), "replay %d differs" % rep
            junk.add_(1.0)                       # eager work between replays
            torch.cuda.synchronize()
    finally:
        ctx.set_stream(torch.cuda.current_stream())


def test_batched_rejects_bad_problem(ctx, gpu_lib):
    A = torch.randn(100, 50, device="cuda")
    with pytest.raises(gpu_lib.RpcaError):
        ctx.svd_batched([dict(A=A, k=5), dict(A=A, k=60)])   # k > min(m, n)
