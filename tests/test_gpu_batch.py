"""Batched fit/predict (gp_fit_batch / gp_predict_batch, one persistent Gram
launch for all mixed problems, direct launches or one captured graph) and the
autotuner.

* every batched result equals the same problem fitted alone (bitwise: the
  batch uses the same per-problem chunking and reduction order);
* a sample of problems matches the FP64 oracle within the mixed tolerances;
* a failing problem (non-finite input) leaves the others intact.
"""
import numpy as np
import pytest

from _errs import TOL64, TOL_MEAN_MIXED, TOL_VAR_MIXED, assert_within, errs, fmt
from oracle import mercer_gp as o
from paper_2403_12797_amd import binding as B
from paper_2403_12797_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def batch_problems(count=24, N_max=20_000):
    # the batched workload's distribution (p in 1..3, n in 4..12, log-uniform N) at oracle-friendly sizes
    return wl.batched_problems(count, N_max=N_max)


def single(ctx, torch, P, prec):
    x, y, xs = dev(torch, P.x), dev(torch, P.y), dev(torch, P.xs)
    m = ctx.fit(x, y, p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha, precision=prec)
    mean = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    var = torch.empty_like(mean)
    ctx.predict(m, xs, mean, var)
    torch.cuda.synchronize()
    w = m.get(B.MODEL_W)
    m.free()
    return w, mean.cpu().numpy(), var.cpu().numpy()


@pytest.mark.parametrize("prec", [B.PREC_MIXED, B.PREC_MIXED_F16, B.PREC_FP64, "all three"])
def test_batch_equals_single_and_oracle(torch_cuda, prec):
    """Every problem of a batch equals its single fit bitwise; "all three"
    mixes FP16-Gram, BF16-Gram and FP64 problems in one batch (one persistent
    Gram launch per split scheme)."""
    torch = torch_cuda
    Ps = batch_problems()
    modes = (B.PREC_MIXED_F16, B.PREC_MIXED, B.PREC_FP64)
    precs = [modes[k % 3] for k in range(len(Ps))] if prec == "all three" else [prec] * len(Ps)
    with B.Context(0) as ctx:
        dx = [(dev(torch, P.x), dev(torch, P.y), P.p, P.n, P.sigma, P.eps, P.alpha) for P in Ps]
        models = ctx.fit_batch(dx, precision=precs)
        xs = [dev(torch, P.xs) for P in Ps]
        means = [torch.empty(P.Ns, dtype=torch.float64, device="cuda") for P in Ps]
        vars_ = [torch.empty(P.Ns, dtype=torch.float64, device="cuda") for P in Ps]
        ctx.predict_batch(models, xs, means, vars_)
        torch.cuda.synchronize()
        for k, P in enumerate(Ps):
            print(f"[case] batch {P.name} prec={precs[k]} M={P.M}", flush=True)
            w_s, m_s, v_s = single(ctx, torch, P, precs[k])
            assert np.array_equal(models[k].get(B.MODEL_W), w_s)
            assert np.array_equal(means[k].cpu().numpy(), m_s)
            assert np.array_equal(vars_[k].cpu().numpy(), v_s)
        for k in range(0, len(Ps), 6):
            P = Ps[k]
            f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
            om, ov = o.predict(f, P.xs)
            em, ev = errs(means[k].cpu().numpy(), om), errs(vars_[k].cpu().numpy(), ov)
            print(f"[err] batch {P.name} prec={precs[k]} mean={fmt(em)} var={fmt(ev)}", flush=True)
            if precs[k] != B.PREC_FP64:
                assert_within(em, TOL_MEAN_MIXED, "mean")
                assert_within(ev, TOL_VAR_MIXED, "variance")
            else:
                assert_within(em, TOL64, "mean")
                assert_within(ev, TOL64, "variance")
        for m in models:
            m.free()


def test_batch_graph_equals_direct(torch_cuda, monkeypatch):
    """The batch captured in one HIP graph (MGP_BATCH_GRAPH=1) gives the same
    models bitwise as the default direct launches."""
    torch = torch_cuda
    Ps = batch_problems(12)
    precs = [(B.PREC_MIXED_F16, B.PREC_MIXED, B.PREC_FP64)[k % 3] for k in range(len(Ps))]
    with B.Context(0) as ctx:
        xs = [(dev(torch, P.x), dev(torch, P.y)) for P in Ps]
        probs = [(x, y, P.p, P.n, P.sigma, P.eps, P.alpha) for (x, y), P in zip(xs, Ps)]
        got = {}
        for mode in ("0", "1"):
            monkeypatch.setenv("MGP_BATCH_GRAPH", mode)
            models = ctx.fit_batch(probs, precision=precs)
            torch.cuda.synchronize()
            got[mode] = [(m.get(B.MODEL_W), m.get(B.MODEL_LINV)) for m in models]
            for m in models:
                m.free()
    for k, P in enumerate(Ps):
        print(f"[case] batch graph/direct {P.name} prec={precs[k]}", flush=True)
        assert np.array_equal(got["0"][k][0], got["1"][k][0]) and np.array_equal(got["0"][k][1], got["1"][k][1])


def test_batch_failure_isolated(torch_cuda):
    torch = torch_cuda
    Ps = batch_problems(6)
    with B.Context(0) as ctx:
        dx = [(dev(torch, P.x), dev(torch, P.y), P.p, P.n, P.sigma, P.eps, P.alpha) for P in Ps]
        bad = dx[2][0].clone()
        bad[0, 0] = float("nan")
        dx[2] = (bad,) + dx[2][1:]
        with pytest.raises(B.GpError) as ei:
            ctx.fit_batch(dx)
        assert ei.value.status == B.GP_EINVAL and "problem 2" in str(ei.value)
        models = ei.value.models
        assert models[2] is None
        for k in (0, 1, 3, 4, 5):
            assert models[k] is not None
            w = models[k].get(B.MODEL_W)
            assert np.all(np.isfinite(w))
            models[k].free()


def test_autotune_then_fit(torch_cuda):
    torch = torch_cuda
    P = wl.random_problem(31, 3, 8, 40_000, 2_000)
    with B.Context(0) as ctx:
        chunk = ctx.autotune(P.p, P.n, P.N)
        print(f"[case] autotune p=3 n=8 N=40000 -> chunk {chunk}", flush=True)
        assert chunk % 16 == 0 and 1024 <= chunk <= 32768
        w, mean, var = single(ctx, torch, P, B.PREC_MIXED_F16)
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
    om, ov = o.predict(f, P.xs)
    assert_within(errs(mean, om), TOL_MEAN_MIXED, "mean")
    assert_within(errs(var, ov), TOL_VAR_MIXED, "variance")
