"""The periodic (exp-sine-squared) Mercer kernel through the C ABI against the
FP64 oracle's periodic expansion (Jacobi-Anger; the oracle's pins tie it to
the closed-form kernel): fit and predict on the FP64 and both mixed paths
(p = 1 on the direct Gram, p >= 2 on the paired Gram), the log marginal
likelihood, the full predictive covariance, the batched fit, and the
argument checks.  Tolerances as in test_gpu_parity (tests/_errs.py), both
normwise and max-relative: FP64 1e-10 on mean, variance and w; mixed 1e-5 on
the mean, 1e-4 on the variance."""
import numpy as np
import pytest

from _errs import TOL64, TOL_MEAN_MIXED, TOL_VAR_MIXED, assert_within, errs, fmt
from oracle import mercer_gp as o
from paper_2403_12797_amd import binding as B
from paper_2403_12797_amd import workloads as wl

pytestmark = pytest.mark.gpu
KP = B.KERNEL_PERIODIC


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = B.Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def fit(torch, ctx, P, precision):
    return ctx.fit(dev(torch, P.x), dev(torch, P.y), p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha,
                   precision=precision, kernel=KP)


def oracle(P):
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n, kernel="periodic")
    return f, o.predict(f, P.xs)


CASES = [(81, 1, 15, 4000, 500), (82, 2, 7, 20000, 700), (83, 3, 6, 30000, 600), (84, 2, 12, 12000, 400)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_periodic_fit_predict(torch_cuda, ctx, case, precision):
    torch = torch_cuda
    P = wl.periodic_problem(*case)
    print(f"[case] {P.name} precision={precision} N={P.N} Ns={P.Ns} M={P.M}", flush=True)
    m = fit(torch, ctx, P, precision)
    mean = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    var = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    ctx.predict(m, dev(torch, P.xs), mean, var)
    torch.cuda.synchronize()
    f, (om, ov) = oracle(P)
    e_m, e_v, e_w = errs(mean.cpu().numpy(), om), errs(var.cpu().numpy(), ov), errs(m.weights(), f.w)
    print(f"[err] periodic {P.name} prec={precision} mean={fmt(e_m)} var={fmt(e_v)} w={fmt(e_w)}", flush=True)
    if precision == B.PREC_FP64:
        assert_within(e_m, TOL64, "mean")
        assert_within(e_v, TOL64, "variance")
        assert_within(e_w, TOL64, "w")
    else:
        assert_within(e_m, TOL_MEAN_MIXED, "mean")
        assert_within(e_v, TOL_VAR_MIXED, "variance")
    m.free()


@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED_F16])
def test_periodic_lml_and_covariance(torch_cuda, ctx, precision):
    torch = torch_cuda
    P = wl.periodic_problem(85, 2, 6, 6000, 150)
    m = fit(torch, ctx, P, precision)
    f, _ = oracle(P)
    lml, want = m.lml(), o.log_marginal_likelihood(f, P.y)
    cov = torch.empty((P.Ns, P.Ns), dtype=torch.float64, device="cuda")
    ctx.predict_cov(m, dev(torch, P.xs), cov)
    torch.cuda.synchronize()
    e_c = errs(cov.cpu().numpy().ravel(), o.predict_cov(f, P.xs).ravel())
    e_l = abs(lml - want) / abs(want)
    print(f"[err] periodic lml prec={precision} rel={e_l:.3e} cov={fmt(e_c)}", flush=True)
    assert e_l <= (TOL64 if precision == B.PREC_FP64 else 1e-6)
    assert_within(e_c, TOL64 if precision == B.PREC_FP64 else TOL_VAR_MIXED, "covariance")
    m.free()


def test_periodic_batch_equals_single(torch_cuda, ctx):
    torch = torch_cuda
    Ps = [wl.periodic_problem(90 + k, 1 + k % 3, 5 + k, 3000 + 1000 * k, 100) for k in range(4)]
    dx = [(dev(torch, P.x), dev(torch, P.y)) for P in Ps]
    models = ctx.fit_batch([(x, y, P.p, P.n, P.sigma, P.eps, P.alpha) for (x, y), P in zip(dx, Ps)],
                           precision=B.PREC_MIXED_F16, kernel=KP)
    for (x, y), P, mb in zip(dx, Ps, models):
        ms = ctx.fit(x, y, p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha, precision=B.PREC_MIXED_F16,
                     kernel=KP)
        assert np.array_equal(mb.weights(), ms.weights()), P.name
        mb.free()
        ms.free()


def test_periodic_argument_checks(torch_cuda, ctx):
    torch = torch_cuda
    P = wl.periodic_problem(86, 1, 5, 500, 10)
    x, y = dev(torch, P.x), dev(torch, P.y)
    with pytest.raises(B.GpError) as ei:
        ctx.fit(x, y, p=1, n=5, sigma=0.1, eps=17.0, alpha=1.0, kernel=KP)
    assert ei.value.status == B.GP_EINVAL
    with pytest.raises(B.GpError) as ei:
        ctx.fit(x, y, p=1, n=5, sigma=0.1, eps=1.0, alpha=1.0, kernel=7)
    assert ei.value.status == B.GP_EINVAL
