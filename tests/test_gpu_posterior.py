"""Beyond the posterior diagonal, through the C ABI against the FP64 oracle:
the log marginal likelihood of a fit (gp_model_lml), the full predictive
covariance of a block of test points (gp_predict_cov) and hyperparameter
learning (gp_learn).

Tolerances: the FP64 path 1e-10 (log likelihood relative; covariance
normwise and max-relative over the matrix).  Mixed models use their mixed A:
the log likelihood within 1e-6 relative, the covariance within the variance
tolerance 1e-4."""
import numpy as np
import pytest

from _errs import TOL64, TOL_VAR_MIXED, assert_within, errs, fmt
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


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = B.Context(0)
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def fit(torch, ctx, P, precision):
    return ctx.fit(dev(torch, P.x), dev(torch, P.y), p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha,
                   precision=precision)


CASES = [("c1", None), ("rand", (61, 2, 5, 3000, 200)), ("rand", (62, 3, 6, 8000, 300)), ("c2", 20000)]


def problem(kind, arg):
    if kind == "c1":
        return wl.config("c1")
    if kind == "c2":
        return wl.config("c2", N=arg, Ns=400)
    return wl.random_problem(*arg)


@pytest.mark.parametrize("kind,arg", CASES)
@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_log_marginal_likelihood(torch_cuda, ctx, kind, arg, precision):
    P = problem(kind, arg)
    print(f"[case] lml {P.name} precision={precision} N={P.N} M={P.M}", flush=True)
    m = fit(torch_cuda, ctx, P, precision)
    got = m.lml()
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
    want = o.log_marginal_likelihood(f, P.y)
    e = abs(got - want) / abs(want)
    print(f"[err] lml {P.name} prec={precision} got={got:.12e} want={want:.12e} rel={e:.3e}", flush=True)
    assert e <= (TOL64 if precision == B.PREC_FP64 else 1e-6)
    m.free()


@pytest.mark.parametrize("kind,arg", [("rand", (63, 2, 6, 4000, 333)), ("rand", (64, 4, 4, 6000, 130)),
                                      ("c2", 20000)])
@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED_F16])
def test_full_covariance(torch_cuda, ctx, kind, arg, precision):
    torch = torch_cuda
    P = problem(kind, arg)
    print(f"[case] cov {P.name} precision={precision} M={P.M} Ns={P.Ns}", flush=True)
    m = fit(torch, ctx, P, precision)
    xs = dev(torch, P.xs)
    cov = torch.full((P.Ns, P.Ns + 3), float("nan"), dtype=torch.float64, device="cuda")   # pitch > Ns
    ctx.predict_cov(m, xs, cov)
    var = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    ctx.predict(m, xs, None, var)
    torch.cuda.synchronize()
    C = cov.cpu().numpy()
    assert np.isnan(C[:, P.Ns:]).all()          # the padding columns are not written
    C = C[:, :P.Ns]
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
    want = o.predict_cov(f, P.xs)
    e = errs(C.ravel(), want.ravel())
    ed = errs(np.diag(C), var.cpu().numpy())
    print(f"[err] cov {P.name} prec={precision} cov={fmt(e)} diag-vs-predict={fmt(ed)}", flush=True)
    assert_within(e, TOL64 if precision == B.PREC_FP64 else TOL_VAR_MIXED, "covariance")
    assert np.array_equal(C, C.T) or errs(C.ravel(), C.T.ravel())[1] <= 1e-14
    assert_within(ed, 1e-12 if precision == B.PREC_FP64 else TOL_VAR_MIXED, "diagonal vs gp_predict")
    m.free()


def test_covariance_rejects_bad_pitch(torch_cuda, ctx):
    torch = torch_cuda
    P = wl.random_problem(65, 2, 4, 500, 20)
    m = fit(torch, ctx, P, B.PREC_FP64)
    cov = torch.empty((20, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(B.GpError) as ei:
        ctx.predict_cov(m, dev(torch, P.xs), cov)
    assert ei.value.status == B.GP_EINVAL
    m.free()


def test_learn_maximises_the_likelihood(torch_cuda, ctx):
    """gp_learn from a poor start (shared eps and sigma learnt, alpha kept):
    the likelihood it reports is the oracle's at the point it returns, it
    improves on the start, and it reaches the optimum that scipy's
    Nelder-Mead finds on the oracle's likelihood from the same start and
    initial simplex."""
    from scipy.optimize import minimize
    torch = torch_cuda
    P = wl.random_problem(66, 2, 6, 3000, 10, sigma=0.1, eps=1.0, alpha=1.0)
    x, y = dev(torch, P.x), dev(torch, P.y)
    eps0, sig0 = 2.5, 0.4
    e_out, a_out, s_out, lml, evals = ctx.learn(x, y, p=P.p, n=P.n, sigma=sig0, eps=eps0, alpha=1.0,
                                                precision=B.PREC_FP64, max_evals=120, learn_alpha=False,
                                                learn_sigma=True, tol=1e-7)

    def olml(le, ls):
        f = o.fit(P.x, P.y, float(np.exp(ls)), float(np.exp(le)), 1.0, P.n)
        return o.log_marginal_likelihood(f, P.y)

    at_result = olml(np.log(e_out[0]), np.log(s_out))
    start = olml(np.log(eps0), np.log(sig0))
    th0 = np.array([np.log(eps0), np.log(sig0)])
    res = minimize(lambda th: -olml(*th), th0, method="Nelder-Mead",
                   options={"initial_simplex": np.array([th0, th0 + [0.3, 0], th0 + [0, 0.3]]),
                            "xatol": 1e-6, "fatol": 1e-7, "maxfev": 400})
    print(f"[err] learn evals={evals} eps={e_out[0]:.6f} sigma={s_out:.6f} lml={lml:.9e} oracle-at-result="
          f"{at_result:.9e} start={start:.6e} scipy-opt={-res.fun:.9e} (eps={np.exp(res.x[0]):.6f}, "
          f"sigma={np.exp(res.x[1]):.6f})", flush=True)
    assert abs(lml - at_result) <= 1e-10 * abs(at_result)
    assert lml > start
    assert np.allclose(a_out, 1.0)
    assert abs(lml - (-res.fun)) <= 1e-6 * abs(res.fun)
