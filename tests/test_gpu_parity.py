"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Tolerances, each asserted both normwise (||got - want||_2 / ||want||_2) and
as max|got - want| / max|want| per result vector (tests/_errs.py):
  FP64 path: 1e-10 on mean, variance and w.
  Mixed paths (Gram as split-BF16 with three terms or as scaled split-FP16
  with two terms; split-BF16 variance; FP64 factorisation, one FP64
  refinement step): 1e-5 on the mean, 1e-4 on the variance.
"""
import os

import numpy as np
import pytest

from _errs import TOL64, TOL_MEAN_MIXED, TOL_VAR_MIXED, assert_within, errs, fmt
from oracle import mercer_gp as o
from paper_2403_12797_amd import binding as B
from paper_2403_12797_amd import workloads as wl

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


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


def gpu_fit_predict(torch, ctx, P, precision):
    print(f"[case] {P.name} precision={precision} N={P.N} Ns={P.Ns} M={P.M}", flush=True)
    x, y, xs = dev(torch, P.x), dev(torch, P.y), dev(torch, P.xs)
    m = ctx.fit(x, y, p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha, precision=precision)
    mean = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    var = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    ctx.predict(m, xs, mean, var)
    torch.cuda.synchronize()
    return m, mean.cpu().numpy(), var.cpu().numpy()


def oracle_fit_predict(P):
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
    mean, var = o.predict(f, P.xs)
    return f, mean, var


def check(P, got, want, precision, extra="", w_ref=None):
    """Assert the mean and variance (and, FP64, w) within tolerance, both
    normwise and max-relative; print both (norm/max) on the [err] line."""
    m, gmean, gvar = got
    omean, ovar = want[1], want[2]
    e_mean, e_var = errs(gmean, omean), errs(gvar, ovar)
    w = m.weights()
    e_w = errs(w, want[0].w if w_ref is None else w_ref)
    print(f"[err] {P.name} prec={precision} mean={fmt(e_mean)} var={fmt(e_var)} w={fmt(e_w)} {extra}", flush=True)
    if precision == B.PREC_FP64:
        assert_within(e_mean, TOL64, "mean")
        assert_within(e_var, TOL64, "variance")
        assert_within(e_w, TOL64, "w")
    else:
        assert_within(e_mean, TOL_MEAN_MIXED, "mean")
        assert_within(e_var, TOL_VAR_MIXED, "variance")
    return e_mean, e_var


@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_c1_full(torch_cuda, ctx, precision):
    P = wl.config("c1")
    got = gpu_fit_predict(torch_cuda, ctx, P, precision)
    want = oracle_fit_predict(P)
    check(P, got, want, precision)
    lam = got[0].get(B.MODEL_LAMBDA)
    assert rel(lam, want[0].lam) <= 1e-14


def test_c1_stages_fp64(torch_cuda, ctx):
    """Per-stage parity: Lambda, A = Phi^T Phi + sigma^2 Lambda^-1, b = Phi^T y,
    and L L^T = A, L^-1 L = I."""
    P = wl.config("c1")
    m, _, _ = gpu_fit_predict(torch_cuda, ctx, P, B.PREC_FP64)
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
    assert rel(m.get(B.MODEL_A), f.A) <= 1e-13
    assert rel(m.get(B.MODEL_B), f.b) <= 1e-13
    L = m.get(B.MODEL_L)
    assert np.allclose(np.triu(L, 1), 0.0)
    assert rel(L @ L.T, f.A) <= 1e-13
    Li = m.get(B.MODEL_LINV)
    assert np.abs(Li @ L - np.eye(P.M)).max() <= 1e-10


@pytest.mark.parametrize("seed,p,n,N", [(21, 2, 17, 3000), (22, 3, 11, 6000), (23, 1, 64, 500), (24, 2, 45, 8000)])
def test_factor_stages_multiblock(torch_cuda, ctx, seed, p, n, N):
    """Cholesky and L^-1 across several 64-blocks and recursion levels,
    including ragged last blocks (M = 289, 1331, 64, 2025)."""
    P = wl.random_problem(seed, p, n, N, 10)
    m, _, _ = gpu_fit_predict(torch_cuda, ctx, P, B.PREC_FP64)
    A = m.get(B.MODEL_A)
    L = m.get(B.MODEL_L)
    Li = m.get(B.MODEL_LINV)
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
    assert rel(A, f.A) <= 1e-12
    assert np.allclose(np.triu(L, 1), 0.0) and np.allclose(np.triu(Li, 1), 0.0)
    assert rel(L @ L.T, A) <= 1e-13
    # L^-1 L = I to rounding, measured against |L^-1| |L| (scale-free)
    E = np.abs(Li @ L - np.eye(P.M)) / (np.abs(Li) @ np.abs(L) + 1e-300)
    print(f"[err] stages {P.name}: max |Li L - I| / (|Li||L|) = {E.max():.3e}", flush=True)
    assert E.max() <= 1e-12


@pytest.mark.parametrize("knob", [("MGP_SYRK_ORDER", "0"), ("MGP_CHOL_DIAG", "block")])
def test_factor_stages_alternative_paths(torch_cuda, ctx, monkeypatch, knob):
    """The non-default factorisation paths behind the tuning knobs: the
    trailing update in plain column order, and the 512-thread diagonal
    factor (M = 2025: eight outer panels, a ragged last block)."""
    monkeypatch.setenv(*knob)
    P = wl.random_problem(28, 2, 45, 8000, 10)
    m, _, _ = gpu_fit_predict(torch_cuda, ctx, P, B.PREC_FP64)
    A = m.get(B.MODEL_A)
    L = m.get(B.MODEL_L)
    Li = m.get(B.MODEL_LINV)
    assert rel(L @ L.T, A) <= 1e-13
    E = np.abs(Li @ L - np.eye(P.M)) / (np.abs(Li) @ np.abs(L) + 1e-300)
    print(f"[err] stages {knob[0]}={knob[1]} {P.name}: max |Li L - I| / (|Li||L|) = {E.max():.3e}", flush=True)
    assert E.max() <= 1e-12


@pytest.mark.parametrize("seed,p,n,N,Ns", [
    (1, 1, 1, 1, 1),          # smallest problem
    (2, 1, 7, 5, 3),          # M > N
    (3, 2, 5, 257, 65),       # ragged tails
    (4, 2, 12, 1000, 300),    # M = 144: two 128-tiles, ragged
    (5, 3, 6, 3000, 1000),    # M = 216
    (6, 4, 5, 2000, 777),     # M = 625
    (7, 5, 3, 4097, 129),     # M = 243
    (8, 1, 40, 600, 100),     # long 1-D expansion
    (9, 8, 2, 1500, 200),     # p = 8, M = 256
    (10, 3, 11, 5000, 513),   # M = 1331 (several 256-tiles, ragged)
    (11, 7, 3, 3000, 300),    # M = 2187: prediction reads prefix digits from global memory
    (12, 2, 64, 4000, 300),   # M = 4096, 128 table rows: 128-point prediction tiles
])
@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_random_shapes(torch_cuda, ctx, seed, p, n, N, Ns, precision):
    P = wl.random_problem(seed, p, n, N, Ns)
    got = gpu_fit_predict(torch_cuda, ctx, P, precision)
    want = oracle_fit_predict(P)
    check(P, got, want, precision)


@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_c2_shape(torch_cuda, ctx, precision):
    """p = 3, n = 8 (M = 512), x ~ N(0, I): N reduced to 20000 for the oracle."""
    P = wl.config("c2", N=20_000, Ns=4_000)
    got = gpu_fit_predict(torch_cuda, ctx, P, precision)
    check(P, got, oracle_fit_predict(P), precision)


@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_c3_shape_reduced(torch_cuda, ctx, precision):
    """p = 4, n = 8 (M = 4096), alpha = 1.2: N reduced to 30000 for the oracle."""
    P = wl.config("c3", N=30_000, Ns=3_000)
    got = gpu_fit_predict(torch_cuda, ctx, P, precision)
    check(P, got, oracle_fit_predict(P), precision)


def test_empty_predict_and_null_outputs(torch_cuda, ctx):
    torch = torch_cuda
    P = wl.random_problem(11, 2, 4, 100, 10)
    m, mean, var = gpu_fit_predict(torch, ctx, P, B.PREC_FP64)
    xs = dev(torch, P.xs)
    ctx.predict(m, xs[:0], None, None)                         # Ns = 0
    only_mean = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    ctx.predict(m, xs, only_mean, None)
    only_var = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    ctx.predict(m, xs, None, only_var)
    torch.cuda.synchronize()
    assert np.array_equal(only_mean.cpu().numpy(), mean)
    assert np.array_equal(only_var.cpu().numpy(), var)


def test_invalid_arguments(torch_cuda, ctx):
    torch = torch_cuda
    x = torch.zeros((10, 2), dtype=torch.float64, device="cuda")
    y = torch.zeros(10, dtype=torch.float64, device="cuda")
    bad = [dict(p=0, n=4), dict(p=2, n=0), dict(p=2, n=65), dict(p=9, n=2), dict(p=2, n=200),
           dict(p=3, n=26)]  # 26^3 > 16384
    for kw in bad:
        with pytest.raises(B.GpError) as ei:
            ctx.fit(x, y, sigma=0.1, eps=1.0, alpha=1.0, **kw)
        assert ei.value.status == B.GP_EINVAL
    for sig, e, a in [(0.0, 1.0, 1.0), (-1.0, 1.0, 1.0), (float("nan"), 1.0, 1.0), (0.1, 0.0, 1.0),
                      (0.1, 1.0, -2.0), (0.1, float("inf"), 1.0)]:
        with pytest.raises(B.GpError) as ei:
            ctx.fit(x, y, p=2, n=3, sigma=sig, eps=e, alpha=a)
        assert ei.value.status == B.GP_EINVAL
    with pytest.raises(B.GpError):
        ctx.fit(x, y, p=2, n=3, sigma=0.1, eps=1.0, alpha=1.0, precision=7)
    xn = x.clone()
    xn[3, 1] = float("nan")
    with pytest.raises(B.GpError) as ei:
        ctx.fit(xn, y, p=2, n=3, sigma=0.1, eps=1.0, alpha=1.0)
    assert ei.value.status == B.GP_EINVAL and "non-finite" in str(ei.value)
    yn = y.clone()
    yn[0] = float("inf")
    with pytest.raises(B.GpError):
        ctx.fit(x, yn, p=2, n=3, sigma=0.1, eps=1.0, alpha=1.0)


@pytest.mark.parametrize("precision", [B.PREC_MIXED, B.PREC_MIXED_F16])
def test_deterministic_repeat(torch_cuda, ctx, precision):
    """Same inputs twice give bitwise-equal results (fixed reduction orders)."""
    P = wl.random_problem(12, 3, 6, 20000, 2000)
    a = gpu_fit_predict(torch_cuda, ctx, P, precision)
    b = gpu_fit_predict(torch_cuda, ctx, P, precision)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", [B.PREC_MIXED, B.PREC_MIXED_F16])
@pytest.mark.parametrize("seed,p,n,spread,shift,eps,alpha", [
    (31, 3, 8, 3.0, 2.0, None, None),   # wide inputs: |Phi| up to ~2e3
    (33, 4, 6, 2.0, -3.0, None, None),  # shifted, one-sided
    (37, 2, 16, 1.5, 1.0, 2.0, 1.0),    # long 1-D expansions, |Phi| up to ~7e2
    (39, 4, 6, 2.5, 0.0, 1.0, 1.5),     # |Phi| up to ~8e4: beyond FP16 without the scaling
])
def test_mixed_gram_range(torch_cuda, ctx, precision, seed, p, n, spread, shift, eps, alpha):
    """The Gram of both mixed schemes against the oracle's A (normwise 1e-6)
    and the end results within the mixed tolerances, on inputs whose 1-D
    eigenfunction values span many orders of magnitude (the FP16 scheme's
    per-row power-of-two scaling has to keep them in range)."""
    Q = wl.random_problem(seed, p, n, 6000, 500, dist="normal", eps=eps, alpha=alpha)
    x = Q.x * spread
    x[:, 0] += shift
    xs = Q.xs * spread
    xs[:, 0] += shift
    y = np.cos(x).sum(axis=1) + np.random.default_rng(seed).normal(0.0, Q.sigma, size=x.shape[0])
    P = wl.Problem(f"range{seed}_p{p}_n{n}", p, n, Q.sigma, Q.eps, Q.alpha, x, y, xs)
    got = gpu_fit_predict(torch_cuda, ctx, P, precision)
    want = oracle_fit_predict(P)
    e_A = rel(got[0].get(B.MODEL_A), want[0].A)
    check(P, got, want, precision, extra=f"A={e_A:.3e}")
    assert e_A <= 1e-6


@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_c5_largest_request_shape(torch_cuda, ctx, precision):
    """The served stream's largest expansion, p = 5, n = 6 (M = 7776), at
    N = 50000, N_* = 2000, against the oracle's values in
    golden/c5_p5_oracle.npz (written by golden/make_shape_goldens.py)."""
    g = np.load(os.path.join(GOLDEN, "c5_p5_oracle.npz"))
    P = wl.config("c5")
    assert int(g["N"]) == P.N and int(g["Ns"]) == P.Ns and int(g["M"]) == P.M
    got = gpu_fit_predict(torch_cuda, ctx, P, precision)
    e_b = errs(got[0].get(B.MODEL_B), g["b"])
    check(P, got, (None, g["mean"], g["var"]), precision, extra=f"b={fmt(e_b)}", w_ref=g["w"])
    assert_within(e_b, 1e-12, "b")


@pytest.mark.parametrize("precision", [B.PREC_FP64, B.PREC_MIXED, B.PREC_MIXED_F16])
def test_paper_shape(torch_cuda, ctx, precision):
    """The paper's data-set shape (Sec. 3, the Sec. 4 headline): p = 4, n = 11
    (M = 14641), N = N_* = 10000, against golden/paper_oracle.npz."""
    g = np.load(os.path.join(GOLDEN, "paper_oracle.npz"))
    P = wl.config("paper")
    assert int(g["N"]) == P.N and int(g["Ns"]) == P.Ns and int(g["M"]) == P.M
    got = gpu_fit_predict(torch_cuda, ctx, P, precision)
    e_b = errs(got[0].get(B.MODEL_B), g["b"])
    check(P, got, (None, g["mean"], g["var"]), precision, extra=f"b={fmt(e_b)}", w_ref=g["w"])
    assert_within(e_b, 1e-12, "b")
