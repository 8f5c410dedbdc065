"""Pins of the FP64 CPU oracle against facts that do not come from the oracle
itself: closed forms, textbook/library routines, exactness of Gauss-Hermite
quadrature, and the paper's alternative formulations of the same posterior.

Each pin is chosen so that a plausible mistake (wrong delta^2, wrong Hermite
convention, dropped normalisation, wrong multi-index order, dropped noise
term, transposed operand) fails at least one of them; the tests at the end
plant such mistakes in a copy of the oracle and check that a pin catches them.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as sps
from numpy.polynomial.hermite import hermgauss

from oracle import mercer_gp as o

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# ---------------------------------------------------------------- 1-D pins
@pytest.mark.parametrize("alpha", [1.0, 1.2])
def test_mercer_sum_reproduces_se_kernel_1d(alpha):
    """Eq. (5)/(6) with (15)-(16): 40 terms reproduce exp(-eps^2 (x-x')^2),
    the closed form (13), to 1e-12 on |x|, |x'| <= 3."""
    x = np.linspace(-3.0, 3.0, 73)
    phi = o.eigenfunctions_1d(x, 1.0, alpha, 40)
    lam = o.eigenvalues_1d(1.0, alpha, 40)
    K = (phi * lam) @ phi.T
    Kt = np.exp(-(x[:, None] - x[None, :]) ** 2)
    assert np.abs(K - Kt).max() <= 1e-12


@pytest.mark.parametrize("eps,alpha", [(1.0, 1.0), (2.0, 1.0), (1.0, 1.2), (1.0, 0.5), (0.8, 1.0)])
def test_orthonormality_gauss_hermite(eps, alpha):
    """phi_k are orthonormal under rho(x) = alpha/sqrt(pi) exp(-alpha^2 x^2).
    In u = alpha beta x the integrand is (polynomial) * exp(-u^2) exactly when
    alpha^2 + 2 delta^2 = alpha^2 beta^2, so a 20-node Gauss-Hermite rule is
    exact for n = 12 and the Gram of the quadrature must be the identity."""
    n = 12
    u, wq = hermgauss(20)
    beta, _ = o.se_scalars(eps, alpha)
    xq = u / (alpha * beta)
    phi = o.eigenfunctions_1d(xq, eps, alpha, n)
    rho = alpha / math.sqrt(math.pi) * np.exp(-(alpha * xq) ** 2)
    wts = wq * np.exp(u * u) * rho / (alpha * beta)
    G = (phi * wts[:, None]).T @ phi
    assert np.abs(G - np.eye(n)).max() <= 1e-13


@pytest.mark.parametrize("eps,alpha", [(1.0, 1.0), (2.0, 1.0), (1.0, 1.2), (1.0, 0.5), (0.6, 1.7)])
def test_eigenvalue_trace_is_one(eps, alpha):
    """sum_k lambda_k = integral k(x,x) rho(x) dx = 1 (k(x,x)=1 for (13)).
    Geometric series: lambda_1 / (1 - eps^2/D)."""
    lam = o.eigenvalues_1d(eps, alpha, 3)
    ratio = lam[1] / lam[0]
    assert abs(lam[0] / (1.0 - ratio) - 1.0) <= 1e-14


def test_closed_form_golden_ratio():
    """At eps = alpha = 1: beta = 5^(1/4), delta^2 = (sqrt5 - 1)/2,
    D = (3 + sqrt5)/2 and lambda_k = g^-(2k-1) with g the golden ratio
    (hand derivation: eps^2/D = 1/g^2, sqrt(1/D) = 1/g)."""
    beta, d2 = o.se_scalars(1.0, 1.0)
    assert abs(beta - 5.0 ** 0.25) <= 1e-15
    assert abs(d2 - (math.sqrt(5.0) - 1.0) / 2.0) <= 1e-15
    lam = o.eigenvalues_1d(1.0, 1.0, 12)
    want = GOLDEN ** -(2.0 * np.arange(1, 13) - 1.0)
    assert np.abs(lam / want - 1.0).max() <= 1e-14
    # phi_1 = sqrt(beta) exp(-delta^2 x^2); phi_2 = sqrt(beta/2) exp(-delta^2 x^2) 2 beta x
    x = np.array([-0.7, 0.0, 0.3, 1.9])
    phi = o.eigenfunctions_1d(x, 1.0, 1.0, 2)
    e = np.exp(-d2 * x * x)
    assert np.allclose(phi[:, 0], 5.0 ** 0.125 * e, rtol=1e-15, atol=0)
    assert np.allclose(phi[:, 1], math.sqrt(beta / 2.0) * e * 2.0 * beta * x, rtol=1e-15, atol=1e-300)


def test_diagonal_sum_is_one():
    """sum_k lambda_k phi_k(x)^2 -> k(x, x) = 1 at 40 terms, |x| <= 3."""
    x = np.linspace(-3.0, 3.0, 61)
    for alpha in (1.0, 1.2):
        phi = o.eigenfunctions_1d(x, 1.0, alpha, 40)
        lam = o.eigenvalues_1d(1.0, alpha, 40)
        assert np.abs((phi * phi) @ lam - 1.0).max() <= 1e-12


def test_hermite_matches_scipy():
    t = np.linspace(-4.0, 4.0, 33)
    H = o.hermite_physicists(t, 25)
    for k in range(25):
        ref = sps.eval_hermite(k, t)
        assert np.allclose(H[:, k], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------- p-variate pins
def test_multi_index_c_order():
    """n = 2, p = 3 enumerates binary counting with the last digit fastest."""
    idx = o.multi_indices(2, 3)
    want = np.array([[(m >> 2) & 1, (m >> 1) & 1, m & 1] for m in range(8)])
    assert np.array_equal(idx, want)
    idx = o.multi_indices(3, 2)
    assert np.array_equal(idx, np.array([[a, b] for a in range(3) for b in range(3)]))


def test_tensor_factorisation():
    """sum_m Lambda_m Phi_m(x) Phi_m(x') = prod_j sum_k lambda_jk phi_jk phi_jk
    (eqs. (18)-(20)); any n, p."""
    rng = np.random.default_rng(3)
    p, n = 3, 5
    eps, alpha = [1.0, 0.7, 1.4], [1.2, 0.9, 1.0]
    X1 = rng.uniform(-1, 1, (7, p))
    X2 = rng.uniform(-1, 1, (6, p))
    K = o.truncated_kernel(X1, X2, eps, alpha, n)
    prod = np.ones((7, 6))
    for j in range(p):
        a = o.eigenfunctions_1d(X1[:, j], eps[j], alpha[j], n)
        b = o.eigenfunctions_1d(X2[:, j], eps[j], alpha[j], n)
        prod *= (a * o.eigenvalues_1d(eps[j], alpha[j], n)) @ b.T
    assert np.abs(K - prod).max() <= 1e-14


def test_truncated_kernel_tends_to_ard():
    """Eq. (18) -> eq. (17) as n grows (p = 2, 30 terms per dim)."""
    rng = np.random.default_rng(4)
    X1 = rng.uniform(-1.5, 1.5, (20, 2))
    X2 = rng.uniform(-1.5, 1.5, (15, 2))
    K = o.truncated_kernel(X1, X2, [1.0, 0.7], [1.0, 1.2], 30)
    assert np.abs(K - o.se_ard_kernel(X1, X2, [1.0, 0.7])).max() <= 1e-12


# ---------------------------------------------------------------- posterior pins
def _small(seed, p, N=50, Ns=20):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (N, p))
    y = np.cos(X).sum(1) + 0.1 * rng.normal(size=N)
    Xs = rng.uniform(-1, 1, (Ns, p))
    return X, y, Xs


@pytest.mark.parametrize("p,n,eps,alpha", [(1, 10, 1.0, 1.0), (2, 5, [1.0, 1.3], [1.2, 0.9]),
                                           (3, 3, 0.8, 1.0)])
def test_weight_space_equals_nxn_truncated_posterior(p, n, eps, alpha):
    """F1 (M x M) vs F3 (eqs. (8)-(9), N x N): <= 1e-10 on mean and variance."""
    X, y, Xs = _small(p, p)
    f = o.fit(X, y, 0.1, eps, alpha, n)
    m1, v1 = o.predict(f, Xs)
    m3, C3 = o.posterior_truncated_nxn(X, y, Xs, 0.1, eps, alpha, n)
    assert rel(m1, m3) <= 1e-10
    assert rel(v1, np.diag(C3)) <= 1e-10


@pytest.mark.parametrize("p,n", [(1, 10), (2, 5)])
def test_weight_space_equals_paper_W_form(p, n):
    """F1 vs the paper's literal FAGP form (11)-(12) (F2).  F2 subtracts the
    explained variance from the prior one and divides by sigma^4, so the
    variance only agrees to ~1e-8."""
    X, y, Xs = _small(10 + p, p)
    f = o.fit(X, y, 0.1, 1.0, 1.2, n)
    m1, v1 = o.predict(f, Xs)
    m2, C2 = o.posterior_woodbury_W(X, y, Xs, 0.1, 1.0, 1.2, n)
    assert rel(m1, m2) <= 1e-10
    assert rel(v1, np.diag(C2)) <= 1e-8


def test_weight_space_tends_to_exact_se_posterior():
    """p = 1, n = 40, N = 50, |x| <= 2: F1 vs the exact GP posterior (3)-(4)
    with the closed-form kernel (13)."""
    rng = np.random.default_rng(5)
    X = rng.uniform(-2, 2, (50, 1))
    y = np.sin(3 * X[:, 0]) + 0.1 * rng.normal(size=50)
    Xs = np.linspace(-2, 2, 30)[:, None]
    f = o.fit(X, y, 0.1, 1.0, 1.0, 40)
    m1, v1 = o.predict(f, Xs)
    me, Ce = o.posterior_exact_se(X, y, Xs, 0.1, 1.0)
    assert rel(m1, me) <= 1e-10
    assert rel(v1, np.diag(Ce)) <= 1e-10


def test_weight_space_tends_to_exact_ard_posterior_p2():
    rng = np.random.default_rng(6)
    X = rng.uniform(-1.5, 1.5, (50, 2))
    y = np.cos(X).sum(1)
    Xs = rng.uniform(-1.5, 1.5, (20, 2))
    f = o.fit(X, y, 0.1, [1.0, 0.7], [1.0, 1.2], 30)
    m1, v1 = o.predict(f, Xs)
    me, Ce = o.posterior_exact_se(X, y, Xs, 0.1, [1.0, 0.7])
    assert rel(m1, me) <= 1e-10
    assert rel(v1, np.diag(Ce)) <= 1e-9


def test_multi_index_permutation_invariance():
    """Permuting the enumeration of (18) permutes w and leaves mu_*, v_* fixed."""
    X, y, Xs = _small(7, 3)
    f = o.fit(X, y, 0.1, 1.0, 1.2, 4)
    perm = np.random.default_rng(0).permutation(4 ** 3)
    g = o.fit(X, y, 0.1, 1.0, 1.2, 4, order=o.multi_indices(4, 3)[perm])
    mf, vf = o.predict(f, Xs)
    mg, vg = o.predict(g, Xs)
    assert rel(mg, mf) <= 1e-13 and rel(vg, vf) <= 1e-13
    assert np.allclose(g.w, f.w[perm], rtol=1e-11, atol=1e-13 * np.abs(f.w).max())


def test_single_term_closed_form():
    """p = 1, n = 1: w = sum phi_i y_i / (sum phi_i^2 + sigma^2/lambda_1)."""
    rng = np.random.default_rng(8)
    X = rng.uniform(-1, 1, (40, 1))
    y = rng.normal(size=40)
    f = o.fit(X, y, 0.3, 1.1, 0.9, 1)
    beta, d2 = o.se_scalars(1.1, 0.9)
    phi = math.sqrt(beta) * np.exp(-d2 * X[:, 0] ** 2)
    lam1 = o.eigenvalues_1d(1.1, 0.9, 1)[0]
    w = (phi @ y) / (phi @ phi + 0.09 / lam1)
    assert abs(f.w[0] - w) <= 1e-14 * abs(w)
    xs = np.array([[0.25]])
    m, v = o.predict(f, xs)
    ps = math.sqrt(beta) * math.exp(-d2 * 0.0625)
    assert abs(m[0] - ps * w) <= 1e-14 * abs(ps * w)
    assert abs(v[0] - 0.09 * ps * ps / (phi @ phi + 0.09 / lam1)) <= 1e-14 * v[0]


def test_lu_solution_matches_cholesky_solve():
    """The oracle's LU solve of A agrees with a library Cholesky solve."""
    X, y, Xs = _small(9, 2, N=300)
    f = o.fit(X, y, 0.05, 1.0, 1.2, 8)
    w = sla.cho_solve(sla.cho_factor(f.A, lower=True), f.b)
    assert rel(f.w, w) <= 1e-11


def test_chunked_gram_equals_one_shot():
    X, y, _ = _small(11, 2, N=1000)
    f1 = o.fit(X, y, 0.1, 1.0, 1.0, 6, chunk=97)
    Phi = o.eigenfunctions_nd(X, 1.0, 1.0, 6)
    A = Phi.T @ Phi + np.diag(0.01 / o.eigenvalues_nd(1.0, 1.0, 6, 2))
    assert rel(f1.A, A) <= 1e-14
    assert rel(f1.b, Phi.T @ y) <= 1e-14


# ---------------------------------------------------------------- planted mistakes
def _with(monkeypatch, name, fn):
    monkeypatch.setattr(o, name, fn)


def test_pin_catches_literal_delta_reading(monkeypatch):
    """The literal delta^2 = rho/2 (beta^2 - 1) fails orthonormality and the
    trace at rho != 1 (and is invisible at rho = 1)."""
    def literal(eps, alpha):
        beta = (1.0 + (2.0 * eps / alpha) ** 2) ** 0.25
        return beta, alpha / 2.0 * (beta * beta - 1.0)
    _with(monkeypatch, "se_scalars", literal)
    with pytest.raises(AssertionError):
        test_orthonormality_gauss_hermite(1.0, 1.2)
    with pytest.raises(AssertionError):
        test_eigenvalue_trace_is_one(1.0, 0.5)
    test_orthonormality_gauss_hermite(1.0, 1.0)   # rho = 1: indistinguishable


def test_pin_catches_probabilists_hermite(monkeypatch):
    def he(t, n):
        t = np.asarray(t, dtype=np.float64)
        H = np.empty(t.shape + (n,))
        H[..., 0] = 1.0
        if n > 1:
            H[..., 1] = t
        for k in range(1, n - 1):
            H[..., k + 1] = t * H[..., k] - k * H[..., k - 1]
        return H
    _with(monkeypatch, "hermite_physicists", he)
    with pytest.raises(AssertionError):
        test_orthonormality_gauss_hermite(1.0, 1.0)
    with pytest.raises(AssertionError):
        test_mercer_sum_reproduces_se_kernel_1d(1.0)


def test_pin_catches_dropped_noise_term(monkeypatch):
    real_fit = o.fit

    def bad_fit(X, y, sigma, eps, alpha, n, chunk=8192, order=None):
        f = real_fit(X, y, sigma, eps, alpha, n, chunk, order)
        A = f.A - np.diag(sigma * sigma / f.lam) + np.diag(sigma * sigma * f.lam)
        lu = sla.lu_factor(A)
        return o.Fit(f.p, f.n, f.sigma, f.eps, f.alpha, f.lam, A, f.b, lu, sla.lu_solve(lu, f.b), order)
    _with(monkeypatch, "fit", bad_fit)
    with pytest.raises(AssertionError):
        test_weight_space_equals_nxn_truncated_posterior(2, 5, [1.0, 1.3], [1.2, 0.9])


def test_pin_catches_wrong_multi_index_order(monkeypatch):
    """A multi-index table that pairs Lambda of one order with Phi of
    another breaks the tensor factorisation."""
    real = o.eigenfunctions_nd

    def swapped(X, eps, alpha, n, order=None, kernel="se"):
        X = np.atleast_2d(X)
        idx = o.multi_indices(n, X.shape[1])[:, ::-1] if order is None else order
        return real(X, eps, alpha, n, idx, kernel=kernel)
    _with(monkeypatch, "eigenfunctions_nd", swapped)
    with pytest.raises(AssertionError):
        test_tensor_factorisation()


# ---------------------------------------------------------------- full covariance and log marginal likelihood
@pytest.mark.parametrize("p,n,eps,alpha", [(1, 10, 1.0, 1.0), (2, 5, [1.0, 1.3], [1.2, 0.9]), (3, 3, 0.8, 1.0)])
def test_full_covariance_equals_nxn_truncated_posterior(p, n, eps, alpha):
    """predict_cov (weight space, eq. (12)) vs the N x N form (eq. (9)) on the
    whole N* x N* matrix, and its diagonal is predict()'s variance."""
    X, y, Xs = _small(30 + p, p)
    f = o.fit(X, y, 0.1, eps, alpha, n)
    C1 = o.predict_cov(f, Xs)
    _, C3 = o.posterior_truncated_nxn(X, y, Xs, 0.1, eps, alpha, n)
    assert rel(C1, C3) <= 1e-10
    assert np.allclose(C1, C1.T, rtol=0, atol=1e-15 * np.abs(C1).max())
    _, v1 = o.predict(f, Xs)
    assert rel(np.diag(C1), v1) <= 1e-13
    # positive semi-definite up to rounding
    assert np.linalg.eigvalsh(0.5 * (C1 + C1.T)).min() >= -1e-12 * np.abs(C1).max()


@pytest.mark.parametrize("p,n,sigma,eps,alpha", [(1, 10, 0.1, 1.0, 1.0), (2, 5, 0.05, [1.0, 1.3], [1.2, 0.9]),
                                                 (3, 3, 0.2, 0.8, 1.0), (2, 6, 0.1, 1.0, 1.2)])
def test_log_marginal_likelihood_equals_gaussian_density(p, n, sigma, eps, alpha):
    """The weight-space log marginal likelihood (Woodbury + determinant lemma)
    against log N(y; 0, K~ + sigma^2 I) evaluated two ways on the N x N
    covariance: by its Cholesky, and by scipy's multivariate normal."""
    from scipy.stats import multivariate_normal
    X, y, _ = _small(40 + p, p)
    f = o.fit(X, y, sigma, eps, alpha, n)
    lml = o.log_marginal_likelihood(f, y)
    ref = o.log_marginal_likelihood_nxn(X, y, sigma, eps, alpha, n)
    S = o.truncated_kernel(X, X, eps, alpha, n) + sigma * sigma * np.eye(len(y))
    lib = multivariate_normal(mean=np.zeros(len(y)), cov=S).logpdf(y)
    assert abs(lml - ref) <= 1e-10 * abs(ref)
    assert abs(ref - lib) <= 1e-10 * abs(lib)


def test_log_marginal_likelihood_single_term_closed_form():
    """p = 1, n = 1: S = lambda_1 phi phi^T + sigma^2 I, so by the determinant
    lemma log det S = N log sigma^2 + log(1 + lambda_1 |phi|^2 / sigma^2) and
    y^T S^-1 y = (|y|^2 - (phi.y)^2 lambda_1 / (sigma^2 + lambda_1 |phi|^2)) / sigma^2."""
    X, y, _ = _small(50, 1)
    sigma = 0.3
    f = o.fit(X, y, sigma, 1.0, 1.0, 1)
    phi = o.eigenfunctions_1d(X[:, 0], 1.0, 1.0, 1)[:, 0]
    lam = o.eigenvalues_1d(1.0, 1.0, 1)[0]
    s2, N = sigma * sigma, len(y)
    pp, py = float(phi @ phi), float(phi @ y)
    logdet = N * np.log(s2) + np.log1p(lam * pp / s2)
    quad = (float(y @ y) - py * py * lam / (s2 + lam * pp)) / s2
    want = -0.5 * quad - 0.5 * logdet - 0.5 * N * np.log(2 * np.pi)
    assert abs(o.log_marginal_likelihood(f, y) - want) <= 1e-12 * abs(want)


def test_pin_catches_dropped_eigenvalue_logdet(monkeypatch):
    """A log marginal likelihood that forgets the sum of log Lambda in
    log det S must fail the Gaussian-density pin."""
    real = o.log_marginal_likelihood

    def broken(f, y):
        return real(f, y) + 0.5 * float(np.sum(np.log(f.lam)))
    monkeypatch.setattr(o, "log_marginal_likelihood", broken)
    with pytest.raises(AssertionError):
        test_log_marginal_likelihood_equals_gaussian_density(2, 5, 0.05, [1.0, 1.3], [1.2, 0.9])


# ---------------------------------------------------------------- periodic kernel (other Mercer kernels)
def periodic_1d(x1, x2, eps, alpha):
    """exp(-2 eps^2 sin^2(alpha (x - x') / 2)), written out."""
    return np.exp(-2.0 * eps ** 2 * np.sin(alpha * (x1[:, None] - x2[None, :]) / 2.0) ** 2)


@pytest.mark.parametrize("eps,alpha", [(0.5, 1.0), (1.0, 2.0), (2.0, 0.7)])
def test_periodic_expansion_reproduces_kernel(eps, alpha):
    """Jacobi-Anger: the expansion (1, sqrt2 cos, sqrt2 sin with e^-a I_k(a))
    truncated at 61 columns is the periodic kernel to rounding."""
    x = np.linspace(-4.0, 4.0, 41)
    K = periodic_1d(x, x, eps, alpha)
    lam = o.periodic_eigenvalues_1d(eps, 61)
    Phi = o.periodic_eigenfunctions_1d(x, eps, alpha, 61)
    assert np.max(np.abs((Phi * lam) @ Phi.T - K)) < 1e-14


@pytest.mark.parametrize("eps", [0.3, 1.0, 3.0])
def test_periodic_eigenvalues_power_series(eps):
    """e^-a I_k(a) against its power series e^-a sum_m (a/2)^(2m+k) / (m! (m+k)!)
    summed here in log space (not the library routine the oracle calls)."""
    a = eps * eps
    lam = o.periodic_eigenvalues_1d(eps, 21)
    for c in range(21):
        k = (c + 1) // 2
        ser = sum(math.exp((2 * m + k) * math.log(a / 2.0) - math.lgamma(m + 1) - math.lgamma(m + k + 1) - a)
                  for m in range(200))
        assert abs(lam[c] - ser) <= 1e-14 * ser


@pytest.mark.parametrize("eps", [0.7, 2.0])
def test_periodic_eigenvalue_trace_is_one(eps):
    """sum of all eigenvalues = k(x, x) = 1; cos and sin of a harmonic share theirs."""
    lam = o.periodic_eigenvalues_1d(eps, 81)
    assert abs(lam.sum() - 1.0) < 1e-14
    assert np.array_equal(lam[1::2][:40], lam[2::2][:40])
    assert np.all(np.diff(lam[::2]) < 0)


def test_periodic_eigenfunctions_orthonormal():
    """Mean of phi_i phi_j over one period (a uniform grid of 256 points
    integrates trigonometric polynomials of degree < 256 exactly) = delta_ij."""
    alpha = 1.7
    x = np.arange(256) * (2.0 * math.pi / alpha) / 256 - 3.0
    Phi = o.periodic_eigenfunctions_1d(x, 1.0, alpha, 31)
    assert np.max(np.abs(Phi.T @ Phi / 256 - np.eye(31))) < 1e-13


def test_periodic_closed_form_p2():
    x1 = np.random.default_rng(5).uniform(-3, 3, (30, 2))
    x2 = np.random.default_rng(6).uniform(-3, 3, (20, 2))
    K = periodic_1d(x1[:, 0], x2[:, 0], 0.8, 1.1) * periodic_1d(x1[:, 1], x2[:, 1], 1.3, 2.0)
    assert np.max(np.abs(o.periodic_ard_kernel(x1, x2, [0.8, 1.3], [1.1, 2.0]) - K)) < 1e-15
    Kt = o.truncated_kernel(x1, x2, [0.8, 1.3], [1.1, 2.0], 41, "periodic")
    assert np.max(np.abs(Kt - K)) < 1e-14


@pytest.mark.parametrize("p,n", [(1, 7), (2, 5)])
def test_periodic_weight_space_equals_nxn_truncated_posterior(p, n):
    rng = np.random.default_rng(11 + p)
    X = rng.uniform(-3, 3, (150, p))
    y = np.sin(1.5 * X).sum(axis=1) + 0.05 * rng.standard_normal(150)
    Xs = rng.uniform(-3, 3, (40, p))
    f = o.fit(X, y, 0.1, 0.9, 1.5, n, kernel="periodic")
    mean, var = o.predict(f, Xs)
    m3, c3 = o.posterior_truncated_nxn(X, y, Xs, 0.1, 0.9, 1.5, n, "periodic")
    assert rel(mean, m3) < 1e-10
    assert rel(var, np.diag(c3)) < 1e-9
    assert rel(o.predict_cov(f, Xs), c3) < 1e-9
    lml = o.log_marginal_likelihood(f, y)
    assert abs(lml - o.log_marginal_likelihood_nxn(X, y, 0.1, 0.9, 1.5, n, "periodic")) < 1e-9 * abs(lml)


def test_periodic_weight_space_tends_to_exact_posterior():
    """With 41 columns the truncated-kernel posterior is the exact periodic
    GP posterior (eqs. 3-4 with the closed-form kernel)."""
    rng = np.random.default_rng(3)
    X = rng.uniform(-3, 3, (120, 1))
    y = np.cos(2.0 * X[:, 0]) + 0.05 * rng.standard_normal(120)
    Xs = rng.uniform(-3, 3, (30, 1))
    f = o.fit(X, y, 0.1, 1.2, 2.0, 41, kernel="periodic")
    mean, var = o.predict(f, Xs)
    me, ce = o.posterior_exact(X, y, Xs, 0.1, 1.2, 2.0, "periodic")
    assert rel(mean, me) < 1e-9
    assert np.max(np.abs(var - np.diag(ce))) < 1e-9


def test_pin_catches_periodic_without_sqrt2(monkeypatch):
    """Unnormalised cos/sin features (or e^-a dropped from I_k) break the
    closed-form pin and orthonormality."""
    real = o.periodic_eigenfunctions_1d
    _with(monkeypatch, "periodic_eigenfunctions_1d",
          lambda x, eps, alpha, n: real(x, eps, alpha, n) / np.where(np.arange(n) > 0, math.sqrt(2.0), 1.0))
    with pytest.raises(AssertionError):
        test_periodic_expansion_reproduces_kernel(1.0, 2.0)
    with pytest.raises(AssertionError):
        test_periodic_eigenfunctions_orthonormal()


def test_pin_catches_unscaled_bessel(monkeypatch):
    _with(monkeypatch, "periodic_eigenvalues_1d",
          lambda eps, n: sps.iv((np.arange(n) + 1) // 2, eps * eps))
    with pytest.raises(AssertionError):
        test_periodic_expansion_reproduces_kernel(1.0, 2.0)
    with pytest.raises(AssertionError):
        test_periodic_eigenvalue_trace_is_one(0.7)
