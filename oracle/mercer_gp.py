"""Plain FP64 CPU oracle for the decomposed-kernel (Mercer) Gaussian process.

TEST INFRASTRUCTURE ONLY.  This module is the yardstick the GPU library is
checked against.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path (the HIP library and its Python
binding) never does, and this module imports nothing from the product.

Source: D. Carminati, "Parallel Gaussian Process with Kernel Approximation in
CUDA" (arXiv 2403.12797).  Equation numbers follow the paper's numbered
displays in order:
  (3)-(4)   exact GP posterior mean / covariance            (Sec. 2.1)
  (7)       k(X,X') ~ Phi Lambda Phi^T                      (Sec. 2.2)
  (8)-(9)   posterior with the truncated kernel, N x N form (Sec. 2.2)
  (10)      Woodbury identity, Lambda_bar                   (Sec. 2.2)
  (11)-(12) FAGP posterior with W                           (Sec. 2.2)
  (13)      1-D squared-exponential kernel                  (Sec. 2.3)
  (14)      beta, gamma_i, delta^2                          (Sec. 2.3)
  (15)      eigenfunctions phi_i                            (Sec. 2.3)
  (16)      eigenvalues lambda_i                            (Sec. 2.3)
  (17)      ARD kernel                                      (Sec. 2.3)
  (18)-(20) tensor-product expansion over all n^p indices   (Sec. 2.3)

The paper's global scale factor rho is called ``alpha`` here (one per input
dimension, as in (19)-(20)); its length scale is ``eps``.

Readings where the paper is garbled or silent (each one pinned by a test):
  * delta^2 in (14) prints as rho/2 (beta^2 - 1); the Fasshauer-McCourt value
    rho^2/2 (beta^2 - 1) is used.  Only that value makes the eigenfunctions
    orthonormal under the weight (rho/sqrt(pi)) exp(-rho^2 x^2) and makes the
    eigenvalues sum to k(x, x) = 1.  The two readings agree at rho = 1.
  * "classical" Hermite polynomials in (15) are the physicists' H_k
    (leading coefficient 2^k), matching gamma_i's 2^(i-1) Gamma(i).
  * The n^p multi-indices of (18) are enumerated in C order (last input
    dimension varies fastest).  Posterior mean and variance do not depend on
    the order; only the layout of the weight vector does.
  * The prior mean m(.) of (3), (8), (11) is zero.
  * The variance returned is that of the latent f_* (no added noise sigma^2).

Main formulation (F1, weight space).  With A = Phi^T Phi + sigma^2 Lambda^-1
(= sigma^2 Lambda_bar of (10)) the FAGP posterior (11)-(12) equals
    mu_* = Phi_* w,  w = A^-1 Phi^T y,   Sigma_* = sigma^2 Phi_* A^-1 Phi_*^T,
because W of (11) simplifies to Phi_* A^-1 Phi^T and I - A^-1 Phi^T Phi equals
sigma^2 A^-1 Lambda^-1.  The oracle solves A with an LU factorisation (the
factorisation the paper uses, Sec. 3); the paper's own W form (F2) and the
N x N truncated-kernel form (F3) are here too, for small N, and the tests pin
F1 to both and to the exact SE posterior.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

__all__ = [
    "se_scalars", "gamma_coeffs", "eigenvalues_1d", "hermite_physicists",
    "eigenfunctions_1d", "multi_indices", "eigenvalues_nd", "eigenfunctions_nd",
    "se_ard_kernel", "truncated_kernel", "Fit", "fit", "predict", "predict_cov",
    "log_marginal_likelihood", "log_marginal_likelihood_nxn",
    "posterior_woodbury_W", "posterior_truncated_nxn", "posterior_exact_se",
]


def _as_dim_array(v, p):
    a = np.asarray(v, dtype=np.float64).reshape(-1)
    if a.size == 1:
        a = np.full(p, float(a[0]))
    if a.size != p:
        raise ValueError(f"expected {p} per-dimension values, got {a.size}")
    return a


# --------------------------------------------------------------------------
# 1-D squared-exponential eigenpairs, Sec. 2.3 eqs. (14)-(16)
# --------------------------------------------------------------------------
def se_scalars(eps: float, alpha: float):
    """beta and delta^2 of eq. (14) for one input dimension.

    beta    = (1 + (2 eps / alpha)^2)^(1/4)
    delta^2 = alpha^2 / 2 * (beta^2 - 1)        (Fasshauer-McCourt reading)
    """
    beta = (1.0 + (2.0 * eps / alpha) ** 2) ** 0.25
    delta2 = alpha * alpha / 2.0 * (beta * beta - 1.0)
    return beta, delta2


def gamma_coeffs(beta: float, n: int) -> np.ndarray:
    """gamma_i = sqrt(beta / (2^(i-1) Gamma(i))), i = 1..n (eq. (14))."""
    i = np.arange(1, n + 1)
    logs = np.array([0.5 * (math.log(beta) - (k - 1) * math.log(2.0) - math.lgamma(k))
                     for k in i])
    return np.exp(logs)


def eigenvalues_1d(eps: float, alpha: float, n: int) -> np.ndarray:
    """lambda_i of eq. (16), i = 1..n:
    sqrt(alpha^2 / D) * (eps^2 / D)^(i-1),  D = alpha^2 + delta^2 + eps^2."""
    _, delta2 = se_scalars(eps, alpha)
    D = alpha * alpha + delta2 + eps * eps
    i = np.arange(n, dtype=np.float64)
    return math.sqrt(alpha * alpha / D) * (eps * eps / D) ** i


def hermite_physicists(t: np.ndarray, n: int) -> np.ndarray:
    """H_0(t) .. H_{n-1}(t), physicists' convention, by the textbook
    three-term recurrence H_0 = 1, H_1 = 2t, H_{k+1} = 2t H_k - 2k H_{k-1}.
    Returns shape t.shape + (n,)."""
    t = np.asarray(t, dtype=np.float64)
    H = np.empty(t.shape + (n,), dtype=np.float64)
    if n >= 1:
        H[..., 0] = 1.0
    if n >= 2:
        H[..., 1] = 2.0 * t
    for k in range(1, n - 1):
        H[..., k + 1] = 2.0 * t * H[..., k] - 2.0 * k * H[..., k - 1]
    return H


def eigenfunctions_1d(x: np.ndarray, eps: float, alpha: float, n: int) -> np.ndarray:
    """phi_i(x) = gamma_i exp(-delta^2 x^2) H_{i-1}(alpha beta x), eq. (15).
    x: any shape; returns x.shape + (n,), column i-1 holding phi_i."""
    beta, delta2 = se_scalars(eps, alpha)
    x = np.asarray(x, dtype=np.float64)
    g = gamma_coeffs(beta, n)
    H = hermite_physicists(alpha * beta * x, n)
    return g * np.exp(-delta2 * x * x)[..., None] * H


# --------------------------------------------------------------------------
# p-variate tensor-product expansion, Sec. 2.3 eqs. (17)-(20)
# --------------------------------------------------------------------------
def multi_indices(n: int, p: int) -> np.ndarray:
    """All n^p multi-indices (0-based digits k_1..k_p) of eq. (18), in C
    order: the last dimension varies fastest.  Shape (n^p, p)."""
    grids = np.meshgrid(*([np.arange(n)] * p), indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def eigenvalues_nd(eps, alpha, n: int, p: int, order: np.ndarray | None = None) -> np.ndarray:
    """Lambda_m = prod_j lambda_{k_j(m)}(eps_j, alpha_j), eq. (20)."""
    eps = _as_dim_array(eps, p)
    alpha = _as_dim_array(alpha, p)
    idx = multi_indices(n, p) if order is None else order
    lam = np.ones(idx.shape[0])
    for j in range(p):
        lam = lam * eigenvalues_1d(eps[j], alpha[j], n)[idx[:, j]]
    return lam


def eigenfunctions_nd(X: np.ndarray, eps, alpha, n: int,
                      order: np.ndarray | None = None) -> np.ndarray:
    """Phi[i, m] = prod_j phi_{k_j(m)}(x_ij; eps_j, alpha_j), eq. (19).
    X: (N, p).  Returns (N, n^p)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    p = X.shape[1]
    eps = _as_dim_array(eps, p)
    alpha = _as_dim_array(alpha, p)
    idx = multi_indices(n, p) if order is None else order
    Phi = np.ones((X.shape[0], idx.shape[0]))
    for j in range(p):
        phij = eigenfunctions_1d(X[:, j], eps[j], alpha[j], n)
        Phi *= phij[:, idx[:, j]]
    return Phi


def se_ard_kernel(X1: np.ndarray, X2: np.ndarray, eps) -> np.ndarray:
    """Closed-form ARD squared-exponential kernel, eq. (17) (eq. (13) at p=1)."""
    X1 = np.atleast_2d(np.asarray(X1, dtype=np.float64))
    X2 = np.atleast_2d(np.asarray(X2, dtype=np.float64))
    eps = _as_dim_array(eps, X1.shape[1])
    d2 = np.zeros((X1.shape[0], X2.shape[0]))
    for j in range(X1.shape[1]):
        d2 += (eps[j] * (X1[:, j][:, None] - X2[:, j][None, :])) ** 2
    return np.exp(-d2)


def truncated_kernel(X1, X2, eps, alpha, n: int) -> np.ndarray:
    """Phi(X1) Lambda Phi(X2)^T, eq. (7) with the expansion (18)."""
    X1 = np.atleast_2d(X1)
    p = X1.shape[1]
    lam = eigenvalues_nd(eps, alpha, n, p)
    return (eigenfunctions_nd(X1, eps, alpha, n) * lam) @ eigenfunctions_nd(X2, eps, alpha, n).T


# --------------------------------------------------------------------------
# Posterior, weight-space form F1 (eqs. (10)-(12) reassociated)
# --------------------------------------------------------------------------
@dataclass
class Fit:
    p: int
    n: int
    sigma: float
    eps: np.ndarray
    alpha: np.ndarray
    lam: np.ndarray          # (M,)  Lambda, eq. (20)
    A: np.ndarray            # (M, M) Phi^T Phi + sigma^2 Lambda^-1
    b: np.ndarray            # (M,)  Phi^T y
    lu: tuple                # LU factorisation of A (scipy lu_factor)
    w: np.ndarray            # (M,)  A^-1 Phi^T y  (C-order multi-index)
    order: np.ndarray | None = None   # multi-index table if not C order


def fit(X, y, sigma: float, eps, alpha, n: int, chunk: int = 8192,
        order: np.ndarray | None = None) -> Fit:
    """Weight-space fit.  A = sigma^2 Lambda_bar with Lambda_bar of (10);
    the Gram Phi^T Phi and Phi^T y are summed over row blocks of `chunk`
    samples in natural order (only to bound memory: Phi itself is N x n^p).
    `order` optionally replaces the C-order multi-index table (same rows,
    any permutation), which permutes w accordingly."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    N, p = X.shape
    if y.shape[0] != N:
        raise ValueError("x and y disagree on N")
    eps = _as_dim_array(eps, p)
    alpha = _as_dim_array(alpha, p)
    lam = eigenvalues_nd(eps, alpha, n, p, order)
    M = lam.shape[0]
    G = np.zeros((M, M))
    b = np.zeros(M)
    for s in range(0, N, chunk):
        Phi = eigenfunctions_nd(X[s:s + chunk], eps, alpha, n, order)
        G += Phi.T @ Phi
        b += Phi.T @ y[s:s + chunk]
    A = G + np.diag(sigma * sigma / lam)
    lu = sla.lu_factor(A)
    w = sla.lu_solve(lu, b)
    return Fit(p, n, float(sigma), eps, alpha, lam, A, b, lu, w, order)


def predict(f: Fit, Xs, chunk: int = 4096):
    """mu_* = Phi_* w and v_* = sigma^2 diag(Phi_* A^-1 Phi_*^T) (latent f_*),
    eqs. (11)-(12) in weight-space form.  Returns (mean, var)."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64))
    mean = np.empty(Xs.shape[0])
    var = np.empty(Xs.shape[0])
    for s in range(0, Xs.shape[0], chunk):
        Ps = eigenfunctions_nd(Xs[s:s + chunk], f.eps, f.alpha, f.n, f.order)
        mean[s:s + chunk] = Ps @ f.w
        Z = sla.lu_solve(f.lu, Ps.T)                   # A^-1 Phi_*^T
        var[s:s + chunk] = f.sigma ** 2 * np.einsum("im,mi->i", Ps, Z)
    return mean, var


def predict_cov(f: Fit, Xs, chunk: int = 4096):
    """Full predictive covariance of the latent f_* (eq. (12) in weight-space
    form): Sigma_* = sigma^2 Phi_* A^-1 Phi_*^T, N_* x N_*.  Its diagonal is
    predict()'s variance."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64))
    Ps = eigenfunctions_nd(Xs, f.eps, f.alpha, f.n, f.order)
    Z = sla.lu_solve(f.lu, Ps.T)                        # A^-1 Phi_*^T
    return f.sigma ** 2 * (Ps @ Z)


def log_marginal_likelihood(f: Fit, y):
    """log p(y) under the truncated-kernel GP prior of (7)-(8):
    y ~ N(0, S), S = Phi Lambda Phi^T + sigma^2 I (zero prior mean), written
    with the M x M system of the weight-space form instead of S itself:
      y^T S^-1 y = (y^T y - b^T w) / sigma^2            (Woodbury, as (10))
      log det S  = (N - M) log sigma^2 + sum_m log Lambda_m + log det A
    (the matrix determinant lemma with A = Phi^T Phi + sigma^2 Lambda^-1), so
      log p(y) = -(y^T y - b^T w) / (2 sigma^2) - log det S / 2 - N log(2 pi) / 2.
    log det A is the sum of log |u_ii| over the LU factor of A (A is SPD)."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    N, M = y.shape[0], f.lam.shape[0]
    s2 = f.sigma * f.sigma
    logdet_A = float(np.sum(np.log(np.abs(np.diag(f.lu[0])))))
    logdet_S = (N - M) * math.log(s2) + float(np.sum(np.log(f.lam))) + logdet_A
    quad = (float(y @ y) - float(f.b @ f.w)) / s2
    return -0.5 * quad - 0.5 * logdet_S - 0.5 * N * math.log(2.0 * math.pi)


# --------------------------------------------------------------------------
# Alternative formulations (small N only), used to pin F1
# --------------------------------------------------------------------------
def log_marginal_likelihood_nxn(X, y, sigma, eps, alpha, n):
    """log N(y; 0, K~ + sigma^2 I) with the N x N truncated kernel (7),
    evaluated by its definition (Cholesky of the N x N covariance)."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    S = truncated_kernel(X, X, eps, alpha, n) + sigma * sigma * np.eye(y.shape[0])
    L = np.linalg.cholesky(S)
    a = sla.solve_triangular(L, y, lower=True)
    return -0.5 * float(a @ a) - float(np.sum(np.log(np.diag(L)))) - 0.5 * y.shape[0] * math.log(2.0 * math.pi)


def posterior_woodbury_W(X, y, Xs, sigma, eps, alpha, n):
    """F2: the paper's literal FAGP form (11)-(12) with
    Lambda_bar = Lambda^-1 + Phi^T Sigma^-1 Phi and
    W = Phi_* Lambda Phi^T (Sigma^-1 - Sigma^-1 Phi Lambda_bar^-1 Phi^T Sigma^-1),
    Sigma = sigma^2 I.  Returns (mean, full covariance)."""
    X = np.atleast_2d(X)
    p = X.shape[1]
    lam = eigenvalues_nd(eps, alpha, n, p)
    Phi = eigenfunctions_nd(X, eps, alpha, n)
    Ps = eigenfunctions_nd(Xs, eps, alpha, n)
    Lam = np.diag(lam)
    s2inv = 1.0 / (sigma * sigma)
    Lbar = np.diag(1.0 / lam) + s2inv * Phi.T @ Phi
    inner = s2inv * np.eye(X.shape[0]) - s2inv * s2inv * Phi @ np.linalg.solve(Lbar, Phi.T)
    W = Ps @ Lam @ Phi.T @ inner
    mean = W @ np.asarray(y, dtype=np.float64)
    cov = Ps @ Lam @ Ps.T - W @ Phi @ Lam @ Ps.T
    return mean, cov


def posterior_truncated_nxn(X, y, Xs, sigma, eps, alpha, n):
    """F3: eqs. (8)-(9), the GP posterior with the truncated kernel (7) and
    the N x N system (K~ + sigma^2 I).  Returns (mean, full covariance)."""
    K = truncated_kernel(X, X, eps, alpha, n)
    Ks = truncated_kernel(Xs, X, eps, alpha, n)
    Kss = truncated_kernel(Xs, Xs, eps, alpha, n)
    S = K + sigma * sigma * np.eye(K.shape[0])
    mean = Ks @ np.linalg.solve(S, np.asarray(y, dtype=np.float64))
    cov = Kss - Ks @ np.linalg.solve(S, Ks.T)
    return mean, cov


def posterior_exact_se(X, y, Xs, sigma, eps):
    """Eqs. (3)-(4) with the closed-form ARD kernel (17) and m = 0."""
    K = se_ard_kernel(X, X, eps)
    Ks = se_ard_kernel(Xs, X, eps)
    Kss = se_ard_kernel(Xs, Xs, eps)
    S = K + sigma * sigma * np.eye(K.shape[0])
    mean = Ks @ np.linalg.solve(S, np.asarray(y, dtype=np.float64))
    cov = Kss - Ks @ np.linalg.solve(S, Ks.T)
    return mean, cov
