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

Other Mercer kernels (Sec. 2.3 notes that expansions exist for kernels other
than the SE, e.g. periodic ones, without giving them).  ``kernel="periodic"``
selects the periodic (exp-sine-squared) kernel, per input dimension
    k(x, x') = exp(-2 eps^2 sin^2(alpha (x - x') / 2)),
period 2 pi / alpha, length scale 1 / eps.  With a = eps^2 and
2 sin^2(u/2) = 1 - cos u, the Jacobi-Anger expansion
exp(a cos u) = I_0(a) + 2 sum_{k>=1} I_k(a) cos(k u) gives its exact Mercer
expansion on one period (uniform measure): eigenfunctions 1, sqrt(2) cos(k alpha x),
sqrt(2) sin(k alpha x) (orthonormal), eigenvalues e^-a I_0(a), then
e^-a I_k(a) twice (cos and sin).  Truncation to n columns per dimension and
the tensor product over dimensions (eqs. (18)-(20)) are as for the SE.

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
    "eigenfunctions_1d", "periodic_eigenvalues_1d", "periodic_eigenfunctions_1d",
    "multi_indices", "eigenvalues_nd", "eigenfunctions_nd",
    "se_ard_kernel", "periodic_ard_kernel", "truncated_kernel", "Fit", "fit", "predict", "predict_cov",
    "log_marginal_likelihood", "log_marginal_likelihood_nxn",
    "posterior_woodbury_W", "posterior_truncated_nxn", "posterior_exact_se", "posterior_exact",
]

KERNELS = ("se", "periodic")


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
# 1-D periodic eigenpairs (Jacobi-Anger; see the module docstring)
# --------------------------------------------------------------------------
def periodic_eigenvalues_1d(eps: float, n: int) -> np.ndarray:
    """lambda_1 = e^-a I_0(a); lambda_{2k} = lambda_{2k+1} = e^-a I_k(a),
    a = eps^2 (scipy's exponentially scaled Bessel function ive)."""
    from scipy.special import ive
    a = eps * eps
    k = (np.arange(n) + 1) // 2
    return ive(k, a)


def periodic_eigenfunctions_1d(x: np.ndarray, eps: float, alpha: float, n: int) -> np.ndarray:
    """phi_1 = 1, phi_{2k} = sqrt(2) cos(k alpha x), phi_{2k+1} = sqrt(2) sin(k alpha x).
    x: any shape; returns x.shape + (n,), column i-1 holding phi_i."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape + (n,), dtype=np.float64)
    for c in range(n):
        k = (c + 1) // 2
        if c == 0:
            out[..., c] = 1.0
        elif c % 2 == 1:
            out[..., c] = math.sqrt(2.0) * np.cos(k * alpha * x)
        else:
            out[..., c] = math.sqrt(2.0) * np.sin(k * alpha * x)
    return out


def _eigvals_1d(kernel, eps, alpha, n):
    if kernel == "se":
        return eigenvalues_1d(eps, alpha, n)
    if kernel == "periodic":
        return periodic_eigenvalues_1d(eps, n)
    raise ValueError(f"unknown kernel {kernel!r}")


def _eigfuns_1d(kernel, x, eps, alpha, n):
    if kernel == "se":
        return eigenfunctions_1d(x, eps, alpha, n)
    if kernel == "periodic":
        return periodic_eigenfunctions_1d(x, eps, alpha, n)
    raise ValueError(f"unknown kernel {kernel!r}")


# --------------------------------------------------------------------------
# p-variate tensor-product expansion, Sec. 2.3 eqs. (17)-(20)
# --------------------------------------------------------------------------
def multi_indices(n: int, p: int) -> np.ndarray:
    """All n^p multi-indices (0-based digits k_1..k_p) of eq. (18), in C
    order: the last dimension varies fastest.  Shape (n^p, p)."""
    grids = np.meshgrid(*([np.arange(n)] * p), indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def eigenvalues_nd(eps, alpha, n: int, p: int, order: np.ndarray | None = None,
                   kernel: str = "se") -> np.ndarray:
    """Lambda_m = prod_j lambda_{k_j(m)}(eps_j, alpha_j), eq. (20)."""
    eps = _as_dim_array(eps, p)
    alpha = _as_dim_array(alpha, p)
    idx = multi_indices(n, p) if order is None else order
    lam = np.ones(idx.shape[0])
    for j in range(p):
        lam = lam * _eigvals_1d(kernel, eps[j], alpha[j], n)[idx[:, j]]
    return lam


def eigenfunctions_nd(X: np.ndarray, eps, alpha, n: int,
                      order: np.ndarray | None = None, kernel: str = "se") -> np.ndarray:
    """Phi[i, m] = prod_j phi_{k_j(m)}(x_ij; eps_j, alpha_j), eq. (19).
    X: (N, p).  Returns (N, n^p)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    p = X.shape[1]
    eps = _as_dim_array(eps, p)
    alpha = _as_dim_array(alpha, p)
    idx = multi_indices(n, p) if order is None else order
    Phi = np.ones((X.shape[0], idx.shape[0]))
    for j in range(p):
        phij = _eigfuns_1d(kernel, X[:, j], eps[j], alpha[j], n)
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


def periodic_ard_kernel(X1: np.ndarray, X2: np.ndarray, eps, alpha) -> np.ndarray:
    """Closed-form product periodic kernel:
    prod_j exp(-2 eps_j^2 sin^2(alpha_j (x_j - x'_j) / 2))."""
    X1 = np.atleast_2d(np.asarray(X1, dtype=np.float64))
    X2 = np.atleast_2d(np.asarray(X2, dtype=np.float64))
    p = X1.shape[1]
    eps = _as_dim_array(eps, p)
    alpha = _as_dim_array(alpha, p)
    e = np.zeros((X1.shape[0], X2.shape[0]))
    for j in range(p):
        s = np.sin(alpha[j] * (X1[:, j][:, None] - X2[:, j][None, :]) / 2.0)
        e += 2.0 * eps[j] ** 2 * s * s
    return np.exp(-e)


def truncated_kernel(X1, X2, eps, alpha, n: int, kernel: str = "se") -> np.ndarray:
    """Phi(X1) Lambda Phi(X2)^T, eq. (7) with the expansion (18)."""
    X1 = np.atleast_2d(X1)
    p = X1.shape[1]
    lam = eigenvalues_nd(eps, alpha, n, p, kernel=kernel)
    return (eigenfunctions_nd(X1, eps, alpha, n, kernel=kernel) * lam) @ \
        eigenfunctions_nd(X2, eps, alpha, n, kernel=kernel).T


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
    kernel: str = "se"                # "se" (eqs. 13-20) or "periodic"


def fit(X, y, sigma: float, eps, alpha, n: int, chunk: int = 8192,
        order: np.ndarray | None = None, kernel: str = "se") -> Fit:
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
    lam = eigenvalues_nd(eps, alpha, n, p, order, kernel=kernel)
    M = lam.shape[0]
    G = np.zeros((M, M))
    b = np.zeros(M)
    for s in range(0, N, chunk):
        Phi = eigenfunctions_nd(X[s:s + chunk], eps, alpha, n, order, kernel=kernel)
        G += Phi.T @ Phi
        b += Phi.T @ y[s:s + chunk]
    A = G + np.diag(sigma * sigma / lam)
    lu = sla.lu_factor(A)
    w = sla.lu_solve(lu, b)
    return Fit(p, n, float(sigma), eps, alpha, lam, A, b, lu, w, order, kernel)


def predict(f: Fit, Xs, chunk: int = 4096):
    """mu_* = Phi_* w and v_* = sigma^2 diag(Phi_* A^-1 Phi_*^T) (latent f_*),
    eqs. (11)-(12) in weight-space form.  Returns (mean, var)."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64))
    mean = np.empty(Xs.shape[0])
    var = np.empty(Xs.shape[0])
    for s in range(0, Xs.shape[0], chunk):
        Ps = eigenfunctions_nd(Xs[s:s + chunk], f.eps, f.alpha, f.n, f.order, kernel=f.kernel)
        mean[s:s + chunk] = Ps @ f.w
        Z = sla.lu_solve(f.lu, Ps.T)                   # A^-1 Phi_*^T
        var[s:s + chunk] = f.sigma ** 2 * np.einsum("im,mi->i", Ps, Z)
    return mean, var


def predict_cov(f: Fit, Xs, chunk: int = 4096):
    """Full predictive covariance of the latent f_* (eq. (12) in weight-space
    form): Sigma_* = sigma^2 Phi_* A^-1 Phi_*^T, N_* x N_*.  Its diagonal is
    predict()'s variance."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64))
    Ps = eigenfunctions_nd(Xs, f.eps, f.alpha, f.n, f.order, kernel=f.kernel)
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
def log_marginal_likelihood_nxn(X, y, sigma, eps, alpha, n, kernel: str = "se"):
    """log N(y; 0, K~ + sigma^2 I) with the N x N truncated kernel (7),
    evaluated by its definition (Cholesky of the N x N covariance)."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    S = truncated_kernel(X, X, eps, alpha, n, kernel) + sigma * sigma * np.eye(y.shape[0])
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


def posterior_truncated_nxn(X, y, Xs, sigma, eps, alpha, n, kernel: str = "se"):
    """F3: eqs. (8)-(9), the GP posterior with the truncated kernel (7) and
    the N x N system (K~ + sigma^2 I).  Returns (mean, full covariance)."""
    K = truncated_kernel(X, X, eps, alpha, n, kernel)
    Ks = truncated_kernel(Xs, X, eps, alpha, n, kernel)
    Kss = truncated_kernel(Xs, Xs, eps, alpha, n, kernel)
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


def posterior_exact(X, y, Xs, sigma, eps, alpha, kernel: str = "se"):
    """Eqs. (3)-(4) with m = 0 and the closed-form kernel of the family: the
    ARD SE kernel (17) or the product periodic kernel."""
    if kernel == "se":
        return posterior_exact_se(X, y, Xs, sigma, eps)
    if kernel != "periodic":
        raise ValueError(f"unknown kernel {kernel!r}")
    K = periodic_ard_kernel(X, X, eps, alpha)
    Ks = periodic_ard_kernel(Xs, X, eps, alpha)
    Kss = periodic_ard_kernel(Xs, Xs, eps, alpha)
    S = K + sigma * sigma * np.eye(K.shape[0])
    mean = Ks @ np.linalg.solve(S, np.asarray(y, dtype=np.float64))
    cov = Kss - Ks @ np.linalg.solve(S, Ks.T)
    return mean, cov
