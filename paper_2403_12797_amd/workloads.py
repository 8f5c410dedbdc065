"""Seeded synthetic inputs for the Mercer-GP workloads.

Holds none of the method's arithmetic: only input shapes, value
distributions and the synthetic target functions.  Both the GPU library's
tests/benchmark and the CPU oracle are fed from here.

The paper's own data set (Sec. 3: N = 10000 samples, y = sum_i cos x_i + noise,
p and n swept) fixes neither the x distribution, the noise level nor N_*;
"paper_shape" below picks x ~ U[-1,1]^p, sigma = 0.1, N_* = N.  The larger
workloads keep the paper's form (a smooth sum of cosines/sines of the inputs
plus white noise) at the sizes the GPU targets.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Problem", "config", "CONFIG_NAMES", "random_problem", "batched_problems",
           "served_stream"]

SEED_BASE = 12797


@dataclass
class Problem:
    name: str
    p: int
    n: int
    sigma: float
    eps: np.ndarray          # (p,)
    alpha: np.ndarray        # (p,)
    x: np.ndarray            # (N, p) float64, row-major
    y: np.ndarray            # (N,)
    xs: np.ndarray           # (Ns, p)
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.n ** self.p

    @property
    def N(self) -> int:
        return self.x.shape[0]

    @property
    def Ns(self) -> int:
        return self.xs.shape[0]


def _rng(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + k)))


def _c1(N=1000, Ns=1000):
    g = _rng(1)
    x = g.uniform(-1.0, 1.0, size=(N, 1))
    y = np.sin(3.0 * x[:, 0]) + g.normal(0.0, 0.1, size=N)
    xs = np.linspace(-1.0, 1.0, Ns).reshape(Ns, 1)
    return Problem("c1_p1_n10", 1, 10, 0.1, np.array([1.0]), np.array([1.0]), x, y, xs,
                   {"recipe": "x~U[-1,1], y=sin(3x)+N(0,0.1^2), x* uniform grid, eps=1, alpha=1"})


def _c2(N=100_000, Ns=100_000):
    g = _rng(2)
    x = g.normal(size=(N, 3))
    y = np.sin(2.0 * x).sum(axis=1) + g.normal(0.0, 0.05, size=N)
    xs = g.normal(size=(Ns, 3))
    return Problem("c2_p3_n8", 3, 8, 0.05, np.full(3, 0.8), np.ones(3), x, y, xs,
                   {"recipe": "x,x*~N(0,I_3), y=sum_d sin(2x_d)+N(0,0.05^2), eps=0.8, alpha=1"})


def _c3(N=1_000_000, Ns=1_000_000):
    g = _rng(3)
    x = g.uniform(-1.0, 1.0, size=(N, 4))
    y = (np.exp(-(x * x).sum(axis=1)) + np.cos(3.0 * x[:, 0] * x[:, 1])
         + g.normal(0.0, 0.05, size=N))
    xs = g.uniform(-1.0, 1.0, size=(Ns, 4))
    return Problem("c3_p4_n8", 4, 8, 0.05, np.ones(4), np.full(4, 1.2), x, y, xs,
                   {"recipe": "x,x*~U[-1,1]^4, y=exp(-|x|^2)+cos(3x1x2)+N(0,0.05^2), eps=1, alpha=1.2"})


def _paper_shape(N=10_000, Ns=10_000):
    g = _rng(6)
    x = g.uniform(-1.0, 1.0, size=(N, 4))
    y = np.cos(x).sum(axis=1) + g.normal(0.0, 0.1, size=N)
    xs = g.uniform(-1.0, 1.0, size=(Ns, 4))
    return Problem("paper_p4_n11", 4, 11, 0.1, np.ones(4), np.ones(4), x, y, xs,
                   {"recipe": "x,x*~U[-1,1]^4, y=sum_i cos(x_i)+N(0,0.1^2), eps=1, alpha=1"})


def _c5_shape(N=50_000, Ns=2_000, p=5):
    """One request of the served stream at its largest expansion: p = 5, n = 6
    (M = 7776), x ~ U[-1,1]^p, y = exp(-|x|^2) + cos(3 x_1 x_2) + N(0, 0.05^2),
    sigma = 0.05, eps = 1, alpha = 1.2 (the served stream's values), at an N
    and N_* the oracle finishes in about a minute."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + 5, p])))
    x = g.uniform(-1.0, 1.0, size=(N, p))
    y = (np.exp(-(x * x).sum(axis=1)) + np.cos(3.0 * x[:, 0] * x[:, 1])
         + g.normal(0.0, 0.05, size=N))
    xs = g.uniform(-1.0, 1.0, size=(Ns, p))
    return Problem(f"c5_p{p}_n6", p, 6, 0.05, np.ones(p), np.full(p, 1.2), x, y, xs,
                   {"recipe": f"x,x*~U[-1,1]^{p}, y=exp(-|x|^2)+cos(3x1x2)+N(0,0.05^2), eps=1, alpha=1.2"})


_CONFIGS = {"c1": _c1, "c2": _c2, "c3": _c3, "c5": _c5_shape, "paper": _paper_shape}
CONFIG_NAMES = tuple(_CONFIGS)


def config(name: str, N: int | None = None, Ns: int | None = None) -> Problem:
    """Named workload.  N / Ns override the sizes (a prefix-stable subset is
    NOT implied: changing N changes the draw)."""
    kw = {}
    if N is not None:
        kw["N"] = N
    if Ns is not None:
        kw["Ns"] = Ns
    return _CONFIGS[name](**kw)


def random_problem(seed: int, p: int, n: int, N: int, Ns: int, *, dist: str = "uniform",
                   sigma: float = 0.1, eps=None, alpha=None) -> Problem:
    """A small random problem for parity sweeps (shapes chosen by the caller)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 99, seed])))
    draw = (lambda s: g.uniform(-1.0, 1.0, size=s)) if dist == "uniform" else (lambda s: g.normal(size=s))
    x = draw((N, p))
    xs = draw((Ns, p))
    y = np.cos(2.0 * x).sum(axis=1) + g.normal(0.0, sigma, size=N)
    eps = g.uniform(0.5, 2.0, size=p) if eps is None else np.broadcast_to(np.asarray(eps, float), (p,)).copy()
    alpha = g.uniform(0.8, 1.5, size=p) if alpha is None else np.broadcast_to(np.asarray(alpha, float), (p,)).copy()
    return Problem(f"rand{seed}_p{p}_n{n}_N{N}", p, n, sigma, eps, alpha, x, y, xs)


def periodic_problem(seed: int, p: int, n: int, N: int, Ns: int, *, sigma: float = 0.1, eps=None,
                     alpha=None) -> Problem:
    """A random problem for the periodic kernel: x, x* ~ U[-3, 3]^p (a few
    periods at the drawn angular frequencies alpha ~ U[0.8, 2]),
    y = sum_d sin(alpha_d x_d + d) + N(0, sigma^2), eps ~ U[0.5, 1.5]."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 77, seed])))
    x = g.uniform(-3.0, 3.0, size=(N, p))
    xs = g.uniform(-3.0, 3.0, size=(Ns, p))
    eps = g.uniform(0.5, 1.5, size=p) if eps is None else np.broadcast_to(np.asarray(eps, float), (p,)).copy()
    alpha = g.uniform(0.8, 2.0, size=p) if alpha is None else np.broadcast_to(np.asarray(alpha, float), (p,)).copy()
    y = np.sin(alpha * x + np.arange(p)).sum(axis=1) + g.normal(0.0, sigma, size=N)
    return Problem(f"per{seed}_p{p}_n{n}_N{N}", p, n, sigma, eps, alpha, x, y, xs, meta={"kernel": "periodic"})


def batched_problems(count: int = 256, *, N_max: int = 200_000) -> list[Problem]:
    """Many independent problems of uneven shape: p ~ U{1,2,3}, one n ~ U{4..12}
    for all dims, N log-uniform in [1e3, N_max], N_* = N, x ~ N(0, I_p),
    y = sum_d sin(k_d x_d) + N(0, 0.1^2) with k_d ~ U[1,4], eps ~ U[0.5,2], alpha = 1."""
    root = np.random.SeedSequence(SEED_BASE + 4)
    out = []
    for i, ss in enumerate(root.spawn(count)):
        g = np.random.Generator(np.random.PCG64(ss))
        p = int(g.integers(1, 4))
        n = int(g.integers(4, 13))
        N = int(round(10 ** g.uniform(3.0, np.log10(N_max))))
        k = g.uniform(1.0, 4.0, size=p)
        eps = float(g.uniform(0.5, 2.0))
        x = g.normal(size=(N, p))
        y = np.sin(k * x).sum(axis=1) + g.normal(0.0, 0.1, size=N)
        xs = g.normal(size=(N, p))
        out.append(Problem(f"b{i}_p{p}_n{n}_N{N}", p, n, 0.1, np.full(p, eps), np.ones(p), x, y, xs))
    return out


def served_stream(rate: float = 200.0, duration: float = 30.0, *, N_max: int = 500_000,
                  Ns_max: int = 100_000, seed_offset: int = 5):
    """Poisson arrivals of fit+predict requests: p ~ U{2..5}, n = 6, N log-U[1e3, N_max],
    N_* log-U[1e2, Ns_max], x ~ U[-1,1]^p, y = exp(-|x|^2) + cos(3 x_1 x_2) + N(0, 0.05^2),
    sigma = 0.05, eps = 1, alpha = 1.2.  Returns a list of (arrival_time_s, lazy factory)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + seed_offset)))
    t = 0.0
    out = []
    i = 0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        p = int(g.integers(2, 6))
        N = int(round(10 ** g.uniform(3.0, np.log10(N_max))))
        Ns = int(round(10 ** g.uniform(2.0, np.log10(Ns_max))))
        sub = int(g.integers(0, 2**62))

        def make(p=p, N=N, Ns=Ns, sub=sub, i=i):
            h = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + seed_offset, sub])))
            x = h.uniform(-1.0, 1.0, size=(N, p))
            y = (np.exp(-(x * x).sum(axis=1)) + np.cos(3.0 * x[:, 0] * x[:, 1])
                 + h.normal(0.0, 0.05, size=N))
            xs = h.uniform(-1.0, 1.0, size=(Ns, p))
            return Problem(f"s{i}_p{p}_N{N}_Ns{Ns}", p, 6, 0.05, np.ones(p), np.full(p, 1.2), x, y, xs)

        out.append((t, make))
        i += 1
    return out
