"""Write the FP64 oracle's posterior for two large-M shapes the GPU parity
tests check in full:

  c5_p5_oracle.npz     the served stream's largest expansion: p = 5, n = 6
                       (M = 7776), N = 50000, N_* = 2000 (workloads.config("c5"))
  paper_oracle.npz     the paper's own data-set shape (Sec. 3, headline of
                       Sec. 4): p = 4, n = 11 (M = 14641), N = N_* = 10000
                       (workloads.config("paper"))

Each file holds w, b, diag(A) and mean/var at every test point.  Calls only
oracle/ (inputs from the seeded workload generators).  About five minutes on
8 cores.

    python tests/golden/make_shape_goldens.py [c5] [paper]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mercer_gp as o  # noqa: E402
from paper_2403_12797_amd import workloads as wl  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SHAPES = {"c5": "c5_p5_oracle.npz", "paper": "paper_oracle.npz"}


def make(name):
    P = wl.config(name)
    t0 = time.time()
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n, chunk=4096)
    t1 = time.time()
    mean, var = o.predict(f, P.xs, chunk=2048)
    t2 = time.time()
    out = os.path.join(HERE, SHAPES[name])
    np.savez_compressed(out, mean=mean, var=var, w=f.w, b=f.b, diagA=np.diag(f.A).copy(),
                        N=P.N, Ns=P.Ns, M=P.M, fit_s=t1 - t0, predict_s=t2 - t1)
    print(f"wrote {out}: M={P.M} N={P.N} Ns={P.Ns}: fit {t1 - t0:.1f} s, predict {t2 - t1:.1f} s", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(SHAPES)):
        make(name)
