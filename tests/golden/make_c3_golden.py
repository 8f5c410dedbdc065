"""Write tests/golden/c3_oracle.npz: the FP64 oracle's posterior for the full
c3 workload (p = 4, n = 8, M = 4096, N = 1e6) at a seeded sample of 2000 of
its 1e6 test points, plus w.  Calls only oracle/ (inputs from the seeded
workload generator).  Takes a few minutes on 8 cores.

    python tests/golden/make_c3_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mercer_gp as o  # noqa: E402
from paper_2403_12797_amd import workloads as wl  # noqa: E402

SAMPLE_SEED = 12800 + 100
SAMPLE = 2000


def sample_indices(Ns):
    g = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return np.sort(g.choice(Ns, size=SAMPLE, replace=False))


def main():
    P = wl.config("c3")
    idx = sample_indices(P.Ns)
    t0 = time.time()
    f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
    t1 = time.time()
    mean, var = o.predict(f, P.xs[idx])
    t2 = time.time()
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle.npz")
    np.savez_compressed(out, idx=idx, mean=mean, var=var, w=f.w, b=f.b,
                        diagA=np.diag(f.A).copy(), fit_s=t1 - t0, predict_s=t2 - t1)
    print(f"wrote {out}: fit {t1 - t0:.1f} s, predict {t2 - t1:.1f} s")


if __name__ == "__main__":
    main()
