"""Benchmark: train+test points/s of one fit + predict (mean and variance) of
the Mercer GP on one MI355X: the mixed path (Gram as split-FP16 MFMA on scaled
Phi by default, or as split-BF16 with --gram bf16), the other Gram scheme and
the plain FP64 GPU path beside it, plus the FP64 CPU oracle on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (default): p = 4, n = 8 (M = 4096), N = N_* = 1e6, x ~ U[-1,1]^4,
y = exp(-|x|^2) + cos(3 x1 x2) + N(0, 0.05^2), eps = 1, alpha = 1.2.  A step is
gp_fit + gp_predict(mean, var) with inputs resident in HBM; value =
(N + N_*) / seconds per step.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "train+test points/s at p=4,M=4096 (mixed vs FP64 GPU); p50/p99 request latency"
PEAK_16 = 2.5e15        # dense FP16 / BF16 MFMA, MI355X
PEAK_FP64 = 78.6e12     # FP64 MFMA, MI355X


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--Ns", type=int, default=None)
    ap.add_argument("--gram", choices=("f16", "bf16"), default="f16",
                    help="Gram scheme of the timed mixed path: two FP16 terms (3 products) or three BF16 terms "
                         "(6 products)")
    ap.add_argument("--no-alt", action="store_true", help="skip timing the other Gram scheme")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU comparison path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-target-s", type=float, default=15.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the served Poisson stream (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--batched", type=int, default=256,
                    help="problems of the batched leg (0 = skip)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched leg and print its JSON (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    return ap.parse_args()


def run_path(ctx, torch, P, dev, precision, steps, warmup):
    from paper_2403_12797_amd import binding as B
    x, y, xs = dev
    mean = torch.empty(P.Ns, dtype=torch.float64, device="cuda")
    var = torch.empty(P.Ns, dtype=torch.float64, device="cuda")

    def step():
        m = ctx.fit(x, y, p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha, precision=precision)
        ctx.predict(m, xs, mean, var)
        torch.cuda.synchronize()
        m.free()

    for _ in range(warmup):
        step()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    return dt, prof, (mean, var)


def served_stream(torch, rate, seconds, warm=2.0):
    """Poisson arrivals of fit+predict requests through gp_submit / gp_poll:
    p ~ U{2..5}, n = 6, N log-U[1e3, 5e5], N* log-U[1e2, 1e5], x ~ U[-1,1]^p,
    y = exp(-|x|^2) + cos(3 x1 x2) + N(0, 0.05^2), sigma = 0.05, eps = 1,
    alpha = 1.2, mixed precision (FP16 Gram).  Inputs are slices of seeded device-resident
    pools (drawn before the stream starts).  Returns latency percentiles and
    sustained points/s over the requests that arrived after the warm-up."""
    import threading
    from paper_2403_12797_amd import binding as B
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(12797 + 5)))
    NMAX, NSMAX = 500_000, 100_000
    pools = {}
    for p in range(2, 6):
        x = g.uniform(-1.0, 1.0, size=(NMAX, p))
        y = np.exp(-(x * x).sum(axis=1)) + np.cos(3.0 * x[:, 0] * x[:, 1]) + g.normal(0.0, 0.05, size=NMAX)
        xs = g.uniform(-1.0, 1.0, size=(NSMAX, p))
        pools[p] = tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (x, y, xs))
    out_mean = torch.empty(NSMAX, dtype=torch.float64, device="cuda")
    total = warm + seconds
    reqs = []
    t = 0.0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= total:
            break
        p = int(g.integers(2, 6))
        N = int(round(10 ** g.uniform(3.0, np.log10(NMAX))))
        Ns = int(round(10 ** g.uniform(2.0, np.log10(NSMAX))))
        off = int(g.integers(0, NMAX - N + 1))
        offs = int(g.integers(0, NSMAX - Ns + 1))
        reqs.append((t, p, N, Ns, off, offs))
    torch.cuda.synchronize()
    ctx = B.Context(0)
    prm = {p: B.make_params(p, 6, 0.05, 1.0, 1.2, B.PREC_MIXED_F16) for p in range(2, 6)}
    means = [torch.empty(r[3], dtype=torch.float64, device="cuda") for r in reqs]
    vars_ = [torch.empty(r[3], dtype=torch.float64, device="cuda") for r in reqs]
    ids = [None] * len(reqs)
    t_sub = [0.0] * len(reqs)
    t_done = [0.0] * len(reqs)
    status = [None] * len(reqs)
    submitted = threading.Semaphore(0)

    def submitter():
        t0 = time.perf_counter()
        for k, (ta, p, N, Ns, off, offs) in enumerate(reqs):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            x, y, xs = pools[p]
            t_sub[k] = time.perf_counter()
            ids[k] = ctx.submit(B.REQ_FIT_PREDICT, x=x[off:off + N], y=y[off:off + N], params=prm[p],
                                xs=xs[offs:offs + Ns], mean=means[k], var=vars_[k])
            submitted.release()

    th = threading.Thread(target=submitter)
    t_start = time.perf_counter()
    th.start()
    # poll every outstanding request without blocking, so each completion is
    # stamped when it happens (requests can finish out of order)
    outstanding = []
    nxt = 0
    done_count = 0
    while done_count < len(reqs):
        while submitted.acquire(blocking=False):
            outstanding.append(nxt)
            nxt += 1
        progressed = False
        for k in list(outstanding):
            try:
                st, _ = ctx.poll(ids[k], wait_us=0)
            except B.GpError as e:
                st = e.status
            if st != B.GP_PENDING:
                t_done[k] = time.perf_counter()
                status[k] = st
                outstanding.remove(k)
                done_count += 1
                progressed = True
        if not progressed:
            time.sleep(0.0002)
    th.join()
    t_end = time.perf_counter()
    ctx.close()
    sel = [k for k in range(len(reqs)) if reqs[k][0] >= warm]
    lat = np.array([t_done[k] - t_sub[k] for k in sel]) * 1e3
    pts = sum(reqs[k][2] + reqs[k][3] for k in sel)
    span = max(t_done[k] for k in sel) - min(t_sub[k] for k in sel)
    return {"requests": len(sel), "rate_req_s": rate, "seconds": seconds,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "points_per_s": pts / span,
            "failed": int(sum(1 for k in sel if status[k] != B.GP_OK)),
            "wall_s": t_end - t_start,
            # time to serve every arrival / arrival window: > 1 means the offered
            # load exceeds what the device sustains, and p99 grows with run length
            "rho": (t_end - t_start) / (warm + seconds),
            "workload": "Poisson 200 req/s fit+predict, p~U{2..5}, n=6 (M<=7776), N log-U[1e3,5e5], "
                        "N* log-U[1e2,1e5], mixed precision (FP16 Gram), stream slots from the HBM budget "
                        "(MGP_SLOTS to override)"}


def batched_leg(torch, count, steps=2):
    """The batched workload: `count` independent problems with p ~ U{1,2,3},
    one n ~ U{4..12} per problem, N log-uniform in [1e3, 2e5], N* = N,
    x ~ N(0, I_p), y = sum_d sin(k_d x_d) + N(0, 0.1^2), eps ~ U[0.5, 2],
    alpha = 1, sigma = 0.1; mixed precision (FP16 Gram).  A step is one
    gp_fit_batch (one persistent Gram launch per kernel group, the rest on
    four forked streams) and one gp_predict_batch over all problems, inputs
    resident in HBM; value = sum(N + N*) / seconds per step."""
    from paper_2403_12797_amd import binding as B
    from paper_2403_12797_amd import workloads as wl
    Ps = wl.batched_problems(count)

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    dx = [(d(P.x), d(P.y), P.p, P.n, P.sigma, P.eps, P.alpha) for P in Ps]
    xs = [d(P.xs) for P in Ps]
    means = [torch.empty(P.Ns, dtype=torch.float64, device="cuda") for P in Ps]
    vars_ = [torch.empty(P.Ns, dtype=torch.float64, device="cuda") for P in Ps]
    torch.cuda.synchronize()
    ctx = B.Context(0)

    def step():
        models = ctx.fit_batch(dx, precision=B.PREC_MIXED_F16)
        ctx.predict_batch(models, xs, means, vars_)
        torch.cuda.synchronize()
        for m in models:
            m.free()

    step()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    dt = (time.perf_counter() - t0) / steps
    ctx.close()
    pts = sum(P.N + P.Ns for P in Ps)
    Ms = sorted(P.M for P in Ps)
    return {"problems": count, "points": pts, "value": pts / dt, "unit": "points/s", "ms_per_step": dt * 1e3,
            "steps": steps, "M_median": Ms[len(Ms) // 2], "M_max": Ms[-1],
            "workload": "256 independent problems, p~U{1,2,3}, n~U{4..12}, N log-U[1e3,2e5], N*=N, x~N(0,I_p), "
                        "mixed precision (FP16 Gram); gp_fit_batch + gp_predict_batch"}


def cpu_baseline(P_full, target_s):
    """The FP64 oracle (as it is) on bounded samples of the same workload.

    It is timed at two sample sizes with the workload's N : N* ratio; the
    time is modelled as t = F + c (N + N*): F the fixed part (eigen tables,
    the M x M factorisation), c the cost per train or test point.  `value`
    is the full workload's (N + N*) / (F + c (N + N*)) from that fit; the
    per-point rate 1/c and F are reported beside it, with the raw samples.
    The two smaller workloads (p = 1, M = 10 and p = 3, M = 512) are timed
    in full."""
    from oracle import mercer_gp as o
    from paper_2403_12797_amd import workloads as wl
    try:
        from threadpoolctl import threadpool_info
        cores = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:
        cores = os.cpu_count() or 1
    base = P_full.name.split("_")[0]
    ratio = P_full.Ns / max(P_full.N, 1)

    def timed(name, N=None, Ns=None):
        P = wl.config(name, N=N, Ns=Ns)
        t0 = time.perf_counter()
        f = o.fit(P.x, P.y, P.sigma, P.eps, P.alpha, P.n)
        t1 = time.perf_counter()
        o.predict(f, P.xs)
        t2 = time.perf_counter()
        return P, t1 - t0, t2 - t1

    n1 = 4096
    _, f1, p1 = timed(base, n1, max(128, int(n1 * ratio)))
    t1 = f1 + p1
    # grow the second sample so both together take about target_s
    scale = max(2.0, min(16.0, (target_s - t1) / max(t1, 1e-3)))
    n2 = int(n1 * scale) // 1024 * 1024
    _, f2, p2 = timed(base, n2, max(128, int(n2 * ratio)))
    t2 = f2 + p2
    pts1, pts2 = n1 + max(128, int(n1 * ratio)), n2 + max(128, int(n2 * ratio))
    c = max((t2 - t1) / (pts2 - pts1), 1e-12)
    F = max(t1 - c * pts1, 0.0)
    full = P_full.N + P_full.Ns
    small = {}
    for name in ("c1", "c2"):
        P, fs, ps = timed(name)
        small[name] = {"N": P.N, "Ns": P.Ns, "M": P.M, "fit_s": round(fs, 3), "predict_s": round(ps, 3),
                       "points_per_s": (P.N + P.Ns) / (fs + ps)}
    return {"value": full / (F + c * full), "unit": "points/s", "cores": int(cores), "kind": "oracle",
            "per_point_rate": 1.0 / c, "fixed_s": F,
            "samples": [{"N": n1, "Ns": pts1 - n1, "fit_s": round(f1, 3), "predict_s": round(p1, 3)},
                        {"N": n2, "Ns": pts2 - n2, "fit_s": round(f2, 3), "predict_s": round(p2, 3)}],
            "other_configs": small,
            "sample": f"{P_full.name} shape (p={P_full.p}, n={P_full.n}, M={P_full.M}) timed at N={n1} and N={n2} "
                      f"(N*:N as in the workload), FP64 numpy/scipy oracle (Gram, LU, mean, variance); value = "
                      f"full workload from t = F + c (N + N*) fitted to the two samples"}


# Source sections whose code a counter record is tied to: (file, first
# banner, end marker); the fingerprint is the sha256 of the code between
# them with comment lines, trailing comments and blank lines dropped.
SECTIONS = {
    "variance": ("mixed_path.hip", "// ================================================================ a5 mixed predict",
                 "__global__ void predict_mixed_reduce_kernel"),
    "gram_pair": ("pair_gram.hip", "constexpr int kPgT", "// Single problem: grid"),
}


def source_fingerprint(section):
    fname, start, end = SECTIONS[section]
    src = open(os.path.join(ROOT, "paper_2403_12797_amd", "csrc", fname)).read()
    code = []
    for line in src[src.index(start):src.index(end)].splitlines():
        line = line.split("//", 1)[0].rstrip()
        if line:
            code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()


def kernel_traffic(P, section, record):
    """HBM bytes per launch of a kernel from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record (profiles/<record>), scaled by the copy-kernel
    calibration; None when the record is for another workload or the
    kernel's code has changed since."""
    path = os.path.join(ROOT, "profiles", record)
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None, "no counter record"
    if rec.get("N") != P.N or rec.get("Ns") != P.Ns or rec.get("M") != P.M or rec.get("workload") != P.name:
        return None, "counter record is for another workload"
    if rec.get("source_fingerprint") != source_fingerprint(section):
        return None, "kernel changed since the counters were taken"
    kib = sum(rec["fetch_kib_per_launch"]) * rec["fetch_factor"] + sum(rec["write_kib_per_launch"]) * rec["write_factor"]
    return kib * 1024.0 / len(rec["fetch_kib_per_launch"]), "bytes per launch, " + os.path.basename(path)


def gram_layout(P, f16):
    """The Gram layout the library picks for this shape (mirrors pair_plan in
    pair_gram.hip): paired when p >= 2, the tabulated digit counts and the
    LDS fit, and it has fewer 256 x 128 work items per chunk than the direct
    upper triangle; MGP_GRAM_LAYOUT=direct forces the direct layout."""
    if os.environ.get("MGP_GRAM_LAYOUT") == "direct" or P.p < 2:
        return None
    n, p = P.n, P.p
    s, p1 = n * (n + 1) // 2, p // 2
    S1, S2 = s ** p1, s ** (p - p1)
    if n ** p1 > 1024 or n ** (p - p1) > 1024:
        return None
    npre1 = min(S1, 256) // s + 2 if p1 > 1 else 0
    npre2 = min(S2, 128) // s + 2 if p - p1 > 1 else 0
    ndi = 2 * s + npre1 + npre2
    lds = 2 * (2 if f16 else 3) * 384 * 16 * 2 + 3 * (p * n + 1) * 20 * 4 + 2 * (ndi + 2) * 20 * 4 + 384 * 4 + ndi * 12 + 16
    T = -(-P.M // 256)
    T1, T2 = -(-S1 // 256), -(-S2 // 128)
    if lds > 159 * 1024 or T1 * T2 >= T * (T + 1):
        return None
    F = 2 * max(1, p - p1 - 1)
    return {"s": s, "p1": p1, "S1": S1, "S2": S2, "T1": T1, "T2": T2, "F": F}


def variance_issued_flops(P):
    """MFMA flops the variance kernel issues: three products per pair over
    256-point tiles x 256-wide L^-1 row blocks x the 16-column stages each
    row block reaches (columns c <= its last row)."""
    Mc = -(-P.M // 16)
    RB = -(-P.M // 256)
    stages = sum(min((rb + 1) * 16, Mc) for rb in range(RB))
    pts = -(-P.Ns // 256) * 256
    return 3 * 2 * pts * 256 * 16 * stages


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU design is described "
              f"in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_12797_amd import binding as B
    from paper_2403_12797_amd import workloads as wl
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                          "launches": 3}))
        return
    if a.batched_only:
        print(json.dumps(batched_leg(torch, a.batched, steps=a.steps)), flush=True)
        return
    P = wl.config(a.config, N=a.N, Ns=a.Ns)
    dev = tuple(torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in (P.x, P.y, P.xs))
    torch.cuda.synchronize()
    ctx = B.Context(0)
    f16 = a.gram == "f16"
    prec = B.PREC_MIXED_F16 if f16 else B.PREC_MIXED
    print(f"[bench] {P.name} N={P.N} Ns={P.Ns} M={P.M}: mixed path, {a.gram} Gram", file=sys.stderr, flush=True)
    dt_mx, prof_mx, _ = run_path(ctx, torch, P, dev, prec, a.steps, a.warmup)
    print(f"[bench] mixed {dt_mx * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
    alt = None
    if not a.no_alt:
        k_alt = max(1, min(a.steps, 2))
        dt_alt, prof_alt, _ = run_path(ctx, torch, P, dev, B.PREC_MIXED if f16 else B.PREC_MIXED_F16, k_alt, 1)
        print(f"[bench] other Gram scheme {dt_alt * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
        alt = {"gram": "bf16x3 (3 terms, 6 products)" if f16 else "f16x2 (2 terms, 3 products)",
               "value": (P.N + P.Ns) / dt_alt, "ms_per_step": dt_alt * 1e3, "steps": k_alt,
               "phases_ms": {k: round(v[0] / k_alt, 3) for k, v in prof_alt.items() if v[1]}}
    fp64 = None
    if not a.no_fp64:
        k64 = max(1, min(a.steps, 2))
        dt64, prof64, _ = run_path(ctx, torch, P, dev, B.PREC_FP64, k64, 1)
        print(f"[bench] fp64 {dt64 * 1e3:.1f} ms/step", file=sys.stderr, flush=True)
        g64 = prof64["gram"][0] / k64
        fp64 = {"value": (P.N + P.Ns) / dt64, "ms_per_step": dt64 * 1e3, "steps": k64,
                "gram_frac_fp64_peak": (P.N * P.M * (P.M + 1)) / (g64 * 1e-3) / PEAK_FP64,
                "phases_ms": {k: round(v[0] / k64, 3) for k, v in prof64.items() if v[1]}}
    ctx.close()

    steps = a.steps
    # dominant kernel: the variance contraction (a5); the Gram (a3) beside it
    pv_ms, pv_cnt = prof_mx["predict"]
    var_launch_ms = pv_ms / pv_cnt
    var_flops = P.Ns * P.M * (P.M + 1)        # per launch: per test point M(M+1) (triangular L^-1 phi, squares)
    var_achieved = var_flops / (var_launch_ms * 1e-3)
    var_traffic, var_traffic_note = kernel_traffic(P, "variance", f"predict_var_mixed_kernel_{P.name}_hbm.json")
    tn = 256 if (P.p * P.n + 1 + 2 * (15 // P.n + 2)) * 256 * 4 + 2 * 2 * 16 * 512 * 2 + 2 * 256 * 8 + 8192 <= 159 * 1024 \
        else 128
    var_kernel = f"predict_var_mixed_kernel<{tn}, {P.p}, {'true' if P.n % (16 * tn // 512) == 0 else 'false'}>"
    g_ms, g_cnt = prof_mx["gram"]
    gram_launch_ms = g_ms / g_cnt
    lay = gram_layout(P, f16)
    nt = 3 if f16 else 6
    if lay:
        gram_flops = 2 * P.N * lay["s"] ** P.p            # H = Psi1^T Psi2: N s^p multiply-adds
        ceil32 = lambda v: -(-v // 32) * 32
        gram_issued = nt * 2 * P.N * ceil32(lay["S1"]) * ceil32(lay["S2"])
        gram_kernel = f"gram_pair_kernel<{'true' if f16 else 'false'}, {lay['F']}, 0>"
    else:
        gram_flops = P.N * P.M * (P.M + 1)
        T = -(-P.M // 256)
        gram_issued = nt * 2 * P.N * 65536 * T * (T + 1) // 2
        gram_kernel = f"gram_mixed_kernel<{'true' if f16 else 'false'}>"
    out = {
        "metric": METRIC, "value": (P.N + P.Ns) / dt_mx, "unit": "points/s", "n_gpus": 1, "steps": steps,
        "warmup": a.warmup, "ms_per_step": dt_mx * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ("f16x2 Gram" if f16 else "bf16x3 Gram") + ", bf16x2 variance, fp32 acc, fp64 factor",
        "data": "synthetic",
        "config": {"workload": f"{P.name}: p={P.p}, n={P.n}, M={P.M}, N={P.N}, N*={P.Ns}, "
                               f"{P.meta.get('recipe', '')}; "
                               f"fit + predict(mean, var); Gram "
                               + ("paired (pair tuples of two dimension groups) " if lay else "direct ")
                               + ("split-FP16 MFMA on power-of-two-scaled operands (2 terms, 3 products)" if f16 else
                                  "split-BF16 MFMA (3 terms, 6 products)")
                               + "; variance split-BF16 MFMA (2 terms, 3 products); FP64 Cholesky + 1 refinement",
                   "precision": "mixed_f16" if f16 else "mixed"},
        "roofline": {"kernel": var_kernel, "bound": "mfma", "achieved": var_achieved / 1e12,
                     "peak": PEAK_16 / 1e12, "unit": "TFLOP/s", "frac": var_achieved / PEAK_16,
                     "traffic": var_traffic, "traffic_note": var_traffic_note, "launches_per_step": pv_cnt / steps,
                     "avg_launch_ms": var_launch_ms, "algorithmic_flops_per_launch": var_flops,
                     "mfma_issue_frac": variance_issued_flops(P) / (var_launch_ms * 1e-3) / PEAK_16},
        "gram": {"kernel": gram_kernel, "layout": "paired" if lay else "direct", "bound": "mfma",
                 "avg_launch_ms": gram_launch_ms, "launches_per_step": g_cnt / steps,
                 "algorithmic_flops_per_launch": gram_flops,
                 "achieved": gram_flops / (gram_launch_ms * 1e-3) / 1e12, "unit": "TFLOP/s",
                 "frac": gram_flops / (gram_launch_ms * 1e-3) / PEAK_16,
                 "mfma_issue_frac": gram_issued / (gram_launch_ms * 1e-3) / PEAK_16,
                 "direct_gram_equivalent_frac": P.N * P.M * (P.M + 1) / (gram_launch_ms * 1e-3) / PEAK_16},
        "phases_ms": {k: round(v[0] / steps, 3) for k, v in prof_mx.items() if v[1]},
        "other_gram_scheme": alt,
        "fp64_path": fp64,
        "served": None,
        "batched": None,
        "cpu_baseline": None if a.no_cpu else cpu_baseline(P, a.cpu_target_s),
    }
    if a.batched > 0:
        print(f"[bench] batched leg: {a.batched} problems", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(torch, a.batched)
    if a.serve_seconds > 0:
        print(f"[bench] served stream {a.serve_seconds:.0f} s at {a.serve_rate:.0f} req/s", file=sys.stderr,
              flush=True)
        out["served"] = served_stream(torch, a.serve_rate, a.serve_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
