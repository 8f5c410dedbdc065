"""gp_predict_noalloc (the prediction entry point that allocates nothing)
against gp_predict through the C ABI: same kernels on the same inputs, so the
outputs must agree bitwise, on two calls in a row (the second with a smaller
input, so it reuses the fixed scratch array after a larger call), for a
mixed-precision and an FP64 model; and the host-side rejection of an input
too large for the array."""
import numpy as np
import pytest

from paper_2403_12797_amd import binding as B
from paper_2403_12797_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("precision", [B.PREC_MIXED_F16, B.PREC_FP64])
def test_noalloc_matches_predict(torch_cuda, precision):
    torch = torch_cuda
    P = wl.random_problem(71, 3, 7, 20000, 6000)
    print(f"[case] noalloc precision={precision} M={P.M} Ns={P.Ns} then {P.Ns // 3}", flush=True)
    with B.Context(0) as ctx:
        m = ctx.fit(_dev(torch, P.x), _dev(torch, P.y), p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha,
                    precision=precision)
        for Ns in (P.Ns, P.Ns // 3):          # second call smaller than the first
            xs = _dev(torch, P.xs[:Ns])
            ref_m = torch.empty(Ns, dtype=torch.float64, device="cuda")
            ref_v = torch.empty_like(ref_m)
            ctx.predict(m, xs, ref_m, ref_v)
            got_m = torch.full_like(ref_m, float("nan"))
            got_v = torch.full_like(ref_m, float("nan"))
            ctx.predict_noalloc(m, xs, got_m, got_v)
            torch.cuda.synchronize()
            assert torch.equal(got_m, ref_m) and torch.equal(got_v, ref_v), Ns
        m.free()


def test_noalloc_rejects_oversized_input(torch_cuda):
    torch = torch_cuda
    P = wl.random_problem(72, 2, 4, 500, 10)
    with B.Context(0) as ctx:
        m = ctx.fit(_dev(torch, P.x), _dev(torch, P.y), p=P.p, n=P.n, sigma=P.sigma, eps=P.eps, alpha=P.alpha,
                    precision=B.PREC_MIXED_F16)
        Ns = (32 << 20) // 8 + 1                 # one more partial sum than the array holds
        xs = torch.zeros((Ns, P.p), dtype=torch.float64, device="cuda")
        out = torch.empty(Ns, dtype=torch.float64, device="cuda")
        with pytest.raises(B.GpError) as ei:
            ctx.predict_noalloc(m, xs, None, out)
        assert ei.value.status == B.GP_EINVAL and "scratch" in str(ei.value)
        m.free()
