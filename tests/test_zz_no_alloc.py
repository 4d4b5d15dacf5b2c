"""The allocation-free likelihood call (pcmd_loglike_noalloc) through the C ABI against
pcmd_loglike on the same inputs: identical kernels and block order, so identical results, on two
calls in a row (the second with fewer bins, so the static scratch holds the first call's sums)."""
import ctypes as C

import numpy as np
import pytest

from oracle import loglike as ol

pytestmark = pytest.mark.gpu


def _call_noalloc(ctx, hm, hd, mm, md, out, mode, eps):
    import torch
    lib = ctx.lib
    f = lib.pcmd_loglike_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                  C.c_void_p, C.c_void_p]
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return f(ctx.h, C.c_void_p(hm.data_ptr()), C.c_void_p(hd.data_ptr()), int(hm.numel()), C.c_void_p(mm.data_ptr()),
             C.c_void_p(md.data_ptr()), int(mode), float(eps), C.c_void_p(out.data_ptr()), s)


def test_noalloc_loglike_matches_pcmd_loglike():
    import torch
    import paper_1904_00011_amd as P
    ctx = P.Context(0)
    dev = torch.device("cuda")
    r = np.random.default_rng(99)
    try:
        for nb in (40000, 7, 10000):  # the second and third calls are smaller than the first
            hm = r.poisson(2.5, nb)
            hd = r.poisson(2.5, nb)
            hm[-1] += 1
            mom_m = np.array([40.0 * hm.sum(), 2e3 * hm.sum(), float(hm.sum())])
            mom_d = np.array([41.0 * hd.sum(), 2.01e3 * hd.sum(), float(hd.sum())])
            a = torch.from_numpy(hm.astype(np.int32)).to(dev)
            b = torch.from_numpy(hd.astype(np.int32)).to(dev)
            mm = torch.from_numpy(mom_m).to(dev)
            md = torch.from_numpy(mom_d).to(dev)
            for mode in (0, 1, 2):
                print(f"[case] noalloc loglike nbins={nb} mode={mode}", flush=True)
                want = torch.empty(1, dtype=torch.float64, device=dev)
                got = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
                ctx.loglike(a, b, mm, md, want, mode, 0.01)
                assert _call_noalloc(ctx, a, b, mm, md, got, mode, 0.01) == 0, ctx.lib.pcmd_last_error(ctx.h)
                ctx.sync()
                assert got.item() == want.item()
                lo = ol.loglike(hm, hd, mom_m, mom_d, mode)
                assert abs(got.item() - lo) <= max(1e-9 * abs(lo), 1e-9)
        # sizes beyond the static scratch are refused before anything runs
        big = torch.zeros(65537, dtype=torch.int32, device=dev)
        out = torch.zeros(1, dtype=torch.float64, device=dev)
        mm = torch.ones(3, dtype=torch.float64, device=dev)
        assert _call_noalloc(ctx, big, big, mm, mm, out, 0, 0.01) == P._lib.E_INVAL
        assert b"65536" in ctx.lib.pcmd_last_error(ctx.h)
    finally:
        ctx.close()
