"""The allocation-free solve (pipe_poisson_solve_noalloc) against the ordinary
solve (pipe_poisson_solve with a caller workspace), through the C ABI.

Both run the same kernels on the same inputs, so their outputs must agree
exactly; the ordinary solve is itself checked against the oracle elsewhere,
and once more here on the small mesh.  Two calls in a row, the second on a
smaller mesh (the scratch keeps the first call's contents), then the
benchmark's 128 x 128 x 512 FP32 mesh, whose workspace nearly fills the
scratch, and a plan too large for it (FP64 at that size).
"""
import ctypes

import numpy as np
import pytest

from helpers import TOL, log, oracle_input, rel_l2, rel_max

pytestmark = pytest.mark.gpu


def _plan(shape, prec, kind=1):
    from paper_1111_4971_amd import pipe
    nx, ny, nz = shape
    a, b = 1.0, 1.2
    return pipe.GreenPlan(nx, ny, nz, a / (nx + 1), b / (ny + 1), 0.05, a, b, kind=kind, precision=prec)


def _noalloc(plan, x, out):
    from paper_1111_4971_amd import pipe
    import torch
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return pipe.lib().pipe_poisson_solve_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), st)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_the_workspace_solve(prec):
    import torch
    from oracle import fourterm
    assert torch.cuda.is_available()
    big, small = (40, 36, 100), (12, 10, 24)
    plans = {s: _plan(s, prec) for s in (big, small)}
    rng = np.random.default_rng(3)
    rhos = {s: rng.standard_normal(s) for s in (big, small)}
    for s in (big, small, big):   # the second call is on the smaller mesh
        p = plans[s]
        x = torch.from_numpy(rhos[s]).to("cuda", p.dtype)
        log("noalloc %s shape=%s" % (prec, s))
        out = torch.full_like(x, float("nan"))
        assert _noalloc(p, x, out) == 0, p_err()
        ref = p.solve(x)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), float((out - ref).abs().max())
    # the small mesh against the oracle too
    p = plans[small]
    x = torch.from_numpy(rhos[small]).to("cuda", p.dtype)
    out = torch.empty_like(x)
    assert _noalloc(p, x, out) == 0, p_err()
    torch.cuda.synchronize()
    nx, ny, nz = small
    ref = fourterm.solve(oracle_input(rhos[small], prec), 1.0 / (nx + 1), 1.2 / (ny + 1), 0.05, 1.0, 1.2,
                         2 * nx, 2 * ny, 1)
    got = out.double().cpu().numpy()
    assert rel_l2(got, ref) <= TOL[prec] and rel_max(got, ref) <= TOL[prec]
    for q in plans.values():
        q.close()


def p_err():
    from paper_1111_4971_amd import pipe
    return pipe.lib().pipe_last_error().decode()


def test_noalloc_at_the_benchmark_size_and_beyond():
    import torch
    shape = (128, 128, 512)
    p32 = _plan(shape, "fp32")
    assert p32.info.workspace_bytes <= 256 << 20
    x = torch.from_numpy(np.random.default_rng(9).standard_normal(shape)).to("cuda", torch.float32)
    out = torch.empty_like(x)
    log("noalloc fp32 %s" % (shape,))
    assert _noalloc(p32, x, out) == 0, p_err()
    ref = p32.solve(x)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    p32.close()
    p64 = _plan(shape, "fp64")
    assert p64.info.workspace_bytes > 256 << 20
    x64 = x.double()
    out64 = torch.empty_like(x64)
    log("noalloc fp64 %s (too large)" % (shape,))
    assert _noalloc(p64, x64, out64) == 2   # PIPE_ERR_UNSUPPORTED_SIZE
    assert "scratch" in p_err()
    p64.close()
    from paper_1111_4971_amd import pipe
    assert pipe.lib().pipe_poisson_solve_noalloc(ctypes.c_void_p(16), ctypes.c_void_p(x.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), None) == 1
