"""Launch schedules (kz tile of the x pass, row pitches of the y- and
z-transformed arrays, block cap of the persistent z passes, FP64 non-temporal
stores) change no result: every forced
schedule against the literal Eq. 10 oracle, element by element, and the
timed choice is reported, cached and grouped correctly in batches.
"""
import numpy as np
import pytest

from helpers import TOL, gpu_solve, log, oracle_input, rel_l2, rel_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _mk(shape, prec, kind=1, **kw):
    from paper_1111_4971_amd import pipe
    nx, ny, nz = shape
    a, b = 1.0, 1.3
    return pipe.GreenPlan(nx, ny, nz, a / (nx + 1), 0.9 * b / (ny + 1), 0.06, a, b, kind=kind, precision=prec,
                          mx=2 * nx + 1, my=2 * ny + 3, **kw)


def _ref(shape, rho, prec, kind=1):
    from oracle import fourterm
    nx, ny, nz = shape
    a, b = 1.0, 1.3
    return fourterm.solve(oracle_input(rho, prec), a / (nx + 1), 0.9 * b / (ny + 1), 0.06, a, b, 2 * nx + 1,
                          2 * ny + 3, kind)


# ragged kz tiles, a radix-3 length, an odd lz/2, the four-stage 384
SHAPES = [(13, 11, 40), (24, 12, 70), (9, 5, 81), (150, 3, 9)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_forced_schedule_matches_eq10_oracle(torch_cuda, monkeypatch, shape, prec):
    rho = np.random.default_rng(sum(shape)).standard_normal(shape)
    ref = _ref(shape, rho, prec)
    monkeypatch.setenv("PIPE_SCHEDULE", "fixed")
    T = _mk(shape, prec).info.xtile
    tiles = [T, T // 2] if T > 1 else [T]
    for t in tiles:
        for pad in (0, 16, 32):
            for cap, nt, a1 in ((1, 0, 16), (7, 1, 0), (2048, 0, 0), (4096, 1, 16)):
                if prec == "fp32":
                    nt = 0          # non-temporal stores are an FP64 option
                monkeypatch.setenv("PIPE_SCHEDULE", "%d,%d,%d,%d,%d" % (t, pad, cap, nt, a1))
                log("schedule %s %s T=%d pad=%d cap=%d nt=%d a1=%d" % (prec, shape, t, pad, cap, nt, a1))
                plan = _mk(shape, prec)
                i = plan.info
                assert (i.xtile, i.apad, i.zblocks, i.xnt, i.a1pad) == (t, pad, cap, nt, a1)
                got = gpu_solve(plan, rho)
                assert rel_l2(got, ref) <= TOL[prec] and rel_max(got, ref) <= TOL[prec], (t, pad, cap, nt, a1)
                plan.close()


def test_bad_forced_schedule_is_rejected(torch_cuda, monkeypatch):
    from paper_1111_4971_amd import pipe
    monkeypatch.setenv("PIPE_SCHEDULE", "3,0,2048")    # not a compiled tile
    with pytest.raises(pipe.PipeError) as e:
        _mk((13, 11, 40), "fp32")
    assert e.value.status == 1
    monkeypatch.setenv("PIPE_SCHEDULE", "8,-1,2048")
    with pytest.raises(pipe.PipeError):
        _mk((13, 11, 40), "fp32")
    monkeypatch.setenv("PIPE_SCHEDULE", "8,0,2048,2")
    with pytest.raises(pipe.PipeError):
        _mk((13, 11, 40), "fp32")
    monkeypatch.setenv("PIPE_SCHEDULE", "8,0,2048,1")     # an FP64-only option
    with pytest.raises(pipe.PipeError):
        _mk((13, 11, 40), "fp32")
    for bad in ("8,0,2048,0,3", "8,0,2048,0,258", "8,0,2048,0,-2"):   # the A1 pad: even, 0 .. 256
        monkeypatch.setenv("PIPE_SCHEDULE", bad)
        with pytest.raises(pipe.PipeError):
            _mk((13, 11, 40), "fp32")


def test_timed_schedule_is_cached_and_adjoint_agrees(torch_cuda, monkeypatch):
    torch = torch_cuda
    monkeypatch.delenv("PIPE_SCHEDULE", raising=False)
    shape = (40, 36, 100)
    p1 = _mk(shape, "fp32")
    p2 = _mk(shape, "fp32")
    s1 = (p1.info.xtile, p1.info.apad, p1.info.zblocks)
    assert s1 == (p2.info.xtile, p2.info.apad, p2.info.zblocks)
    assert p1.info.apad in (0, 16, 32) and p1.info.zblocks in (1024, 2048, 4096) and p1.info.a1pad in (0, 16)
    assert p1.info.a1pad == p2.info.a1pad
    rho = np.random.default_rng(4).standard_normal(shape)
    got = gpu_solve(p1, rho)
    ref = _ref(shape, rho, "fp32")
    assert rel_l2(got, ref) <= 1e-5 and rel_max(got, ref) <= 1e-5
    x = torch.from_numpy(rho).to("cuda", torch.float32)
    assert rel_l2(p1.adjoint(x).double().cpu().numpy(), got) <= 1e-5


def test_batch_groups_plans_by_schedule(torch_cuda, monkeypatch):
    """Plans of one mesh with different schedules go to different grouped
    launches; every member equals its own single solve."""
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    shape = (20, 18, 50)
    plans = []
    for sched in ("8,0,2048", "8,16,1024,0", "4,32,7", "8,0,2048,0", "8,0,2048,0,16"):
        monkeypatch.setenv("PIPE_SCHEDULE", sched)
        plans.append(_mk(shape, "fp32"))
    rng = np.random.default_rng(6)
    rhos = [torch.from_numpy(rng.standard_normal(shape)).to("cuda", torch.float32) for _ in plans]
    log("batch with mixed schedules")
    b = pipe.Batch(plans)
    outs = b.solve(rhos)
    torch.cuda.synchronize()
    for p, r, o in zip(plans, rhos, outs):
        assert torch.equal(o, p.solve(r))
    b.close()
