"""Batched solves (pipe_batch_*): 96 uneven meshes in one replay of a captured HIP graph.

Each member must equal its own single solve, and the oracle at sampled
members; replaying the graph must give the same result every time, also
with the program's own work between replays; new pointers rebuild it.
"""
import numpy as np
import pytest

from helpers import log, oracle_input, rel_l2, rel_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def batch_setup(torch_cuda):
    torch = torch_cuda
    from paper_1111_4971_amd import pipe, workloads
    man = workloads.batch_manifest()
    log("batch: building %d plans" % len(man))
    members = [workloads.batch_member(d) for d in man]
    plans = [pipe.GreenPlan(w.nx, w.ny, w.nz, w.hx, w.hy, w.hz, w.a, w.b, kind=w.kind, precision="fp32",
                            mx=w.mx, my=w.my) for w in members]
    rhos = [torch.from_numpy(w.rho).to("cuda", torch.float32) for w in members]
    return members, plans, rhos


def test_batch_equals_single_solves_and_replays(torch_cuda, batch_setup):
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    members, plans, rhos = batch_setup
    shapes = sorted({w.shape for w in members})
    assert len(shapes) == 4
    log("batch: single solves")
    singles = [p.solve(r).double().cpu().numpy() for p, r in zip(plans, rhos)]
    log("batch: graph create + solve")
    b = pipe.Batch(plans)
    outs = [torch.empty_like(r) for r in rhos]
    b.solve(rhos, outs)
    torch.cuda.synchronize()
    first = [o.double().cpu().numpy() for o in outs]
    for s, f in zip(singles, first):
        assert rel_l2(f, s) <= 1e-6 and rel_max(f, s) <= 1e-6
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        _ = (rhos[0] * 2).sum().item()     # unrelated eager work between replays
        b.solve(rhos, outs)
        torch.cuda.synchronize()
        for f, o in zip(first, outs):
            assert np.array_equal(f, o.double().cpu().numpy())
    # new output buffers: the descriptors are copied again, the graph replayed
    outs2 = [torch.empty_like(r) for r in rhos]
    b.solve(rhos, outs2)
    torch.cuda.synchronize()
    for f, o in zip(first, outs2):
        assert np.array_equal(f, o.double().cpu().numpy())
    # alternate between the two output sets, back to back with no host wait,
    # then on a second stream: every call must write its own outputs
    side = torch.cuda.Stream()
    for rep in range(3):
        for o in outs + outs2:
            o.zero_()
        b.solve(rhos, outs)
        b.solve(rhos, outs2)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            outs3 = [torch.empty_like(r) for r in rhos]
            b.solve(rhos, outs3, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        for f, o1, o2, o3 in zip(first, outs, outs2, outs3):
            assert np.array_equal(f, o1.double().cpu().numpy())
            assert np.array_equal(f, o2.double().cpu().numpy())
            assert np.array_equal(f, o3.double().cpu().numpy())
    b.close()


def test_batch_members_match_the_oracle(torch_cuda, batch_setup):
    from oracle import modespace
    members, plans, rhos = batch_setup
    from paper_1111_4971_amd import pipe
    b = pipe.Batch(plans)
    outs = b.solve(rhos)
    import torch
    torch.cuda.synchronize()
    seen = set()
    for w, o in zip(members, outs):
        if w.shape in seen:
            continue
        seen.add(w.shape)
        log("batch: oracle check %s" % (w.shape,))
        ref = modespace.solve(oracle_input(w.rho, "fp32"), **w.geometry())
        got = o.double().cpu().numpy()
        assert rel_l2(got, ref) <= 1e-5 and rel_max(got, ref) <= 1e-5
    b.close()


def test_batch_rejects_bad_arguments(torch_cuda, batch_setup):
    torch = torch_cuda
    import ctypes
    from paper_1111_4971_amd import pipe
    members, plans, rhos = batch_setup
    L = pipe.lib()
    h = ctypes.c_void_p()
    mixed = pipe.GreenPlan(8, 8, 8, 0.1, 0.1, 0.1, 1.0, 1.0, precision="fp64")
    arr = (ctypes.c_void_p * 2)(plans[0].handle, mixed.handle)
    assert L.pipe_batch_create(arr, 2, ctypes.byref(h)) == 1     # mixed precision
    b = pipe.Batch(plans[:2])
    ws = b.workspace()
    ra = (ctypes.c_void_p * 2)(rhos[0].data_ptr(), rhos[1].data_ptr())
    pa = (ctypes.c_void_p * 2)(rhos[0].data_ptr(), rhos[1].data_ptr())   # phi aliases rho
    assert L.pipe_batch_solve(b._h, ra, pa, ctypes.c_void_p(ws.data_ptr()), None) == 6
    b.close()
    assert L.pipe_batch_destroy(h) == 1


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_same_plan_many_charges(torch_cuda, prec):
    """A batch holding one plan several times (many charges, one cached Green
    function): every member equals that plan's single solve."""
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    plan = pipe.GreenPlan(24, 20, 48, 1.0 / 25, 1.0 / 21, 0.05, 1.0, 1.0, kind=pipe.IGF_Z, precision=prec)
    rng = np.random.default_rng(77)
    rhos = [torch.tensor(rng.standard_normal(plan.shape), device="cuda", dtype=plan.dtype) for _ in range(5)]
    log("same plan x5 %s" % prec)
    outs = pipe.Batch([plan] * 5).solve(rhos)
    torch.cuda.synchronize()
    for r, o in zip(rhos, outs):
        ref = plan.solve(r)
        assert torch.equal(o, ref)


def test_autotuned_batch_members_match_the_oracle(torch_cuda):
    """The batch the benchmark times: 96 uneven FP32 plans whose padded lengths
    the throughput-mode autotuner picked (e.g. 96x96x192 -> 256x192x384), one
    replay of the graph.  One member per mesh shape against the mode-space
    oracle (exact for these full-aperture meshes), every member against its
    own single solve."""
    torch = torch_cuda
    from oracle import modespace
    from paper_1111_4971_amd import pipe, workloads
    man = workloads.batch_manifest()
    members = [workloads.batch_member(d) for d in man]
    log("autotuned batch: building %d plans" % len(members))
    plans = [pipe.GreenPlan(w.nx, w.ny, w.nz, w.hx, w.hy, w.hz, w.a, w.b, kind=w.kind, precision="fp32",
                            mx=w.mx, my=w.my, autotune="batch") for w in members]
    rhos = [torch.from_numpy(w.rho).to("cuda", torch.float32) for w in members]
    lengths = {w.shape: (p.info.lx, p.info.ly, p.info.lz) for w, p in zip(members, plans)}
    log("autotuned batch: lengths %s" % lengths)
    for w, p in zip(members, plans):
        assert (p.info.lx, p.info.ly, p.info.lz) == lengths[w.shape]
    b = pipe.Batch(plans)
    outs = b.solve(rhos)
    torch.cuda.synchronize()
    seen = set()
    for w, p, r, o in zip(members, plans, rhos, outs):
        got = o.double().cpu().numpy()
        single = p.solve(r).double().cpu().numpy()
        assert rel_l2(got, single) <= 1e-6 and rel_max(got, single) <= 1e-6
        if w.shape in seen:
            continue
        seen.add(w.shape)
        log("autotuned batch: oracle check %s at %s" % (w.shape, lengths[w.shape]))
        ref = modespace.solve(oracle_input(w.rho, "fp32"), **w.geometry())
        assert rel_l2(got, ref) <= 1e-5 and rel_max(got, ref) <= 1e-5, (w.shape, rel_l2(got, ref))
    assert len(seen) == 4
    b.close()
    for p in plans:
        p.close()
