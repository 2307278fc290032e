"""Shared helpers for the GPU parity tests (comparison metrics, plan construction)."""
import sys

import numpy as np


def log(msg):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def rel_max(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


# Tolerances: FP64 path <= 1e-12, FP32 path <= 1e-5, both in relative L2 and in
# max-norm relative to max|phi| (the FP32 error measured against the FP64
# oracle run on the FP32-rounded input, so input rounding is not counted).
TOL = {"fp64": 1e-12, "fp32": 1e-5}


def plan_for(wl, precision, **kw):
    from paper_1111_4971_amd import pipe
    return pipe.GreenPlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, wl.a, wl.b, kind=wl.kind,
                          precision=precision, mx=wl.mx, my=wl.my, **kw)


def gpu_solve(plan, rho_np):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(rho_np)).to(device="cuda", dtype=plan.dtype)
    y = plan.solve(x)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def oracle_input(rho_np, precision):
    """The values the GPU actually sees, upcast to FP64."""
    if precision == "fp32":
        return rho_np.astype(np.float32).astype(np.float64)
    return np.asarray(rho_np, dtype=np.float64)
