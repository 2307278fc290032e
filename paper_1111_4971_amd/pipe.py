"""Python binding of libpipe (ctypes): argument marshalling only.

Every step of a solve runs in the HIP kernels of libpipe.so.  PyTorch supplies
device memory (tensors) and streams.  If the shared library is missing this
module raises at load time; there is no fallback.

Entry points mirror include/pipe_poisson.h:
  GreenPlan(...)            -> pipe_green_plan_ex
  GreenPlan.solve(rho)      -> pipe_poisson_solve
  GreenPlan.adjoint(dphi)   -> pipe_poisson_adjoint
  Batch(plans).solve(rhos)  -> pipe_batch_create / pipe_batch_solve
  PipePoissonFn.apply(rho, plan): autograd function whose backward is the adjoint.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpipe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pipe_poisson.h")

POINT, IGF_Z, FREE = 0, 1, 2
PREC_FP64, PREC_FP32 = 0x00, 0x10
KEEP_GREEN = 0x100
AUTOTUNE = 0x200
AUTOTUNE_BATCH = 0x400
BAND_FASTEST = 0x800

STATUS = {0: "PIPE_OK", 1: "PIPE_ERR_INVALID_ARG", 2: "PIPE_ERR_UNSUPPORTED_SIZE", 3: "PIPE_ERR_OUT_OF_MEMORY",
          4: "PIPE_ERR_NO_DEVICE", 5: "PIPE_ERR_HIP", 6: "PIPE_ERR_ALIASING"}


class PipeError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status
        self.message = message


class PlanInfo(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_int), ("ly", ctypes.c_int), ("lz", ctypes.c_int),
                ("mx", ctypes.c_int), ("my", ctypes.c_int), ("kind", ctypes.c_int),
                ("real_bytes", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("norm", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t), ("spectra_bytes", ctypes.c_size_t),
                ("model_bytes", ctypes.c_double), ("pass_bytes", ctypes.c_double * 5),
                ("build_ms", ctypes.c_double), ("tune_ms", ctypes.c_double), ("band", ctypes.c_int),
                ("band_speedup", ctypes.c_double),
                ("xtile", ctypes.c_int), ("apad", ctypes.c_int), ("zblocks", ctypes.c_int), ("xnt", ctypes.c_int),
                ("a1pad", ctypes.c_int)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["pass_bytes"] = list(self.pass_bytes)
        return d


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def lib():
    """Load libpipe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpipe.so is not built (%s); run `python -m paper_1111_4971_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "pipe_green_plan": ([_I, _I, _I, _D, _D, _D, _D, _D, _I, ctypes.POINTER(_P)], _I),
        "pipe_green_plan_ex": ([_I, _I, _I, _D, _D, _D, _D, _D, _I, _I, _I, _I, _I, _I, _P,
                                ctypes.POINTER(_P)], _I),
        "pipe_green_plan_region": ([_I, _I, _I, _D, _D, _D, _D, _D, _D, _D, _I, _I, _I, _I, _I, _I, _P,
                                    ctypes.POINTER(_P)], _I),
        "pipe_green_plan_banded": ([_I, _I, _I, _D, _D, _D, _D, _D, _D, _D, _I, _I, _I, _I, _I, _I, _D, _P,
                                    ctypes.POINTER(_P)], _I),
        "pipe_free_plan": ([_I, _I, _I, _D, _D, _D, _D, _I, _I, _I, _I, _P, ctypes.POINTER(_P)], _I),
        "pipe_fft3d": ([_I, _I, _I, _I, ctypes.c_char_p, _P, _P, _P], _I),
        "pipe_plan_info": ([_P, ctypes.POINTER(PlanInfo)], _I),
        "pipe_default_lengths": ([_I, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)], _I),
        "pipe_poisson_solve": ([_P, _P, _P, _P, _P], _I),
        "pipe_poisson_adjoint": ([_P, _P, _P, _P, _P], _I),
        "pipe_poisson_solve_noalloc": ([_P, _P, _P, _P], _I),
        "pipe_poisson_solve_timed": ([_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_float)], _I),
        "pipe_batch_create": ([ctypes.POINTER(_P), _I, ctypes.POINTER(_P)], _I),
        "pipe_batch_workspace": ([_P, ctypes.POINTER(ctypes.c_size_t)], _I),
        "pipe_batch_solve": ([_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _P, _P], _I),
        "pipe_plan_destroy": ([_P], _I),
        "pipe_batch_destroy": ([_P], _I),
        "pipe_status_string": ([_I], ctypes.c_char_p),
        "pipe_last_error": ([], ctypes.c_char_p),
        "pipe_plan_green_table": ([_P, _P, _P], _I),
        "pipe_plan_spectra": ([_P, _P, _P], _I),
        "pipe_fft_lines": ([_I, _I, _I, _I, _I, _P, _P, _P], _I),
        "pipe_plan_timing": ([_P, _I, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_I)], _I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def header_functions():
    """Names of the functions include/pipe_poisson.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pipe_[a-z_0-9]+)\s*\(", txt)))


def check(status):
    if status != 0:
        raise PipeError(status, lib().pipe_last_error().decode())


def default_lengths(nx, ny, nz, precision="fp64"):
    """(lx, ly, lz) a default plan of this mesh and precision gets
    (pipe_default_lengths; host only)."""
    if precision not in ("fp32", "fp64"):
        raise ValueError("precision must be 'fp32' or 'fp64'")
    out = [_I(), _I(), _I()]
    check(lib().pipe_default_lengths(int(nx), int(ny), int(nz), PREC_FP32 if precision == "fp32" else PREC_FP64,
                                     *[ctypes.byref(v) for v in out]))
    return tuple(v.value for v in out)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype(real_bytes):
    torch = _torch()
    return torch.float64 if real_bytes == 8 else torch.float32


def _check_workspace_tensor(ws, need, device, owner):
    torch = _torch()
    if not isinstance(ws, torch.Tensor):
        raise TypeError("workspace: expected a tensor")
    if not ws.is_contiguous():
        raise ValueError("workspace: must be contiguous")
    nbytes = ws.numel() * ws.element_size()
    if nbytes < need:
        raise ValueError("workspace: %d bytes, %s needs %d" % (nbytes, owner, need))
    if not ws.is_cuda or ws.device != device:
        raise TypeError("workspace: expected a CUDA tensor on %s" % device)
    if ws.data_ptr() % 256:
        raise ValueError("workspace: must be 256-byte aligned")


class GreenPlan:
    """Cached Green spectra for one mesh (pipe_green_plan_ex).

    kind: POINT or IGF_Z; precision: 'fp64' or 'fp32'.  mx, my default to
    2 nx, 2 ny; L = (lx, ly, lz) defaults to the smallest supported lengths
    >= 2n (lx, ly: any 2^p 3^q in [8, 1024]; lz: even, lz/2 of that form).  autotune: False, True (time single solves) or "batch"
    (time 16 concurrent solves) to pick the padded lengths.  offset = (x0, y0)
    places the mesh on a sub-region of the cross-section (node i at
    x0 + (i+1) hx).  band = N keeps only plane distances |k - k'| <= N
    (pipe_green_plan_banded, Eq. 18); band = "auto" picks N from the decay
    of the mode sum with tolerance band_tol.  L is then (lx, ly).
    band_fastest=True returns the 3-D plan instead when it solves faster
    (info.band_speedup holds the measured ratio either way).
    """

    def __init__(self, nx, ny, nz, hx, hy, hz, a, b, kind=IGF_Z, precision="fp64", mx=None, my=None,
                 L=None, keep_green=False, autotune=False, stream=None, offset=(0.0, 0.0), band=None,
                 band_tol=1e-6, band_fastest=False):
        flags = int(kind) | (PREC_FP32 if precision == "fp32" else PREC_FP64) | (KEEP_GREEN if keep_green else 0)
        if band_fastest:
            flags |= BAND_FASTEST
        h = _P()
        st = _stream_ptr(stream) if stream is not None else None
        if band is not None:
            lx, ly = L[:2] if L is not None else (0, 0)
            nb = -1 if band == "auto" else int(band)
            if nb < 0 and band != "auto":
                raise ValueError("band must be >= 0 or 'auto'")
            check(lib().pipe_green_plan_banded(nx, ny, nz, hx, hy, hz, a, b, float(offset[0]), float(offset[1]),
                                               flags, mx or 2 * nx, my or 2 * ny, lx, ly, nb, float(band_tol), st,
                                               ctypes.byref(h)))
        else:
            flags |= {False: 0, True: AUTOTUNE, "batch": AUTOTUNE_BATCH}[autotune]
            lx, ly, lz = L if L is not None else (0, 0, 0)
            check(lib().pipe_green_plan_region(nx, ny, nz, hx, hy, hz, a, b, float(offset[0]), float(offset[1]),
                                               flags, mx or 2 * nx, my or 2 * ny, lx, ly, lz, st, ctypes.byref(h)))
        self._h = h
        info = PlanInfo()
        check(lib().pipe_plan_info(h, ctypes.byref(info)))
        self.info = info
        self.shape = (nx, ny, nz)
        self.dtype = _dtype(info.real_bytes)
        self._ws = None

    @property
    def band(self):
        """Planes kept on each side of the z sum (banded plans), else None."""
        return self.info.band if self.info.band >= 0 else None

    @property
    def handle(self):
        if self._h is None:
            raise PipeError(1, "plan already destroyed")
        return self._h

    def workspace(self, device="cuda", stream=None):
        """The plan's cached workspace for one stream (256-byte aligned view).

        Solves that run concurrently must not share a workspace, so the cache
        holds one buffer per (device, stream); stream None means the current
        stream of that device."""
        torch = _torch()
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        key = (dev.index, s.cuda_stream)
        if self._ws is None:
            self._ws = {}
        t = self._ws.get(key)
        if t is None:
            t = torch.empty(self.info.workspace_bytes + 256, dtype=torch.uint8, device=dev)
            self._ws[key] = t
        return self._aligned(t)

    @staticmethod
    def _aligned(t):
        off = (-t.data_ptr()) % 256
        return t[off:]

    def _check_array(self, x, what):
        torch = _torch()
        if not isinstance(x, torch.Tensor):
            raise TypeError("%s: expected a tensor" % what)
        if tuple(x.shape) != self.shape:
            raise ValueError("%s: expected shape %s, got %s" % (what, self.shape, tuple(x.shape)))
        if x.dtype != self.dtype:
            raise TypeError("%s: expected %s, got %s" % (what, self.dtype, x.dtype))
        if not x.is_cuda:
            raise TypeError("%s: expected a CUDA tensor" % what)

    def _prep(self, x):
        self._check_array(x, "input")
        return x.contiguous()

    def _check_out(self, out, x):
        self._check_array(out, "out")
        if not out.is_contiguous():
            raise ValueError("out: must be contiguous")
        if out.device != x.device:
            raise ValueError("out: on %s, input on %s" % (out.device, x.device))

    def _check_workspace(self, ws, x):
        _check_workspace_tensor(ws, self.info.workspace_bytes, x.device, "the plan")

    def _buffers(self, x, out, workspace, stream):
        torch = _torch()
        x = self._prep(x)
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_out(out, x)
        if workspace is None:
            ws = self.workspace(x.device, stream)
        else:
            self._check_workspace(workspace, x)
            ws = workspace
        return x, out, ws

    def _run(self, fn, x, out, workspace, stream):
        x, out, ws = self._buffers(x, out, workspace, stream)
        check(fn(self.handle, _P(x.data_ptr()), _P(out.data_ptr()), _P(ws.data_ptr()), _stream_ptr(stream)))
        return out

    def solve(self, rho, out=None, workspace=None, stream=None):
        return self._run(lib().pipe_poisson_solve, rho, out, workspace, stream)

    def solve_noalloc(self, rho, out, stream=None):
        """pipe_poisson_solve_noalloc: phi = A rho using the library's fixed
        device scratch instead of a workspace (out must be given)."""
        x = self._prep(rho)
        self._check_out(out, x)
        check(lib().pipe_poisson_solve_noalloc(self.handle, _P(x.data_ptr()), _P(out.data_ptr()),
                                                _stream_ptr(stream)))
        return out

    def adjoint(self, dphi, out=None, workspace=None, stream=None):
        return self._run(lib().pipe_poisson_adjoint, dphi, out, workspace, stream)

    def solve_timed(self, rho, out=None, workspace=None, stream=None):
        x, out, ws = self._buffers(rho, out, workspace, stream)
        ms = (ctypes.c_float * 5)()
        check(lib().pipe_poisson_solve_timed(self.handle, _P(x.data_ptr()), _P(out.data_ptr()),
                                             _P(ws.data_ptr()), _stream_ptr(stream), ms))
        return out, list(ms)

    def timing_start(self, max_solves):
        check(lib().pipe_plan_timing(self.handle, int(max_solves), None, None))

    def timing_stop(self):
        """Mean ms of each of the five kernels over the recorded solves, and their count."""
        ms = (ctypes.c_float * 5)()
        n = _I()
        check(lib().pipe_plan_timing(self.handle, 0, ms, ctypes.byref(n)))
        return list(ms), n.value

    def green_table(self):
        """R at [differences p hx (p < nx), sums 2 x0 + (p + 2) hx (p <= 2nx - 2)] x [same in y] x [r hz]
        (r < nz; r <= N for a banded plan)."""
        torch = _torch()
        nx, ny, nz = self.shape
        nr = self.band + 1 if self.band is not None else nz
        out = torch.empty((3 * nx - 1, 3 * ny - 1, nr), dtype=torch.float64, device="cuda")
        check(lib().pipe_plan_green_table(self.handle, _P(out.data_ptr()), _stream_ptr()))
        return out

    def spectra(self):
        """(table, nyquist) as tensors of shape (9, lx/2+1, ly/2+1, lz/2) and (9, lx/2+1, ly/2+1);
        for a banded plan its coefficient table K0..K9, shape (ly/2+1, N+1, 10, lx/2+1)."""
        torch = _torch()
        i = self.info
        kx, ky, nh = i.lx // 2 + 1, i.ly // 2 + 1, i.lz // 2
        if self.band is not None:
            out = torch.empty((ky, self.band + 1, 10, kx), dtype=self.dtype, device="cuda")
            check(lib().pipe_plan_spectra(self.handle, _P(out.data_ptr()), _stream_ptr()))
            return out
        flat = torch.empty(9 * kx * ky * (nh + 1), dtype=self.dtype, device="cuda")
        check(lib().pipe_plan_spectra(self.handle, _P(flat.data_ptr()), _stream_ptr()))
        n1 = 9 * kx * ky * nh
        return flat[:n1].view(9, kx, ky, nh), flat[n1:].view(9, kx, ky)

    def close(self):
        if self._h is not None:
            check(lib().pipe_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if self._h is not None:
                lib().pipe_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


class FreePlan(GreenPlan):
    """Free-space (isolated) plan: Hockney's zero-padded convolution with G = 1/r
    (pipe_free_plan, Sec. 1 Eq. 3-5); g0 is the value used at zero separation.
    Solves, adjoints, batches and timing work as for GreenPlan."""

    def __init__(self, nx, ny, nz, hx, hy, hz, g0, precision="fp64", L=None, autotune=False, stream=None):
        flags = (PREC_FP32 if precision == "fp32" else PREC_FP64)
        flags |= {False: 0, True: AUTOTUNE, "batch": AUTOTUNE_BATCH}[autotune]
        lx, ly, lz = L if L is not None else (0, 0, 0)
        h = _P()
        st = _stream_ptr(stream) if stream is not None else None
        check(lib().pipe_free_plan(nx, ny, nz, hx, hy, hz, float(g0), flags, lx, ly, lz, st, ctypes.byref(h)))
        self._h = h
        info = PlanInfo()
        check(lib().pipe_plan_info(h, ctypes.byref(info)))
        self.info = info
        self.shape = (nx, ny, nz)
        self.dtype = _dtype(info.real_bytes)
        self._ws = None


def fft3d(x, dirs, out=None, stream=None):
    """Unscaled 3-D DFT of a complex CUDA tensor with a direction per dimension
    (pipe_fft3d): dirs[d] = 'f' sums a_n W^{nk}, 'b' sums a_n W^{-nk},
    W = e^{-2 pi i/N}.  out may be x itself (in place)."""
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dim() != 3:
        raise TypeError("expected a 3-D CUDA tensor")
    if x.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("expected complex64 or complex128")
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    rb = 8 if x.dtype == torch.complex128 else 4
    check(lib().pipe_fft3d(rb, x.shape[0], x.shape[1], x.shape[2], dirs.encode(), _P(x.data_ptr()),
                           _P(out.data_ptr()), _stream_ptr(stream)))
    return out


class Batch:
    """Many plans solved by one replay of a captured HIP graph (pipe_batch_*)."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (_P * len(self.plans))(*[p.handle for p in self.plans])
        h = _P()
        check(lib().pipe_batch_create(arr, len(self.plans), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        check(lib().pipe_batch_workspace(h, ctypes.byref(n)))
        self.workspace_bytes = n.value
        self._ws = None
        self._outs = None

    def workspace(self, device="cuda", stream=None):
        """The batch's cached workspace for one stream (see GreenPlan.workspace)."""
        torch = _torch()
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        key = (dev.index, s.cuda_stream)
        if self._ws is None:
            self._ws = {}
        t = self._ws.get(key)
        if t is None:
            t = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
            self._ws[key] = t
        return GreenPlan._aligned(t)

    def solve(self, rhos, outs=None, workspace=None, stream=None):
        """phi_s = A_s rho_s for every member.  outs=None reuses the batch's own
        output tensors from the previous call (new ones only on the first call
        or when the input device changes), so repeated calls replay the
        captured graph unchanged; copy the results if they must outlive the
        next call."""
        torch = _torch()
        n = len(self.plans)
        rhos = list(rhos)
        if len(rhos) != n:
            raise ValueError("expected %d charge arrays, got %d" % (n, len(rhos)))
        for i, (p, r) in enumerate(zip(self.plans, rhos)):
            p._check_array(r, "rhos[%d]" % i)
            if not r.is_contiguous():
                raise ValueError("rhos[%d]: must be contiguous" % i)
            if r.device != rhos[0].device:
                raise ValueError("rhos[%d]: every member must be on one device" % i)
        if outs is None:
            if self._outs is None or self._outs[0].device != rhos[0].device:
                self._outs = [torch.empty_like(r) for r in rhos]
            outs = self._outs
        else:
            outs = list(outs)
            if len(outs) != n:
                raise ValueError("expected %d output arrays, got %d" % (n, len(outs)))
            for i, (p, r, o) in enumerate(zip(self.plans, rhos, outs)):
                p._check_out(o, r)
        if workspace is None:
            ws = self.workspace(rhos[0].device, stream)
        else:
            _check_workspace_tensor(workspace, self.workspace_bytes, rhos[0].device, "the batch")
            ws = workspace
        ra = (_P * n)(*[r.data_ptr() for r in rhos])
        pa = (_P * n)(*[o.data_ptr() for o in outs])
        check(lib().pipe_batch_solve(self._h, ra, pa, _P(ws.data_ptr()), _stream_ptr(stream)))
        return outs

    def close(self):
        if self._h is not None:
            check(lib().pipe_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if self._h is not None:
                lib().pipe_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass


def fft_lines(x, length, direction=-1, stream=None):
    """Batched 1-D DFT of the rows of a complex (howmany, n_in) CUDA tensor, zero-padded to `length`."""
    torch = _torch()
    if x.dtype not in (torch.complex64, torch.complex128) or x.dim() != 2:
        raise TypeError("expected a 2-D complex tensor")
    x = x.contiguous()
    rb = 8 if x.dtype == torch.complex128 else 4
    out = torch.empty((x.shape[0], length), dtype=x.dtype, device=x.device)
    check(lib().pipe_fft_lines(rb, length, x.shape[1], x.shape[0], direction, _P(x.data_ptr()),
                               _P(out.data_ptr()), _stream_ptr(stream)))
    return out


def _make_fn():
    torch = _torch()

    class PipePoissonFn(torch.autograd.Function):
        """phi = A rho on a GreenPlan; backward applies the adjoint kernel to dL/dphi."""

        @staticmethod
        def forward(ctx, rho, plan):
            ctx.plan = plan
            return plan.solve(rho)

        @staticmethod
        def backward(ctx, grad_phi):
            return ctx.plan.adjoint(grad_phi.contiguous()), None

    return PipePoissonFn


class _Lazy:
    _fn = None

    def __getattr__(self, item):
        if _Lazy._fn is None:
            _Lazy._fn = _make_fn()
        return getattr(_Lazy._fn, item)


PipePoissonFn = _Lazy()
