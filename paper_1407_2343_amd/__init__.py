"""Separable PatchLift non-local means on AMD Instinct MI355X (gfx950).

Thin Python binding of ``libsnlm.so`` (C ABI in ``include/snlm.h``): it only
marshals PyTorch device tensors, streams and parameters into the library.
Every step of the denoiser runs in the library's HIP kernels; there is no CPU
or PyTorch fallback, and importing a call without the built library raises.

    import torch, paper_1407_2343_amd as snlm
    y = snlm.denoise(x_cuda_f32, S=10, K=3, h=200.0, kernel="box", order="row_col")

Method (Ghosh & Chaudhury, "Fast Separable Non-Local Means"): 1D NLM (eq.
1dNLM) along every row and then every column (RC) or the reverse (CR, Sec. 3),
with patch distances (eq. distanceSquared) computed by lifting each offset-s
diagonal and summing it over the patch with running sums (PatchLift, Sec.
2.1-2.2, eq. recursion).
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsnlm.so")

OK, PENDING, EINVAL, ENOMEM, EDEVICE, ENOTICKET, ECLOSED, EBUSY = 0, 1, -1, -2, -3, -4, -5, -6
KERNELS = {"box": 0, "gauss": 1, "gauss_iir": 2}
ORDERS = {"row_col": 0, "col_row": 1}
SUMS = {"block": 0, "kahan": 1, "plain": 2}
DTYPES = {"f32": 0, "f16": 1}
MAX_S, MAX_K = 16, 8


class SnlmError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__("snlm status %d (%s)%s" % (status, strerror(status),
                                                     (": " + detail) if detail else ""))


class Job(ctypes.Structure):
    """Mirror of ``snlm_job`` in include/snlm.h."""
    _fields_ = [
        ("img", ctypes.c_void_p), ("out", ctypes.c_void_p),
        ("H", ctypes.c_int), ("W", ctypes.c_int), ("ld_in", ctypes.c_int), ("ld_out", ctypes.c_int),
        ("dtype", ctypes.c_int), ("S", ctypes.c_int), ("K", ctypes.c_int),
        ("h", ctypes.c_float), ("beta", ctypes.c_float),
        ("kernel", ctypes.c_int), ("order", ctypes.c_int), ("sum", ctypes.c_int),
        ("seg_len", ctypes.c_int),
    ]


_lib = None
_lib_lock = threading.Lock()


def lib():
    """The loaded ``libsnlm.so``; raises if it has not been built."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libsnlm.so is not built (%s); run "
                                   "`python -m paper_1407_2343_amd.build`" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
            jp = ctypes.POINTER(Job)
            L.snlm_create.argtypes = [ctypes.POINTER(vp), i, vp, vp, sz]
            L.snlm_destroy.argtypes = [vp]
            L.snlm_workspace_bytes.argtypes = [i, i, i]
            L.snlm_workspace_bytes.restype = sz
            L.snlm_serving_bytes.argtypes = [i, i, i]
            L.snlm_serving_bytes.restype = sz
            L.snlm_denoise.argtypes = [vp, vp, vp, i, i, i, i, ctypes.c_float, i, i]
            L.snlm_denoise_ex.argtypes = [vp, jp]
            L.snlm_denoise_batch.argtypes = [vp, jp, i]
            L.snlm_enqueue_ex.argtypes = [vp, jp]
            L.snlm_enqueue_static.argtypes = [jp, vp]
            L.snlm_issue_rate.argtypes = [i, i, i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
            L.snlm_enqueue_batch.argtypes = [vp, jp, i]
            L.snlm_submit_many.argtypes = [vp, jp, i, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint64)]
            L.snlm_job_device_ms.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
            L.snlm_serving_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                             ctypes.POINTER(ctypes.c_double)]
            L.snlm_sync.argtypes = [vp]
            L.snlm_submit.argtypes = [vp, jp, ctypes.POINTER(ctypes.c_uint64)]
            L.snlm_poll.argtypes = [vp, ctypes.c_uint64]
            L.snlm_job_times.argtypes = [vp, ctypes.c_uint64] + [ctypes.POINTER(ctypes.c_double)] * 3
            L.snlm_validate.argtypes = [jp, ctypes.POINTER(ctypes.c_char_p)]
            L.snlm_autotune.argtypes = [vp, jp, ctypes.POINTER(i)]
            L.snlm_autotune_batch.argtypes = [vp, jp, i, ctypes.POINTER(i)]
            L.snlm_autotune_batch.restype = ctypes.c_int
            L.snlm_autotune_save.argtypes = [vp, ctypes.c_char_p]
            L.snlm_autotune_load.argtypes = [vp, ctypes.c_char_p]
            L.snlm_plan_seg_len.argtypes = [vp, jp, i]
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            L.snlm_timing.argtypes = [vp, i, dp, ip, dp, ip]
            L.snlm_timing.restype = ctypes.c_int
            L.snlm_denoise_sure.argtypes = [vp, jp, ctypes.c_float, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double)]
            L.snlm_denoise_sure.restype = ctypes.c_int
            L.snlm_sure_workspace_bytes.argtypes = [i, i]
            L.snlm_sure_workspace_bytes.restype = sz
            L.snlm_sure_layout.argtypes = [i, i, ctypes.POINTER(sz)]
            L.snlm_sure_layout.restype = ctypes.c_int
            fp = ctypes.POINTER(ctypes.c_float)
            L.snlm_bilateral.argtypes = [vp, vp, i, vp, i, i, i, ctypes.c_float, ctypes.c_float]
            L.snlm_bilateral.restype = ctypes.c_int
            L.snlm_bilateral_params.argtypes = [ctypes.c_float, fp, fp]
            L.snlm_bilateral_params.restype = None
            L.snlm_denoise_full.argtypes = [vp, jp, ctypes.c_float, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double)]
            L.snlm_denoise_full.restype = ctypes.c_int
            L.snlm_full_workspace_bytes.argtypes = [i, i]
            L.snlm_full_workspace_bytes.restype = sz
            L.snlm_denoise3d.argtypes = [vp, vp, i, i, vp, i, i, i, i, i, i, ctypes.c_float, i,
                                         ctypes.POINTER(ctypes.c_int)]
            L.snlm_denoise3d.restype = ctypes.c_int
            L.snlm_workspace3d_bytes.argtypes = [i, i, i]
            L.snlm_workspace3d_bytes.restype = sz
            L.snlm_strerror.argtypes = [i]
            L.snlm_strerror.restype = ctypes.c_char_p
            L.snlm_last_error.argtypes = [vp]
            L.snlm_last_error.restype = ctypes.c_char_p
            L.snlm_version.restype = ctypes.c_char_p
            for name in ("snlm_create", "snlm_destroy", "snlm_denoise", "snlm_denoise_ex",
                         "snlm_denoise_batch", "snlm_enqueue_ex", "snlm_enqueue_batch",
                         "snlm_submit_many", "snlm_job_device_ms", "snlm_serving_stats", "snlm_sync", "snlm_submit", "snlm_poll",
                         "snlm_job_times", "snlm_validate", "snlm_autotune", "snlm_autotune_save",
                         "snlm_autotune_load", "snlm_plan_seg_len"):
                getattr(L, name).restype = ctypes.c_int
            _lib = L
        return _lib


def strerror(status: int) -> str:
    return lib().snlm_strerror(int(status)).decode()


def version() -> str:
    return lib().snlm_version().decode()


def workspace_bytes(H: int, W: int, dtype: str = "f32") -> int:
    return int(lib().snlm_workspace_bytes(H, W, DTYPES[dtype]))


def sure_workspace_bytes(H: int, W: int) -> int:
    return int(lib().snlm_sure_workspace_bytes(H, W))


def workspace3d_bytes(D: int, H: int, W: int) -> int:
    return int(lib().snlm_workspace3d_bytes(D, H, W))


AXES = {"x": 0, "y": 1, "z": 2}


def full_workspace_bytes(H: int, W: int) -> int:
    return int(lib().snlm_full_workspace_bytes(H, W))


def bilateral_params(sigma: float):
    """(sigma_s, sigma_r) of the paper's bilateral rules for noise level sigma."""
    a, b = ctypes.c_float(), ctypes.c_float()
    lib().snlm_bilateral_params(float(sigma), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def sure_layout(H: int, W: int) -> list:
    """Byte offsets of the SURE workspace regions (see snlm_sure_layout)."""
    off = (ctypes.c_size_t * 8)()
    rc = lib().snlm_sure_layout(H, W, off)
    if rc != OK:
        raise SnlmError(rc, "snlm_sure_layout")
    return list(off)


def make_job(img=0, out=0, H=1, W=1, S=0, K=0, h=1.0, kernel="box", order="row_col",
             sum="block", dtype="f32", beta=0.0, seg_len=0, ld_in=None, ld_out=None) -> Job:
    """A ``snlm_job`` from plain values (pointers as integers)."""
    return Job(img, out, H, W, W if ld_in is None else ld_in, W if ld_out is None else ld_out,
               DTYPES[dtype], S, K, float(h), float(beta or 0.0), KERNELS[kernel], ORDERS[order],
               SUMS[sum], seg_len)


def validate(job: Job) -> tuple[int, str]:
    """Host-side check of a job (no device access): (status, reason)."""
    why = ctypes.c_char_p()
    rc = lib().snlm_validate(ctypes.byref(job), ctypes.byref(why))
    return rc, why.value.decode() if why.value else ""


def _torch():
    import torch
    return torch


def _check_image(x):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dim() != 2:
        raise ValueError("expected a 2D torch tensor")
    if not x.is_cuda:
        raise ValueError("expected a device (cuda/hip) tensor")
    if x.dtype not in (torch.float32, torch.float16):
        raise ValueError("expected float32 or float16")
    if x.stride(1) != 1:
        raise ValueError("rows must be contiguous (stride(1) == 1)")
    return "f16" if x.dtype == torch.float16 else "f32"


class Context:
    """A library context bound to one device, one stream and one arena tensor.

    The arena (a uint8 device tensor) holds the workspaces of direct calls and
    the slots of served jobs; it grows on demand for direct calls, but never
    while served jobs are outstanding (the context would be rebuilt under
    them).  Calls on a Context are stream-ordered (asynchronous) like PyTorch
    ops unless they say otherwise."""

    def __init__(self, arena_bytes: int = 64 << 20, device: int | None = None, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self._ptr = ctypes.c_void_p()
        self.arena = None
        self._tickets = set()
        self._create(max(int(arena_bytes), 256))

    def _create(self, nbytes: int):
        torch = _torch()
        if self._ptr.value:
            self.close()
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda:%d" % self.device)
        rc = lib().snlm_create(ctypes.byref(self._ptr), self.device,
                               ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.c_void_p(self.arena.data_ptr()), nbytes)
        if rc != OK:
            raise SnlmError(rc, "snlm_create")

    def ensure_arena(self, nbytes: int):
        if self.arena is None or self.arena.numel() < nbytes:
            if self._tickets:
                raise SnlmError(EBUSY, "the arena cannot grow while %d served jobs are outstanding"
                                % len(self._tickets))
            self._create(nbytes)

    @property
    def handle(self):
        return self._ptr

    def last_error(self) -> str:
        return lib().snlm_last_error(self._ptr).decode()

    def check(self, rc: int, what: str):
        if rc not in (OK, PENDING):
            raise SnlmError(rc, "%s: %s" % (what, self.last_error()))
        return rc

    def sync(self):
        self.check(lib().snlm_sync(self._ptr), "snlm_sync")

    def close(self):
        if self._ptr.value:
            lib().snlm_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()
            self._tickets = set()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ------------------------------------------------------------
    def job_for(self, x, out, S, K, h, kernel="box", order="row_col", sum="block", beta=None,
                seg_len=0) -> Job:
        dt = _check_image(x)
        H, W = x.shape
        return make_job(x.data_ptr(), out.data_ptr(), H, W, S, K, h, kernel, order, sum, dt,
                        beta or 0.0, seg_len, ld_in=x.stride(0), ld_out=out.stride(0))

    def denoise(self, x, S: int, K: int, h: float, kernel="box", order="row_col", sum="block",
                beta=None, seg_len: int = 0, out=None, sync: bool = False):
        torch = _torch()
        H, W = x.shape
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=x.device)
        self.ensure_arena(workspace_bytes(H, W))
        job = self.job_for(x, out, S, K, h, kernel, order, sum, beta, seg_len)
        self.check(lib().snlm_enqueue_ex(self._ptr, ctypes.byref(job)), "snlm_enqueue_ex")
        if sync:
            self.sync()
        return out

    def denoise_sure(self, x, S: int, K: int, h: float, sigma: float, kernel="box", beta=None,
                     seg_len: int = 0, out=None):
        """SURE-optimal combination of the two orders (Alg. 4).  Returns
        (out, theta, stats); waits for the result."""
        torch = _torch()
        H, W = x.shape
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=x.device)
        self.ensure_arena(sure_workspace_bytes(H, W))
        job = self.job_for(x, out, S, K, h, kernel, "row_col", "block", beta, seg_len)
        theta = (ctypes.c_double * 2)()
        stats = (ctypes.c_double * 7)()
        self.check(lib().snlm_denoise_sure(self._ptr, ctypes.byref(job), float(sigma), theta, stats),
                   "snlm_denoise_sure")
        return out, list(theta), list(stats)

    def bilateral(self, x, sigma_s: float, sigma_r: float, out=None):
        """Bilateral filter of eq. BF on an FP32 device image."""
        torch = _torch()
        H, W = x.shape
        if x.dtype != torch.float32 or x.stride(1) != 1:
            raise ValueError("expected an FP32 image with unit column stride")
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=x.device)
        self.check(lib().snlm_bilateral(self._ptr, ctypes.c_void_p(x.data_ptr()), x.stride(0),
                                        ctypes.c_void_p(out.data_ptr()), out.stride(0), H, W,
                                        float(sigma_s), float(sigma_r)), "snlm_bilateral")
        return out

    def denoise_full(self, x, S: int, K: int, h: float, sigma: float, kernel="box", beta=None,
                     seg_len: int = 0, out=None):
        """SNLM[f]: the SURE combination followed by the bilateral filter with
        the paper's parameter rules.  Returns (out, theta, stats)."""
        torch = _torch()
        H, W = x.shape
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=x.device)
        self.ensure_arena(full_workspace_bytes(H, W))
        job = self.job_for(x, out, S, K, h, kernel, "row_col", "block", beta, seg_len)
        theta = (ctypes.c_double * 2)()
        stats = (ctypes.c_double * 7)()
        self.check(lib().snlm_denoise_full(self._ptr, ctypes.byref(job), float(sigma), theta, stats),
                   "snlm_denoise_full")
        return out, list(theta), list(stats)

    def denoise3d(self, x, S: int, K: int, h: float, kernel="box", axes="xyz", out=None):
        """Separable NLM of a D x H x W volume along the axes in the given order
        (a string over x, y, z; x is the contiguous axis)."""
        torch = _torch()
        if x.dim() != 3 or x.stride(2) != 1 or x.stride(0) != x.shape[1] * x.stride(1):
            raise ValueError("expected a D x H x W volume with contiguous slices")
        dt = {torch.float32: "f32", torch.float16: "f16"}[x.dtype]
        D, H, W = x.shape
        if out is None:
            out = torch.empty((D, H, W), dtype=torch.float32, device=x.device)
        self.ensure_arena(workspace3d_bytes(D, H, W))
        ax = (ctypes.c_int * 3)(*[AXES[a] for a in axes])
        self.check(lib().snlm_denoise3d(self._ptr, ctypes.c_void_p(x.data_ptr()), x.stride(1), DTYPES[dt],
                                        ctypes.c_void_p(out.data_ptr()), out.stride(1), D, H, W, S, K,
                                        float(h), KERNELS[kernel], ax), "snlm_denoise3d")
        return out

    def sure_planes(self, H: int, W: int) -> dict:
        """Views of the SURE workspace after a call: f_cr and the divergences
        of f_rc and f_cr (H x W FP32)."""
        torch = _torch()
        off = sure_layout(H, W)
        Wp = (W + 15) // 16 * 16
        out = {}
        for k, name in ((2, "f_cr"), (3, "d_rc"), (4, "d_cr")):
            plane = self.arena[off[k]:off[k] + H * Wp * 4].view(torch.float32).view(H, Wp)
            out[name] = plane[:, :W]
        return out

    def denoise_job(self, job: Job):
        """Plain launch of a prepared ``Job``, stream-ordered (snlm_enqueue_ex)."""
        self.check(lib().snlm_enqueue_ex(self._ptr, ctypes.byref(job)), "snlm_enqueue_ex")

    def denoise_job_sync(self, job: Job):
        """Plain launch of a prepared ``Job`` that returns with the result in
        place (snlm_denoise_ex)."""
        self.check(lib().snlm_denoise_ex(self._ptr, ctypes.byref(job)), "snlm_denoise_ex")

    def denoise_batch(self, xs, S: int, K: int, hs, kernel="box", order="row_col", beta=None,
                      outs=None, sync: bool = False):
        """One batched launch per kernel class over a list of images; ``hs`` is
        one h per image (or a single float)."""
        torch = _torch()
        if not isinstance(hs, (list, tuple)):
            hs = [hs] * len(xs)
        if outs is None:
            outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in xs]
        need = sum(workspace_bytes(*x.shape) for x in xs)
        self.ensure_arena(need)
        arr = (Job * len(xs))()
        for i, (x, o, h) in enumerate(zip(xs, outs, hs)):
            arr[i] = self.job_for(x, o, S, K, h, kernel, order, "block", beta, 0)
        self.check(lib().snlm_enqueue_batch(self._ptr, arr, len(xs)), "snlm_enqueue_batch")
        if sync:
            self.sync()
        return outs

    def denoise_jobs(self, jobs, sync: bool = False):
        """Batched launch over prepared ``Job`` structures (a list, or a ctypes
        array built once with ``job_array``)."""
        arr = jobs if isinstance(jobs, ctypes.Array) else job_array(jobs)
        self.check(lib().snlm_enqueue_batch(self._ptr, arr, len(arr)), "snlm_enqueue_batch")
        if sync:
            self.sync()

    def denoise_jobs_sync(self, jobs):
        """Batched launch that returns with every result in place (snlm_denoise_batch)."""
        arr = jobs if isinstance(jobs, ctypes.Array) else job_array(jobs)
        self.check(lib().snlm_denoise_batch(self._ptr, arr, len(arr)), "snlm_denoise_batch")

    def autotune(self, x, S, K, h, kernel="box", order="row_col") -> int:
        torch = _torch()
        out = torch.empty(x.shape, dtype=torch.float32, device=x.device)
        self.ensure_arena(workspace_bytes(*x.shape))
        job = self.job_for(x, out, S, K, h, kernel, order)
        best = ctypes.c_int()
        self.check(lib().snlm_autotune(self._ptr, ctypes.byref(job), ctypes.byref(best)),
                   "snlm_autotune")
        return best.value

    def autotune_batch(self, jobs) -> int:
        """Pick the persistent waves per SIMD of batched launches for the classes of these jobs."""
        arr = jobs if isinstance(jobs, ctypes.Array) else job_array(jobs)
        best = ctypes.c_int()
        self.check(lib().snlm_autotune_batch(self._ptr, arr, len(arr), ctypes.byref(best)),
                   "snlm_autotune_batch")
        return best.value

    def plan_seg_len(self, job: Job, pass_: int) -> int:
        return lib().snlm_plan_seg_len(self._ptr, ctypes.byref(job), pass_)

    def save_tuning(self, path: str):
        self.check(lib().snlm_autotune_save(self._ptr, path.encode()), "autotune_save")

    def load_tuning(self, path: str):
        self.check(lib().snlm_autotune_load(self._ptr, path.encode()), "autotune_load")

    def timing_start(self):
        self.check(lib().snlm_timing(self._ptr, 1, None, None, None, None), "snlm_timing")

    def timing_stop(self):
        """(batch_ms, batch_launches, direct_ms, direct_launches) since timing_start."""
        bm, bn, dm, dn = ctypes.c_double(), ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        self.check(lib().snlm_timing(self._ptr, 0, ctypes.byref(bm), ctypes.byref(bn),
                                     ctypes.byref(dm), ctypes.byref(dn)), "snlm_timing")
        return bm.value, bn.value, dm.value, dn.value

    # -- serving ----------------------------------------------------------
    def submit(self, job: Job) -> int:
        t = ctypes.c_uint64()
        self.check(lib().snlm_submit(self._ptr, ctypes.byref(job), ctypes.byref(t)), "snlm_submit")
        self._tickets.add(t.value)
        return t.value

    def submit_many(self, jobs, arrivals_s=None) -> list:
        """Submits prepared jobs from the library's own loop, job i at
        arrivals_s[i] seconds after the call (all at once when None)."""
        arr = jobs if isinstance(jobs, ctypes.Array) else job_array(jobs)
        n = len(arr)
        tickets = (ctypes.c_uint64 * n)()
        at = None
        if arrivals_s is not None:
            at = (ctypes.c_double * n)(*[float(a) * 1e6 for a in arrivals_s])
        rc = lib().snlm_submit_many(self._ptr, arr, n, at, tickets)
        got = [t for t in tickets if t]
        self._tickets.update(got)
        self.check(rc, "snlm_submit_many")
        return list(tickets)

    def poll(self, ticket: int) -> int:
        rc = lib().snlm_poll(self._ptr, ctypes.c_uint64(ticket))
        if rc != PENDING:
            self._tickets.discard(ticket)
        return rc

    def job_device_ms(self, ticket: int) -> float:
        """Device-measured latency of a finished served job (submit event to
        the end of its round), in milliseconds."""
        v = ctypes.c_double()
        rc = lib().snlm_job_device_ms(self._ptr, ctypes.c_uint64(ticket), ctypes.byref(v))
        if rc != OK:
            raise SnlmError(rc, "snlm_job_device_ms")
        return v.value

    def serving_stats(self):
        """(rounds, jobs, scheduler host microseconds) since creation."""
        r, j, us = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_double(0.0)
        self.check(lib().snlm_serving_stats(self._ptr, ctypes.byref(r), ctypes.byref(j), ctypes.byref(us)),
                   "snlm_serving_stats")
        return int(r.value), int(j.value), float(us.value)

    def job_times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().snlm_job_times(self._ptr, ctypes.c_uint64(ticket), ctypes.byref(a),
                                  ctypes.byref(b), ctypes.byref(c))
        if rc != OK:
            raise SnlmError(rc, "snlm_job_times")
        return a.value, b.value, c.value


def job_array(jobs):
    """A ctypes array of ``Job`` for repeated batched launches."""
    return (Job * len(jobs))(*jobs)


_default_ctx = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def denoise(x, S: int, K: int, h: float, kernel: str = "box", order: str = "row_col",
            sum: str = "block", beta=None, seg_len: int = 0, out=None):
    """Separable NLM of a 2D float32/float16 device tensor; returns float32.
    Ordered on the current stream like any PyTorch op."""
    return default_context().denoise(x, S, K, h, kernel, order, sum, beta, seg_len, out)


def enqueue_static(job: Job, stream=None) -> int:
    """``snlm_enqueue_static``: both passes of one job on ``stream`` (a
    torch.cuda.Stream, or the current stream) with the intermediate in the
    library's static device array; no context, no allocation.  Returns the
    status code."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    return lib().snlm_enqueue_static(ctypes.byref(job), ctypes.c_void_p(st.cuda_stream))


def issue_rate(mode: int, waves_per_simd: int, iters: int = 4000):
    """``snlm_issue_rate``: (clock cycles per pair body per SIMD, shader
    clock lower bound in GHz) on the current device."""
    clk, ghz = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().snlm_issue_rate(mode, waves_per_simd, iters, ctypes.byref(clk), ctypes.byref(ghz))
    if rc != OK:
        raise SnlmError(rc, "snlm_issue_rate")
    return clk.value, ghz.value


def denoise_batch(xs, S: int, K: int, hs, kernel: str = "box", order: str = "row_col", beta=None):
    return default_context().denoise_batch(xs, S, K, hs, kernel, order, beta)


def h_from_sigma(sigma: float, factor: float = 10.0) -> float:
    """The classic h = 10 sigma rule used by the benchmark workloads."""
    return factor * sigma


__all__ = ["Context", "Job", "SnlmError", "denoise", "denoise_batch", "default_context", "lib",
           "make_job", "validate", "workspace_bytes", "strerror", "version", "h_from_sigma",
           "MAX_S", "MAX_K"]
