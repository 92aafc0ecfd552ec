"""ctypes binding of ``libpm.so`` (the C ABI declared in ``include/pm.h``).

Argument marshalling only: each function has the name of its C entry point,
takes torch tensors for device arrays (``torch.int64`` or ``torch.uint64``,
contiguous, on a HIP device) and Python integers or sequences for host values,
and raises ``PMError`` when the library returns an error code. Every step of
the computation runs in the library's HIP kernels; there is no fallback: if
``libpm.so`` is missing or cannot be loaded, calls raise.

Streams: ``stream=None`` uses torch's current stream on the tensor's device.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpm.so")

PM_OK, PM_EINVAL, PM_EUNSUPPORTED, PM_ENOMEM, PM_EHIP = 0, -1, -2, -3, -4
OP_NTT_FWD, OP_NTT_INV, OP_POLYMUL = 0, 1, 2

_lock = threading.Lock()
_lib = None


class ProbeEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("lane_ops_per_s", ctypes.c_double)]


class ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


class Job(ctypes.Structure):
    """pm_job: `count` pairs sharing N = 2^log2n and q (device pointers)."""
    _fields_ = [("log2n", ctypes.c_uint32), ("count", ctypes.c_uint32), ("q", ctypes.c_uint64),
                ("psi_br", ctypes.c_void_p), ("psi_inv_br", ctypes.c_void_p),
                ("a", ctypes.c_void_p), ("b", ctypes.c_void_p), ("c", ctypes.c_void_p)]


class PMError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__("%s failed (%d): %s" % (func, code, msg))
        self.code = code


def load():
    """Load libpm.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        import torch  # noqa: F401  (loads libamdhip64 first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpm.so is not built; run: python -m paper_2209_01290_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, u64, sz, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        sig = {
            "pm_last_error": (ctypes.c_char_p, []),
            "pm_barrett_mulmod": (i32, [vp, vp, vp, sz, u64, vp]),
            "pm_ntt_fwd": (i32, [vp, sz, sz, sz, u64p, vp, vp]),
            "pm_ntt_inv": (i32, [vp, sz, sz, sz, u64p, vp, vp]),
            "pm_polymul": (i32, [vp, vp, vp, sz, sz, sz, u64p, vp, vp, vp, vp]),
            "pm_polymul_workspace_bytes": (sz, [sz, sz, sz]),
            "pm_polymul_noalloc": (i32, [vp, vp, vp, sz, sz, sz, u64p, vp, vp, vp]),
            "pm_polymul_fused": (i32, [vp, vp, vp, sz, sz, sz, u64p, vp, vp, vp, vp]),
            "pm_polymul_stagewise": (i32, [vp, vp, vp, sz, sz, sz, u64p, vp, vp, vp, vp]),
            "pm_polymul_stagewise_workspace_bytes": (sz, [sz, sz, sz]),
            "pm_tune_set": (i32, [i32, ctypes.c_uint, ctypes.c_uint]),
            "pm_tune_get": (i32, [i32, ctypes.c_uint]),
            "pm_tune_set_small": (i32, [i32, ctypes.c_uint, ctypes.c_uint, ctypes.c_uint]),
            "pm_tune_get_small": (i32, [i32, ctypes.c_uint, ctypes.POINTER(ctypes.c_uint),
                                        ctypes.POINTER(ctypes.c_uint)]),
            "pm_tune_set_small_batch": (i32, [sz]),
            "pm_tune_get_small_batch": (sz, []),
            "pm_tune_set_small_limit": (i32, [i32, ctypes.c_uint, sz]),
            "pm_tune_get_small_limit": (sz, [i32, ctypes.c_uint]),
            "pm_tune_set_pipeline": (i32, [i32]),
            "pm_tune_get_pipeline": (i32, []),
            "pm_tune_set_pipeline_rows": (i32, [ctypes.c_uint, sz]),
            "pm_tune_get_pipeline_rows": (sz, [ctypes.c_uint]),
            "pm_tune_set_jobs_pipeline": (i32, [i32]),
            "pm_tune_get_jobs_pipeline": (i32, []),
            "pm_ntt_primes": (sz, [u64, ctypes.c_uint, sz, u64p]),
            "pm_find_psi": (u64, [u64, sz]),
            "pm_make_tables": (i32, [u64, sz, u64, u64p, u64p]),
            "pm_prof_enable": (i32, [i32]),
            "pm_polymul_jobs_workspace_bytes": (sz, [ctypes.POINTER(Job), sz]),
            "pm_polymul_jobs": (i32, [ctypes.POINTER(Job), sz, vp, sz, vp]),
            "pm_plan_create": (i32, [ctypes.POINTER(vp), ctypes.POINTER(Job), sz, ctypes.c_uint]),
            "pm_plan_launch": (i32, [vp, vp]),
            "pm_plan_destroy": (i32, [vp]),
            "pm_plan_device_bytes": (sz, [vp]),
            "pm_reduce_apply": (i32, [i32, ctypes.c_uint, vp, vp, vp, vp, sz, u64, vp]),
            "pm_reduce_chain": (i32, [i32, ctypes.c_uint, vp, sz, u64, i32, u64, vp]),
            "pm_prof_read": (i32, [ctypes.POINTER(ProfEntry), sz, ctypes.POINTER(sz), i32]),
            "pm_probe_valu": (i32, [ctypes.POINTER(ProbeEntry), sz, ctypes.POINTER(sz),
                                    ctypes.POINTER(ctypes.c_double)]),
            "pm_ntt_fwd_il": (i32, [vp, sz, sz, sz, u64p, vp, vp]),
            "pm_ntt_inv_il": (i32, [vp, sz, sz, sz, u64p, vp, vp]),
            "pm_polymul_il": (i32, [vp, vp, vp, sz, sz, sz, u64p, vp, vp, vp, vp]),
            "pm_polymul_il_workspace_bytes": (sz, [sz, sz, sz]),
            "pm_ntt_fwd_u32": (i32, [vp, sz, sz, sz, u32p, vp, vp]),
            "pm_ntt_inv_u32": (i32, [vp, sz, sz, sz, u32p, vp, vp]),
            "pm_polymul_u32": (i32, [vp, vp, vp, sz, sz, sz, u32p, vp, vp, vp, vp]),
            "pm_polymul_fused_u32": (i32, [vp, vp, vp, sz, sz, sz, u32p, vp, vp, vp, vp]),
            "pm_polymul_u32_workspace_bytes": (sz, [sz, sz, sz]),
            "pm_make_tables_u32": (i32, [ctypes.c_uint32, sz, ctypes.c_uint32, u32p, u32p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def exported_symbols():
    """Names of the C entry points this binding declares."""
    return ["pm_last_error", "pm_barrett_mulmod", "pm_ntt_fwd", "pm_ntt_inv", "pm_polymul", "pm_polymul_fused",
            "pm_polymul_workspace_bytes", "pm_polymul_noalloc", "pm_polymul_stagewise",
            "pm_polymul_stagewise_workspace_bytes", "pm_tune_set", "pm_tune_get",
            "pm_ntt_primes", "pm_find_psi", "pm_make_tables", "pm_prof_enable", "pm_prof_read", "pm_probe_valu",
            "pm_polymul_jobs_workspace_bytes", "pm_polymul_jobs", "pm_plan_create", "pm_plan_launch",
            "pm_plan_destroy", "pm_plan_device_bytes", "pm_reduce_apply", "pm_reduce_chain",
            "pm_ntt_fwd_u32", "pm_ntt_inv_u32", "pm_polymul_u32", "pm_polymul_fused_u32",
            "pm_polymul_u32_workspace_bytes",
            "pm_make_tables_u32", "pm_ntt_fwd_il", "pm_ntt_inv_il", "pm_polymul_il",
            "pm_polymul_il_workspace_bytes", "pm_tune_set_small", "pm_tune_get_small",
            "pm_tune_set_small_batch", "pm_tune_get_small_batch", "pm_tune_set_small_limit",
            "pm_tune_get_small_limit", "pm_tune_set_pipeline", "pm_tune_get_pipeline",
            "pm_tune_set_pipeline_rows", "pm_tune_get_pipeline_rows", "pm_tune_set_jobs_pipeline",
            "pm_tune_get_jobs_pipeline"]


def _check(rc: int, func: str):
    if rc != PM_OK:
        raise PMError(rc, func, load().pm_last_error().decode())


def _dptr(t, name):
    """Device pointer of a contiguous 64-bit tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on a HIP device" % name)
    if t.element_size() != 8 or t.dtype.is_floating_point:
        raise TypeError("%s must be int64 or uint64" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _dptr32(t, name):
    """Device pointer of a contiguous 32-bit integer tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must live on a HIP device" % name)
    if t.element_size() != 4 or t.dtype.is_floating_point:
        raise TypeError("%s must be int32 or uint32" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _wptr(t):
    """Device pointer of a workspace tensor of any integer type (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("workspace must be a contiguous tensor on a HIP device")
    return t.data_ptr()


def _stream(stream, like=None):
    import torch
    if stream is None:
        dev = like.device if like is not None else None
        return torch.cuda.current_stream(dev).cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _qarr(q, limbs):
    qs = [int(x) for x in (q if hasattr(q, "__len__") else [q])]
    if len(qs) != limbs:
        raise ValueError("need %d moduli, got %d" % (limbs, len(qs)))
    return (ctypes.c_uint64 * limbs)(*qs)


def _qarr32(q, limbs):
    qs = [int(x) for x in (q if hasattr(q, "__len__") else [q])]
    if len(qs) != limbs:
        raise ValueError("need %d moduli, got %d" % (limbs, len(qs)))
    if any(x < 0 or x >= 1 << 32 for x in qs):
        raise ValueError("32-bit moduli expected")
    return (ctypes.c_uint32 * limbs)(*qs)


# ------------------------------------------------------------ entry points --

def pm_barrett_mulmod(a, b, c, q, n=None, stream=None):
    n = a.numel() if n is None else n
    _check(load().pm_barrett_mulmod(_dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"), n, int(q),
                                    _stream(stream, a)), "pm_barrett_mulmod")


def pm_ntt_fwd(x, N, limbs, polys_per_limb, q, psi_br, stream=None):
    _check(load().pm_ntt_fwd(_dptr(x, "x"), N, limbs, polys_per_limb, _qarr(q, limbs),
                             _dptr(psi_br, "psi_br"), _stream(stream, x)), "pm_ntt_fwd")


def pm_ntt_inv(x, N, limbs, polys_per_limb, q, psi_inv_br, stream=None):
    _check(load().pm_ntt_inv(_dptr(x, "x"), N, limbs, polys_per_limb, _qarr(q, limbs),
                             _dptr(psi_inv_br, "psi_inv_br"), _stream(stream, x)), "pm_ntt_inv")


def pm_polymul_workspace_bytes(N, limbs, polys_per_limb):
    return int(load().pm_polymul_workspace_bytes(N, limbs, polys_per_limb))


def pm_polymul_stagewise_workspace_bytes(N, limbs, polys_per_limb):
    return int(load().pm_polymul_stagewise_workspace_bytes(N, limbs, polys_per_limb))


def pm_polymul(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace=None, stream=None):
    _check(load().pm_polymul(_dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"), N, limbs, polys_per_limb,
                             _qarr(q, limbs), _dptr(psi_br, "psi_br"), _dptr(psi_inv_br, "psi_inv_br"),
                             _dptr(workspace, "workspace"), _stream(stream, a)), "pm_polymul")


def pm_polymul_noalloc(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, stream=None):
    """pm_polymul with its workspace in the library's fixed per-GPU scratch array (no allocation)."""
    _check(load().pm_polymul_noalloc(_dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"), N, limbs, polys_per_limb,
                                     _qarr(q, limbs), _dptr(psi_br, "psi_br"), _dptr(psi_inv_br, "psi_inv_br"),
                                     _stream(stream, a)), "pm_polymul_noalloc")


PM_NOALLOC_SCRATCH_BYTES = 64 << 20


def pm_polymul_fused(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace=None, stream=None):
    _check(load().pm_polymul_fused(_dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"), N, limbs, polys_per_limb,
                                   _qarr(q, limbs), _dptr(psi_br, "psi_br"), _dptr(psi_inv_br, "psi_inv_br"),
                                   _dptr(workspace, "workspace"), _stream(stream, a)), "pm_polymul_fused")


def pm_polymul_stagewise(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace=None,
                         stream=None):
    _check(load().pm_polymul_stagewise(_dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"), N, limbs,
                                       polys_per_limb, _qarr(q, limbs), _dptr(psi_br, "psi_br"),
                                       _dptr(psi_inv_br, "psi_inv_br"), _dptr(workspace, "workspace"),
                                       _stream(stream, a)), "pm_polymul_stagewise")


def pm_ntt_fwd_il(x, N, limbs, polys_per_limb, q, psi_br, stream=None):
    """Forward transform of a coefficient-major batch x[limb][N][polys_per_limb]."""
    _check(load().pm_ntt_fwd_il(_dptr(x, "x"), N, limbs, polys_per_limb, _qarr(q, limbs),
                                _dptr(psi_br, "psi_br"), _stream(stream, x)), "pm_ntt_fwd_il")


def pm_ntt_inv_il(x, N, limbs, polys_per_limb, q, psi_inv_br, stream=None):
    _check(load().pm_ntt_inv_il(_dptr(x, "x"), N, limbs, polys_per_limb, _qarr(q, limbs),
                                _dptr(psi_inv_br, "psi_inv_br"), _stream(stream, x)), "pm_ntt_inv_il")


def pm_polymul_il_workspace_bytes(N, limbs, polys_per_limb):
    return int(load().pm_polymul_il_workspace_bytes(N, limbs, polys_per_limb))


def pm_polymul_il(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace=None, stream=None):
    _check(load().pm_polymul_il(_dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"), N, limbs, polys_per_limb,
                                _qarr(q, limbs), _dptr(psi_br, "psi_br"), _dptr(psi_inv_br, "psi_inv_br"),
                                _wptr(workspace), _stream(stream, a)), "pm_polymul_il")


def pm_ntt_fwd_u32(x, N, limbs, polys_per_limb, q, psi_br, stream=None):
    _check(load().pm_ntt_fwd_u32(_dptr32(x, "x"), N, limbs, polys_per_limb, _qarr32(q, limbs),
                                 _dptr32(psi_br, "psi_br"), _stream(stream, x)), "pm_ntt_fwd_u32")


def pm_ntt_inv_u32(x, N, limbs, polys_per_limb, q, psi_inv_br, stream=None):
    _check(load().pm_ntt_inv_u32(_dptr32(x, "x"), N, limbs, polys_per_limb, _qarr32(q, limbs),
                                 _dptr32(psi_inv_br, "psi_inv_br"), _stream(stream, x)), "pm_ntt_inv_u32")


def pm_polymul_u32_workspace_bytes(N, limbs, polys_per_limb):
    return int(load().pm_polymul_u32_workspace_bytes(N, limbs, polys_per_limb))


def pm_polymul_u32(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace=None, stream=None):
    _check(load().pm_polymul_u32(_dptr32(a, "a"), _dptr32(b, "b"), _dptr32(c, "c"), N, limbs, polys_per_limb,
                                 _qarr32(q, limbs), _dptr32(psi_br, "psi_br"), _dptr32(psi_inv_br, "psi_inv_br"),
                                 _wptr(workspace), _stream(stream, a)), "pm_polymul_u32")


PM_PLAN_NO_GRAPH = 1


def make_job(log2n, count, q, psi_br, psi_inv_br, a, b, c):
    """A pm_job from tensors (device pointers are taken, the tensors must outlive its use)."""
    return Job(log2n, count, int(q), _dptr(psi_br, "psi_br"), _dptr(psi_inv_br, "psi_inv_br"),
               _dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"))


def _jobarr(jobs):
    arr = (Job * len(jobs))(*jobs)
    return arr, len(jobs)


def pm_polymul_jobs_workspace_bytes(jobs):
    arr, n = _jobarr(jobs)
    return int(load().pm_polymul_jobs_workspace_bytes(arr, n))


def pm_polymul_jobs(jobs, workspace, stream=None):
    arr, n = _jobarr(jobs)
    _check(load().pm_polymul_jobs(arr, n, _dptr(workspace, "workspace"),
                                  workspace.numel() * workspace.element_size(), _stream(stream, workspace)),
           "pm_polymul_jobs")


def pm_polymul_jobs_workspace_bytes_raw(jobs_ptr, njobs):
    """As pm_polymul_jobs_workspace_bytes, for a host array of pm_job records at jobs_ptr."""
    return int(load().pm_polymul_jobs_workspace_bytes(ctypes.cast(jobs_ptr, ctypes.POINTER(Job)), njobs))


def pm_polymul_raw(a_ptr, b_ptr, c_ptr, N, limbs, polys_per_limb, q_arr, psi_br_ptr, psi_inv_br_ptr,
                   workspace_ptr, stream):
    """As pm_polymul, for raw device pointers, a ctypes uint64 array of at
    least `limbs` moduli and a raw stream handle (no tensor checks)."""
    _check(load().pm_polymul(a_ptr, b_ptr, c_ptr, N, limbs, polys_per_limb, q_arr, psi_br_ptr, psi_inv_br_ptr,
                             workspace_ptr, stream), "pm_polymul")


def pm_polymul_jobs_raw(jobs_ptr, njobs, workspace_ptr, workspace_bytes, stream):
    """As pm_polymul_jobs, for a host array of pm_job records at jobs_ptr and raw
    device / stream handles."""
    _check(load().pm_polymul_jobs(ctypes.cast(jobs_ptr, ctypes.POINTER(Job)), njobs, workspace_ptr,
                                  workspace_bytes, stream), "pm_polymul_jobs")


def pm_plan_create(jobs, flags=0):
    """Returns an opaque plan handle (int); free it with pm_plan_destroy."""
    arr, n = _jobarr(jobs)
    h = ctypes.c_void_p()
    _check(load().pm_plan_create(ctypes.byref(h), arr, n, flags), "pm_plan_create")
    return h.value


def pm_plan_launch(plan, stream=None):
    _check(load().pm_plan_launch(plan, _stream(stream)), "pm_plan_launch")


def pm_plan_destroy(plan):
    _check(load().pm_plan_destroy(plan), "pm_plan_destroy")


def pm_plan_device_bytes(plan):
    return int(load().pm_plan_device_bytes(plan))


def pm_reduce_apply(variant, word_bits, a, b, c, hist, q, n=None, stream=None):
    """Barrett variant study: c = a*b mod q by variant (0 = %, 2, 3, 4 = Alg. number);
    hist (int32/uint32 device tensor, 3 per 256 indices) receives correction counts."""
    n = a.numel() if n is None else n
    if hist.element_size() != 4 or not hist.is_cuda or not hist.is_contiguous():
        raise TypeError("hist must be a contiguous 32-bit device tensor")
    _check(load().pm_reduce_apply(variant, word_bits, _dptr(a, "a"), _dptr(b, "b"), _dptr(c, "c"),
                                  hist.data_ptr(), n, int(q), _stream(stream, a)), "pm_reduce_apply")


def pm_reduce_chain(variant, word_bits, out, y, iters, q, stream=None):
    _check(load().pm_reduce_chain(variant, word_bits, _dptr(out, "out"), out.numel(), int(y), iters, int(q),
                                  _stream(stream, out)), "pm_reduce_chain")


def pm_tune_set(op, log2n, logc):
    _check(load().pm_tune_set(op, log2n, logc), "pm_tune_set")


def pm_tune_get(op, log2n):
    r = load().pm_tune_get(op, log2n)
    if r < 0:
        _check(r, "pm_tune_get")
    return r


def pm_tune_set_small(op, log2n, logc, words_per_thread):
    _check(load().pm_tune_set_small(op, log2n, logc, words_per_thread), "pm_tune_set_small")


def pm_tune_get_small(op, log2n):
    """(logc, words_per_thread) of the small-batch plan, (0, 0) if none."""
    lc, wpt = ctypes.c_uint(), ctypes.c_uint()
    _check(load().pm_tune_get_small(op, log2n, ctypes.byref(lc), ctypes.byref(wpt)), "pm_tune_get_small")
    return lc.value, wpt.value


def pm_tune_set_small_batch(max_words):
    _check(load().pm_tune_set_small_batch(max_words), "pm_tune_set_small_batch")


def pm_tune_get_small_batch():
    return int(load().pm_tune_get_small_batch())


def pm_tune_set_small_limit(op, log2n, max_words):
    """Batch limit (words) of the small-batch plan of (op, N); 0 = the global threshold."""
    _check(load().pm_tune_set_small_limit(op, log2n, max_words), "pm_tune_set_small_limit")


def pm_tune_get_small_limit(op, log2n):
    return int(load().pm_tune_get_small_limit(op, log2n))


def pm_tune_set_pipeline(chunks):
    """Limb chunks of the software-pipelined product: -1 = built-in choice,
    0 or 1 = off, G >= 2 = G chunks."""
    _check(load().pm_tune_set_pipeline(int(chunks)), "pm_tune_set_pipeline")


def pm_tune_set_pipeline_rows(logr, min_rows):
    """Rows of 2^12 words from which the default pipelines a product with column
    radix 2^logr (3..5); 0 = built-in value."""
    _check(load().pm_tune_set_pipeline_rows(int(logr), int(min_rows)), "pm_tune_set_pipeline_rows")


def pm_tune_get_pipeline_rows(logr):
    return int(load().pm_tune_get_pipeline_rows(int(logr)))


def pm_tune_set_jobs_pipeline(chunks):
    """Chunks of the software-pipelined job tables: -1 automatic, 0 off, G >= 2 forced."""
    _check(load().pm_tune_set_jobs_pipeline(int(chunks)), "pm_tune_set_jobs_pipeline")


def pm_tune_get_jobs_pipeline():
    return int(load().pm_tune_get_jobs_pipeline())


def pm_tune_get_pipeline():
    return int(load().pm_tune_get_pipeline())


def apply_tune_db(path=None):
    """Install the pass plans of an autotuner database (see tune.py; default:
    $PM_TUNE_DB, else the packaged MI355X database): the
    throughput plans ("choices") and, if present, the small-batch plans
    ("small": {"max_words": W, "choices": {op: {log2n: [logc, words_per_thread]}},
    "limits": {op: {log2n: words}}}, the limits replacing W for their (op, N))
    and the pipelining thresholds ("pipeline": {"min_rows": {logr: rows}});
    returns the number of entries applied, 0 if the file does not exist."""
    import json
    if path is None:
        path = os.environ.get("PM_TUNE_DB") or os.path.join(PKG, "tune_db", "gfx950.json")
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        db = json.load(f)
    ops = {"polymul": OP_POLYMUL, "ntt_fwd": OP_NTT_FWD, "ntt_inv": OP_NTT_INV}
    n = 0
    for name, table in db.get("choices", {}).items():
        for log2n, logc in table.items():
            pm_tune_set(ops[name], int(log2n), int(logc))
            n += 1
    small = db.get("small")
    if small:
        for name, table in small.get("choices", {}).items():
            for log2n, (logc, wpt) in table.items():
                pm_tune_set_small(ops[name], int(log2n), int(logc), int(wpt))
                n += 1
        for name, table in small.get("limits", {}).items():
            for log2n, words in table.items():
                pm_tune_set_small_limit(ops[name], int(log2n), int(words))
                n += 1
        pm_tune_set_small_batch(int(small["max_words"]))
    pipe = db.get("pipeline")
    if pipe:
        for logr, rows in pipe.get("min_rows", {}).items():
            pm_tune_set_pipeline_rows(int(logr), int(rows))
            n += 1
    return n


def pm_prof_enable(on=True):
    _check(load().pm_prof_enable(1 if on else 0), "pm_prof_enable")


def pm_prof_read(reset=True):
    """{kernel name: (launches, total_ms)} for launches timed since the last reset."""
    lib = load()
    cap = 64
    buf = (ProfEntry * cap)()
    n = ctypes.c_size_t(0)
    _check(lib.pm_prof_read(buf, cap, ctypes.byref(n), 1 if reset else 0), "pm_prof_read")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
            for i in range(min(n.value, cap))}


def pm_probe_valu():
    """({instruction: lane-ops/s}, shader clock MHz under load) on the current device."""
    lib = load()
    cap = 16
    buf = (ProbeEntry * cap)()
    n = ctypes.c_size_t(0)
    mhz = ctypes.c_double(0)
    _check(lib.pm_probe_valu(buf, cap, ctypes.byref(n), ctypes.byref(mhz)), "pm_probe_valu")
    return {buf[i].name.decode(): float(buf[i].lane_ops_per_s) for i in range(min(n.value, cap))}, mhz.value


def pm_ntt_primes(N, count, bits=60):
    out = (ctypes.c_uint64 * count)()
    got = load().pm_ntt_primes(2 * N, bits, count, out)
    return [int(out[i]) for i in range(got)]


def pm_find_psi(q, N):
    return int(load().pm_find_psi(q, N))


def pm_make_tables(q, N, psi=None):
    """(psi_br, psi_inv_br) as numpy uint64 arrays of N words."""
    if psi is None:
        psi = pm_find_psi(q, N)
    fwd = np.empty(N, dtype=np.uint64)
    inv = np.empty(N, dtype=np.uint64)
    p = ctypes.POINTER(ctypes.c_uint64)
    _check(load().pm_make_tables(q, N, psi, fwd.ctypes.data_as(p), inv.ctypes.data_as(p)),
           "pm_make_tables")
    return fwd, inv


def pm_polymul_fused_u32(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace=None, stream=None):
    _check(load().pm_polymul_fused_u32(_dptr32(a, "a"), _dptr32(b, "b"), _dptr32(c, "c"), N, limbs, polys_per_limb,
                                       _qarr32(q, limbs), _dptr32(psi_br, "psi_br"),
                                       _dptr32(psi_inv_br, "psi_inv_br"), _wptr(workspace), _stream(stream, a)),
           "pm_polymul_fused_u32")


def pm_make_tables_u32(q, N, psi=None):
    """(psi_br, psi_inv_br) as numpy uint32 arrays of N words (q < 2^30)."""
    if psi is None:
        psi = pm_find_psi(q, N)
    fwd = np.empty(N, dtype=np.uint32)
    inv = np.empty(N, dtype=np.uint32)
    p = ctypes.POINTER(ctypes.c_uint32)
    _check(load().pm_make_tables_u32(q, N, psi, fwd.ctypes.data_as(p), inv.ctypes.data_as(p)),
           "pm_make_tables_u32")
    return fwd, inv


# ------------------------------------------------------------- helpers ----

def to_device(arr: np.ndarray, device="cuda"):
    """numpy uint64 -> torch int64 tensor on the device (same bits)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint64).view(np.int64)).to(device)


def to_host(t) -> np.ndarray:
    """torch 64-bit tensor -> numpy uint64 (same bits)."""
    return t.detach().to("cpu").contiguous().numpy().view(np.uint64)


def to_device32(arr: np.ndarray, device="cuda"):
    """numpy array of values < 2^31 -> torch int32 tensor on the device."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint32).view(np.int32)).to(device)


def to_host32(t) -> np.ndarray:
    """torch 32-bit tensor -> numpy uint32 (same bits)."""
    return t.detach().to("cpu").contiguous().numpy().view(np.uint32)


class Params:
    """Moduli and device-resident twiddle tables for `limbs` limbs of size N.

    Limb l uses the l-th largest prime q < 2^bits with q = 1 mod 2N (the
    library's own generator) and psi from pm_find_psi."""

    def __init__(self, N, limbs, bits=60, device="cuda", primes=None):
        self.N, self.limbs = N, limbs
        self.q = list(primes) if primes is not None else pm_ntt_primes(N, limbs, bits)
        if len(self.q) != limbs:
            raise ValueError("not enough primes")
        fw = np.empty((limbs, N), dtype=np.uint64)
        iv = np.empty((limbs, N), dtype=np.uint64)
        for l, q in enumerate(self.q):
            fw[l], iv[l] = pm_make_tables(q, N)
        self.psi_br_host, self.psi_inv_br_host = fw, iv
        self.psi_br = to_device(fw, device)
        self.psi_inv_br = to_device(iv, device)


class Params32:
    """Moduli (< 2^30) and device-resident 32-bit twiddle tables for `limbs`
    limbs of size N: the l-th largest prime q < 2^bits with q = 1 mod 2N."""

    def __init__(self, N, limbs, bits=30, device="cuda", primes=None):
        if bits > 30:
            raise ValueError("32-bit words take moduli of at most 30 bits")
        self.N, self.limbs = N, limbs
        self.q = list(primes) if primes is not None else pm_ntt_primes(N, limbs, bits)
        if len(self.q) != limbs:
            raise ValueError("not enough primes")
        fw = np.empty((limbs, N), dtype=np.uint32)
        iv = np.empty((limbs, N), dtype=np.uint32)
        for l, q in enumerate(self.q):
            fw[l], iv[l] = pm_make_tables_u32(q, N)
        self.psi_br_host, self.psi_inv_br_host = fw, iv
        self.psi_br = to_device32(fw, device)
        self.psi_inv_br = to_device32(iv, device)
