"""Python API over libsp.so: contexts, barriers, mutexes, semaphores, microbenchmarks.

Thin wrappers: they allocate output tensors with torch (device memory), pass raw
pointers and torch's current HIP stream to the C ABI, and convert statistics.  Every
primitive runs in the library's kernels; nothing here computes a result.
"""

from __future__ import annotations

import ctypes

import torch

from . import _native as N
from ._native import check, lib


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA (HIP) tensor")
    return ctypes.c_void_p(t.data_ptr())


def _u32(t: torch.Tensor) -> torch.Tensor:
    """View an int32 tensor's bits as uint32 values in an int64 CPU tensor."""
    return t.cpu().to(torch.int64) & 0xFFFFFFFF


def make_params(**kw) -> N.Params:
    p = N.Params()
    lib.sp_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "backoff" and isinstance(v, str):
            v = N.BACKOFF[v]
        if k == "backoff_unit" and isinstance(v, str):
            v = N.BACKOFF_UNIT[v]
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, int(v))
    return p


class Context:
    """A libsp context bound to one HIP device (torch's current device by default)."""

    def __init__(self, device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: libsp needs an MI355X (gfx950) GPU")
        self.device = torch.cuda.current_device() if device is None else device
        torch.cuda.set_device(self.device)
        torch.cuda.init()
        h = ctypes.c_void_p()
        check(lib.sp_init(self.device, ctypes.byref(h)), "sp_init")
        self.h = h
        info = N.DeviceInfo()
        check(lib.sp_device_info_get(self.h, ctypes.byref(info)), "sp_device_info_get", self.h)
        self.info = {
            "name": info.name.decode(), "arch": info.arch.decode(), "cu_count": info.cu_count,
            "xcd_count": info.xcd_count, "wall_clock_khz": info.wall_clock_khz,
            "clock_khz": info.clock_khz, "hbm_bytes": info.hbm_bytes,
            "max_threads_per_cu": info.max_threads_per_cu,
        }

    def close(self):
        if self.h:
            lib.sp_fini(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_default(self, primitive: str, bucket: int, kind: str, **params):
        prim = {"barrier": 0, "mutex": 1, "semaphore": 2}[primitive]
        kinds = [N.BARRIER_KINDS, N.MUTEX_KINDS, N.SEM_KINDS][prim]
        p = make_params(**params)
        check(lib.sp_set_default(self.h, prim, bucket, kinds[kind], ctypes.byref(p)),
              "sp_set_default", self.h)

    def probe_xcc(self, nwg: int, lanes: int = 64) -> torch.Tensor:
        out = torch.zeros(nwg, dtype=torch.int32, device="cuda")
        check(lib.sp_probe_xcc(self.h, nwg, lanes, _ptr(out), _stream()), "sp_probe_xcc", self.h)
        return out.cpu()


class Barrier:
    """Global barrier among `nwg` co-resident workgroups (Section 5, Barrier)."""

    def __init__(self, ctx: Context, kind: str, nwg: int, **params):
        self.ctx, self.kind, self.nwg = ctx, kind, nwg
        p = make_params(**params)
        h = ctypes.c_void_p()
        check(lib.sp_barrier_create(ctx.h, N.BARRIER_KINDS[kind], nwg, ctypes.byref(p),
                                    ctypes.byref(h)), "sp_barrier_create", ctx.h)
        self.h = h

    def run_hash(self, lanes: int, rounds: int, seed: int, out: torch.Tensor | None = None):
        """Hash-exchange workload; returns (checksums uint32 as int64 CPU tensor, stats)."""
        if out is None:
            out = torch.zeros(self.nwg, dtype=torch.int32, device="cuda")
        st = N.Stats()
        check(lib.sp_barrier_run_hash(self.h, lanes, rounds, seed & 0xFFFFFFFF, _ptr(out),
                                      ctypes.byref(st), _stream()), "sp_barrier_run_hash", self.ctx.h)
        return _u32(out), st.as_dict()

    def close(self):
        if self.h:
            lib.sp_barrier_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def barrier_hash_launches(ctx: Context, nwg: int, lanes: int, rounds: int, seed: int,
                          graph: bool = False):
    """Kernel-boundary comparator of the hash exchange (one launch per round)."""
    slots = torch.zeros(2 * nwg, dtype=torch.int32, device="cuda")
    out = torch.zeros(nwg, dtype=torch.int32, device="cuda")
    st = N.Stats()
    check(lib.sp_barrier_run_hash_launches(ctx.h, nwg, lanes, rounds, seed & 0xFFFFFFFF,
                                           int(graph), _ptr(slots), _ptr(out), ctypes.byref(st),
                                           _stream()), "sp_barrier_run_hash_launches", ctx.h)
    return _u32(out), st.as_dict()


class Mutex:
    """`nlocks` mutexes each guarding `words_per_lock` words (Section 5, Mutex)."""

    def __init__(self, ctx: Context, kind: str, nlocks: int, words_per_lock: int, **params):
        self.ctx, self.kind, self.nlocks, self.W = ctx, kind, nlocks, words_per_lock
        p = make_params(**params)
        h = ctypes.c_void_p()
        check(lib.sp_mutex_create(ctx.h, N.MUTEX_KINDS[kind], nlocks, words_per_lock,
                                  ctypes.byref(p), ctypes.byref(h)), "sp_mutex_create", ctx.h)
        self.h = h

    def run(self, nwg: int, lanes: int, total: int, max_delay: int, seed: int,
            finish: bool = False):
        words = torch.zeros(self.nlocks * self.W, dtype=torch.int32, device="cuda")
        fin = torch.zeros(nwg, dtype=torch.int64, device="cuda") if finish else None
        st = N.Stats()
        check(lib.sp_mutex_run(self.h, nwg, lanes, total, max_delay, seed & 0xFFFFFFFF,
                               _ptr(words), _ptr(fin), ctypes.byref(st), _stream()),
              "sp_mutex_run", self.ctx.h)
        out = _u32(words).reshape(self.nlocks, self.W)
        return (out, st.as_dict(), fin.cpu() if fin is not None else None)

    def close(self):
        if self.h:
            lib.sp_mutex_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Semaphore:
    """Counting semaphore with initial value K (Section 5, Semaphore)."""

    def __init__(self, ctx: Context, kind: str, K: int, **params):
        self.ctx, self.kind, self.K = ctx, kind, K
        p = make_params(**params)
        h = ctypes.c_void_p()
        check(lib.sp_sem_create(ctx.h, N.SEM_KINDS[kind], K, ctypes.byref(p), ctypes.byref(h)),
              "sp_sem_create", ctx.h)
        self.h = h

    def run(self, nwg: int, lanes: int, total: int, max_hold: int, seed: int, track: bool = True):
        chk = torch.zeros(nwg, dtype=torch.int32, device="cuda")
        state = torch.zeros(8, dtype=torch.int32, device="cuda")
        st = N.Stats()
        check(lib.sp_sem_run(self.h, nwg, lanes, total, max_hold, seed & 0xFFFFFFFF, int(track),
                             _ptr(chk), _ptr(state), ctypes.byref(st), _stream()),
              "sp_sem_run", self.ctx.h)
        s = [int(x) for x in _u32(state)]
        return {"chk": _u32(chk), "maxocc": s[0], "state": (s[1], s[2], s[3], s[4]),
                "count": s[5], "occ": s[6], "stats": st.as_dict()}

    def close(self):
        if self.h:
            lib.sp_sem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- microbenchmarks -----------------------------------------------------------------

def bench_atomic(ctx: Context, op: str, nwg: int, lanes: int, T: int, stride: int, mode: str,
                 n: int, seed: int, perm: torch.Tensor, buf: torch.Tensor | None = None):
    """Returns (finals uint32 as int64 CPU tensor [T], sum (int), stats)."""
    words = T * stride // 4
    if buf is None or buf.numel() < words:
        buf = torch.empty(words, dtype=torch.int32, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = N.Stats()
    check(lib.sp_bench_atomic(ctx.h, N.OPS[op], nwg, lanes, T, stride, N.ISSUE[mode], n,
                              seed & 0xFFFFFFFF, _ptr(perm), _ptr(buf), _ptr(out),
                              ctypes.byref(st), _stream()), "sp_bench_atomic", ctx.h)
    finals = _u32(buf[: words].view(T, stride // 4)[:, 0].contiguous())
    return finals, int(out.cpu().item()) & 0xFFFFFFFFFFFFFFFF, st.as_dict()


def paper12(ctx: Context, test: str, nwg: int, lanes: int = 64, n_ops: int = 1000,
            stride: int = 256, buf: torch.Tensor | None = None):
    words = nwg * stride // 4
    if buf is None or buf.numel() < words:
        buf = torch.empty(words, dtype=torch.int32, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = N.Stats()
    check(lib.sp_bench_paper12(ctx.h, N.PAPER12[test], nwg, lanes, n_ops, stride, _ptr(buf),
                               _ptr(out), ctypes.byref(st), _stream()), "sp_bench_paper12", ctx.h)
    return int(out.cpu().item()), buf, st.as_dict()


def stream_read(ctx: Context, buf: torch.Tensor, reps: int = 1, nwg: int = 0):
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = N.Stats()
    nbytes = buf.numel() * buf.element_size()
    check(lib.sp_bench_stream(ctx.h, _ptr(buf), nbytes, nwg, reps, _ptr(out), ctypes.byref(st),
                              _stream()), "sp_bench_stream", ctx.h)
    return int(out.cpu().item()) & 0xFFFFFFFFFFFFFFFF, st.as_dict()


def pingpong(ctx: Context, rounds: int):
    words = torch.zeros(512, dtype=torch.int32, device="cuda")
    out = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = N.Stats()
    check(lib.sp_bench_pingpong(ctx.h, rounds, _ptr(words), _ptr(out), ctypes.byref(st),
                                _stream()), "sp_bench_pingpong", ctx.h)
    return [int(x) for x in _u32(out)], st.as_dict()
