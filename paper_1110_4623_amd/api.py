"""Python API over libsp.so: contexts, barriers, mutexes, semaphores, microbenchmarks.

Thin wrappers: they allocate device buffers, pass raw pointers and a HIP stream to the
C ABI, and read results back as numpy arrays.  Every primitive runs in the library's
kernels; nothing here computes a result.

Device memory comes from PyTorch (CUDA tensors, launched on torch's current stream)
when torch is in the process, otherwise from the library's own sp_buffer_alloc
(launched on the null stream); see _native.USE_TORCH.
"""

from __future__ import annotations

import atexit
import ctypes
import weakref

import numpy as np

from . import _native as N
from ._native import check, lib

_NP = {"u32": np.uint32, "u64": np.uint64, "i64": np.int64}


class DeviceBuffer:
    """Zero-filled device memory from sp_buffer_alloc (the torch-free path)."""

    def __init__(self, ctx: "Context", nbytes: int):
        self.ctx, self.nbytes = ctx, nbytes
        self.p = None
        p = ctypes.c_void_p()
        check(lib.sp_buffer_alloc(ctx.h, nbytes, ctypes.byref(p)), "sp_buffer_alloc", ctx.h)
        self.p = p
        ctx._own(self)

    def ptr(self) -> ctypes.c_void_p:
        return self.p

    def read(self, dtype, count: int) -> np.ndarray:
        out = np.empty(count, dtype=dtype)
        check(lib.sp_buffer_read(self.ctx.h, out.ctypes.data_as(ctypes.c_void_p), self.p,
                                 out.nbytes), "sp_buffer_read", self.ctx.h)
        return out

    def write(self, arr: np.ndarray) -> None:
        arr = np.ascontiguousarray(arr)
        check(lib.sp_buffer_write(self.ctx.h, self.p, arr.ctypes.data_as(ctypes.c_void_p),
                                  arr.nbytes), "sp_buffer_write", self.ctx.h)

    def close(self):
        if self.p:
            if self.ctx.h:
                lib.sp_buffer_free(self.ctx.h, self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Contexts still open; closed before the interpreter tears down its objects (and before
# the HIP runtime and any profiler attached to it finalize), so that no device memory or
# state object is released in the middle of process exit.
_LIVE: "weakref.WeakSet[Context]" = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    for c in list(_LIVE):
        c.close()


class Context:
    """A libsp context bound to one HIP device."""

    def __init__(self, device: int | None = None):
        self.torch = None
        if N.USE_TORCH:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no HIP device visible: libsp needs an MI355X (gfx950) GPU")
            self.torch = torch
            device = torch.cuda.current_device() if device is None else device
            torch.cuda.set_device(device)
            torch.cuda.init()
        self.device = 0 if device is None else device
        self.h = None
        # buffers and state objects made from this context: closed before sp_fini
        self._owned = weakref.WeakSet()
        h = ctypes.c_void_p()
        check(lib.sp_init(self.device, ctypes.byref(h)), "sp_init")
        self.h = h
        _LIVE.add(self)
        info = N.DeviceInfo()
        check(lib.sp_device_info_get(self.h, ctypes.byref(info)), "sp_device_info_get", self.h)
        self.info = {
            "name": info.name.decode(), "arch": info.arch.decode(), "cu_count": info.cu_count,
            "xcd_count": info.xcd_count, "wall_clock_khz": info.wall_clock_khz,
            "clock_khz": info.clock_khz, "hbm_bytes": info.hbm_bytes,
            "max_threads_per_cu": info.max_threads_per_cu,
        }

    # ---- memory and streams --------------------------------------------------------
    def stream(self) -> ctypes.c_void_p:
        if getattr(self, "_record_stream", None) is not None:
            return self._record_stream
        if self.torch is not None:
            return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)

    def zeros(self, count: int, dtype: str = "u32"):
        """Zero-filled device array of `count` elements (u32, u64 or i64)."""
        size = np.dtype(_NP[dtype]).itemsize
        if self.torch is not None:
            tdt = {"u32": self.torch.int32, "u64": self.torch.int64, "i64": self.torch.int64}[dtype]
            return self.torch.zeros(max(count, 1), dtype=tdt, device="cuda")
        return DeviceBuffer(self, max(count, 1) * size)

    def upload(self, arr: np.ndarray):
        arr = np.ascontiguousarray(arr)
        if self.torch is not None:
            view = arr.view(np.int32) if arr.dtype == np.uint32 else arr
            return self.torch.from_numpy(view.copy()).cuda()
        buf = DeviceBuffer(self, arr.nbytes)
        buf.write(arr)
        return buf

    def read(self, buf, dtype: str, count: int | None = None) -> np.ndarray:
        npdt = _NP[dtype]
        if isinstance(buf, DeviceBuffer):
            n = buf.nbytes // np.dtype(npdt).itemsize if count is None else count
            return buf.read(npdt, n)
        a = buf.detach().cpu().numpy()
        a = a.view(np.uint32) if dtype == "u32" and a.dtype == np.int32 else a
        a = a.view(np.uint64) if dtype == "u64" and a.dtype == np.int64 else a
        return (a if count is None else a[:count]).astype(npdt, copy=False)

    @staticmethod
    def ptr(buf) -> ctypes.c_void_p:
        if buf is None:
            return ctypes.c_void_p(0)
        if isinstance(buf, DeviceBuffer):
            return buf.ptr()
        if not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("expected a contiguous device tensor")
        return ctypes.c_void_p(buf.data_ptr())

    def synchronize(self):
        if self.torch is not None:
            self.torch.cuda.synchronize()

    # ---- lifetime ------------------------------------------------------------------
    def _own(self, obj) -> None:
        self._owned.add(obj)

    def close(self):
        """Releases every buffer, state object and graph made from this context, waits for
        the device, then the context itself.  Idempotent."""
        if self.h:
            for obj in list(self._owned):
                obj.close()
            lib.sp_fini(self.h)
            self.h = None
        _LIVE.discard(self)

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

    def get_default(self, primitive: str, bucket: int) -> str:
        """The kind name that a DEFAULT object of this class resolves to in this bucket."""
        prim = {"barrier": 0, "mutex": 1, "semaphore": 2}[primitive]
        kinds = [N.BARRIER_KINDS, N.MUTEX_KINDS, N.SEM_KINDS][prim]
        k = ctypes.c_uint32(0)
        check(lib.sp_get_default(self.h, prim, bucket, ctypes.byref(k), None),
              "sp_get_default", self.h)
        return {v: n for n, v in kinds.items()}[k.value]

    def probe_xcc(self, nwg: int, lanes: int = 64) -> np.ndarray:
        out = self.zeros(nwg)
        check(lib.sp_probe_xcc(self.h, nwg, lanes, self.ptr(out), self.stream()), "sp_probe_xcc",
              self.h)
        return self.read(out, "u32", nwg)


def make_params(**kw) -> N.Params:
    p = N.Params()
    lib.sp_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "backoff" and isinstance(v, str):
            v = N.BACKOFF[v]
        if k == "backoff_unit" and isinstance(v, str):
            v = N.BACKOFF_UNIT[v]
        if not hasattr(p, k) or k == "reserved":
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, int(v))
    return p


class _Handle:
    _destroy = None

    def close(self):
        if getattr(self, "h", None):
            type(self)._destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Barrier(_Handle):
    """Global barrier among `nwg` co-resident workgroups (Section 5, Barrier)."""

    _destroy = staticmethod(lambda h: lib.sp_barrier_destroy(h))

    def __init__(self, ctx: Context, kind: str, nwg: int, **params):
        self.ctx, self.kind, self.nwg = ctx, kind, nwg
        p = make_params(**params)
        h = ctypes.c_void_p()
        check(lib.sp_barrier_create(ctx.h, N.BARRIER_KINDS[kind], nwg, ctypes.byref(p),
                                    ctypes.byref(h)), "sp_barrier_create", ctx.h)
        self.h = h
        ctx._own(self)
        self._out = ctx.zeros(nwg)

    def launch(self, lanes: int, rounds: int, seed: int) -> dict:
        """Runs (or, inside a Graph recording, records) the hash exchange; the checksums
        stay on the device until `checksums()`.  Returns the stats."""
        st = N.Stats()
        check(lib.sp_barrier_run_hash(self.h, lanes, rounds, seed & 0xFFFFFFFF,
                                      self.ctx.ptr(self._out), ctypes.byref(st), self.ctx.stream()),
              "sp_barrier_run_hash", self.ctx.h)
        return st.as_dict()

    def checksums(self) -> np.ndarray:
        return self.ctx.read(self._out, "u32", self.nwg)

    def info(self) -> dict:
        """How the last run synchronized (per-XCD path used, or why not)."""
        i = N.BarrierInfo()
        check(lib.sp_barrier_info_get(self.h, ctypes.byref(i)), "sp_barrier_info_get", self.ctx.h)
        names = {v: k for k, v in N.BARRIER_KINDS.items()}
        return {"kind": names.get(i.kind, i.kind), "xcd_path": bool(i.xcd_path),
                "misplaced": i.misplaced, "cu_overflow": i.cu_overflow,
                "near_placed": i.near_placed}

    def run_hash(self, lanes: int, rounds: int, seed: int):
        """Hash-exchange workload; returns (checksums as uint32 numpy array, stats)."""
        st = self.launch(lanes, rounds, seed)
        return self.checksums(), st


def barrier_hash_launches(ctx: Context, nwg: int, lanes: int, rounds: int, seed: int,
                          graph: bool = False):
    """Kernel-boundary comparator of the hash exchange (one launch per round)."""
    slots = ctx.zeros(2 * nwg)
    out = ctx.zeros(nwg)
    st = N.Stats()
    check(lib.sp_barrier_run_hash_launches(ctx.h, nwg, lanes, rounds, seed & 0xFFFFFFFF,
                                           int(graph), ctx.ptr(slots), ctx.ptr(out),
                                           ctypes.byref(st), ctx.stream()),
          "sp_barrier_run_hash_launches", ctx.h)
    return ctx.read(out, "u32", nwg), st.as_dict()


class Mutex(_Handle):
    """`nlocks` mutexes each guarding `words_per_lock` words (Section 5, Mutex)."""

    _destroy = staticmethod(lambda h: lib.sp_mutex_destroy(h))

    def __init__(self, ctx: Context, kind: str, nlocks: int, words_per_lock: int, **params):
        self.ctx, self.kind, self.nlocks, self.W = ctx, kind, nlocks, words_per_lock
        p = make_params(**params)
        h = ctypes.c_void_p()
        check(lib.sp_mutex_create(ctx.h, N.MUTEX_KINDS[kind], nlocks, words_per_lock,
                                  ctypes.byref(p), ctypes.byref(h)), "sp_mutex_create", ctx.h)
        self.h = h
        ctx._own(self)
        self._words = ctx.zeros(nlocks * words_per_lock)

    def launch(self, nwg: int, lanes: int, total: int, max_delay: int, seed: int,
               finish=None) -> dict:
        """Runs (or records) the contention workload; results stay on the device until
        `words()`.  finish: optional device buffer of nwg uint64.  Returns the stats."""
        st = N.Stats()
        check(lib.sp_mutex_run(self.h, nwg, lanes, total, max_delay, seed & 0xFFFFFFFF,
                               self.ctx.ptr(self._words), self.ctx.ptr(finish), ctypes.byref(st),
                               self.ctx.stream()), "sp_mutex_run", self.ctx.h)
        return st.as_dict()

    def words(self) -> np.ndarray:
        return self.ctx.read(self._words, "u32", self.nlocks * self.W).reshape(self.nlocks, self.W)

    def run(self, nwg: int, lanes: int, total: int, max_delay: int, seed: int,
            finish: bool = False):
        """Returns (words[nlocks, W] uint32, stats, finish ticks uint64 or None)."""
        fin = self.ctx.zeros(nwg, "u64") if finish else None
        st = self.launch(nwg, lanes, total, max_delay, seed, fin)
        return self.words(), st, (self.ctx.read(fin, "u64", nwg) if finish else None)


class Semaphore(_Handle):
    """Counting semaphore with initial value K (Section 5, Semaphore)."""

    _destroy = staticmethod(lambda h: lib.sp_sem_destroy(h))

    def __init__(self, ctx: Context, kind: str, K: int, **params):
        self.ctx, self.kind, self.K = ctx, kind, K
        p = make_params(**params)
        h = ctypes.c_void_p()
        check(lib.sp_sem_create(ctx.h, N.SEM_KINDS[kind], K, ctypes.byref(p), ctypes.byref(h)),
              "sp_sem_create", ctx.h)
        self.h = h
        ctx._own(self)
        self._state = ctx.zeros(8)

    def launch(self, nwg: int, lanes: int, total: int, max_hold: int, seed: int,
               track: bool = True, data: bool = False) -> dict:
        """Runs (or records) the wait/post workload; results stay on the device until
        `result()`.  data=True also updates the guarded data words.  Returns the stats."""
        if getattr(self, "_chk_n", None) != nwg:
            self._chk, self._chk_n = self.ctx.zeros(nwg), nwg
        if data and getattr(self, "_data", None) is None:
            self._data = self.ctx.zeros(self.K)
        self._with_data = data
        st = N.Stats()
        check(lib.sp_sem_run(self.h, nwg, lanes, total, max_hold, seed & 0xFFFFFFFF, int(track),
                             self.ctx.ptr(self._chk), self.ctx.ptr(self._state),
                             self.ctx.ptr(self._data if data else None), ctypes.byref(st),
                             self.ctx.stream()), "sp_sem_run", self.ctx.h)
        return st.as_dict()

    def result(self) -> dict:
        s = [int(x) for x in self.ctx.read(self._state, "u32", 8)]
        r = {"chk": self.ctx.read(self._chk, "u32", self._chk_n), "maxocc": s[0],
             "state": (s[1], s[2], s[3], s[4]), "count": s[5], "occ": s[6], "unserved": s[7]}
        if getattr(self, "_with_data", False):
            r["data"] = self.ctx.read(self._data, "u32", self.K)
        return r

    def run(self, nwg: int, lanes: int, total: int, max_hold: int, seed: int, track: bool = True,
            data: bool = False):
        st = self.launch(nwg, lanes, total, max_hold, seed, track, data)
        return dict(self.result(), stats=st)


def bounded_buffer(ctx: Context, mutex_kind: str, nwg: int, producers: int, capacity: int,
                   items: int, seed: int, lanes: int = 64, values: bool = False,
                   noalloc: bool = False, **params) -> dict:
    """Producer/consumer ring on a mutex and two condition variables
    (sp_cond_run_bounded_buffer, or with noalloc=True the allocation-free
    sp_cond_run_bounded_buffer_noalloc).  values=True also returns every value taken."""
    out = ctx.zeros(6, "u64")
    taken = ctx.zeros(items) if values else None
    p = make_params(**params)
    st = N.Stats()
    name = "sp_cond_run_bounded_buffer_noalloc" if noalloc else "sp_cond_run_bounded_buffer"
    check(getattr(lib, name)(ctx.h, N.MUTEX_KINDS[mutex_kind], nwg, producers, lanes, capacity,
                             items, seed & 0xFFFFFFFF, ctypes.byref(p), ctx.ptr(out),
                             ctx.ptr(taken), ctypes.byref(st), ctx.stream()), name, ctx.h)
    v = [int(x) for x in ctx.read(out, "u64", 6)]
    r = {"xor": v[0], "sum": v[1], "taken": v[2], "put": v[3], "max_count": v[4],
         "left": v[5], "stats": st.as_dict()}
    if values:
        r["values"] = ctx.read(taken, "u32", items)
    return r


class Graph:
    """Records the primitive runs made inside a `with` block into one HIP graph
    (sp_graph_begin/end) and replays them with `launch`.  Inside the block, use the
    wrappers' `launch` methods (results stay on the device); read results after a
    replay with `checksums()`, `words()` or `result()`."""

    def __init__(self, ctx: Context):
        self.ctx, self.h = ctx, None

    def __enter__(self):
        cs = ctypes.c_void_p()
        # record on the context's own stream, so that nothing else (torch's work on its
        # current stream) is captured
        check(lib.sp_graph_begin(self.ctx.h, None, ctypes.byref(cs)), "sp_graph_begin",
              self.ctx.h)
        self._cs = cs
        self.ctx._record_stream = cs
        return self

    def __exit__(self, exc_type, exc, tb):
        self.ctx._record_stream = None
        g = ctypes.c_void_p()
        rc = lib.sp_graph_end(self.ctx.h, self._cs, ctypes.byref(g))
        if exc_type is None:
            check(rc, "sp_graph_end", self.ctx.h)
            self.h = g
            self.ctx._own(self)
        elif rc == 0:
            lib.sp_graph_destroy(g)
        return False

    def launch(self, replays: int = 1) -> dict:
        st = N.Stats()
        check(lib.sp_graph_launch(self.h, replays, ctypes.byref(st), self.ctx.stream()),
              "sp_graph_launch", self.ctx.h)
        return st.as_dict()

    def close(self):
        if self.h:
            lib.sp_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- microbenchmarks -----------------------------------------------------------------

def bench_atomic(ctx: Context, op: str, nwg: int, lanes: int, T: int, stride: int, mode: str,
                 n: int, seed: int, perm, buf=None):
    """perm: uint32 numpy array or device buffer of T entries.  Returns (finals uint32
    numpy [T], sum, stats); sum is the uint64 total of returned values (plus the final
    words for EXCH)."""
    if isinstance(perm, np.ndarray):
        perm = ctx.upload(perm.astype(np.uint32))
    words = T * stride // 4
    if buf is None:
        buf = ctx.zeros(words)
    out = ctx.zeros(1, "u64")
    st = N.Stats()
    check(lib.sp_bench_atomic(ctx.h, N.OPS[op], nwg, lanes, T, stride, N.ISSUE[mode], n,
                              seed & 0xFFFFFFFF, ctx.ptr(perm), ctx.ptr(buf), ctx.ptr(out),
                              ctypes.byref(st), ctx.stream()), "sp_bench_atomic", ctx.h)
    finals = ctx.read(buf, "u32", words).reshape(T, stride // 4)[:, 0].copy()
    return finals, int(ctx.read(out, "u64", 1)[0]), st.as_dict()


def paper12(ctx: Context, test: str, nwg: int, lanes: int = 64, n_ops: int = 1000,
            stride: int = 256, buf=None):
    """Returns (sum of loaded values, final buffer words uint32 numpy, stats)."""
    words = nwg * stride // 4
    if buf is None:
        buf = ctx.zeros(words)
    out = ctx.zeros(1, "u64")
    st = N.Stats()
    check(lib.sp_bench_paper12(ctx.h, N.PAPER12[test], nwg, lanes, n_ops, stride, ctx.ptr(buf),
                               ctx.ptr(out), ctypes.byref(st), ctx.stream()), "sp_bench_paper12",
          ctx.h)
    return int(ctx.read(out, "u64", 1)[0]), ctx.read(buf, "u32", words), st.as_dict()


def stream_read(ctx: Context, buf, nbytes: int, reps: int = 1, nwg: int = 0):
    out = ctx.zeros(1, "u64")
    st = N.Stats()
    check(lib.sp_bench_stream(ctx.h, ctx.ptr(buf), nbytes, nwg, reps, ctx.ptr(out),
                              ctypes.byref(st), ctx.stream()), "sp_bench_stream", ctx.h)
    return int(ctx.read(out, "u64", 1)[0]), st.as_dict()


def copy(ctx: Context, dst, src, nbytes: int, reps: int = 1):
    st = N.Stats()
    check(lib.sp_bench_copy(ctx.h, ctx.ptr(dst), ctx.ptr(src), nbytes, reps, ctypes.byref(st),
                            ctx.stream()), "sp_bench_copy", ctx.h)
    return st.as_dict()


LITMUS = {"mp": (0, {"fenced": 0, "no_acquire": 1, "no_release": 2, "none": 3,
                    "release_wg_invalidate": 4}),
          "sb": (1, {"fenced": 0, "none": 1})}


def litmus(ctx: Context, test: str, variant: str, pairs: int, iters: int) -> dict:
    """Memory-model litmus test (sp_bench_litmus); returns forbidden outcomes and trials."""
    t, variants = LITMUS[test]
    out = ctx.zeros(1, "u64")
    st = N.Stats()
    check(lib.sp_bench_litmus(ctx.h, t, variants[variant], pairs, iters, ctx.ptr(out),
                              ctypes.byref(st), ctx.stream()), "sp_bench_litmus", ctx.h)
    return {"forbidden": int(ctx.read(out, "u64", 1)[0]), "trials": pairs * iters,
            "stats": st.as_dict()}


def shader_clock_mhz(ctx: Context, ms: int = 20) -> float:
    """Shader clock rate observed by one spinning lane over `ms` of wall clock."""
    out = ctx.zeros(2, "u64")
    mhz = ctypes.c_double(0)
    check(lib.sp_bench_clock(ctx.h, ms, ctx.ptr(out), ctypes.byref(mhz), ctx.stream()),
          "sp_bench_clock", ctx.h)
    return mhz.value


def bench_fence(ctx: Context, kind: str, nwg: int, lanes: int = 64, reps: int = 1,
                lines: int = 1) -> dict:
    """Fence cost (sp_bench_fence).  kind: "release" or "acquire" (agent scope) or
    "wg_invalidate" (a workgroup-scope invalidate).  Returns
    per-fence shader clocks (mean and max over workgroups) and the wall-clock span from
    the first workgroup's start to the last one's end."""
    out = ctx.zeros(4 * nwg, "u64")
    st = N.Stats()
    check(lib.sp_bench_fence(ctx.h, {"release": 0, "acquire": 1, "wg_invalidate": 2}[kind], nwg, lanes, reps, lines,
                             ctx.ptr(out), ctypes.byref(st), ctx.stream()),
          "sp_bench_fence", ctx.h)
    v = ctx.read(out, "u64", 4 * nwg).reshape(nwg, 4).astype(np.float64)
    per = v[:, 0] / reps
    span_ticks = float(v[:, 2].max() - v[:, 1].min())
    return {"clk_per_fence_mean": float(per.mean()), "clk_per_fence_max": float(per.max()),
            "span_us": span_ticks / ctx.info["wall_clock_khz"] * 1e3, "stats": st.as_dict()}


def pingpong(ctx: Context, rounds: int, fenced: bool = True, same_xcd: bool = False,
             offset_bytes: int = 0):
    """Token ping-pong between two workgroups (`sp_bench_pingpong`): returns ([partner's
    word, workgroup 0's word, XCC of workgroup 0, XCC of the partner], stats); one-way
    latency = kernel_ms / (2 * rounds).  offset_bytes (a multiple of 128) places the two
    words that far into a fresh buffer, to reach other memory channels."""
    if offset_bytes < 0 or offset_bytes % 128:
        raise ValueError("offset_bytes must be a non-negative multiple of 128")
    words = ctx.zeros(512 + offset_bytes // 4)
    out = ctx.zeros(4)
    st = N.Stats()
    mode = (N.PINGPONG_FENCED if fenced else 0) | (N.PINGPONG_SAME_XCD if same_xcd else 0)
    base = ctx.ptr(words).value + offset_bytes
    check(lib.sp_bench_pingpong(ctx.h, rounds, mode, ctypes.c_void_p(base), ctx.ptr(out),
                                ctypes.byref(st), ctx.stream()), "sp_bench_pingpong", ctx.h)
    return [int(x) for x in ctx.read(out, "u32", 4)], st.as_dict()


def _serve_args(ctx: Context, reqs: dict, nwg: int, lanes: int, budget_units: int,
                unit_bytes: int, seed: int, **cfg):
    L = np.ascontiguousarray(reqs["L"], dtype=np.uint32)
    nbytes = np.ascontiguousarray(reqs["nbytes"], dtype=np.uint64)
    t_arr = np.ascontiguousarray(reqs["t_arr"], dtype=np.float64)
    n = len(L)
    if len(nbytes) != n or len(t_arr) != n:
        raise ValueError("request table columns differ in length")
    c = N.ServeCfg()
    c.nwg, c.lanes, c.budget_units, c.unit_bytes, c.seed = nwg, lanes, budget_units, unit_bytes, seed
    for k, v in cfg.items():
        if not hasattr(c, k) or k == "reserved":
            raise TypeError(f"unknown serving option {k}")
        setattr(c, k, int(v))
    out = np.zeros(n, dtype=np.uint32)
    lat = np.zeros(n, dtype=np.float64)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    return c, n, (vp(L), vp(nbytes), vp(t_arr), vp(out), vp(lat)), out, lat, (L, nbytes, t_arr)


def _serve_result(r: N.ServeResult) -> dict:
    return {k: getattr(r, k) for k, _ in N.ServeResult._fields_ if k != "reserved"}


def serve(ctx: Context, reqs: dict, nwg: int = 1024, lanes: int = 64,
          budget_units: int = 16384, unit_bytes: int = 65536, seed: int = 42, **cfg):
    """Persistent serving queue (sp_serve_run) over a request table from
    sp_inputs.request_table.  Returns (out, latency_us, result dict)."""
    c, n, ptrs, out, lat, keep = _serve_args(ctx, reqs, nwg, lanes, budget_units, unit_bytes,
                                             seed, **cfg)
    res = N.ServeResult()
    check(lib.sp_serve_run(ctx.h, ctypes.byref(c), n, *ptrs, ctypes.byref(res)),
          "sp_serve_run", ctx.h)
    del keep
    return out, lat, _serve_result(res)


def serve_launch_per_request(ctx: Context, reqs: dict, lanes: int = 64,
                             budget_units: int = 16384, unit_bytes: int = 65536, seed: int = 42,
                             **cfg):
    """Comparator: one kernel launch per request (batch = 1) or per arrival batch."""
    c, n, ptrs, out, lat, keep = _serve_args(ctx, reqs, 0, lanes, budget_units, unit_bytes,
                                             seed, **cfg)
    res = N.ServeResult()
    check(lib.sp_serve_run_launch_per_request(ctx.h, ctypes.byref(c), n, *ptrs,
                                              ctypes.byref(res)),
          "sp_serve_run_launch_per_request", ctx.h)
    del keep
    return out, lat, _serve_result(res)
