"""ctypes binding of libsp.so (the C ABI declared in include/sp.h).

Argument marshalling only: every primitive runs in the library's HIP kernels.  There is
no fallback: if libsp.so is missing or fails to load, importing this module raises.
"""

from __future__ import annotations

import ctypes
import os

# PyTorch's wheel bundles its own HIP runtime (soname libamdhip64.so.7).  Importing torch
# before libsp.so is loaded makes libsp.so bind to that same runtime, so device pointers
# and streams created by torch are valid in the library.  A process that never uses
# torch sets SP_NO_TORCH=1 and the library binds to the system ROCm runtime instead; it
# then allocates device memory through sp_buffer_alloc.
USE_TORCH = os.environ.get("SP_NO_TORCH", "0") != "1"
if USE_TORCH:
    try:
        import torch  # noqa: F401
    except ImportError:
        USE_TORCH = False

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsp.so")

# error codes
SP_OK = 0
SP_E_INVAL = -1
SP_E_HIP = -2
SP_E_NORESIDENT = -3
SP_E_TIMEOUT = -4
SP_E_PARITY = -5
SP_E_RANGE = -6

BARRIER_KINDS = {"central": 0, "central_split": 1, "tree": 2, "flag": 3, "grid_sync": 4,
                 "xcd": 5, "default": 15}
MUTEX_KINDS = {"spin_cas": 0, "spin_exch": 1, "spin_backoff": 2, "ticket": 3, "sleep": 4,
               "ring": 5, "array": 6, "adaptive": 7, "cohort": 8, "mcs": 9, "cu_cohort": 10,
               "default": 15}
SEM_KINDS = {"spin": 0, "spin_backoff": 1, "ticket": 2, "sleep": 3, "counters": 4,
             "adaptive": 5, "cohort": 6, "array": 7, "chain": 8, "xcd_chain": 9, "cu_lock": 10,
             "default": 15}
BACKOFF = {"none": 0, "paper": 1, "exp": 2}
BACKOFF_UNIT = {"sleep": 0, "load": 1}
OPS = {"add": 0, "cas": 1, "exch": 2, "ld": 3, "st": 4}
ISSUE = {"per_lane": 0, "wave_leader": 1}
PINGPONG_FENCED = 1
PINGPONG_SAME_XCD = 2
PAPER12 = {
    "cont_vol_read": 0, "cont_vol_write": 1, "noncont_vol_read": 2, "noncont_vol_write": 3,
    "cont_atom_read": 4, "cont_atom_write": 5, "noncont_atom_read": 6,
    "noncont_atom_write": 7, "cont_vol_read_after_atom": 8, "cont_vol_write_after_atom": 9,
    "noncont_vol_read_after_atom": 10, "noncont_vol_write_after_atom": 11,
}


class Params(ctypes.Structure):
    _fields_ = [
        ("backoff", ctypes.c_uint32),
        ("backoff_min", ctypes.c_uint32),
        ("backoff_max", ctypes.c_uint32),
        ("backoff_unit", ctypes.c_uint32),
        ("poll_sleep", ctypes.c_uint32),
        ("fan_in", ctypes.c_uint32),
        ("pad_bytes", ctypes.c_uint32),
        ("flags_packed", ctypes.c_uint32),
        ("timeout_ms", ctypes.c_uint32),
        ("verify", ctypes.c_uint32),
        ("cooperative", ctypes.c_uint32),
        ("coherent_cs", ctypes.c_uint32),
        ("xcd_copies", ctypes.c_uint32),
        ("cohort_passes", ctypes.c_uint32),
        ("flag_placement", ctypes.c_uint32),
        ("post_backoff", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 3),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("kernel_ms", ctypes.c_double),
        ("nwg", ctypes.c_uint32),
        ("lanes", ctypes.c_uint32),
        ("resident_per_cu", ctypes.c_uint32),
        ("device_error", ctypes.c_uint32),
        ("ops", ctypes.c_uint64),
        ("reserved", ctypes.c_uint64 * 4),
    ]

    def as_dict(self) -> dict:
        return {"kernel_ms": self.kernel_ms, "nwg": self.nwg, "lanes": self.lanes,
                "resident_per_cu": self.resident_per_cu, "device_error": self.device_error,
                "ops": self.ops}


class DeviceInfo(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 64),
        ("arch", ctypes.c_char * 64),
        ("cu_count", ctypes.c_uint32),
        ("xcd_count", ctypes.c_uint32),
        ("wall_clock_khz", ctypes.c_uint32),
        ("clock_khz", ctypes.c_uint32),
        ("hbm_bytes", ctypes.c_uint64),
        ("max_threads_per_cu", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 7),
    ]


class BarrierInfo(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_uint32),
        ("nwg", ctypes.c_uint32),
        ("xcd_path", ctypes.c_uint32),
        ("misplaced", ctypes.c_uint32),
        ("cu_overflow", ctypes.c_uint32),
        ("near_placed", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 2),
    ]


class ServeCfg(ctypes.Structure):
    _fields_ = [
        ("nwg", ctypes.c_uint32),
        ("lanes", ctypes.c_uint32),
        ("ring_slots", ctypes.c_uint32),
        ("budget_units", ctypes.c_uint32),
        ("unit_bytes", ctypes.c_uint64),
        ("seed", ctypes.c_uint32),
        ("poll_sleep", ctypes.c_uint32),
        ("far_sleep", ctypes.c_uint32),
        ("timeout_ms", ctypes.c_uint32),
        ("streams", ctypes.c_uint32),
        ("batch", ctypes.c_uint32),
        ("track", ctypes.c_uint32),
        ("graph_batch", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 4),
    ]


class ServeResult(ctypes.Structure):
    _fields_ = [
        ("wall_s", ctypes.c_double),
        ("p50_us", ctypes.c_double),
        ("p99_us", ctypes.c_double),
        ("mean_us", ctypes.c_double),
        ("max_us", ctypes.c_double),
        ("req_per_s", ctypes.c_double),
        ("publish_lag_max_us", ctypes.c_double),
        ("completed", ctypes.c_uint64),
        ("launches", ctypes.c_uint64),
        ("max_units_in_use", ctypes.c_uint32),
        ("device_error", ctypes.c_uint32),
        ("units_issued", ctypes.c_uint64),
        ("units_released", ctypes.c_uint64),
        ("reserved", ctypes.c_uint64 * 2),
    ]


class Occupancy(ctypes.Structure):
    _fields_ = [
        ("runtime_per_cu", ctypes.c_uint32),
        ("vgprs", ctypes.c_uint32),
        ("lds_bytes", ctypes.c_uint32),
        ("lanes", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 4),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
            "g.build()'` (hipcc, gfx950).  There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "sp_init": (i32, [i32, P(vp)]),
        "sp_fini": (i32, [vp]),
        "sp_device_info_get": (i32, [vp, P(DeviceInfo)]),
        "sp_params_default": (None, [P(Params)]),
        "sp_set_default": (i32, [vp, u32, u32, u32, P(Params)]),
        "sp_get_default": (i32, [vp, u32, u32, P(u32), P(Params)]),
        "sp_strerror": (ctypes.c_char_p, [i32]),
        "sp_last_hip_error": (i32, [vp]),
        "sp_probe_xcc": (i32, [vp, u32, u32, vp, vp]),
        "sp_resident_per_cu": (u32, [P(Occupancy)]),
        "sp_buffer_alloc": (i32, [vp, u64, P(vp)]),
        "sp_buffer_free": (i32, [vp, vp]),
        "sp_buffer_read": (i32, [vp, vp, vp, u64]),
        "sp_buffer_write": (i32, [vp, vp, vp, u64]),
        "sp_barrier_create": (i32, [vp, u32, u32, P(Params), P(vp)]),
        "sp_barrier_destroy": (i32, [vp]),
        "sp_barrier_info_get": (i32, [vp, P(BarrierInfo)]),
        "sp_barrier_run_hash": (i32, [vp, u32, u32, u32, vp, P(Stats), vp]),
        "sp_barrier_run_hash_launches": (i32, [vp, u32, u32, u32, u32, u32, vp, vp, P(Stats), vp]),
        "sp_mutex_create": (i32, [vp, u32, u32, u32, P(Params), P(vp)]),
        "sp_mutex_destroy": (i32, [vp]),
        "sp_mutex_run": (i32, [vp, u32, u32, u64, u32, u32, vp, vp, P(Stats), vp]),
        "sp_sem_create": (i32, [vp, u32, u32, P(Params), P(vp)]),
        "sp_sem_destroy": (i32, [vp]),
        "sp_sem_run": (i32, [vp, u32, u32, u64, u32, u32, u32, vp, vp, vp, P(Stats), vp]),
        "sp_bench_atomic": (i32, [vp, u32, u32, u32, u32, u32, u32, u64, u32, vp, vp, vp,
                                  P(Stats), vp]),
        "sp_bench_paper12": (i32, [vp, u32, u32, u32, u32, u32, vp, vp, P(Stats), vp]),
        "sp_bench_stream": (i32, [vp, vp, u64, u32, u32, vp, P(Stats), vp]),
        "sp_bench_pingpong": (i32, [vp, u32, u32, vp, vp, P(Stats), vp]),
        "sp_bench_copy": (i32, [vp, vp, vp, u64, u32, P(Stats), vp]),
        "sp_bench_litmus": (i32, [vp, u32, u32, u32, u32, vp, P(Stats), vp]),
        "sp_bench_fence": (i32, [vp, u32, u32, u32, u32, u32, vp, P(Stats), vp]),
        "sp_bench_clock": (i32, [vp, u32, vp, P(ctypes.c_double), vp]),
        "sp_cond_run_bounded_buffer": (i32, [vp, u32, u32, u32, u32, u32, u64, u32, P(Params),
                                              vp, vp, P(Stats), vp]),
        "sp_cond_run_bounded_buffer_noalloc": (i32, [vp, u32, u32, u32, u32, u32, u64, u32,
                                                      P(Params), vp, vp, P(Stats), vp]),
        "sp_graph_begin": (i32, [vp, vp, P(vp)]),
        "sp_graph_end": (i32, [vp, vp, P(vp)]),
        "sp_graph_launch": (i32, [vp, u32, P(Stats), vp]),
        "sp_graph_destroy": (i32, [vp]),
        "sp_serve_run": (i32, [vp, P(ServeCfg), u32, vp, vp, vp, vp, vp, P(ServeResult)]),
        "sp_serve_run_launch_per_request": (i32, [vp, P(ServeCfg), u32, vp, vp, vp, vp, vp,
                                                  P(ServeResult)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name, None)
        if f is None:
            continue  # optional entry points are checked by the ABI test
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class SpError(RuntimeError):
    def __init__(self, code: int, where: str, hip: int = 0):
        self.code = code
        msg = lib.sp_strerror(code).decode()
        super().__init__(f"{where}: {msg} (code {code}{', hip error ' + str(hip) if hip else ''})")


class SpTimeout(SpError):
    pass


class SpNotResident(SpError):
    pass


def check(rc: int, where: str, ctx=None) -> None:
    if rc == SP_OK:
        return
    hip = lib.sp_last_hip_error(ctx) if ctx else 0
    if rc == SP_E_TIMEOUT:
        raise SpTimeout(rc, where, hip)
    if rc == SP_E_NORESIDENT:
        raise SpNotResident(rc, where, hip)
    raise SpError(rc, where, hip)
