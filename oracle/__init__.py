"""CPU oracle for the synchronization primitives of Stuart & Owens (2011).

TEST INFRASTRUCTURE ONLY.  The test-suite, the package smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports this package
and this package never imports the GPU library; they share only the seeded input
generators of ``sp_inputs``.

Three parts:

* closed forms (sequential definitions of each workload's output, in ``sp_oracle.cpp``),
* a threaded reference (one ``std::thread`` per agent, ``std::atomic`` shared words, the
  algorithms of Section 5 and the appendix, in ``sp_oracle.cpp``),
* an exhaustive-interleaving model checker (``modelcheck.py``).

The C++ part is built by :func:`build` into ``liboracle.so`` beside this file.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sp_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

BARRIER_KINDS = {"central": 0, "tree": 1, "flag": 2, "xcd": 3, "split": 4}
MUTEX_KINDS = {"spin_cas": 0, "spin_exch": 1, "spin_backoff": 2, "ticket": 3, "sleep": 4,
               "ring": 5, "array": 6, "adaptive": 7, "cohort": 8, "mcs": 9,
               "cu_cohort": 10}
SEM_KINDS = {"spin": 0, "spin_backoff": 1, "ticket": 2, "sleep": 3, "counters": 4,
             "adaptive": 5, "spin_backoff_wait_only": 6, "cohort": 7,
             "array": 8, "chain": 9,
             "xcd_chain": 10}
BENCH_OPS = {"add": 0, "cas": 1, "exch": 2, "ld": 3, "st": 4}


def build() -> str:
    """Compile ``sp_oracle.cpp`` with g++ into ``liboracle.so`` (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++20", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
           _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        p32 = ctypes.POINTER(ctypes.c_uint32)
        p64 = ctypes.POINTER(ctypes.c_uint64)
        pd = ctypes.POINTER(ctypes.c_double)
        sig = {
            "or_fmix32": (u32, [u32]),
            "or_sm32": (u32, [u32]),
            "or_key": (u32, [u32, u32, u32, u32]),
            "or_chain": (u32, [u32, u32]),
            "or_chain_batch": (None, [u32, p32, u32, p32]),
            "or_ops_for_agent": (u64, [u32, u64, u32]),
            "or_barrier_closed": (None, [u32, u32, u32, p32]),
            "or_mutex_closed": (None, [u32, u32, u64, u32, u32, p32]),
            "or_sem_closed": (None, [u32, u32, u64, p32]),
            "or_bench_counts": (None, [u32, u64, u32, p32, p64]),
            "or_bench_count_one": (u64, [u32, u64, u32, u32]),
            "or_sum_increments": (u64, [u32, u64]),
            "or_exch_value": (u32, [u32, u32, u32]),
            "or_prefill": (u32, [u32, u32]),
            "or_bench_closed": (i32, [i32, u32, u32, u64, u32, p32, p32, p64]),
            "or_hardware_threads": (ctypes.c_uint, []),
            "or_barrier_threaded": (i32, [i32, u32, u32, u32, u32, p32, pd]),
            "or_mutex_threaded": (i32, [i32, u32, u32, u64, u32, u32, u32, u32, p32, pd]),
            "or_sem_threaded": (i32, [i32, u32, u32, u32, u64, u32, u32, p32, p32, p32, pd]),
            "or_bench_threaded": (i32, [i32, u32, u32, u64, u32, p32, u32, p32, p64, pd]),
            "or_serve_threaded": (i32, [u32, p32, p32, u32, u32, u32, p32, p32, p64, pd]),
            "or_bb_closed": (None, [u32, u32, u64, p64]),
            "or_bb_values": (None, [u32, u32, u64, p32]),
            "or_exch_finals_invalid": (u64, [u32, u32, u64, u32, p32, p32]),
            "or_bb_threaded": (i32, [u32, u32, u32, u64, u32, p64, pd]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p32(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p64(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


# ---- hashing -------------------------------------------------------------------------

def fmix32(z: int) -> int:
    return lib().or_fmix32(z & 0xFFFFFFFF)


def sm32(x: int) -> int:
    return lib().or_sm32(x & 0xFFFFFFFF)


def key(seed: int, b: int, j: int, s: int) -> int:
    return lib().or_key(seed & 0xFFFFFFFF, b, j, s)


def chain(x: int, L: int) -> int:
    return lib().or_chain(x & 0xFFFFFFFF, L)


def chain_batch(seed: int, lengths: np.ndarray) -> np.ndarray:
    lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
    out = np.zeros(len(lengths), dtype=np.uint32)
    lib().or_chain_batch(seed & 0xFFFFFFFF, _p32(lengths), len(lengths), _p32(out))
    return out


def ops_for_agent(nwg: int, total: int, b: int) -> int:
    return lib().or_ops_for_agent(nwg, total, b)


# ---- closed forms --------------------------------------------------------------------

def barrier_closed(seed: int, N: int, R: int) -> np.ndarray:
    out = np.zeros(N, dtype=np.uint32)
    lib().or_barrier_closed(seed & 0xFFFFFFFF, N, R, _p32(out))
    return out


def mutex_closed(seed: int, nwg: int, total: int, L: int, W: int) -> np.ndarray:
    out = np.zeros(L * W, dtype=np.uint32)
    lib().or_mutex_closed(seed & 0xFFFFFFFF, nwg, total, L, W, _p32(out))
    return out.reshape(L, W)


def sem_closed(seed: int, nwg: int, total: int) -> np.ndarray:
    out = np.zeros(nwg, dtype=np.uint32)
    lib().or_sem_closed(seed & 0xFFFFFFFF, nwg, total, _p32(out))
    return out


def bench_counts(U: int, n: int, perm: np.ndarray) -> np.ndarray:
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    out = np.zeros(len(perm), dtype=np.uint64)
    lib().or_bench_counts(U, n, len(perm), _p32(perm), _p64(out))
    return out


def bench_count_one(U: int, n: int, T: int, p: int) -> int:
    return lib().or_bench_count_one(U, n, T, p)


def sum_increments(a: int, c: int) -> int:
    return lib().or_sum_increments(a & 0xFFFFFFFF, c)


def exch_value(seed: int, u: int, i: int) -> int:
    return lib().or_exch_value(seed & 0xFFFFFFFF, u, i)


def prefill(seed: int, t: int) -> int:
    return lib().or_prefill(seed & 0xFFFFFFFF, t)


def bench_closed(op: str, seed: int, U: int, n: int, perm: np.ndarray):
    """Returns (finals[T] uint32, sum uint64).  For 'exch' finals are not unique (zeros
    are returned) and sum is the conserved quantity sum(initial) + sum(written)."""
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    finals = np.zeros(len(perm), dtype=np.uint32)
    s = ctypes.c_uint64(0)
    rc = lib().or_bench_closed(BENCH_OPS[op], seed & 0xFFFFFFFF, U, n, len(perm), _p32(perm),
                               _p32(finals), ctypes.byref(s))
    if rc != 0:
        raise ValueError(f"or_bench_closed({op}) failed: {rc}")
    return finals, s.value


def exch_finals_invalid(seed: int, U: int, n: int, perm: np.ndarray, finals: np.ndarray) -> int:
    """Words whose final value after the exchange benchmark is neither their initial value
    nor a value some exchange wrote to them (0 for a valid outcome)."""
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    finals = np.ascontiguousarray(finals, dtype=np.uint32)
    return lib().or_exch_finals_invalid(seed & 0xFFFFFFFF, U, n, len(perm), _p32(perm),
                                        _p32(finals))


def bb_values(seed: int, producers: int, items: int) -> np.ndarray:
    """Every value the bounded buffer's producers put (uint32, producer order)."""
    out = np.zeros(items, dtype=np.uint32)
    lib().or_bb_values(seed & 0xFFFFFFFF, producers, items, _p32(out))
    return out


# ---- threaded reference ----------------------------------------------------------------

def hardware_threads() -> int:
    return lib().or_hardware_threads()


def barrier_threaded(kind: str, seed: int, N: int, R: int, groups: int = 8):
    """Returns (checksums, rc, seconds); rc = -2 means a phase violation was seen."""
    out = np.zeros(N, dtype=np.uint32)
    secs = ctypes.c_double(0)
    rc = lib().or_barrier_threaded(BARRIER_KINDS[kind], seed & 0xFFFFFFFF, N, R, groups,
                                   _p32(out), ctypes.byref(secs))
    return out, rc, secs.value


def mutex_threaded(kind: str, seed: int, nwg: int, total: int, L: int, W: int,
                   imin: int = 1, imax: int = 32):
    """Returns (words[L, W], rc, seconds); rc = -2 means mutual exclusion was violated."""
    out = np.zeros(L * W, dtype=np.uint32)
    secs = ctypes.c_double(0)
    rc = lib().or_mutex_threaded(MUTEX_KINDS[kind], seed & 0xFFFFFFFF, nwg, total, L, W,
                                 imin, imax, _p32(out), ctypes.byref(secs))
    return out.reshape(L, W), rc, secs.value


def sem_threaded(kind: str, K: int, seed: int, nwg: int, total: int, imin: int = 1,
                 imax: int = 32):
    """Returns dict(chk, maxocc, state=(S-or-count, ticket, turn, admissions), rc, seconds)."""
    chk = np.zeros(nwg, dtype=np.uint32)
    maxocc = np.zeros(1, dtype=np.uint32)
    state = np.zeros(4, dtype=np.uint32)
    secs = ctypes.c_double(0)
    rc = lib().or_sem_threaded(SEM_KINDS[kind], K, seed & 0xFFFFFFFF, nwg, total, imin, imax,
                               _p32(chk), _p32(maxocc), _p32(state), ctypes.byref(secs))
    return {"chk": chk, "maxocc": int(maxocc[0]), "state": tuple(int(x) for x in state),
            "rc": rc, "seconds": secs.value}


def bench_threaded(op: str, seed: int, U: int, n: int, perm: np.ndarray, threads: int):
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    finals = np.zeros(len(perm), dtype=np.uint32)
    s = ctypes.c_uint64(0)
    secs = ctypes.c_double(0)
    rc = lib().or_bench_threaded(BENCH_OPS[op], seed & 0xFFFFFFFF, U, n, len(perm), _p32(perm),
                                 threads, _p32(finals), ctypes.byref(s), ctypes.byref(secs))
    if rc != 0:
        raise ValueError(f"or_bench_threaded({op}) failed: {rc}")
    return finals, s.value, secs.value


def serve_threaded(seed: int, lengths: np.ndarray, units: np.ndarray, K: int, agents: int):
    """Threaded serving queue; returns dict(out, maxuse, issued, released, rc, seconds)."""
    lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
    units = np.ascontiguousarray(units, dtype=np.uint32)
    out = np.zeros(len(lengths), dtype=np.uint32)
    maxuse = np.zeros(1, dtype=np.uint32)
    counters = np.zeros(2, dtype=np.uint64)
    secs = ctypes.c_double(0)
    rc = lib().or_serve_threaded(seed & 0xFFFFFFFF, _p32(lengths), _p32(units), len(lengths), K,
                                 agents, _p32(out), _p32(maxuse), _p64(counters),
                                 ctypes.byref(secs))
    return {"out": out, "maxuse": int(maxuse[0]), "issued": int(counters[0]),
            "released": int(counters[1]), "rc": rc, "seconds": secs.value}


def bb_closed(seed: int, producers: int, items: int) -> tuple[int, int]:
    """(xor, sum) of every value the bounded buffer's producers put."""
    out = np.zeros(2, dtype=np.uint64)
    lib().or_bb_closed(seed & 0xFFFFFFFF, producers, items, _p64(out))
    return int(out[0]), int(out[1])


def bb_threaded(seed: int, producers: int, consumers: int, items: int, capacity: int) -> dict:
    out = np.zeros(6, dtype=np.uint64)
    secs = ctypes.c_double(0)
    rc = lib().or_bb_threaded(seed & 0xFFFFFFFF, producers, consumers, items, capacity, _p64(out),
                              ctypes.byref(secs))
    v = [int(x) for x in out]
    return {"xor": v[0], "sum": v[1], "taken": v[2], "put": v[3], "max_count": v[4],
            "left": v[5], "rc": rc, "seconds": secs.value}
