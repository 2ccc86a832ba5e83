"""Teardown in any order: state objects that outlive their context are destroyed safely
(the context's memory stays until the last of them goes), every call on a closed context
is refused, and a process that exits with live contexts and objects ends with status 0."""

import ctypes
import os
import subprocess
import sys

import pytest

from conftest import announce

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_objects_destroyed_after_their_context():
    from paper_1110_4623_amd import _native as N
    lib = N.lib
    announce("teardown", "objects after sp_fini", "barrier, mutex, semaphore", {})
    ctx = ctypes.c_void_p()
    assert lib.sp_init(0, ctypes.byref(ctx)) == N.SP_OK
    p = N.Params()
    lib.sp_params_default(ctypes.byref(p))
    bar, mtx, sem = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.sp_barrier_create(ctx, N.BARRIER_KINDS["xcd"], 64, ctypes.byref(p),
                                 ctypes.byref(bar)) == N.SP_OK
    assert lib.sp_mutex_create(ctx, N.MUTEX_KINDS["ticket"], 1, 4, ctypes.byref(p),
                               ctypes.byref(mtx)) == N.SP_OK
    assert lib.sp_sem_create(ctx, N.SEM_KINDS["adaptive"], 4, ctypes.byref(p),
                             ctypes.byref(sem)) == N.SP_OK
    assert lib.sp_fini(ctx) == N.SP_OK
    # the context is closed: calls on it are refused, a second fini too
    assert lib.sp_fini(ctx) == N.SP_E_INVAL
    h = ctypes.c_void_p()
    assert lib.sp_barrier_create(ctx, N.BARRIER_KINDS["xcd"], 64, ctypes.byref(p),
                                 ctypes.byref(h)) == N.SP_E_INVAL
    # the objects still release their own memory, the last one the context's
    assert lib.sp_sem_destroy(sem) == N.SP_OK
    assert lib.sp_mutex_destroy(mtx) == N.SP_OK
    assert lib.sp_barrier_destroy(bar) == N.SP_OK
    # and a new context works
    ctx2 = ctypes.c_void_p()
    assert lib.sp_init(0, ctypes.byref(ctx2)) == N.SP_OK
    assert lib.sp_fini(ctx2) == N.SP_OK


def test_python_close_releases_owned_objects_first():
    import paper_1110_4623_amd as sp
    announce("teardown", "Context.close with live objects", "", {})
    c = sp.Context(0)
    b = sp.Barrier(c, "xcd", 64)
    m = sp.Mutex(c, "ticket", 1, 4)
    buf = c.zeros(1024)
    c.close()
    assert b.h is None and m.h is None
    c.close()  # idempotent
    del buf


def test_process_exit_with_live_objects():
    """A process that never closes anything: the exit handler closes the context and its
    objects before the runtime unloads."""
    announce("teardown", "process exit", "live context, barrier, mutex, semaphore, buffer", {})
    code = ("import paper_1110_4623_amd as sp\n"
            "c = sp.Context(0)\n"
            "b = sp.Barrier(c, 'xcd', 64); chk, st = b.run_hash(64, 10, 1)\n"
            "m = sp.Mutex(c, 'ticket', 1, 4); s = sp.Semaphore(c, 'adaptive', 4)\n"
            "buf = c.zeros(4096)\n"
            "print('last line', flush=True)\n")
    env = dict(os.environ, SP_NO_TORCH="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "last line" in r.stdout
