"""The C ABI library loads and exports every entry point include/sp.h declares (CPU:
loading only, no compute calls)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^(?:int|void|uint32_t|const char\*)\s+(sp_\w+)\(", text,
                                re.M)
    return names


def test_header_declares_entry_points():
    names = _declared()
    assert len(names) >= 20
    assert len(names) == len(set(names))


def test_library_exports_every_declared_symbol():
    from paper_1110_4623_amd import _native
    missing = [n for n in _declared() if not hasattr(_native.lib, n)]
    assert not missing, missing


def test_error_strings():
    from paper_1110_4623_amd import _native
    lib = _native.lib
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.sp_strerror(code).decode()
    assert lib.sp_strerror(-99).decode() == "unknown error"


def test_params_default_roundtrip():
    import ctypes
    from paper_1110_4623_amd import _native, api
    p = api.make_params(backoff="paper", backoff_min=2, backoff_max=64, poll_sleep=3)
    assert (p.backoff, p.backoff_min, p.backoff_max, p.poll_sleep) == (1, 2, 64, 3)
    assert p.pad_bytes == 128 and p.timeout_ms == 20000 and p.xcd_copies == 64
    assert p.flag_placement == 0 and p.cohort_passes in (0, 64)
    assert ctypes.sizeof(_native.Params) == 76
    assert ctypes.sizeof(_native.Stats) == 64


def test_bad_arguments_rejected_without_gpu():
    import ctypes
    from paper_1110_4623_amd import _native
    lib = _native.lib
    h = ctypes.c_void_p()
    # null context / null out pointers are argument errors, checked before any HIP call
    assert lib.sp_barrier_create(None, 0, 16, None, ctypes.byref(h)) == _native.SP_E_INVAL
    assert lib.sp_mutex_create(None, 0, 1, 1, None, ctypes.byref(h)) == _native.SP_E_INVAL
    assert lib.sp_sem_create(None, 0, 1, None, ctypes.byref(h)) == _native.SP_E_INVAL
    assert lib.sp_fini(None) == _native.SP_E_INVAL
    assert lib.sp_barrier_run_hash(None, 64, 1, 0, None, None, None) == _native.SP_E_INVAL


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of the C structs have the sizes and field offsets a C compiler
    gives them from include/sp.h."""
    import ctypes
    import subprocess
    from paper_1110_4623_amd import _native as N
    structs = {"sp_params": N.Params, "sp_stats": N.Stats, "sp_device_info": N.DeviceInfo,
               "sp_serve_cfg": N.ServeCfg, "sp_serve_result": N.ServeResult,
               "sp_barrier_info": N.BarrierInfo, "sp_occupancy": N.Occupancy}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "sp.h"', "int main(void) {"]
    for cname, py in structs.items():
        src.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            src.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append("  return 0;\n}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o",
                           str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).split("\n")
               if line)
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_serve_rejects_bad_tables_without_gpu():
    import ctypes
    from paper_1110_4623_amd import _native as N
    c = N.ServeCfg()
    r = N.ServeResult()
    assert N.lib.sp_serve_run(None, ctypes.byref(c), 1, None, None, None, None, None,
                              ctypes.byref(r)) == N.SP_E_INVAL
    assert N.lib.sp_serve_run_launch_per_request(None, ctypes.byref(c), 1, None, None, None,
                                                 None, None, ctypes.byref(r)) == N.SP_E_INVAL


def test_newer_entry_points_reject_bad_arguments_without_gpu():
    import ctypes
    from paper_1110_4623_amd import _native as N
    lib = N.lib
    st = N.Stats()
    p = N.Params()
    lib.sp_params_default(ctypes.byref(p))
    # no context / no output / no consumers: argument errors before any HIP call
    assert lib.sp_cond_run_bounded_buffer(None, 3, 4, 2, 64, 8, 100, 1, ctypes.byref(p), None,
                                          None, ctypes.byref(st), None) == N.SP_E_INVAL
    g = ctypes.c_void_p()
    assert lib.sp_graph_begin(None, None, ctypes.byref(g)) == N.SP_E_INVAL
    assert lib.sp_graph_end(None, None, ctypes.byref(g)) == N.SP_E_INVAL
    assert lib.sp_graph_launch(None, 1, ctypes.byref(st), None) == N.SP_E_INVAL
    assert lib.sp_graph_destroy(None) == N.SP_E_INVAL
    info = N.BarrierInfo()
    assert lib.sp_barrier_info_get(None, ctypes.byref(info)) == N.SP_E_INVAL


def test_kind_tables_match_the_header():
    """The Python name -> kind maps use the enum values include/sp.h defines."""
    import re
    from paper_1110_4623_amd import _native as N
    text = open(os.path.join(ROOT, "include", "sp.h")).read()
    enum = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(SP_\w+)\s*=\s*(\d+)", text)}
    for prefix, table in (("SP_BARRIER_", N.BARRIER_KINDS), ("SP_MUTEX_", N.MUTEX_KINDS),
                          ("SP_SEM_", N.SEM_KINDS)):
        for name, value in table.items():
            assert enum[prefix + name.upper()] == value, (prefix, name)


def test_pingpong_mode_bits_match_the_header():
    import re
    from paper_1110_4623_amd import _native as N
    text = open(os.path.join(ROOT, "include", "sp.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in
            re.finditer(r"#define\s+(SP_PINGPONG_\w+)\s+(\d+)u", text)}
    assert defs == {"SP_PINGPONG_FENCED": N.PINGPONG_FENCED,
                    "SP_PINGPONG_SAME_XCD": N.PINGPONG_SAME_XCD}


def test_pingpong_rejects_bad_arguments_without_gpu():
    import ctypes
    from paper_1110_4623_amd import _native as N
    st = N.Stats()
    assert N.lib.sp_bench_pingpong(None, 10, 0, None, None, ctypes.byref(st), None) == N.SP_E_INVAL


def test_pingpong_offset_must_be_whole_lines():
    """The binding checks the word offset before it touches the device."""
    import paper_1110_4623_amd as sp
    for bad in (-128, 100, 4095):
        with pytest.raises(ValueError):
            sp.pingpong(None, 10, offset_bytes=bad)


def _resident(runtime, vgprs, lds, lanes):
    import ctypes
    from paper_1110_4623_amd import _native as N
    o = N.Occupancy(runtime_per_cu=runtime, vgprs=vgprs, lds_bytes=lds, lanes=lanes)
    return N.lib.sp_resident_per_cu(ctypes.byref(o))


def test_residency_takes_the_smaller_of_runtime_and_own_budget():
    """A fake occupancy provider: the runtime's figure is trusted only as far as the
    kernel's own VGPR and LDS use allows (8 waves and 512 VGPRs per SIMD, 4 SIMDs,
    160 KiB of LDS per CU)."""
    import ctypes
    from paper_1110_4623_amd import _native as N
    # 256 lanes = 4 wavefronts, one per SIMD: 8 workgroups per CU when registers allow
    assert _resident(8, 64, 0, 256) == 8
    # the runtime over-reports: 72 VGPRs leave 512 // 72 = 7 waves per SIMD
    assert _resident(8, 72, 0, 256) == 7
    # 2048 workgroups of 256 lanes then do not fit 256 CUs: a run refuses
    assert _resident(8, 72, 0, 256) * 256 < 2048
    # VGPRs round up to granules of 8: 65 counts as 72
    assert _resident(8, 65, 0, 256) == 7
    # LDS: 48 KiB per workgroup leaves 3 per CU; 40000 B rounds up to 40448 -> 4
    assert _resident(8, 32, 48 * 1024, 256) == 3
    assert _resident(8, 32, 40000, 256) == 4
    # one-wave workgroups: 4 SIMDs x 8 waves, capped by the runtime
    assert _resident(32, 32, 0, 64) == 32
    assert _resident(20, 32, 0, 64) == 20
    # 1024 lanes = 16 wavefronts: 2 per CU at 8 waves per SIMD
    assert _resident(2, 32, 0, 1024) == 2
    assert _resident(0, 32, 0, 256) == 0
    assert _resident(8, 32, 0, 0) == 0
    assert N.lib.sp_resident_per_cu(None) == 0
