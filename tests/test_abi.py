"""The C-ABI library loads, exports every symbol include/dsmc.h declares, and its
host-side argument checks reject bad input before any device work (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsmc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(dsmc_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ("dsmc_plan", "dsmc_smooth", "dsmc_smooth_batch", "dsmc_smooth_conditional",
              "dsmc_model_create",
              "dsmc_server_create", "dsmc_submit", "dsmc_poll", "dsmc_cancel",
              "dsmc_schedule", "dsmc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2202_02264_amd import dsmc
    lib = C.CDLL(dsmc.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors have the header's layout: compile a C probe with gcc
    that prints sizeof/offsetof of every field and compare."""
    import shutil
    import subprocess
    from paper_2202_02264_amd import dsmc
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [dsmc.dsmc_model_callbacks, dsmc.dsmc_model_desc, dsmc.dsmc_plan_desc, dsmc.dsmc_output, dsmc.dsmc_profile,
               dsmc.dsmc_server_desc, dsmc.dsmc_job]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dsmc.h"', "int main(void){"]
    for s in structs:
        lines.append(f'printf("%zu\\n", sizeof({s.__name__}));')
        for f in s._fields_:
            lines.append(f'printf("%zu\\n", offsetof({s.__name__}, {f[0]}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for s in structs:
        want.append(C.sizeof(s))
        want.extend(getattr(s, f[0]).offset for f in s._fields_)
    assert got == want


def test_invalid_arguments_rejected_on_host():
    from paper_2202_02264_amd import dsmc
    lib = dsmc._lib
    d = dsmc.dsmc_model_desc()
    h = C.c_void_p()
    d.K = 0
    assert lib.dsmc_model_create(C.byref(d), C.byref(h)) == dsmc.DSMC_EINVAL
    assert "K must be" in lib.dsmc_last_error().decode()
    d.K, d.d_x, d.d_y = 4, 64, 1
    assert lib.dsmc_model_create(C.byref(d), C.byref(h)) == dsmc.DSMC_EINVAL
    d.d_x = 1
    assert lib.dsmc_model_create(C.byref(d), C.byref(h)) == dsmc.DSMC_EINVAL  # missing arrays
    one = np.ones(4)
    for f in ("m0", "P0_chol", "F", "f", "Q_chol", "y", "q_mean", "q_chol"):
        setattr(d, f, one.ctypes.data_as(C.POINTER(C.c_double)))
    d.obs_kind = 7
    assert lib.dsmc_model_create(C.byref(d), C.byref(h)) == dsmc.DSMC_EINVAL
    d.obs_kind = dsmc.DSMC_OBS_STOCH_VOL
    d.weighting = 5
    assert lib.dsmc_model_create(C.byref(d), C.byref(h)) == dsmc.DSMC_EINVAL
    d.weighting = 0
    bad = np.array([1.0, np.nan, 1.0, 1.0])
    d.q_mean = bad.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.dsmc_model_create(C.byref(d), C.byref(h)) == dsmc.DSMC_EINVAL
    p = dsmc.dsmc_plan_desc()
    hp = C.c_void_p()
    p.N, p.d_x, p.max_K = 0, 1, 4
    assert lib.dsmc_plan(C.byref(p), C.byref(hp)) == dsmc.DSMC_EUNSUPPORTED
    p.N = dsmc.DSMC_MAX_N + 1
    assert lib.dsmc_plan(C.byref(p), C.byref(hp)) == dsmc.DSMC_EUNSUPPORTED
    p.N, p.precision = 64, 9
    assert lib.dsmc_plan(C.byref(p), C.byref(hp)) == dsmc.DSMC_EUNSUPPORTED
    p.precision, p.d_x = dsmc.DSMC_BF16, 8  # bf16 matrix-core rows need d_x >= 9
    assert lib.dsmc_plan(C.byref(p), C.byref(hp)) == dsmc.DSMC_EUNSUPPORTED
    p.precision, p.d_x = dsmc.DSMC_FP32, 1
    p.resampling = 3                        # unknown resampling scheme
    assert lib.dsmc_plan(C.byref(p), C.byref(hp)) == dsmc.DSMC_EINVAL
    p.resampling, p.lazy_param = dsmc.DSMC_RESAMPLE_MH, -1
    assert lib.dsmc_plan(C.byref(p), C.byref(hp)) == dsmc.DSMC_EINVAL
    p.lazy_param, p.precision, p.d_x = 0, dsmc.DSMC_BF16, 32  # lazy plans run no matrix-core rows
    assert lib.dsmc_plan(C.byref(p), C.byref(hp)) == dsmc.DSMC_EUNSUPPORTED
    p.resampling, p.precision, p.d_x = dsmc.DSMC_RESAMPLE_EXACT, dsmc.DSMC_FP32, 1
    assert lib.dsmc_smooth(None, None, 0, None) == dsmc.DSMC_EINVAL
    assert lib.dsmc_smooth_conditional(None, None, 0, None, None) == dsmc.DSMC_EINVAL
    assert lib.dsmc_smooth_batch_conditional(None, 1, None, None, None, None) == dsmc.DSMC_EINVAL
    # serving entry points
    sd = dsmc.dsmc_server_desc()
    hs = C.c_void_p()
    sd.precision = 9
    assert lib.dsmc_server_create(C.byref(sd), C.byref(hs)) == dsmc.DSMC_EUNSUPPORTED
    assert lib.dsmc_server_create(None, C.byref(hs)) == dsmc.DSMC_EINVAL
    jid = C.c_uint64()
    job = dsmc.dsmc_job()
    assert lib.dsmc_submit(None, C.byref(job), C.byref(jid)) == dsmc.DSMC_EINVAL
    assert lib.dsmc_poll(None, 1, None) == dsmc.DSMC_EINVAL
    assert lib.dsmc_cancel(None, 1) == dsmc.DSMC_EINVAL
    assert lib.dsmc_job_times(None, 1, None, None, None) == dsmc.DSMC_EINVAL
