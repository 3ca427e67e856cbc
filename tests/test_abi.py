"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, the ctypes mirrors have the C layouts, and invalid
configurations are rejected before any device work."""
import ctypes as C
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2607_06499_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cemppi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ce_mppi_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libcemppi.so not built")
    return B.load()


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layouts_match_header():
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "cemppi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(ce_mppi_config), sizeof(ce_mppi_info),
         offsetof(ce_mppi_config, seed), offsetof(ce_mppi_config, dh),
         offsetof(ce_mppi_info, margin), offsetof(ce_mppi_info, weight_sum),
         sizeof(ce_mppi_batch_io), offsetof(ce_mppi_batch_io, n_obs), offsetof(ce_mppi_batch_io, u_out),
         offsetof(ce_mppi_batch_io, info), sizeof(ce_mppi_batch_tuning));
  printf("%zu %zu %zu %zu\n", sizeof(ce_mppi_server_config), offsetof(ce_mppi_server_config, memory_budget),
         sizeof(ce_mppi_server_stats), offsetof(ce_mppi_server_stats, session_bytes));
  return 0;
}
'''
    d = tempfile.mkdtemp()
    try:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    finally:
        shutil.rmtree(d, ignore_errors=True)
    assert vals[0] == C.sizeof(B.CeMppiConfig)
    assert vals[1] == C.sizeof(B.CeMppiInfo)
    assert vals[2] == B.CeMppiConfig.seed.offset
    assert vals[3] == B.CeMppiConfig.dh.offset
    assert vals[4] == B.CeMppiInfo.margin.offset
    assert vals[5] == B.CeMppiInfo.weight_sum.offset
    assert vals[6] == C.sizeof(B.CeMppiBatchIO)
    assert vals[7] == B.CeMppiBatchIO.n_obs.offset
    assert vals[8] == B.CeMppiBatchIO.u_out.offset
    assert vals[9] == B.CeMppiBatchIO.info.offset
    assert vals[10] == C.sizeof(B.CeMppiBatchTuning)
    assert vals[11] == C.sizeof(B.CeMppiServerConfig)
    assert vals[12] == B.CeMppiServerConfig.memory_budget.offset
    assert vals[13] == C.sizeof(B.CeMppiServerStats)
    assert vals[14] == B.CeMppiServerStats.session_bytes.offset


def test_config_init_defaults(lib):
    cfg = B.ce_mppi_config_init(B.DYN_UNICYCLE)
    assert cfg.abi_version == B.ABI_VERSION and cfg.horizon == 30 and cfg.num_samples == 1024
    with pytest.raises(B.CeMppiError) as e:
        B.ce_mppi_config_init(7)
    assert e.value.status == B.CE_EINVAL


@pytest.mark.parametrize("field,value", [
    ("horizon", 0), ("horizon", 64), ("num_samples", 0), ("num_samples", 70000), ("dt", 0.0),
    ("lam", -1.0), ("dbscan_eps", 0.0), ("dbscan_min_pts", 0), ("history_len", 0),
    ("history_len", 17), ("max_obstacles", 65), ("ref_mode", 3), ("scene_mode", 2),
    ("abi_version", 99), ("dynamics", 5), ("norm_eps", float("nan")),
])
def test_invalid_config_rejected(lib, field, value):
    cfg = B.ce_mppi_config_init(B.DYN_UNICYCLE)
    setattr(cfg, field, value)
    h = C.c_void_p()
    st = lib.ce_mppi_create(C.byref(cfg), C.byref(h))
    assert st == B.CE_EINVAL, (field, value, st)
    assert h.value is None
    assert lib.ce_mppi_last_error().decode() != ""


def test_flags_validated(lib):
    h = C.c_void_p()
    cfg = B.ce_mppi_config_init(B.DYN_UNICYCLE)
    cfg.flags = 4
    assert lib.ce_mppi_create(C.byref(cfg), C.byref(h)) == B.CE_EINVAL
    cfg.flags = B.FLAG_POSE_COST  # the pose cost is an arm cost
    assert lib.ce_mppi_create(C.byref(cfg), C.byref(h)) == B.CE_EINVAL
    cfg.flags = B.FLAG_OBS_CONST_VEL
    cfg.history_len = 1  # no velocity without two observations
    assert lib.ce_mppi_create(C.byref(cfg), C.byref(h)) == B.CE_EINVAL
    assert h.value is None


def test_dynamic_scene_needs_history(lib):
    cfg = B.ce_mppi_config_init(B.DYN_UNICYCLE)
    cfg.scene_mode = B.SCENE_DYNAMIC
    cfg.history_len = 1
    h = C.c_void_p()
    assert lib.ce_mppi_create(C.byref(cfg), C.byref(h)) == B.CE_EINVAL


def test_arm_spheres_validated(lib):
    cfg = B.ce_mppi_config_init(B.DYN_ARM6)
    cfg.n_link_spheres = 17
    h = C.c_void_p()
    assert lib.ce_mppi_create(C.byref(cfg), C.byref(h)) == B.CE_EINVAL


def test_null_arguments(lib):
    assert lib.ce_mppi_create(None, None) == B.CE_EINVAL
    assert lib.ce_mppi_replan(None, None, None, 0, None, None, None, None) == B.CE_EINVAL
    lib.ce_mppi_destroy(None)  # NULL-safe
    assert B.ce_mppi_status_string(B.CE_EINVAL) == "invalid argument"
    h = C.c_void_p()
    assert lib.ce_mppi_batch_create(None, 1, C.byref(h)) == B.CE_EINVAL
    arr = (C.c_void_p * 1)(None)
    assert lib.ce_mppi_batch_create(arr, 0, C.byref(h)) == B.CE_EINVAL
    assert lib.ce_mppi_batch_create(arr, 1, C.byref(h)) == B.CE_EINVAL  # NULL member
    assert lib.ce_mppi_batch_replan(None, None, None) == B.CE_EINVAL
    t = B.CeMppiBatchTuning(3, 4, 4, 1)
    assert lib.ce_mppi_batch_set_tuning(None, C.byref(t)) == B.CE_EINVAL
    lib.ce_mppi_batch_destroy(None)  # NULL-safe
    assert lib.ce_mppi_server_create(None, None) == B.CE_EINVAL
    cfg = B.CeMppiServerConfig(0, 0, 1, 0, 0)
    assert lib.ce_mppi_server_create(C.byref(cfg), C.byref(h)) == B.CE_EINVAL  # max_batch 0
    cfg = B.CeMppiServerConfig(0, 4, 4, 0, 0)
    assert lib.ce_mppi_server_create(C.byref(cfg), C.byref(h)) == B.CE_EINVAL  # max_inflight 4
    assert lib.ce_mppi_tune_launch(None, None, None, 0, None, 1, None, None, None) == B.CE_EINVAL
    assert lib.ce_mppi_server_start(None) == B.CE_EINVAL
    assert lib.ce_mppi_server_session_planner(None, 0) is None
    lib.ce_mppi_server_destroy(None)  # NULL-safe


def test_no_device_reports_edevice(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg = B.ce_mppi_config_init(B.DYN_UNICYCLE)
    h = C.c_void_p()
    assert lib.ce_mppi_create(C.byref(cfg), C.byref(h)) == B.CE_EDEVICE
