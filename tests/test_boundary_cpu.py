"""The C-ABI library on a machine without a GPU: it loads, exports every call
declared in include/gg.h, its struct layouts agree with the binding, and
argument checks reject bad input on the host before any device work."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2306_01369_amd import gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gg.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_call():
    L = gg.lib()
    names = _declared_functions()
    assert set(gg.EXPORTS) <= set(names)
    for name in names:
        assert hasattr(L, name), f"{name} declared in gg.h but not exported"


def test_struct_layouts_match_binding():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "gg.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(gg_params), sizeof(gg_body), sizeof(gg_stats));
  printf("%zu %zu %zu %zu\n", offsetof(gg_params, hash_size), offsetof(gg_params, flags),
         offsetof(gg_params, stream), offsetof(gg_body, twist));
  printf("%zu %zu\n", offsetof(gg_stats, ms_detect), offsetof(gg_stats, pja_launches));
  printf("%zu %zu %zu\n", sizeof(gg_camera), offsetof(gg_camera, pose), offsetof(gg_camera, params));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "abi.c")
        exe = os.path.join(d, "abi")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    vals = list(map(int, out))
    assert vals[0:3] == [C.sizeof(gg.Params), C.sizeof(gg.Body), C.sizeof(gg.Stats)]
    assert vals[3] == gg.Params.hash_size.offset
    assert vals[4] == gg.Params.flags.offset
    assert vals[5] == gg.Params.stream.offset
    assert vals[6] == gg.Body.twist.offset
    assert vals[7] == gg.Stats.ms_detect.offset
    assert vals[8] == gg.Stats.pja_launches.offset
    assert vals[9:12] == [C.sizeof(gg.Camera), gg.Camera.pose.offset, gg.Camera.params.offset]


def test_status_strings():
    L = gg.lib()
    for st in range(8):
        assert L.gg_status_string(st)
    assert L.gg_status_string(99) == b"unknown status"


def _create(**kw):
    n = kw.pop("n", 8)
    x = kw.pop("x", np.random.default_rng(0).uniform(0, 0.1, (n, 3)).astype(np.float32))
    v = kw.pop("v", np.zeros((n, 3), np.float32))
    r = kw.pop("r", np.full(n, 0.005, np.float32))
    return gg.Sim(x, v, r, **kw)


@pytest.mark.parametrize("kw,status", [
    ({"dt": 0.0}, gg.GG_ERR_INVALID),
    ({"dt": float("nan")}, gg.GG_ERR_INVALID),
    ({"alpha": -1.0}, gg.GG_ERR_INVALID),
    ({"mu": -0.1}, gg.GG_ERR_INVALID),
    ({"n_iters": 0}, gg.GG_ERR_INVALID),
    ({"hash_size": -5}, gg.GG_ERR_INVALID),
    ({"cell_size": 0.005}, gg.GG_ERR_INVALID),           # smaller than 2 r_max
    ({"gravity": (0.0, float("inf"), 0.0)}, gg.GG_ERR_INVALID),
    ({"max_contacts": 1000}, gg.GG_ERR_INVALID),
    ({"relax": 3.0}, gg.GG_ERR_INVALID),
    ({"r": np.array([0.005] * 7 + [0.0], np.float32)}, gg.GG_ERR_INVALID),
    ({"r": np.array([0.005] * 7 + [float("nan")], np.float32)}, gg.GG_ERR_INVALID),
    ({"x": np.array([[0, 0, float("nan")]] * 8, np.float32)}, gg.GG_ERR_NONFINITE),
    ({"v": np.array([[0, float("inf"), 0]] * 8, np.float32)}, gg.GG_ERR_NONFINITE),
    ({"x": np.array([[1e8, 0, 0]] * 8, np.float32)}, gg.GG_ERR_INVALID),   # |x/c| >= 2^30
    ({"env_offsets": [0, 3, 2, 8]}, gg.GG_ERR_INVALID),
    ({"env_offsets": [0, 3, 9]}, gg.GG_ERR_INVALID),
    ({"env_offsets": [1, 8]}, gg.GG_ERR_INVALID),
    ({"fused": True, "differentiable": True}, gg.GG_ERR_INVALID),   # the fused step keeps no tape
])
def test_create_rejects_bad_arguments_on_host(kw, status):
    with pytest.raises(gg.GGError) as e:
        _create(**kw)
    assert e.value.status == status


@pytest.mark.parametrize("precision", [2, -1])
def test_precision_other_than_binary32_or_binary64_is_rejected(precision):
    L = gg.lib()
    P = gg.Params()
    P.dt, P.n_iters, P.precision = 1e-3, 20, precision
    h = C.c_void_p()
    x = np.zeros((1, 3), np.float32)
    r = np.ones(1, np.float32)
    st = L.gg_create(C.byref(P), 1, None, 1, x.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p),
                     r.ctypes.data_as(C.c_void_p), 0, C.byref(h))
    assert st == gg.GG_ERR_INVALID
    assert h.value is None


def test_null_handle_calls_are_rejected():
    L = gg.lib()
    assert L.gg_step(None, 1, None, 0) == gg.GG_ERR_INVALID
    assert L.gg_set_bodies(None, 0, None, 0) == gg.GG_ERR_INVALID
    w = C.c_int64(0)
    assert L.gg_read(None, 0, None, 0, C.byref(w), 0) == gg.GG_ERR_INVALID
    assert L.gg_step_backward(None, None, None, None, None, None, 0) == gg.GG_ERR_INVALID
    assert L.gg_render_depth(None, 0, None, None, 0, 0) == gg.GG_ERR_INVALID
    assert L.gg_goal_reward(None, None, None, None, 0) == gg.GG_ERR_INVALID
    L.gg_destroy(None)
    assert b"NULL" in L.gg_error_detail() or L.gg_error_detail() == b"sim is NULL"


def test_create_with_null_out_is_rejected():
    L = gg.lib()
    P = gg.Params()
    P.dt, P.n_iters = 1e-3, 20
    assert L.gg_create(C.byref(P), 1, None, 0, None, None, None, 0, None) == gg.GG_ERR_INVALID


def test_body_layout_from_scene_dict():
    from paper_2306_01369_amd import scenes
    b = gg.make_body(scenes.box_tool((1, 2, 3), (0.1, 0.2, 0.3), nu=(4, 5, 6), omega=(7, 8, 9), env=2))
    assert b.env == 2 and b.shape == 1
    assert list(b.pose) == [1, 0, 0, 1, 0, 1, 0, 2, 0, 0, 1, 3]
    assert list(b.twist) == [4, 5, 6, 7, 8, 9]


def test_contact_table_beyond_32_bit_slots_is_rejected_on_host():
    # The contact table holds (n rounded up to 64) x capacity slots indexed in
    # 32-bit arithmetic on the device; 2^23 particles at the largest capacity
    # (256) make 2^31 slots, one too many.  The check runs before any device
    # work, so it needs no GPU.
    n = 1 << 23
    x = np.zeros((n, 3), np.float32)
    r = np.full(n, 0.001, np.float32)
    with pytest.raises(gg.GGError) as e:
        gg.Sim(x, x, r, max_contacts=256)
    assert e.value.status == gg.GG_ERR_INVALID
    assert "2^31" in str(e.value)
