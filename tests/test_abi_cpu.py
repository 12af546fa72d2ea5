"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/tb.h declares, and rejects bad configurations before
touching a device."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "tb.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tb_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2112_11991_amd as tb

    names = _declared()
    assert "tb_plan" in names and "tb_get_candidates" in names and len(names) >= 10
    for n in names:
        assert hasattr(tb._L, n), n
    assert sorted(tb.EXPORTS) == names


def test_default_config_and_strerror():
    import paper_2112_11991_amd as tb

    c = tb.tb_default_config()
    assert (c.max_log2n, c.harm_max, c.whiten_window, c.threshold_sigma, c.fmin_hz) == (24, 16, 4096, 6.0, 1.0)
    assert c.ring_capacity == 1 << 20 and c.device == 0 and not c.stream
    assert tb.tb_strerror(tb.TB_OK) == "ok"
    assert "budget" in tb.tb_strerror(tb.TB_ERR_BUDGET)
    assert tb.tb_strerror(-99) == "unknown status"


@pytest.mark.parametrize(
    "field,value",
    [("max_log2n", 9), ("max_log2n", 25), ("harm_max", 3), ("harm_max", 32), ("whiten_window", 0),
     ("whiten_window", 8193), ("threshold_sigma", float("nan")), ("fmin_hz", -1.0), ("ring_capacity", 0),
     ("flags", 2), ("flags", 0x80000001), ("tile_points", 4096), ("tile_points", 12288), ("lanes", 0), ("lanes", 17)],
)
def test_plan_rejects_bad_config(field, value):
    import paper_2112_11991_amd as tb

    c = tb.tb_default_config()
    setattr(c, field, value)
    with pytest.raises(tb.TbError) as e:
        tb.tb_plan(c)
    assert e.value.status == tb.TB_ERR_INVALID_ARG


def test_null_plan_calls_are_rejected():
    import ctypes as C

    import paper_2112_11991_amd as tb

    L = tb._L
    n = C.c_uint64(0)
    assert L.tb_poll(None, 1) == tb.TB_ERR_INVALID_ARG
    assert L.tb_get_candidates(None, 1, None, 0, C.byref(n), 1) == tb.TB_ERR_INVALID_ARG
    assert L.tb_release(None, 1) == tb.TB_ERR_INVALID_ARG
    assert L.tb_destroy(None) == tb.TB_OK
    assert L.tb_plan(None, None) == tb.TB_ERR_INVALID_ARG
    assert L.tb_serve(None, None, 0, 1.0, 0, None, 0, None, None) == tb.TB_ERR_INVALID_ARG
