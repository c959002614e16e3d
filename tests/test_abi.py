"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed); argument errors are reported without a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(slag_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import paper_2505_08124_amd as slag
    L = slag.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(slag.EXPORTS)


def test_null_arguments_are_rejected():
    import paper_2505_08124_amd as slag
    L = slag.lib()
    assert L.slag_create(0, None, None, None) == slag.SLAG_E_INVALID_ARG
    assert L.slag_lift(None) == slag.SLAG_E_INVALID_ARG
    assert L.slag_get_stats(None, None) == slag.SLAG_E_INVALID_ARG
    assert L.slag_codec_clear_pool(None) == slag.SLAG_E_INVALID_ARG
    assert L.slag_lift_codec(None) == slag.SLAG_E_INVALID_ARG
    assert L.slag_codec_train(None, None, None) == slag.SLAG_E_INVALID_ARG
    assert L.slag_stage_name(6) == b"composite"
    assert L.slag_stage_name(10) == b"decode"
    assert L.slag_get_tuning(None, None, 0, None) == slag.SLAG_E_INVALID_ARG
    assert L.slag_variant_name(0).startswith(b"occupancy")
    assert L.slag_stage_name(99) == b""


def test_oracle_library_loads():
    import oracle
    assert oracle.max_threads() >= 1


def test_camera_layout_matches_generator():
    import paper_2505_08124_amd as slag
    from synthetic import camera_dtype
    assert ctypes.sizeof(slag.slag_camera) == camera_dtype.itemsize == 72
    for name, _ in slag.slag_camera._fields_:
        assert getattr(slag.slag_camera, name).offset == camera_dtype.fields[name][1]
