import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running")


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _has_gpu():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


def make_custom_scene(means, scales, quats, opacity, cams, ids, feats, nseg=None,
                      feat_dtype="f32", name="custom"):
    """A Scene from explicit arrays; cams is a list of dicts with keys
    fx, fy, cx, cy, R (3x3), t (3), width, height."""
    from synthetic import Scene, camera_dtype
    C = np.zeros(len(cams), dtype=camera_dtype)
    for i, c in enumerate(cams):
        C[i]["fx"], C[i]["fy"], C[i]["cx"], C[i]["cy"] = c["fx"], c["fy"], c["cx"], c["cy"]
        C[i]["R"] = np.asarray(c.get("R", np.eye(3)), np.float32).reshape(9)
        C[i]["t"] = np.asarray(c.get("t", np.zeros(3)), np.float32)
        C[i]["width"], C[i]["height"] = c["width"], c["height"]
    ids = [np.ascontiguousarray(i, dtype=np.int32) for i in ids]
    if nseg is None:
        nseg = [int(i.max()) + 1 if i.size and i.max() >= 0 else 0 for i in ids]
    return Scene(name, 0, np.asarray(means, np.float32).reshape(-1, 3),
                 np.asarray(scales, np.float32).reshape(-1, 3),
                 np.asarray(quats, np.float32).reshape(-1, 4),
                 np.asarray(opacity, np.float32).reshape(-1),
                 C, ids, np.asarray(nseg, np.int32), feat_dtype,
                 np.ascontiguousarray(feats), {})


@pytest.fixture(scope="session")
def scene_2k():
    from synthetic import make_scene
    return make_scene("plain_fp32_2k")


@pytest.fixture(scope="session")
def oracle_2k(scene_2k):
    import oracle
    return oracle.lift(scene_2k, mode="box", pixels=True)
