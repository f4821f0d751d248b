"""The seeded generators are deterministic and produce the stated shapes."""

import numpy as np

from synth import configs, splitmix64_uniforms


def test_box_room_shapes_and_determinism():
    a = configs.box_room(N=32)
    b = configs.box_room(N=32)
    assert a["grid"].shape == (128, 128, 128) and a["grid"].dtype == np.float32
    assert a["scan"].shape == (512, 3) and a["poses"].shape == (32, 7)
    assert np.array_equal(a["grid"], b["grid"]) and np.array_equal(a["scan"], b["scan"])
    assert np.array_equal(a["poses"], b["poses"]) and a["u"] == b["u"]
    assert np.all(a["poses"][:, 3] >= 0)
    assert np.allclose(np.linalg.norm(a["poses"][:, 3:], axis=1), 1, atol=1e-6)


def test_scan_points_lie_on_surfaces():
    c = configs.box_room(N=4)
    from synth.geometry import quat_to_matrix
    R = quat_to_matrix(c["q_true"])
    world = c["scan"].astype(np.float64) @ R.T + c["t_true"]
    d = c["scene"].distance(world)
    assert np.percentile(d, 99) < 0.08          # 2 cm range noise, 4 sigma


def test_splitmix_stream():
    u = splitmix64_uniforms(1234, 1000)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.05
    assert np.array_equal(u, splitmix64_uniforms(1234, 1000))
