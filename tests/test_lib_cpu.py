"""Host-side checks of libddgs.so that need no GPU: the library loads, it
exports every entry point that include/ddgs.h declares, and its pure host
functions behave (no compute call is made here)."""
import ctypes
import json
import os
import re

import pytest

from paper_2406_02518_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddgs.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2406_02518_amd import build
        build.build()
    return binding.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddgs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    assert len(names) >= 20
    assert set(names) == set(binding.EXPORTED)


def test_every_declared_symbol_is_exported(L):
    cdll = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(cdll, n)]
    assert not missing, missing


def test_param_count_matches_paper(L):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "param_count.json")))
    per, shared = binding.ddgs_param_count(g["k"], g["L"], g["n"])
    assert (per, shared) == (g["per_gaussian"], g["shared"])
    assert per * g["n"] + shared == g["total"]
    assert binding.ddgs_param_count(16, 3, 1) == (27, 16 + 15 * 16)
    with pytest.raises(binding.DDGSError):
        binding.ddgs_param_count(0, 1, 1)


def test_status_strings_and_default_options(L):
    assert binding.status_name(binding.OK) == "ok"
    assert "capacity" in binding.status_name(binding.ERR_CAPACITY)
    o = binding.ddgs_default_options()
    assert (o.tile_w, o.tile_h) == (16, 16)
    assert o.kappa == pytest.approx(3.0) and o.dilation == pytest.approx(0.3)
    assert o.sigma_max == pytest.approx(0.99) and o.t_min == 0.0 and o.z_near == pytest.approx(1.0)
    assert ctypes.sizeof(binding.ddgs_view) == 64
    assert ctypes.sizeof(binding.ddgs_options) == 48
    assert o.split == 256 and o.persistent == 0 and o.capacity == 0


def test_product_path_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "_LIB", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        binding.lib()


def test_registration_metrics():
    """The registration driver's error measures against the FP64 reference on
    random poses, and the target registration error against closed forms."""
    import numpy as np
    from scipy.spatial.transform import Rotation

    from oracle import pose_opt
    from paper_2406_02518_amd import register, synth

    rng = np.random.default_rng(21)
    pts = rng.normal(size=(50, 3)) * 30.0
    P = synth.azimuth_pose(40.0, 600.0)
    for _ in range(5):
        Q = synth.perturbed_pose(P, rng.normal(size=3) * 0.1, rng.normal(size=3) * 10.0)
        ang, dso = pose_opt.pose_errors(Q, P)
        assert register.rotation_error_deg(Q, P) == pytest.approx(ang, abs=1e-9)
        assert register.source_error_mm(Q, P) == pytest.approx(dso, rel=1e-12)
        assert register.projection_distance(Q, P, 800.0, pts) == pytest.approx(
            pose_opt.projection_distance(Q, P, 800.0, pts), rel=1e-12)
    # a shift by tau moves every point by |tau|; a rotation by a about an axis
    # through the origin moves a point at distance r from the axis by 2 r sin(a/2)
    T = P.copy()
    T[:, 3] += [3.0, 4.0, 12.0]
    assert register.target_registration_error(T, P, pts) == pytest.approx(13.0, rel=1e-12)
    Rz = P.copy()
    Rz[:, :3] = P[:, :3] @ Rotation.from_rotvec([0.0, 0.0, 0.3]).as_matrix()
    r = np.linalg.norm(pts[:, :2], axis=1)
    assert register.target_registration_error(Rz, P, pts) == pytest.approx(np.mean(2 * r * np.sin(0.15)), rel=1e-12)


def test_compose_pose_is_the_left_exponential(L):
    """ddgs_compose_pose: Exp(delta) pose with Exp from scipy's rotation-vector
    map (an independent implementation), evaluated in float64 and rounded once;
    zero tangent returns the pose, a translation tangent shifts t only, and
    the small-angle series branch agrees with the closed form."""
    import numpy as np
    from scipy.spatial.transform import Rotation

    from paper_2406_02518_amd import synth

    rng = np.random.default_rng(33)
    P = synth.azimuth_pose(25.0, 600.0).astype(np.float32)
    np.testing.assert_array_equal(binding.ddgs_compose_pose(P, np.zeros(6)), P)
    T = binding.ddgs_compose_pose(P, [1.5, -2.0, 3.25, 0.0, 0.0, 0.0])
    np.testing.assert_array_equal(T[:, :3], P[:, :3])
    np.testing.assert_allclose(T[:, 3], P[:, 3].astype(np.float64) + [1.5, -2.0, 3.25], rtol=0, atol=1e-4)
    for scale in (0.3, 1e-3, 3e-5):
        for _ in range(4):
            d = np.concatenate([rng.normal(size=3) * 10.0, rng.normal(size=3) * scale])
            E = Rotation.from_rotvec(d[3:]).as_matrix()
            P64 = P.astype(np.float64)
            want = np.concatenate([E @ P64[:, :3], (E @ P64[:, 3] + d[:3])[:, None]], axis=1)
            got = binding.ddgs_compose_pose(P, d).astype(np.float64)
            # one rounding to float32 on each side
            tol = 2.0 ** -23 * np.maximum(1.0, np.abs(want))
            assert np.all(np.abs(got - want) <= tol), (scale, np.abs(got - want).max())
    with pytest.raises(binding.DDGSError):
        binding.ddgs_compose_pose(P, [0, 0, 0, np.nan, 0, 0])
