"""Host-side checks of the HIP library and the input generators (no GPU):
the shared library loads and exports every entry point declared in
include/abd.h, and argument validation happens before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2605_15875_amd import abd, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "abd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = abd.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(abd.EXPORTS)


def test_create_rejects_bad_parameters_before_device_use():
    L = abd.lib()
    base = scenes.default_params()
    for key, bad in (("dt", 0.0), ("dhat", -1.0), ("kappa", 0.0),
                     ("max_newton", 0), ("pcg_eta", 0.0),
                     ("newton_theta", -1.0), ("precision", 7),
                     ("list_capacity", -1), ("mixed_switch", -1),
                     ("deterministic", 2)):
        p = dict(base)
        p[key] = bad
        h = C.c_void_p()
        rc = L.abd_create(C.byref(h), C.byref(abd.make_params(p)))
        assert rc == abd.E_INVALID_ARG, key
        assert not h.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(abd, "_lib", None)
    monkeypatch.setattr(abd, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError):
        abd.lib()


def test_scene_shapes_and_determinism():
    c0 = scenes.config(0)
    assert len(c0.bodies) == 8 and c0.n_vertices == 64 and c0.n_triangles == 96
    c1 = scenes.config(1)
    assert len(c1.bodies) == 1001
    assert c1.n_triangles == 1000 * 1280 + 10
    assert c1.bodies[0].xbar.shape == (642, 3)
    again = scenes.config(1)
    for a, b in zip(c1.bodies[:20], again.bodies[:20]):
        np.testing.assert_array_equal(a.q0, b.q0)
        np.testing.assert_array_equal(a.qdot0, b.qdot0)
    # non-overlapping placement with the requested gap
    c = np.array([b.q0[:3] for b in c1.bodies[:-1]])
    r = np.array([np.linalg.norm(b.xbar, axis=1).max() for b in c1.bodies[:-1]])
    d = np.linalg.norm(c[:, None] - c[None], axis=2) + np.eye(len(c)) * 1e9
    assert np.all(d >= r[:, None] + r[None, :] + 0.01 - 1e-12)


def test_hull_scene_worker_share():
    sc = scenes.hulls_in_funnel_scene(0, n_bodies=300, n_lo=30, n_hi=60,
                                      n_shared=25)
    assert sc.shared_ids is not None and len(sc.shared_ids) >= 20
    for b in sc.bodies[:-1]:
        assert b.tris.shape[0] == 2 * b.xbar.shape[0] - 4
