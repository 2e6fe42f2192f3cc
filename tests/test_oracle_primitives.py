"""Pins of the CPU oracle's primitives against closed forms, finite
differences, library routines and brute force (no GPU)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import lsq_linear, minimize

from oracle import oracle as O
from paper_2605_15875_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- barrier
def test_barrier_golden_values():
    """b(d) = -(d - dhat)^2 ln(d / dhat) (IPC barrier on the unsquared
    distance); values written out from the closed form."""
    with open(os.path.join(GOLDEN, "barrier_values.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        b = O.barrier(case["d"], case["dhat"])
        assert b[0] == pytest.approx(case["b"], rel=1e-14, abs=0)


def test_barrier_vanishes_at_dhat_and_is_convex():
    dh = 1e-3
    assert np.all(O.barrier(dh, dh) == 0.0)
    assert np.all(O.barrier(2 * dh, dh) == 0.0)
    for d in np.geomspace(1e-9, dh * (1 - 1e-9), 200):
        b, b1, b2 = O.barrier(d, dh)
        assert b > 0 and b1 < 0 and b2 > 0


def test_barrier_derivatives_fd():
    dh = 1e-3
    for d in np.linspace(0.05 * dh, 0.95 * dh, 19):
        e = 1e-6 * d
        bp, bm = O.barrier(d + e, dh), O.barrier(d - e, dh)
        b = O.barrier(d, dh)
        assert b[1] == pytest.approx((bp[0] - bm[0]) / (2 * e), rel=1e-6)
        assert b[2] == pytest.approx((bp[1] - bm[1]) / (2 * e), rel=1e-6)
    # C2 at dhat: value, slope and curvature all reach zero continuously
    b = O.barrier(dh * (1 - 1e-6), dh)
    assert abs(b[0]) < 1e-20 and abs(b[1]) < 1e-14 and abs(b[2]) < 1e-5


# -------------------------------------------------------------- distances
def _rng():
    return np.random.default_rng(1234)


def _pt_config(kind, rng):
    """Point-triangle configurations that land in a chosen feature."""
    t = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1]])
    t = t + rng.normal(0, 0.05, t.shape)
    c = t.mean(axis=0)
    n = np.cross(t[1] - t[0], t[2] - t[0])
    n /= np.linalg.norm(n)
    if kind == "interior":
        p = c + n * rng.uniform(0.05, 0.5) + 0.05 * (t[1] - c)
    elif kind == "edge":
        m = 0.5 * (t[0] + t[1])
        out = m - c
        p = m + 0.4 * out + n * rng.uniform(-0.3, 0.3)
    else:
        out = t[2] - c
        p = t[2] + 0.5 * out + n * rng.uniform(-0.3, 0.3)
    return np.concatenate([p, t.reshape(-1)])


def _ee_config(kind, rng):
    a0 = np.array([0.0, 0.0, 0.0])
    a1 = np.array([1.0, 0.0, 0.0])
    if kind == "interior":
        b0 = np.array([0.5, -0.5, 0.2])
        b1 = np.array([0.4, 0.6, 0.3])
    elif kind == "edge":
        b0 = np.array([0.5, 0.3, 0.2])
        b1 = np.array([0.6, 1.0, 0.5])
    else:
        b0 = np.array([1.3, 0.2, 0.1])
        b1 = np.array([2.0, 0.9, 0.4])
    x = np.concatenate([a0, a1, b0, b1]) + rng.normal(0, 0.01, 12)
    return x


PT_TYPES = {"interior": {6}, "edge": {3, 4, 5}, "vertex": {0, 1, 2}}
EE_TYPES = {"interior": {8}, "edge": {4, 5, 6, 7}, "vertex": {0, 1, 2, 3}}


def _ref_point_segment(p, a, b):
    r = lsq_linear(np.asarray((b - a)).reshape(3, 1), p - a, bounds=(0, 1),
                   method="bvls", tol=1e-15)
    s = r.x[0]
    return np.linalg.norm(p - (a + s * (b - a)))


def _ref_pt(x):
    p, t0, t1, t2 = x.reshape(4, 3)
    best = min(_ref_point_segment(p, t0, t1), _ref_point_segment(p, t1, t2),
               _ref_point_segment(p, t2, t0))
    f = lambda b: np.sum((p - (t0 + b[0] * (t1 - t0) + b[1] * (t2 - t0))) ** 2)
    cons = [{"type": "ineq", "fun": lambda b: 1 - b[0] - b[1]}]
    for s0 in ([0.3, 0.3], [0.1, 0.1], [0.6, 0.2], [0.2, 0.6]):
        r = minimize(f, s0, method="SLSQP", bounds=[(0, 1), (0, 1)],
                     constraints=cons,
                     options={"ftol": 1e-16, "maxiter": 500})
        best = min(best, math.sqrt(max(r.fun, 0.0)))
    return best


def _ref_ee(x):
    a0, a1, b0, b1 = x.reshape(4, 3)
    A = np.stack([a1 - a0, -(b1 - b0)], axis=1)
    r = lsq_linear(A, b0 - a0, bounds=(0, 1), method="bvls", tol=1e-15)
    s, t = r.x
    return np.linalg.norm(a0 + s * (a1 - a0) - (b0 + t * (b1 - b0)))


@pytest.mark.parametrize("kind", ["interior", "edge", "vertex"])
def test_pt_distance_matches_bruteforce(kind):
    rng = _rng()
    for _ in range(20):
        x = _pt_config(kind, rng)
        D, _, _, dt = O.sqdist(O.PT, x)
        assert dt in PT_TYPES[kind]
        ref = _ref_pt(x)
        assert math.sqrt(D) == pytest.approx(ref, rel=1e-8, abs=1e-12)
        # dense samples never come closer than the oracle's distance
        u = rng.uniform(0, 1, (4000, 2))
        u = np.where(u.sum(1, keepdims=True) > 1, 1 - u, u)
        p, t0, t1, t2 = x.reshape(4, 3)
        pts = t0 + u[:, :1] * (t1 - t0) + u[:, 1:] * (t2 - t0)
        assert np.min(np.linalg.norm(pts - p, axis=1)) >= math.sqrt(D) - 1e-12


@pytest.mark.parametrize("kind", ["interior", "edge", "vertex"])
def test_ee_distance_matches_bruteforce(kind):
    rng = _rng()
    for _ in range(20):
        x = _ee_config(kind, rng)
        D, _, _, dt = O.sqdist(O.EE, x)
        assert dt in EE_TYPES[kind]
        ref = _ref_ee(x)
        assert math.sqrt(D) == pytest.approx(ref, rel=1e-8, abs=1e-12)


def test_distance_special_cases():
    # point straight above the triangle interior: distance = height
    x = np.array([0.25, 0.25, 0.37, 0, 0, 0, 1, 0, 0, 0, 1, 0], float)
    D, _, _, dt = O.sqdist(O.PT, x)
    assert dt == 6 and math.sqrt(D) == pytest.approx(0.37, rel=1e-15)
    # parallel segments offset by h: distance = h (line-line degenerate)
    h = 3e-4
    x = np.array([0, 0, 0, 1, 0, 0, 0.2, h, 0, 0.8, h, 0], float)
    D, _, _, dt = O.sqdist(O.EE, x)
    assert math.sqrt(D) == pytest.approx(h, rel=1e-12)
    # coincident endpoints: distance 0
    x = np.array([0, 0, 0, 1, 0, 0, 1, 0, 0, 1, 1, 1], float)
    D, _, _, _ = O.sqdist(O.EE, x)
    assert D == 0.0


def _fd_grad(f, x, eps):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = eps
        g[i] = (f(x + e) - f(x - e)) / (2 * eps)
    return g


@pytest.mark.parametrize("pk", [O.PT, O.EE])
@pytest.mark.parametrize("kind", ["interior", "edge", "vertex"])
def test_sqdist_derivatives_fd(pk, kind):
    rng = _rng()
    cfg = _pt_config if pk == O.PT else _ee_config
    for _ in range(5):
        x = cfg(kind, rng)
        D, g, H, dt = O.sqdist(pk, x)
        gf = _fd_grad(lambda y: O.sqdist(pk, y)[0], x, 1e-6)
        np.testing.assert_allclose(g, gf, rtol=1e-6, atol=1e-8 * np.abs(g).max())
        Hf = np.stack([_fd_grad(lambda y: O.sqdist(pk, y)[1][i], x, 1e-6)
                       for i in range(12)])
        np.testing.assert_allclose(H, Hf, rtol=1e-5,
                                   atol=1e-7 * np.abs(H).max())
        np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())


def _scaled_pt(rng, d):
    """PT pair at distance ~d inside the plane region, small size."""
    x = _pt_config("interior", rng)
    p, t = x[:3], x[3:].reshape(3, 3)
    n = np.cross(t[1] - t[0], t[2] - t[0])
    n /= np.linalg.norm(n)
    c = t.mean(0)
    p = c + 0.1 * (t[0] - c) + d * n
    return np.concatenate([p, t.reshape(-1)]) * 0.05


@pytest.mark.parametrize("pk", [O.PT, O.EE])
def test_pair_energy_fd(pk):
    rng = _rng()
    dh = 1e-3
    w = 1e-4 * 1e5
    for trial in range(6):
        if pk == O.PT:
            x = _scaled_pt(rng, rng.uniform(0.2, 0.8) * dh / 0.05)
            ex = 0.0
        else:
            # near-parallel edges so the mollifier is active
            a0, a1 = np.zeros(3), np.array([0.1, 0, 0])
            ang = 1e-3 * rng.uniform(0.2, 1.0)
            dd = rng.uniform(0.2, 0.8) * dh
            b0 = np.array([0.03, dd, -0.05 * math.sin(ang)])
            b1 = b0 + 0.1 * np.array([math.cos(ang), 0, math.sin(ang)])
            x = np.concatenate([a0, a1, b0, b1]) + rng.normal(0, 1e-6, 12)
            ex = 1e-3 * 0.1 ** 2 * 0.1 ** 2
        r = O.pair_eval(pk, x, ex, dh, w, project=False)
        assert r["active"]
        f = lambda y: O.pair_eval(pk, y, ex, dh, w, False)["E"]
        eps = 1e-4 * r["d"]
        gf = _fd_grad(f, x, eps)
        sc = np.abs(r["g"]).max()
        np.testing.assert_allclose(r["g"], gf, rtol=1e-5, atol=1e-6 * sc)
        Hf = np.stack([_fd_grad(lambda y: O.pair_eval(pk, y, ex, dh, w,
                                                      False)["g"][i], x, eps)
                       for i in range(12)])
        sh = np.abs(r["H"]).max()
        np.testing.assert_allclose(r["H"], Hf, rtol=1e-4, atol=1e-5 * sh)
        if pk == O.EE:
            # mollifier really engaged: energy below the unmollified one
            r0 = O.pair_eval(pk, x, 0.0, dh, w, project=False)
            assert r["E"] < r0["E"]


def test_pair_energy_translation_invariant_and_psd():
    rng = _rng()
    dh = 1e-3
    x = _scaled_pt(rng, 0.5 * dh / 0.05)
    r = O.pair_eval(O.PT, x, 0.0, dh, 10.0, project=True)
    T = np.tile(np.eye(3), (4, 1))  # uniform translations
    assert np.abs(r["g"].reshape(4, 3).sum(0)).max() < 1e-9 * np.abs(r["g"]).max()
    assert np.abs(r["H"] @ T).max() < 1e-8 * np.abs(r["H"]).max()
    w = np.linalg.eigvalsh(r["H"])
    assert w.min() > -1e-10 * w.max()


# ----------------------------------------------------------------- PSD
def test_psd_matches_numpy_eigh():
    rng = _rng()
    for n in (3, 9, 12):
        for _ in range(10):
            A = rng.normal(size=(n, n))
            A = A + A.T
            A *= 10 ** rng.uniform(-3, 6)
            w, V = np.linalg.eigh(A)
            ref = (V * np.maximum(w, 0)) @ V.T
            out = O.psd(A)
            np.testing.assert_allclose(out, ref, atol=1e-12 * np.abs(A).max())
            ew, _ = O.eig(A)
            np.testing.assert_allclose(np.sort(ew), w,
                                       atol=1e-12 * np.abs(A).max())


# --------------------------------------------------------- orthogonality
def test_orth_zero_at_rotations():
    rng = _rng()
    for _ in range(10):
        R = scenes.random_rotation(rng)
        E, g, H = O.orth(R.reshape(-1))
        assert E < 1e-28 and np.abs(g).max() < 1e-14


def test_orth_uniform_scale_closed_form():
    for s in (0.5, 0.9, 1.0, 1.1, 2.0):
        E, g, _ = O.orth((s * np.eye(3)).reshape(-1))
        assert E == pytest.approx(3 * (s * s - 1) ** 2, rel=1e-13, abs=1e-30)
        # gradient 4 (s^2 - 1) s I
        np.testing.assert_allclose(g, (4 * (s * s - 1) * s * np.eye(3)).reshape(-1),
                                   atol=1e-13)


def test_orth_fd_and_projection():
    rng = _rng()
    for _ in range(5):
        A = np.eye(3) + rng.normal(0, 0.2, (3, 3))
        E, g, H = O.orth(A.reshape(-1))
        f = lambda a: O.orth(a)[0]
        gf = _fd_grad(f, A.reshape(-1), 1e-6)
        np.testing.assert_allclose(g, gf, rtol=1e-7, atol=1e-9)
        Hf = np.stack([_fd_grad(lambda a: O.orth(a)[1][i], A.reshape(-1),
                                1e-6) for i in range(9)])
        np.testing.assert_allclose(H, Hf, rtol=1e-6, atol=1e-8)
        _, _, Hp = O.orth(A.reshape(-1), project=True)
        w, V = np.linalg.eigh(H)
        np.testing.assert_allclose(Hp, (V * np.maximum(w, 0)) @ V.T,
                                   atol=1e-11 * np.abs(H).max())


# ------------------------------------------------------------- mass
def test_unit_cube_mass_closed_form():
    v, t = scenes.cube_mesh(0.5)
    rho = 1000.0
    M, vol = O.mass_props(v, t, rho)
    assert vol == pytest.approx(1.0, rel=1e-15)
    ref = np.diag([rho, rho / 12, rho / 12, rho / 12])
    np.testing.assert_allclose(M, ref, atol=1e-12)
    # shifted cube: first moment m c, second moment rho/12 I + m c c^T
    c = np.array([0.3, -1.2, 2.5])
    M2, _ = O.mass_props(v + c, t, rho)
    np.testing.assert_allclose(M2[0, 1:], rho * c, rtol=1e-13)
    np.testing.assert_allclose(M2[1:, 1:], rho / 12 * np.eye(3) +
                               rho * np.outer(c, c), rtol=1e-12, atol=1e-9)


def test_icosphere_mass_matches_hull_volume_and_sphere_limit():
    from scipy.spatial import ConvexHull
    for lvl in (2, 3, 4):
        v, t = scenes.icosphere_mesh(lvl, 0.1)
        M, vol = O.mass_props(v, t, 1000.0)
        assert vol == pytest.approx(ConvexHull(v).volume, rel=1e-12)
    # level 4 is close to the sphere: V -> 4/3 pi r^3, int x^2 -> 4 pi r^5/15
    r = 0.1
    assert vol == pytest.approx(4 / 3 * math.pi * r ** 3, rel=5e-3)
    assert M[1, 1] / 1000.0 == pytest.approx(4 * math.pi * r ** 5 / 15,
                                             rel=1e-2)
    assert abs(M[1, 2]) < 1e-12 and abs(M[0, 1]) < 1e-12


def test_second_moment_independent_decomposition():
    """Same integrals with tetrahedra fanned from a far apex (numpy)."""
    rng = _rng()
    sc = scenes.hulls_in_funnel_scene(0, n_bodies=3, n_lo=40, n_hi=60,
                                      worker_share=False)
    for b in sc.bodies[:3]:
        v, t = b.xbar, b.tris
        M, vol = O.mass_props(v, t, 700.0)
        apex = rng.normal(0, 1.0, 3)
        a, bb, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
        vt = np.einsum("ij,ij->i", a - apex, np.cross(bb - apex, c - apex)) / 6
        s = apex + a + bb + c
        sec = sum(vt[i] / 20 * (np.outer(apex, apex) + np.outer(a[i], a[i]) +
                                np.outer(bb[i], bb[i]) + np.outer(c[i], c[i]) +
                                np.outer(s[i], s[i])) for i in range(len(t)))
        fst = (vt[:, None] * s / 4).sum(0)
        assert vol == pytest.approx(vt.sum(), rel=1e-12)
        np.testing.assert_allclose(M[0, 1:], 700 * fst, atol=1e-12)
        np.testing.assert_allclose(M[1:, 1:], 700 * sec, rtol=1e-10,
                                   atol=1e-14)


# --------------------------------------------------------------- CCD
def test_accd_point_falling_on_triangle():
    t = np.array([[-1, 0, -1], [1, 0, -1], [0, 0, 1]], float)
    for d0, v in ((0.1, 1.0), (1e-3, 0.5), (0.05, 3.0), (2e-4, 1e-3)):
        x = np.concatenate([[0.1, d0, 0.0], t.reshape(-1)])
        dx = np.zeros(12)
        dx[1] = -v
        toi = O.accd(O.PT, x, dx, 0.1, 1.0)
        exact = d0 / v
        if exact >= 1.0:
            assert toi == 1.0
        else:
            assert 0 < toi <= exact
            assert toi >= 0.5 * exact  # stops once the gap drops under s*d0


def test_accd_conservative_on_random_trajectories():
    rng = _rng()
    for kind in (O.PT, O.EE):
        cfg = _pt_config if kind == O.PT else _ee_config
        for _ in range(30):
            x = cfg(["interior", "edge", "vertex"][rng.integers(3)], rng) * 0.1
            dx = rng.normal(0, 0.1, 12)
            toi = O.accd(kind, x, dx, 0.1, 1.0)
            d0 = math.sqrt(O.sqdist(kind, x)[0])
            ts = np.linspace(0, toi, 400)
            ds = [math.sqrt(O.sqdist(kind, x + s * dx)[0]) for s in ts]
            assert min(ds) > 0
            if toi < 1.0:
                assert ds[-1] >= 0.1 * d0 * (1 - 1e-9)
