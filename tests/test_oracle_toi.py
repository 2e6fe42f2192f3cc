"""Pins of the oracle's exact time of impact and of the Newton stop
criterion's scene scale (CPU only).

The exact TOI (the first contact time along the linear trajectory of a
Newton step, against which every additive-CCD step is checked) is pinned by
closed forms (a falling point, crossing edges), by constructed contacts
(primitives placed to touch at a chosen time t* and moved back along random
velocities: the first contact is at t* or earlier), and by dense sampling
with an independent inside test (a sign change of the coplanarity volume
whose crossing lies inside the triangle, or whose segments cross).  ACCD
(s = 0.1 and s = 1e-3) never exceeds it.

The scene scale l of the stop test |dq|_inf / (h l) < theta (Eq. 8 form) is
the bounding-box diagonal of the dynamic vertices at the step start (static
containers excluded); one Newton iteration of free fall moves q by exactly
h qdot + h^2 g, which pins eps_N.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_15875_amd import scenes


def _rng(seed=7):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- closed forms
def test_exact_toi_falling_point_closed_form():
    tri = np.array([[-1, 0, -1], [1, 0, -1], [0, 0, 1]], float)
    for d0, v in ((0.1, 1.0), (1e-3, 0.5), (0.05, 3.0), (2e-4, 1e-3),
                  (0.3, 0.31)):
        x = np.concatenate([[0.1, d0, 0.0], tri.reshape(-1)])
        dx = np.zeros(12)
        dx[1] = -v
        toi = O.exact_toi(O.PT, x, dx)
        want = d0 / v
        if want > 1.0:
            assert toi == 1.0
        else:
            assert toi == pytest.approx(want, rel=1e-13)
            assert toi <= want * (1 + 1e-15)
        # the triangle rising towards a resting point: same relative motion
        dx2 = np.zeros(12)
        dx2[4::3] = v
        assert O.exact_toi(O.PT, x, dx2) == pytest.approx(min(want, 1.0),
                                                          rel=1e-13)


def test_exact_toi_point_missing_triangle_is_one():
    tri = np.array([[-1, 0, -1], [1, 0, -1], [0, 0, 1]], float)
    # falls past the triangle outside its edge y = ..., x = 2
    x = np.concatenate([[2.0, 0.1, 0.0], tri.reshape(-1)])
    dx = np.zeros(12)
    dx[1] = -1.0
    assert O.exact_toi(O.PT, x, dx) == 1.0
    # moving away
    dx[1] = 1.0
    x[0] = 0.1
    assert O.exact_toi(O.PT, x, dx) == 1.0


def test_exact_toi_crossing_edges_closed_form():
    # edge a along x at height h moving down at speed v, edge b along z at
    # y = 0: they cross at t = h / v
    for h, v in ((0.2, 1.0), (1e-3, 0.25), (0.5, 0.4)):
        x = np.array([-1, h, 0.1, 1, h, 0.1, 0.2, 0, -1, 0.2, 0, 1], float)
        dx = np.zeros(12)
        dx[1] = dx[4] = -v
        want = h / v
        toi = O.exact_toi(O.EE, x, dx)
        if want > 1.0:
            assert toi == 1.0
        else:
            assert toi == pytest.approx(want, rel=1e-13)
    # edge a passes beyond the end of edge b: no contact
    x = np.array([-1, 0.2, 1.5, 1, 0.2, 1.5, 0.2, 0, -1, 0.2, 0, 1], float)
    dx = np.zeros(12)
    dx[1] = dx[4] = -1.0
    assert O.exact_toi(O.EE, x, dx) == 1.0


def test_exact_toi_tilting_edge_closed_form():
    # edge a keeps its foot at (0.3, 0, 0) while its upper end moves to
    # (0.3, 1 - 2t, t); a point s of the edge is (0.3, s(1 - 2t), s t), and
    # it meets the floor edge {(x, 0, 0.5)} only when s(1 - 2t) = 0 and
    # s t = 0.5, i.e. at t = 0.5 with the end on the floor edge
    x = np.array([0.3, 0.0, 0.0, 0.3, 1.0, 0.0,
                  -1.0, 0.0, 0.5, 1.0, 0.0, 0.5], float)
    dx = np.zeros(12)
    dx[3:6] = [0.0, -2.0, 1.0]
    assert O.exact_toi(O.EE, x, dx) == pytest.approx(0.5, rel=1e-12)


# ---------------------------------------------------------- constructed hits
def _random_triangle(rng, scale=0.1):
    while True:
        t = rng.normal(0, scale, (3, 3))
        n = np.cross(t[1] - t[0], t[2] - t[0])
        if np.linalg.norm(n) > 0.2 * scale * scale:
            return t


def _pt_constructed(rng):
    """point and triangle placed to touch at t*: the point sits at a random
    interior point of the triangle at t*, then every vertex moves back along
    its own random velocity"""
    t_star = rng.uniform(0.05, 0.95)
    tri = _random_triangle(rng)
    w = rng.dirichlet([1, 1, 1])
    p = w @ tri
    pts = np.vstack([p, tri])
    vel = rng.normal(0, 0.1, (4, 3))
    x0 = pts - t_star * vel
    return x0.reshape(-1), vel.reshape(-1), t_star


def _ee_constructed(rng):
    """two segments crossing at a common point X at t*"""
    t_star = rng.uniform(0.05, 0.95)
    X = rng.normal(0, 0.1, 3)
    da, db = rng.normal(0, 1, 3), rng.normal(0, 1, 3)
    sa, sb = rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.9)
    la, lb = rng.uniform(0.05, 0.2), rng.uniform(0.05, 0.2)
    da *= la / np.linalg.norm(da)
    db *= lb / np.linalg.norm(db)
    pts = np.array([X - sa * da, X + (1 - sa) * da, X - sb * db,
                    X + (1 - sb) * db])
    vel = rng.normal(0, 0.1, (4, 3))
    x0 = pts - t_star * vel
    return x0.reshape(-1), vel.reshape(-1), t_star


def _dist(kind, x12):
    return math.sqrt(O.sqdist(kind, x12)[0])


@pytest.mark.parametrize("kind", [O.PT, O.EE])
def test_exact_toi_constructed_contacts(kind):
    rng = _rng(11 + kind)
    make = _pt_constructed if kind == O.PT else _ee_constructed
    for _ in range(60):
        x, dx, t_star = make(rng)
        if _dist(kind, x) < 1e-6:
            continue
        toi = O.exact_toi(kind, x, dx)
        # the constructed contact, or an earlier one
        assert toi <= t_star * (1 + 1e-12) + 1e-15
        # a real contact: zero distance at the returned time
        assert _dist(kind, x + toi * dx) < 1e-12 * (np.abs(x).max() +
                                                     np.abs(dx).max())
        # ACCD never beyond it (the CCD contract), and close for small s
        for s in (0.1, 1e-3):
            assert O.accd(kind, x, dx, s, 1.0) <= toi
        assert toi - O.accd(kind, x, dx, 1e-3, 1.0) < 0.05


# ---------------------------------------------------------- dense sampling
def _sampled_first_contact(kind, x, dx, n=4000):
    """first sample interval [t_i, t_i+1] over which the coplanarity volume
    changes sign at a crossing point inside the other primitive (numpy, an
    inside test independent of the oracle's distance code); None if no
    sampled crossing"""
    ts = np.linspace(0.0, 1.0, n + 1)
    P = (x[None, :] + ts[:, None] * dx[None, :]).reshape(-1, 4, 3)
    if kind == O.PT:
        u, v, w = P[:, 2] - P[:, 1], P[:, 3] - P[:, 1], P[:, 0] - P[:, 1]
    else:
        u, v, w = P[:, 1] - P[:, 0], P[:, 3] - P[:, 2], P[:, 2] - P[:, 0]
    f = np.einsum("ij,ij->i", np.cross(u, v), w)
    for i in range(n):
        if f[i] == 0.0 or (f[i] > 0) != (f[i + 1] > 0):
            lam = f[i] / (f[i] - f[i + 1]) if f[i] != f[i + 1] else 0.0
            Q = P[i] + lam * (P[i + 1] - P[i])
            if kind == O.PT:
                p, a, b, c = Q
                nrm = np.cross(b - a, c - a)
                ins = all(np.dot(np.cross(e1 - e0, p - e0), nrm) >= 0
                          for e0, e1 in ((a, b), (b, c), (c, a)))
            else:
                a0, a1, b0, b1 = Q
                # coplanar segments cross iff each separates the other's ends
                nrm = np.cross(a1 - a0, b1 - b0)
                s1 = np.dot(np.cross(a1 - a0, b0 - a0), nrm)
                s2 = np.dot(np.cross(a1 - a0, b1 - a0), nrm)
                s3 = np.dot(np.cross(b1 - b0, a0 - b0), nrm)
                s4 = np.dot(np.cross(b1 - b0, a1 - b0), nrm)
                ins = s1 * s2 <= 0 and s3 * s4 <= 0
            if ins:
                return ts[i], ts[i + 1]
    return None


@pytest.mark.parametrize("kind", [O.PT, O.EE])
def test_exact_toi_against_dense_sampling(kind):
    rng = _rng(23 + kind)
    make = _pt_constructed if kind == O.PT else _ee_constructed
    hits = misses = 0
    for trial in range(80):
        if trial % 2 == 0:
            x, dx, _ = make(rng)
        else:
            # random motion: hits and misses both occur
            x = rng.normal(0, 0.1, 12)
            dx = rng.normal(0, 0.15, 12)
        if _dist(kind, x) < 1e-6:
            continue
        toi = O.exact_toi(kind, x, dx)
        iv = _sampled_first_contact(kind, x, dx)
        if iv is None:
            # no sampled crossing: no contact, or a touch between samples
            # that the distance at the returned time confirms
            if toi < 1.0:
                assert _dist(kind, x + toi * dx) < 1e-10
            misses += toi == 1.0
        else:
            lo, hi = iv
            assert toi <= hi + 1e-12
            # nothing earlier than one sample before the sampled crossing
            # unless it is a real touch
            if toi < lo - 1e-12:
                assert _dist(kind, x + toi * dx) < 1e-10
            hits += 1
        assert O.accd(kind, x, dx, 0.1, 1.0) <= toi
    assert hits > 20 and misses > 5


# ------------------------------------------------------- scene scale, eps_N
def _small_box_scene():
    sc = scenes.spheres_in_box_scene(3, n_bodies=6, level=1, half=0.5,
                                     y_lo=0.3, y_hi=1.2, wall=0.9,
                                     wall_h=2.0)
    return sc


def test_scene_scale_is_dynamic_bounding_box_diagonal():
    sc = _small_box_scene()
    ref = O.Oracle(sc)
    ref.begin_step()
    st = ref.local_solve(check=False)
    xs = []
    allx = []
    for b in sc.bodies:
        A = b.q0[3:].reshape(3, 3)
        x = b.xbar @ A.T + b.q0[:3]
        allx.append(x)
        if b.kind == scenes.DYNAMIC:
            xs.append(x)
    xs = np.vstack(xs)
    want = float(np.linalg.norm(xs.max(0) - xs.min(0)))
    assert st["scene_scale"] == pytest.approx(want, rel=1e-14)
    # the static container is excluded: its box is much larger
    allx = np.vstack(allx)
    assert float(np.linalg.norm(allx.max(0) - allx.min(0))) > 1.5 * want


def test_eps_N_of_one_free_fall_iteration():
    # one unit cube, no ground and no contact: the energy is quadratic in p
    # (the cube is centred at its centre of mass) and the orthogonality
    # term is stationary at A = I, so the first Newton direction is exactly
    # qtilde - q = h qdot + h^2 g in the translation and zero in A
    v, t = scenes.cube_mesh(0.5)
    qd = np.zeros(12)
    qd[0:3] = [0.3, -0.7, 0.2]
    body = scenes.Body(v, t, 1000.0, scenes.identity_q([0.0, 3.0, 0.0]), qd)
    sc = scenes.Scene("cube_fall", scenes.default_params(has_ground=0,
                                                         max_newton=1),
                      [body], 1)
    ref = O.Oracle(sc)
    ref.begin_step()
    st = ref.local_solve(check=False)
    h = sc.params["dt"]
    g = np.array(sc.params["gravity"])
    l = math.sqrt(3.0)   # the unit cube's diagonal
    assert st["scene_scale"] == pytest.approx(l, rel=1e-15)
    want = np.abs(h * qd[:3] + h * h * g).max() / (h * l)
    assert st["final_eps_N"] == pytest.approx(want, rel=1e-10)
    assert st["newton_iters"] == 1


def test_accd_of_a_pair_sliding_into_contact():
    # a point 1e-4 above a wide triangle in y = 0 that slides 2 along x while
    # closing the gap at 2e-4 per unit t: first contact at t = 0.5 (x = 0.5,
    # inside the triangle).  The one-point steps of ACCD shrink the distance
    # by 1e-4 of itself each, so this pair runs well past the one-point
    # phase; its blocked steps must stay below the contact, end within the
    # gap rule's last tenth of the distance, and need far fewer distance
    # evaluations than the cap
    d0 = 1e-4
    x = np.array([-0.5, d0, 0.0, -1.0, 0.0, -1.0, 3.0, 0.0, -1.0, -1.0, 0.0, 3.0])
    dx = np.zeros(12)
    dx[0:3] = [2.0, -2.0 * d0, 0.0]
    toi = O.exact_toi(O.PT, x, dx)
    assert toi == pytest.approx(0.5, rel=1e-12)
    t = O.accd(O.PT, x, dx, 0.1, 1.0)
    assert t <= toi
    # the gap rule stops once the distance would drop below 0.1 d0, whose
    # time is 0.45; the last accepted point lies beyond the previous one
    assert 0.44 < t < 0.5
    # sliding at a constant distance over the triangle: no contact, the
    # blocked steps reach the end of the step
    dx[0:3] = [2.0, 0.0, 0.0]
    x[0] = -0.9
    assert O.accd(O.PT, x, dx, 0.1, 1.0) == 1.0
