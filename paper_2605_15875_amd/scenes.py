"""Seeded synthetic scene generators.

This module only produces *inputs*: rest meshes, initial affine states,
velocities, solver parameters and the random draws that the ADMM
consensus inputs are built from.  It holds none of the method's
arithmetic (no mass matrices, energies, distances or predictions), so
the CPU oracle and the HIP library can both be driven from it without
sharing any code with each other.

Scenes stand in for the paper's large scenes (Sec. 6, Table 1), whose
meshes are not available: unit cubes stacked on a ground plane,
icospheres falling into an open box, and convex hulls in a funnel.

Conventions shared by every consumer:
  * a body is (xbar [nv,3] float64, tris [nt,3] int32, density, q0[12],
    qdot0[12], kind) with kind 0 = dynamic, 1 = static;
  * the affine state is q = [p (3), A row-major (9)];
  * y is up, SI units.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

DYNAMIC = 0
STATIC = 1


@dataclasses.dataclass
class Body:
    xbar: np.ndarray
    tris: np.ndarray
    density: float
    q0: np.ndarray
    qdot0: np.ndarray
    kind: int = DYNAMIC


@dataclasses.dataclass
class Scene:
    name: str
    params: Dict[str, float]
    bodies: List[Body]
    steps: int
    # optional consensus inputs (one worker's share of an ADMM split)
    shared_ids: Optional[np.ndarray] = None
    shared_delta: Optional[np.ndarray] = None   # [n,12] offsets added to q-tilde
    shared_u: Optional[np.ndarray] = None       # [n,12]
    shared_rho: Optional[np.ndarray] = None     # [n]
    shared_kappa: Optional[np.ndarray] = None   # [n] int32

    @property
    def n_vertices(self) -> int:
        return int(sum(b.xbar.shape[0] for b in self.bodies))

    @property
    def n_triangles(self) -> int:
        return int(sum(b.tris.shape[0] for b in self.bodies))

    @property
    def n_dynamic(self) -> int:
        return int(sum(1 for b in self.bodies if b.kind == DYNAMIC))


def default_params(**over) -> Dict[str, float]:
    p = dict(dt=0.01, dhat=1e-3, kappa=1e5, kappa_A=1e8,
             gravity=(0.0, -9.8, 0.0), newton_theta=1e-6, pcg_eta=1e-4,
             max_newton=1000, max_pcg=2000, max_ls=40, has_ground=0,
             ground_y=0.0, mollify_ee=1, precision=0)
    p.update(over)
    return p


def identity_q(p) -> np.ndarray:
    q = np.zeros(12)
    q[0:3] = p
    q[3:12] = np.eye(3).reshape(-1)
    return q


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def cube_mesh(half: float = 0.5):
    """Closed, outward-oriented cube: 8 vertices, 12 triangles."""
    v = np.array([[x, y, z] for x in (-half, half) for y in (-half, half)
                  for z in (-half, half)], dtype=np.float64)
    # vertex index = 4*ix + 2*iy + iz
    quads = [
        (0, 1, 3, 2),  # x = -h
        (4, 6, 7, 5),  # x = +h
        (0, 4, 5, 1),  # y = -h
        (2, 3, 7, 6),  # y = +h
        (0, 2, 6, 4),  # z = -h
        (1, 5, 7, 3),  # z = +h
    ]
    tris = []
    for a, b, c, d in quads:
        tris.append((a, b, c))
        tris.append((a, c, d))
    tris = np.array(tris, dtype=np.int32)
    return v, _orient_outward(v, tris)


def _orient_outward(v: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Flip triangles of a star-shaped closed mesh so normals point away
    from the vertex centroid."""
    c = v.mean(axis=0)
    a, b, d = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    n = np.cross(b - a, d - a)
    m = (a + b + d) / 3.0 - c
    flip = n[:, 0] * m[:, 0] + n[:, 1] * m[:, 1] + n[:, 2] * m[:, 2] < 0
    out = tris.copy()
    out[flip, 1] = tris[flip, 2]
    out[flip, 2] = tris[flip, 1]
    return out


def icosphere_mesh(level: int = 3, radius: float = 1.0):
    """Subdivided icosahedron projected on a sphere.
    level 3 gives 642 vertices and 1280 triangles."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    v = np.array(verts) * radius
    f = np.array(faces, dtype=np.int32)
    return v, _orient_outward(v, f)


def hull_mesh(rng: np.random.Generator, n_points: int, radius: float,
              axis_scale: np.ndarray):
    """Convex hull of n Gaussian directions normalised to the unit sphere,
    scaled by radius and per-axis factors: every point is on the hull, so
    V = n, T = 2n - 4."""
    from scipy.spatial import ConvexHull
    while True:
        p = rng.standard_normal((n_points, 3))
        p /= np.linalg.norm(p, axis=1, keepdims=True)
        p = p * radius * axis_scale[None, :]
        h = ConvexHull(p)
        used = np.unique(h.simplices)
        if used.shape[0] == n_points:
            break
    v = p
    tris = h.simplices.astype(np.int32)
    # centre at the vertex centroid (a star-shaped reference point)
    v = v - v.mean(axis=0)
    return v, _orient_outward(v, tris)


def open_box_mesh(half_x: float, half_z: float, height: float):
    """Static open box: floor at y=0 and four walls, 2 triangles per face."""
    hx, hz, h = half_x, half_z, height
    v = np.array([[-hx, 0, -hz], [hx, 0, -hz], [hx, 0, hz], [-hx, 0, hz],
                  [-hx, h, -hz], [hx, h, -hz], [hx, h, hz], [-hx, h, hz]],
                 dtype=np.float64)
    quads = [(0, 1, 2, 3),  # floor
             (0, 4, 5, 1), (1, 5, 6, 2), (2, 6, 7, 3), (3, 7, 4, 0)]
    tris = []
    for a, b, c, d in quads:
        tris.append((a, b, c))
        tris.append((a, c, d))
    return v, np.array(tris, dtype=np.int32)


def funnel_mesh(top_half: float, top_y: float, neck_half: float,
                neck_y: float, box_half: float, box_h: float):
    """Static funnel: a square frustum of thin triangle walls above an open
    box floor."""
    v = []
    tris = []
    # frustum ring: top 0..3, neck 4..7
    for y, h in ((top_y, top_half), (neck_y, neck_half)):
        v += [[-h, y, -h], [h, y, -h], [h, y, h], [-h, y, h]]
    for i in range(4):
        j = (i + 1) % 4
        tris.append((i, j, 4 + j))
        tris.append((i, 4 + j, 4 + i))
    base = len(v)
    bv, bt = open_box_mesh(box_half, box_half, box_h)
    v += bv.tolist()
    tris += (bt + base).tolist()
    return np.array(v, dtype=np.float64), np.array(tris, dtype=np.int32)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def cubes_scene(seed: int = 0, nx: int = 2, ny: int = 2, nz: int = 2,
                gap: float = 0.05, jitter: float = 0.01, steps: int = 20,
                **over) -> Scene:
    """Unit cubes stacked in an nx*ny*nz grid with `gap` spacing and uniform
    +/-jitter on every position component, above a ground plane at y=0.
    The 2x2x2 case is the 8-cube configuration."""
    rng = np.random.default_rng(seed)
    v, t = cube_mesh(0.5)
    bodies = []
    pitch = 1.0 + gap
    xs = (np.arange(nx) - (nx - 1) / 2.0) * pitch
    zs = (np.arange(nz) - (nz - 1) / 2.0) * pitch
    for iy in range(ny):
        for ix in range(nx):
            for iz in range(nz):
                c = np.array([xs[ix], 0.5 + gap + iy * pitch, zs[iz]])
                c = c + rng.uniform(-jitter, jitter, 3)
                bodies.append(Body(v.copy(), t.copy(), 1000.0, identity_q(c),
                                   np.zeros(12), DYNAMIC))
    params = default_params(has_ground=1, ground_y=0.0)
    params.update(over)
    return Scene(f"cubes{nx}x{ny}x{nz}_s{seed}", params, bodies, steps)


def spheres_in_box_scene(seed: int = 0, n_bodies: int = 1000, level: int = 3,
                         half: float = 2.0, y_lo: float = 0.2,
                         y_hi: float = 8.2, r_lo: float = 0.05,
                         r_hi: float = 0.15, min_gap: float = 0.01,
                         wall: float = 2.2, wall_h: float = 10.0,
                         vel: float = 1.0, steps: int = 50, **over) -> Scene:
    """Icospheres at seeded non-overlapping positions falling into an open
    box.  Defaults give 1000 level-3 icospheres (642 verts, 1280 tris)."""
    rng = np.random.default_rng(seed)
    unit_v, unit_t = icosphere_mesh(level, 1.0)
    centres = np.zeros((n_bodies, 3))
    radii = np.zeros(n_bodies)
    n = 0
    tries = 0
    while n < n_bodies:
        tries += 1
        if tries > 200000 * max(1, n_bodies):
            raise RuntimeError("could not place spheres")
        r = rng.uniform(r_lo, r_hi)
        c = np.array([rng.uniform(-half, half), rng.uniform(y_lo, y_hi),
                      rng.uniform(-half, half)])
        if n:
            d = np.linalg.norm(centres[:n] - c, axis=1)
            if np.any(d < radii[:n] + r + min_gap):
                continue
        centres[n] = c
        radii[n] = r
        n += 1
    bodies = []
    for i in range(n_bodies):
        qd = np.zeros(12)
        qd[0:3] = rng.uniform(-vel, vel, 3)
        bodies.append(Body(unit_v * radii[i], unit_t.copy(), 1000.0,
                           identity_q(centres[i]), qd, DYNAMIC))
    bv, bt = open_box_mesh(wall, wall, wall_h)
    bodies.append(Body(bv, bt, 1000.0, identity_q(np.zeros(3)), np.zeros(12),
                       STATIC))
    params = default_params(has_ground=0)
    params.update(over)
    return Scene(f"spheres{n_bodies}_l{level}_s{seed}", params, bodies, steps)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def hulls_in_funnel_scene(seed: int = 0, n_bodies: int = 2500,
                          n_lo: int = 300, n_hi: int = 1200,
                          worker_share: bool = True, n_shared: int = 200,
                          rho: float = 1e4, steps: int = 50, **over) -> Scene:
    """Seeded convex hulls in a funnel of static triangle walls.  With
    worker_share=True the scene is cut by the plane x=0: the worker keeps
    bodies with centre x<0 plus a slab of bodies around the cut, and the
    ~n_shared bodies in the slab are shared, with seeded consensus draws."""
    rng = np.random.default_rng(seed)
    centres = []
    radii = []
    lo = np.array([-3.5, 8.5, -3.5])
    hi = np.array([3.5, 16.0, 3.5])
    while len(centres) < n_bodies:
        r = rng.uniform(0.05, 0.15)
        c = rng.uniform(lo, hi)
        if centres:
            d = np.linalg.norm(np.array(centres) - c, axis=1)
            if np.any(d < np.array(radii) + r + 0.01):
                continue
        centres.append(c)
        radii.append(r)
    centres = np.array(centres)
    radii = np.array(radii)
    keep = np.ones(n_bodies, dtype=bool)
    shared = np.zeros(n_bodies, dtype=bool)
    if worker_share:
        # slab half-width chosen so that about n_shared bodies meet |x| < w/2
        ext = radii
        order = np.sort(np.abs(centres[:, 0]) - ext)
        w_half = max(order[min(n_shared, n_bodies) - 1], 0.0)
        shared = (np.abs(centres[:, 0]) - ext) <= w_half
        keep = (centres[:, 0] < 0) | shared
    bodies = []
    for i in np.nonzero(keep)[0]:
        n = int(rng.integers(n_lo, n_hi + 1))
        scale = rng.uniform(0.6, 1.0, 3)
        v, t = hull_mesh(rng, n, radii[i], scale)
        q = identity_q(centres[i])
        q[3:12] = random_rotation(rng).reshape(-1)
        bodies.append(Body(v, t, 1000.0, q, np.zeros(12), DYNAMIC))
    fv, ft = funnel_mesh(4.0, 8.0, 0.75, 4.0, 3.0, 4.0)
    bodies.append(Body(fv, ft, 1000.0, identity_q(np.zeros(3)), np.zeros(12),
                       STATIC))
    params = default_params(has_ground=0)
    params.update(over)
    sc = Scene(f"hulls{n_bodies}_s{seed}", params, bodies, steps)
    if worker_share:
        kept = np.nonzero(keep)[0]
        sid = np.nonzero(shared[kept])[0].astype(np.int32)
        ns = sid.shape[0]
        delta = np.zeros((ns, 12))
        delta[:, 0:3] = rng.uniform(-1e-3, 1e-3, (ns, 3))
        delta[:, 3:12] = rng.uniform(-1e-4, 1e-4, (ns, 9))
        sc.shared_ids = sid
        sc.shared_delta = delta
        sc.shared_u = rng.uniform(-1e-5, 1e-5, (ns, 12))
        sc.shared_rho = np.full(ns, rho)
        sc.shared_kappa = np.full(ns, 2, dtype=np.int32)
    return sc


def _place(rng: np.random.Generator, n: int, lo: np.ndarray, hi: np.ndarray,
           r_lo: float, r_hi: float, min_gap: float):
    """n non-overlapping spheres (centres, radii) drawn uniformly in the box
    [lo, hi] by rejection."""
    centres = np.zeros((n, 3))
    radii = np.zeros(n)
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > 200000 * max(1, n):
            raise RuntimeError("could not place bodies")
        r = rng.uniform(r_lo, r_hi)
        c = rng.uniform(lo, hi)
        if k and np.any(np.linalg.norm(centres[:k] - c, axis=1) < radii[:k] + r + min_gap):
            continue
        centres[k] = c
        radii[k] = r
        k += 1
    return centres, radii


def subdomain_scene(seed: int = 0, n_bodies: int = 400, sphere_frac: float = 0.5,
                    level: int = 3, n_lo: int = 300, n_hi: int = 600,
                    width: float = 4.0, shared_frac: float = 0.1,
                    rho: float = 1e4, vel: float = 1.0, steps: int = 50,
                    **over) -> Scene:
    """One ADMM subdomain of a larger scene: icospheres and convex hulls
    (radius 0.05-0.15; hulls of n_lo..n_hi points) at seeded
    non-overlapping positions in the slab 0 < x < width, |z| < width/2,
    with random velocities, falling into an open box.  The bodies nearest
    the two cut planes x = 0 and x = width (a fraction shared_frac) are
    shared, with seeded consensus draws as in the worker share."""
    rng = np.random.default_rng(seed)
    h = max(1.0, 0.004 * n_bodies * (width / 4.0) ** -2)
    m = 0.2
    lo = np.array([m, 0.3, -0.5 * width + m])
    hi = np.array([width - m, 0.3 + h, 0.5 * width - m])
    centres, radii = _place(rng, n_bodies, lo, hi, 0.05, 0.15, 0.01)
    unit_v, unit_t = icosphere_mesh(level, 1.0)
    bodies = []
    for i in range(n_bodies):
        qd = np.zeros(12)
        qd[0:3] = rng.uniform(-vel, vel, 3)
        if rng.uniform() < sphere_frac:
            v, t = unit_v * radii[i], unit_t.copy()
            q = identity_q(centres[i])
        else:
            n = int(rng.integers(n_lo, n_hi + 1))
            v, t = hull_mesh(rng, n, radii[i], rng.uniform(0.6, 1.0, 3))
            q = identity_q(centres[i])
            q[3:12] = random_rotation(rng).reshape(-1)
        bodies.append(Body(v, t, 1000.0, q, qd, DYNAMIC))
    bv, bt = open_box_mesh(0.5 * width + 0.2, 0.5 * width + 0.2, h + 1.0)
    bodies.append(Body(bv, bt, 1000.0, identity_q([0.5 * width, 0.0, 0.0]),
                       np.zeros(12), STATIC))
    params = default_params(has_ground=0)
    params.update(over)
    sc = Scene(f"subdomain{n_bodies}_s{seed}", params, bodies, steps)
    ns = max(1, int(round(shared_frac * n_bodies)))
    edge = np.minimum(centres[:, 0], width - centres[:, 0])
    sid = np.sort(np.argsort(edge, kind="stable")[:ns]).astype(np.int32)
    delta = np.zeros((ns, 12))
    delta[:, 0:3] = rng.uniform(-1e-3, 1e-3, (ns, 3))
    delta[:, 3:12] = rng.uniform(-1e-4, 1e-4, (ns, 9))
    sc.shared_ids = sid
    sc.shared_delta = delta
    sc.shared_u = rng.uniform(-1e-5, 1e-5, (ns, 12))
    sc.shared_rho = np.full(ns, rho)
    sc.shared_kappa = np.full(ns, 2, dtype=np.int32)
    return sc


def cubes_in_box_scene(seed: int = 0, n_cubes: int = 16, gap: float = 0.05,
                       jitter: float = 0.01, steps: int = 20, **over) -> Scene:
    """n unit cubes stacked in layers of k x k (k = round(cbrt(n)), at
    least 2) with `gap` spacing and uniform +/-jitter, in an open box (a
    static body instead of the ground plane, so that these scenes share
    their parameters with the subdomains of a batch)."""
    rng = np.random.default_rng(seed)
    v, t = cube_mesh(0.5)
    k = max(2, int(round(n_cubes ** (1.0 / 3.0))))
    pitch = 1.0 + gap
    xs = (np.arange(k) - (k - 1) / 2.0) * pitch
    bodies = []
    for i in range(n_cubes):
        layer, rest = divmod(i, k * k)
        ix, iz = divmod(rest, k)
        c = np.array([xs[ix], 0.5 + gap + layer * pitch, xs[iz]])
        c = c + rng.uniform(-jitter, jitter, 3)
        bodies.append(Body(v.copy(), t.copy(), 1000.0, identity_q(c),
                           np.zeros(12), DYNAMIC))
    half = 0.5 * k * pitch + 0.3
    layers = (n_cubes + k * k - 1) // (k * k)
    bv, bt = open_box_mesh(half, half, layers * pitch + 1.0)
    bodies.append(Body(bv, bt, 1000.0, identity_q(np.zeros(3)), np.zeros(12),
                       STATIC))
    params = default_params(has_ground=0)
    params.update(over)
    return Scene(f"cubes{n_cubes}_box_s{seed}", params, bodies, steps)


# the batch workload: subdomains of uneven size and independent cube scenes
BATCH_SUBDOMAINS = (200, 220, 250, 300, 400, 600, 1200, 3000)
BATCH_CUBES = tuple(int(round(16 * 32 ** (i / 63))) for i in range(64))


def batch_workload(seed: int = 0, subdomains=BATCH_SUBDOMAINS,
                   cubes=BATCH_CUBES, sub_args: Optional[dict] = None,
                   **over) -> List[Scene]:
    """Problems solved together in one batch: ADMM subdomains of uneven
    size (icospheres and hulls, each a worker's local problem with its
    shared bodies; sub_args: further subdomain_scene arguments) followed
    by independent scenes of stacked cubes, all with the same parameters
    (over)."""
    sa = dict(sub_args or {})
    out = [subdomain_scene(seed * 1000 + i, n, **sa, **over)
           for i, n in enumerate(subdomains)]
    out += [cubes_in_box_scene(seed * 1000 + 500 + i, n, **over)
            for i, n in enumerate(cubes)]
    return out


@dataclasses.dataclass
class Split:
    """Subdomains of one scene: worker scenes plus the replica table.
    Replica k is body rep_body[k] of worker rep_prob[k], a copy of shared
    body rep_group[k]; whole_ids[w][j] is the index in the whole scene of
    worker w's body j."""
    workers: List[Scene]
    rep_prob: np.ndarray
    rep_body: np.ndarray
    rep_group: np.ndarray
    n_groups: int
    whole_ids: List[np.ndarray]


def split_scene(scene: Scene, axis: int = 0, cut: float = 0.0,
                slab: float = 0.0) -> Split:
    """Two subdomains cut by the plane x[axis] = cut: worker 0 keeps the
    dynamic bodies whose centre (q0 translation) lies below cut + slab/2,
    worker 1 those above cut - slab/2, so bodies inside the slab are kept
    by both and shared.  Static bodies go to both workers."""
    keep = [[], []]
    for i, b in enumerate(scene.bodies):
        c = b.q0[axis]
        if b.kind != DYNAMIC or c < cut + 0.5 * slab:
            keep[0].append(i)
        if b.kind != DYNAMIC or c > cut - 0.5 * slab:
            keep[1].append(i)
    workers, whole = [], []
    for w in range(2):
        ids = np.array(keep[w], dtype=np.int64)
        bodies = [dataclasses.replace(scene.bodies[i]) for i in ids]
        workers.append(Scene(f"{scene.name}_w{w}", dict(scene.params), bodies,
                             scene.steps))
        whole.append(ids)
    shared = [i for i in keep[0] if i in set(keep[1])
              and scene.bodies[i].kind == DYNAMIC]
    group_of = {i: g for g, i in enumerate(shared)}
    rp, rb, rg = [], [], []
    for w in range(2):
        for j, i in enumerate(whole[w]):
            if i in group_of:
                rp.append(w)
                rb.append(j)
                rg.append(group_of[i])
    return Split(workers, np.array(rp, dtype=np.int32),
                 np.array(rb, dtype=np.int32), np.array(rg, dtype=np.int32),
                 len(shared), whole)


def config(idx: int, seed: int = 0, **over) -> Scene:
    """The named workloads: 0 = 8 stacked cubes on the ground (20 steps),
    1 = 1000 icospheres in an open box (50 steps), 2 = one worker's share
    of 2500 hulls in a funnel (the batch of subdomains and cube scenes is
    batch_workload)."""
    if idx == 0:
        return cubes_scene(seed, **over)
    if idx == 1:
        return spheres_in_box_scene(seed, **over)
    if idx == 2:
        return hulls_in_funnel_scene(seed, **over)
    raise ValueError(idx)
