"""ctypes binding of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It loads oracle/liboracle.so (built by oracle/build.py) and
exposes the oracle's C API with numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB: another build of the single-threaded library (the sanitized
# one of build.build_sanitized)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
LIB_OMP_PATH = os.path.join(HERE, "liboracle_omp.so")

PT, EE, PG = 0, 1, 2
OK = 0


class OrcParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("dhat", C.c_double),
                ("kappa", C.c_double), ("kappa_A", C.c_double),
                ("gravity", C.c_double * 3), ("newton_theta", C.c_double),
                ("pcg_eta", C.c_double), ("ground_y", C.c_double),
                ("max_newton", C.c_int32), ("max_pcg", C.c_int32),
                ("max_ls", C.c_int32), ("has_ground", C.c_int32),
                ("mollify_ee", C.c_int32), ("dense_max_dof", C.c_int32)]


class OrcStats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters_total", C.c_int32),
                ("ls_halvings", C.c_int32), ("status", C.c_int32),
                ("final_eps_N", C.c_double), ("min_alpha", C.c_double),
                ("min_dist", C.c_double), ("scene_scale", C.c_double),
                ("n_cand_pt", C.c_int64), ("n_cand_ee", C.c_int64),
                ("n_cand_pg", C.c_int64), ("n_active", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_libs = {}


def lib(omp: bool = False):
    """The single-threaded oracle library, or (omp) its OpenMP build, which
    computes bit-identical results on several threads."""
    if omp not in _libs:
        path = LIB_OMP_PATH if omp else LIB_PATH
        if not os.path.exists(path):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        vp = C.c_void_p
        sig = {
            "orc_create": (vp, [C.POINTER(OrcParams)]),
            "orc_destroy": (None, [vp]),
            "orc_last_error": (C.c_char_p, [vp]),
            "orc_add_body": (C.c_int, [vp, dp, C.c_int32, ip, C.c_int32,
                                       C.c_double, dp, dp, C.c_int32]),
            "orc_finalize": (C.c_int, [vp]),
            "orc_sizes": (C.c_int, [vp, lp]),
            "orc_edges": (C.c_int, [vp, ip]),
            "orc_body_mass": (C.c_int, [vp, dp, dp]),
            "orc_set_shared": (C.c_int, [vp, ip, C.c_int32, dp, dp, dp, ip]),
            "orc_set_pair_replication": (C.c_int, [vp, C.c_int32]),
            "orc_set_projection": (C.c_int, [vp, C.c_int32]),
            "orc_begin_step": (C.c_int, [vp]),
            "orc_local_solve": (C.c_int, [vp, C.POINTER(OrcStats)]),
            "orc_end_step": (C.c_int, [vp]),
            "orc_get_state": (C.c_int, [vp, dp, dp]),
            "orc_set_state": (C.c_int, [vp, dp, dp]),
            "orc_get_qtilde": (C.c_int, [vp, dp]),
            "orc_set_step": (C.c_int, [vp, dp, dp, C.c_double]),
            "orc_vertices": (C.c_int, [vp, dp, dp]),
            "orc_candidates": (C.c_int, [vp, C.c_int32, dp, dp, ip, C.c_int64,
                                         lp]),
            "orc_eval": (C.c_int, [vp, dp, dp, dp, dp, C.c_int64, lp, ip, dp,
                                   lp]),
            "orc_direction": (C.c_int, [vp, dp, dp, ip]),
            "orc_ccd": (C.c_int, [vp, dp, dp, dp]),
            "orc_energy_delta": (C.c_int, [vp, dp, dp, C.c_double, dp]),
            "orc_penetration": (C.c_int, [vp, dp, C.c_double, lp, dp]),
            "orc_barrier": (None, [C.c_double, C.c_double, dp]),
            "orc_sqdist": (C.c_int, [C.c_int32, dp, dp, dp, dp, ip]),
            "orc_pair_eval": (C.c_int, [C.c_int32, dp, C.c_double, C.c_double,
                                        C.c_double, C.c_int32, dp, dp, dp, dp,
                                        ip]),
            "orc_orth": (None, [dp, dp, dp, dp, C.c_int32]),
            "orc_mass_props": (C.c_int, [dp, C.c_int32, ip, C.c_int32,
                                         C.c_double, dp, dp]),
            "orc_psd": (None, [C.c_int32, dp, dp]),
            "orc_eig": (None, [C.c_int32, dp, dp, dp]),
            "orc_accd": (C.c_double, [C.c_int32, dp, dp, C.c_double,
                                      C.c_double]),
            "orc_exact_toi": (C.c_double, [C.c_int32, dp, dp, C.c_double]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _libs[omp] = L
    return _libs[omp]


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_params(p: dict, dense_max_dof: int = 2400) -> OrcParams:
    o = OrcParams()
    o.dt = p["dt"]
    o.dhat = p["dhat"]
    o.kappa = p["kappa"]
    o.kappa_A = p["kappa_A"]
    for i in range(3):
        o.gravity[i] = p["gravity"][i]
    o.newton_theta = p["newton_theta"]
    o.pcg_eta = p["pcg_eta"]
    o.ground_y = p.get("ground_y", 0.0)
    o.max_newton = int(p["max_newton"])
    o.max_pcg = int(p["max_pcg"])
    o.max_ls = int(p["max_ls"])
    o.has_ground = int(p.get("has_ground", 0))
    o.mollify_ee = int(p.get("mollify_ee", 1))
    o.dense_max_dof = int(dense_max_dof)
    return o


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


class Oracle:
    """One oracle scene built from a scenes.Scene."""

    def __init__(self, scene, dense_max_dof: int = 2400, finalize=True,
                 omp: bool = False, **param_over):
        """omp: run on the OpenMP build (same results, several threads)."""
        L = self._L = lib(omp)
        p = dict(scene.params)
        p.update(param_over)
        self.params = p
        self._p = make_params(p, dense_max_dof)
        self.h = L.orc_create(C.byref(self._p))
        self.scene = scene
        for b in scene.bodies:
            xb = _f64(b.xbar)
            tr = np.ascontiguousarray(b.tris, dtype=np.int32)
            q0 = _f64(b.q0)
            qd = _f64(b.qdot0)
            rc = L.orc_add_body(self.h, _d(xb), xb.shape[0], _i(tr),
                                tr.shape[0], float(b.density), _d(q0), _d(qd),
                                int(b.kind))
            if rc < 0:
                raise OracleError(rc, self.error())
        sz = np.zeros(4, dtype=np.int64)
        L.orc_sizes(self.h, _l(sz))
        self.B, self.V, self.T, self.E = (int(v) for v in sz)
        if finalize:
            self._check(L.orc_finalize(self.h))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self._L.orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def error(self):
        return self._L.orc_last_error(self.h).decode()

    def _check(self, rc):
        if rc != OK:
            raise OracleError(rc, self.error())
        return rc

    # ---- state ----
    def edges(self):
        out = np.zeros((self.E, 2), dtype=np.int32)
        self._L.orc_edges(self.h, _i(out))
        return out

    def body_mass(self):
        M = np.zeros((self.B, 4, 4))
        v = np.zeros(self.B)
        self._L.orc_body_mass(self.h, _d(M), _d(v))
        return M, v

    def set_shared(self, ids, z, u, rho, kappa_b):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        z = _f64(z, (-1, 12)) if len(ids) else np.zeros((0, 12))
        u = _f64(u, (-1, 12)) if len(ids) else np.zeros((0, 12))
        rho = _f64(rho)
        kb = np.ascontiguousarray(kappa_b, dtype=np.int32)
        return self._check(self._L.orc_set_shared(self.h, _i(ids), len(ids),
                                                _d(z), _d(u), _d(rho),
                                                _i(kb)))

    def set_pair_replication(self, mode):
        return self._check(self._L.orc_set_pair_replication(self.h, mode))

    def set_projection(self, on):
        return self._check(self._L.orc_set_projection(self.h, int(on)))

    def begin_step(self):
        return self._check(self._L.orc_begin_step(self.h))

    def local_solve(self, check=True):
        st = OrcStats()
        rc = self._L.orc_local_solve(self.h, C.byref(st))
        if check:
            self._check(rc)
        return st.as_dict()

    def end_step(self):
        return self._check(self._L.orc_end_step(self.h))

    def step(self):
        self.begin_step()
        st = self.local_solve()
        self.end_step()
        return st

    def get_state(self):
        q = np.zeros((self.B, 12))
        qd = np.zeros((self.B, 12))
        self._L.orc_get_state(self.h, _d(q), _d(qd))
        return q, qd

    def set_state(self, q, qdot=None):
        q = _f64(q, (-1, 12))
        qd = _f64(qdot, (-1, 12)) if qdot is not None else None
        self._L.orc_set_state(self.h, _d(q),
                            _d(qd) if qd is not None else None)

    def qtilde(self):
        out = np.zeros((self.B, 12))
        self._L.orc_get_qtilde(self.h, _d(out))
        return out

    def set_step(self, qt, qtilde, scale):
        qt = _f64(qt, (-1, 12))
        qtilde = _f64(qtilde, (-1, 12))
        self._L.orc_set_step(self.h, _d(qt), _d(qtilde), float(scale))

    # ---- hooks ----
    def vertices(self, q=None):
        x = np.zeros((self.V, 3))
        qq = _f64(q, (-1, 12)) if q is not None else None
        self._L.orc_vertices(self.h, _d(qq) if qq is not None else None, _d(x))
        return x

    def candidates(self, kind, x, dx=None):
        x = _f64(x, (-1, 3))
        dxa = _f64(dx, (-1, 3)) if dx is not None else None
        n = np.zeros(1, dtype=np.int64)
        L = self._L
        L.orc_candidates(self.h, kind, _d(x),
                         _d(dxa) if dxa is not None else None, None, 0, _l(n))
        w = 1 if kind == PG else 2
        out = np.zeros(max(int(n[0]), 1) * w, dtype=np.int32)
        self._check(L.orc_candidates(self.h, kind, _d(x),
                                     _d(dxa) if dxa is not None else None,
                                     _i(out), int(n[0]), _l(n)))
        out = out[: int(n[0]) * w]
        return out.reshape(-1, 2) if w == 2 else out

    def eval(self, q):
        q = _f64(q, (-1, 12))
        E = np.zeros(1)
        g = np.zeros((self.B, 12))
        Hd = np.zeros((self.B, 12, 12))
        n = np.zeros(1, dtype=np.int64)
        na = np.zeros(1, dtype=np.int64)
        L = self._L
        L.orc_eval(self.h, _d(q), _d(E), _d(g), _d(Hd), 0, _l(n), None, None,
                   _l(na))
        cap = max(int(n[0]), 1)
        ij = np.zeros((cap, 2), dtype=np.int32)
        Ho = np.zeros((cap, 12, 12))
        self._check(L.orc_eval(self.h, _d(q), _d(E), _d(g), _d(Hd), cap,
                               _l(n), _i(ij), _d(Ho), _l(na)))
        k = int(n[0])
        return dict(E=float(E[0]), g=g, Hdiag=Hd, off_ij=ij[:k], Hoff=Ho[:k],
                    n_active=int(na[0]))

    def direction(self, q):
        q = _f64(q, (-1, 12))
        dq = np.zeros((self.B, 12))
        it = np.zeros(1, dtype=np.int32)
        self._check(self._L.orc_direction(self.h, _d(q), _d(dq), _i(it)))
        return dq, int(it[0])

    def ccd(self, q, dq):
        q = _f64(q, (-1, 12))
        dq = _f64(dq, (-1, 12))
        a = np.zeros(1)
        self._check(self._L.orc_ccd(self.h, _d(q), _d(dq), _d(a)))
        return float(a[0])

    def energy_delta(self, q, dq, alpha):
        q = _f64(q, (-1, 12))
        dq = _f64(dq, (-1, 12))
        e = np.zeros(1)
        self._check(self._L.orc_energy_delta(self.h, _d(q), _d(dq),
                                           float(alpha), _d(e)))
        return float(e[0])

    def penetration(self, x, pad=None):
        x = _f64(x, (-1, 3))
        nc = np.zeros(1, dtype=np.int64)
        md = np.zeros(1)
        pad = self.params["dhat"] if pad is None else pad
        self._L.orc_penetration(self.h, _d(x), float(pad), _l(nc), _d(md))
        return int(nc[0]), float(md[0])


# ---- primitives ----
def barrier(d, dhat):
    out = np.zeros(3)
    lib().orc_barrier(float(d), float(dhat), _d(out))
    return out


def sqdist(kind, x12):
    x = _f64(x12, (12,))
    D = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros((12, 12))
    t = np.zeros(1, dtype=np.int32)
    lib().orc_sqdist(kind, _d(x), _d(D), _d(g), _d(H), _i(t))
    return float(D[0]), g, H, int(t[0])


def pair_eval(kind, x12, eps_x, dhat, w, project=True):
    x = _f64(x12, (12,))
    E = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros((12, 12))
    d = np.zeros(1)
    t = np.zeros(1, dtype=np.int32)
    act = lib().orc_pair_eval(kind, _d(x), float(eps_x), float(dhat),
                              float(w), int(project), _d(E), _d(g), _d(H),
                              _d(d), _i(t))
    return dict(active=bool(act), E=float(E[0]), g=g, H=H, d=float(d[0]),
                dtype=int(t[0]))


def orth(A, project=False):
    A = _f64(A, (9,))
    E = np.zeros(1)
    g = np.zeros(9)
    H = np.zeros((9, 9))
    lib().orc_orth(_d(A), _d(E), _d(g), _d(H), int(project))
    return float(E[0]), g, H


def mass_props(xbar, tris, density):
    xb = _f64(xbar, (-1, 3))
    tr = np.ascontiguousarray(tris, dtype=np.int32)
    M = np.zeros((4, 4))
    v = np.zeros(1)
    lib().orc_mass_props(_d(xb), xb.shape[0], _i(tr), tr.shape[0],
                         float(density), _d(M), _d(v))
    return M, float(v[0])


def psd(H):
    H = _f64(H)
    n = H.shape[0]
    out = np.zeros_like(H)
    lib().orc_psd(n, _d(H), _d(out))
    return out


def eig(H):
    H = _f64(H)
    n = H.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    lib().orc_eig(n, _d(H), _d(w), _d(V))
    return w, V


def accd(kind, x12, dx12, s=0.1, tmax=1.0):
    x = _f64(x12, (12,))
    d = _f64(dx12, (12,))
    return float(lib().orc_accd(kind, _d(x), _d(d), float(s), float(tmax)))


def exact_toi(kind, x12, dx12, tmax=1.0):
    """Exact first time of impact of a PT or EE pair (tmax: none)."""
    x = _f64(x12, (12,))
    d = _f64(dx12, (12,))
    return float(lib().orc_exact_toi(kind, _d(x), _d(d), float(tmax)))
