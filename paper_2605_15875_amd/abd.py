"""ctypes binding of libabd (include/abd.h): argument marshalling only.

Every step of the solve runs in the HIP library; if libabd.so is missing
or cannot be loaded this module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ABD_LIB: another build of the library (libabd_san.so, the host-code
# sanitizer build); the HIP library is required either way
LIB_PATH = os.environ.get("ABD_LIB") or os.path.join(HERE, "libabd.so")

OK = 0
E_INVALID_ARG, E_MESH, E_INFEASIBLE, E_NOCONV = -1, -2, -3, -4
E_LINESEARCH, E_CAPACITY, E_DEVICE, E_OOM = -5, -6, -7, -8
PT, EE, PG = 0, 1, 2
DYNAMIC, STATIC = 0, 1
PAIRS_ALL_ONE, PAIRS_BY_SHARED = 0, 1
STAGES = ("body", "broad", "barrier", "pcg", "ccd", "linesearch", "other",
          "assemble")


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("dhat", C.c_double),
                ("kappa", C.c_double), ("kappa_A", C.c_double),
                ("gravity", C.c_double * 3), ("newton_theta", C.c_double),
                ("pcg_eta", C.c_double), ("ground_y", C.c_double),
                ("max_newton", C.c_int32), ("max_pcg", C.c_int32),
                ("max_ls", C.c_int32), ("has_ground", C.c_int32),
                ("mollify_ee", C.c_int32), ("precision", C.c_int32),
                ("list_capacity", C.c_int64), ("mixed_switch", C.c_int32),
                ("deterministic", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("pcg_variant", C.c_int32), ("pcg_blocks", C.c_int32),
                ("grid_blocks", C.c_int32), ("assemble_blocks", C.c_int32),
                ("use_graphs", C.c_int32), ("overlap_body", C.c_int32),
                ("pcg_coop", C.c_int32), ("body_pairs", C.c_int32),
                ("pcg_launch_groups", C.c_int32), ("label_rows", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PCG_TWO_BARRIER, PCG_PIPELINED, PCG_LOCAL, PCG_LOCAL1 = 0, 1, 2, 3
BODY_PAIRS_AUTO, BODY_PAIRS_ALL, BODY_PAIRS_SWEEP = 0, 1, 2


class AdmmParams(C.Structure):
    _fields_ = [("beta", C.c_double), ("rho_fixed", C.c_double),
                ("tau", C.c_double), ("mu", C.c_double),
                ("sigma_min", C.c_double), ("sigma_max", C.c_double),
                ("scale", C.c_double), ("adapt_rho", C.c_int32),
                ("merge_check", C.c_int32), ("max_iters", C.c_int32)]


class AdmmReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32),
                ("merge_ok", C.c_int32), ("newton_iters_total", C.c_int32),
                ("eps_newton", C.c_double), ("r_inf", C.c_double),
                ("s_inf", C.c_double), ("min_toi", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters_total", C.c_int32),
                ("ls_halvings", C.c_int32), ("status", C.c_int32),
                ("final_eps_N", C.c_double), ("min_alpha", C.c_double),
                ("min_dist", C.c_double), ("scene_scale", C.c_double),
                ("n_cand_pt", C.c_int64), ("n_cand_ee", C.c_int64),
                ("n_cand_pg", C.c_int64), ("n_active", C.c_int64),
                ("t_solve_ms", C.c_double),
                ("n_body_pairs", C.c_int64), ("n_chunk_pairs", C.c_int64),
                ("n_body_pairs_swept", C.c_int64),
                ("n_chunk_pairs_swept", C.c_int64),
                ("fp64_fallback", C.c_int32), ("newton_fp32", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BalanceState(C.Structure):
    _fields_ = [("k_p", C.c_double), ("k_d", C.c_double),
                ("smooth", C.c_double), ("tau", C.c_double * 2),
                ("T_prev", C.c_double), ("frames", C.c_int32),
                ("pad_", C.c_int32)]


_lib = None
EXPORTS = ["abd_create", "abd_destroy", "abd_last_error", "abd_add_body",
           "abd_finalize", "abd_sizes", "abd_set_shared",
           "abd_set_pair_replication", "abd_begin_step", "abd_local_solve",
           "abd_end_step", "abd_get_state", "abd_set_state", "abd_get_qtilde",
           "abd_set_step", "abd_set_stream", "abd_get_vertices",
           "abd_export_candidates", "abd_eval", "abd_direction", "abd_ccd",
           "abd_energy_delta", "abd_set_timing", "abd_get_timing",
           "abd_reset_timing", "abd_batch_create", "abd_batch_run",
           "abd_batch_solve", "abd_batch_destroy", "abd_get_tuning", "abd_set_tuning",
           "abd_autotune", "abd_consensus_create", "abd_consensus_destroy",
           "abd_consensus_begin", "abd_consensus_update",
           "abd_consensus_adapt", "abd_consensus_merge", "abd_consensus_get",
           "abd_admm_step", "abd_bind_workspace", "abd_workspace_info",
           "abd_balance_update", "abd_check_penetration",
           "abd_get_timing_flops", "abd_local_solve_static"]


TIMING_OFF, TIMING_ALL, TIMING_PCG, TIMING_ASM = 0, 1, 2, 3


def lib():
    """Load libabd.so (built by paper_2605_15875_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libabd.so not built ({LIB_PATH}); run "
                           "python -m paper_2605_15875_amd.build")
    L = C.CDLL(LIB_PATH)
    dp, ip, lp = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                  C.POINTER(C.c_int64))
    vp = C.c_void_p
    sig = {
        "abd_create": (C.c_int, [C.POINTER(vp), C.POINTER(Params)]),
        "abd_destroy": (None, [vp]),
        "abd_last_error": (C.c_char_p, [vp]),
        "abd_add_body": (C.c_int, [vp, dp, C.c_int32, ip, C.c_int32,
                                   C.c_double, dp, dp, C.c_int32, ip]),
        "abd_finalize": (C.c_int, [vp]),
        "abd_sizes": (C.c_int, [vp, lp]),
        "abd_set_shared": (C.c_int, [vp, ip, C.c_int32, dp, dp, dp, ip]),
        "abd_set_pair_replication": (C.c_int, [vp, C.c_int32]),
        "abd_begin_step": (C.c_int, [vp]),
        "abd_local_solve": (C.c_int, [vp, C.POINTER(Stats)]),
        "abd_local_solve_static": (C.c_int, [vp, C.POINTER(Stats)]),
        "abd_end_step": (C.c_int, [vp]),
        "abd_get_state": (C.c_int, [vp, dp, dp]),
        "abd_set_state": (C.c_int, [vp, dp, dp]),
        "abd_get_qtilde": (C.c_int, [vp, dp]),
        "abd_set_step": (C.c_int, [vp, dp, dp, C.c_double]),
        "abd_set_stream": (C.c_int, [vp, vp]),
        "abd_bind_workspace": (C.c_int, [vp, vp, C.c_size_t]),
        "abd_workspace_info": (C.c_int, [vp, lp]),
        "abd_balance_update": (C.c_int, [C.POINTER(BalanceState), C.c_double,
                                         C.c_double, dp]),
        "abd_get_vertices": (C.c_int, [vp, dp, dp, dp, dp]),
        "abd_export_candidates": (C.c_int, [vp, C.c_int32, dp, ip, C.c_int64,
                                            lp]),
        "abd_eval": (C.c_int, [vp, dp, dp, dp, dp, C.c_int64, lp, ip, dp, lp]),
        "abd_direction": (C.c_int, [vp, dp, ip]),
        "abd_ccd": (C.c_int, [vp, dp, dp, dp, C.c_int64, lp]),
        "abd_energy_delta": (C.c_int, [vp, dp, C.c_double, dp]),
        "abd_set_timing": (C.c_int, [vp, C.c_int32]),
        "abd_get_timing": (C.c_int, [vp, C.c_int32, dp, lp, dp]),
        "abd_reset_timing": (C.c_int, [vp]),
        "abd_get_timing_flops": (C.c_int, [vp, C.c_int32, dp]),
        "abd_check_penetration": (C.c_int, [vp, lp, dp]),
        "abd_batch_create": (C.c_int, [C.POINTER(vp), C.c_int32,
                                       C.POINTER(vp)]),
        "abd_batch_run": (C.c_int, [vp, C.POINTER(Stats)]),
        "abd_batch_solve": (C.c_int, [C.POINTER(vp), C.c_int32,
                                      C.POINTER(Stats)]),
        "abd_batch_destroy": (None, [vp]),
        "abd_get_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
        "abd_set_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
        "abd_autotune": (C.c_int, [vp, C.POINTER(Tuning)]),
        "abd_consensus_create": (C.c_int, [vp, ip, ip, ip, C.c_int32,
                                           C.c_int32, C.POINTER(AdmmParams),
                                           C.POINTER(vp)]),
        "abd_consensus_destroy": (None, [vp]),
        "abd_consensus_begin": (C.c_int, [vp]),
        "abd_consensus_update": (C.c_int, [vp, C.POINTER(AdmmReport)]),
        "abd_consensus_adapt": (C.c_int, [vp]),
        "abd_consensus_merge": (C.c_int, [vp]),
        "abd_consensus_get": (C.c_int, [vp, dp, dp, dp]),
        "abd_admm_step": (C.c_int, [vp, C.POINTER(AdmmReport)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


def make_params(p: dict) -> Params:
    o = Params()
    o.dt, o.dhat, o.kappa, o.kappa_A = (p["dt"], p["dhat"], p["kappa"],
                                        p["kappa_A"])
    for i in range(3):
        o.gravity[i] = p["gravity"][i]
    o.newton_theta, o.pcg_eta = p["newton_theta"], p["pcg_eta"]
    o.ground_y = p.get("ground_y", 0.0)
    o.max_newton, o.max_pcg, o.max_ls = (int(p["max_newton"]),
                                         int(p["max_pcg"]), int(p["max_ls"]))
    o.has_ground = int(p.get("has_ground", 0))
    o.mollify_ee = int(p.get("mollify_ee", 1))
    o.precision = int(p.get("precision", 0))
    o.list_capacity = int(p.get("list_capacity", 0))
    o.mixed_switch = int(p.get("mixed_switch", 0))
    o.deterministic = int(p.get("deterministic", 0))
    return o


class AbdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libabd status {code}: {msg}")
        self.code = code


class Solver:
    """One libabd context holding a scenes.Scene on the current device."""

    def __init__(self, scene, finalize=True, workspace=None, **param_over):
        """workspace: optional device memory for every buffer of the
        context, a CUDA tensor (kept alive by the Solver) or a
        (device pointer, bytes) pair."""
        L = lib()
        p = dict(scene.params)
        p.update(param_over)
        self.params = p
        self._p = make_params(p)
        h = C.c_void_p()
        rc = L.abd_create(C.byref(h), C.byref(self._p))
        if rc != OK:
            raise AbdError(rc, "abd_create failed")
        self.h = h
        self.scene = scene
        self._ws = workspace
        if workspace is not None:
            if isinstance(workspace, tuple):
                ptr, nbytes = workspace
            else:
                ptr = workspace.data_ptr()
                nbytes = workspace.numel() * workspace.element_size()
            self._check(L.abd_bind_workspace(h, C.c_void_p(int(ptr)),
                                             int(nbytes)))
        bid = np.zeros(1, dtype=np.int32)
        for b in scene.bodies:
            xb = _f64(b.xbar)
            tr = np.ascontiguousarray(b.tris, dtype=np.int32)
            q0, qd = _f64(b.q0), _f64(b.qdot0)
            self._check(L.abd_add_body(h, _d(xb), xb.shape[0], _i(tr),
                                       tr.shape[0], float(b.density), _d(q0),
                                       _d(qd), int(b.kind), _i(bid)))
        sz = np.zeros(4, dtype=np.int64)
        L.abd_sizes(h, _l(sz))
        self.B, self.V, self.T, self.E = (int(v) for v in sz)
        if finalize:
            self._check(L.abd_finalize(h))

    def close(self):
        if getattr(self, "h", None):
            lib().abd_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_info(self):
        """(usable bytes, bytes in use, most bytes ever in use) of the bound
        workspace; zeros when none is bound."""
        info = np.zeros(3, dtype=np.int64)
        self._check(lib().abd_workspace_info(self.h, _l(info)))
        return tuple(int(v) for v in info)

    def error(self):
        return lib().abd_last_error(self.h).decode()

    def _check(self, rc):
        if rc != OK:
            raise AbdError(rc, self.error())
        return rc

    # ---- simulation ----
    def set_shared(self, ids, z, u, rho, kappa_b):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        n = len(ids)
        z = _f64(z, (-1, 12)) if n else np.zeros((1, 12))
        u = _f64(u, (-1, 12)) if n else np.zeros((1, 12))
        rho = _f64(rho) if n else np.zeros(1)
        kb = np.ascontiguousarray(kappa_b if n else [1], dtype=np.int32)
        return self._check(lib().abd_set_shared(self.h, _i(ids), n, _d(z),
                                                _d(u), _d(rho), _i(kb)))

    def set_pair_replication(self, mode):
        return self._check(lib().abd_set_pair_replication(self.h, mode))

    def set_stream(self, stream_handle):
        return self._check(lib().abd_set_stream(self.h, stream_handle))

    def begin_step(self):
        return self._check(lib().abd_begin_step(self.h))

    def local_solve(self, check=True):
        st = Stats()
        rc = lib().abd_local_solve(self.h, C.byref(st))
        if check:
            self._check(rc)
        return st.as_dict()

    def local_solve_static(self, check=True):
        """The allocation-free solve: lists in the library's static device
        scratch (see abd_local_solve_static)."""
        st = Stats()
        rc = lib().abd_local_solve_static(self.h, C.byref(st))
        if check:
            self._check(rc)
        return st.as_dict()

    def end_step(self):
        return self._check(lib().abd_end_step(self.h))

    def step(self):
        self.begin_step()
        st = self.local_solve()
        self.end_step()
        return st

    def get_state(self):
        q = np.zeros((self.B, 12))
        qd = np.zeros((self.B, 12))
        self._check(lib().abd_get_state(self.h, _d(q), _d(qd)))
        return q, qd

    def set_state(self, q, qdot=None):
        q = _f64(q, (-1, 12))
        qd = _f64(qdot, (-1, 12)) if qdot is not None else None
        self._check(lib().abd_set_state(self.h, _d(q),
                                        _d(qd) if qd is not None else None))

    def qtilde(self):
        out = np.zeros((self.B, 12))
        self._check(lib().abd_get_qtilde(self.h, _d(out)))
        return out

    def set_step(self, qt, qtilde, scale):
        qt, qtilde = _f64(qt, (-1, 12)), _f64(qtilde, (-1, 12))
        self._check(lib().abd_set_step(self.h, _d(qt), _d(qtilde),
                                       float(scale)))

    # ---- hooks ----
    def vertices(self, q=None, dq=None):
        x = np.zeros((self.V, 3))
        dx = np.zeros((self.V, 3)) if dq is not None else None
        qq = _f64(q, (-1, 12)) if q is not None else None
        dd = _f64(dq, (-1, 12)) if dq is not None else None
        self._check(lib().abd_get_vertices(
            self.h, _d(qq) if qq is not None else None,
            _d(dd) if dd is not None else None, _d(x),
            _d(dx) if dx is not None else None))
        return (x, dx) if dq is not None else x

    def candidates(self, kind, dq=None):
        dd = _f64(dq, (-1, 12)) if dq is not None else None
        n = np.zeros(1, dtype=np.int64)
        L = lib()
        self._check(L.abd_export_candidates(
            self.h, kind, _d(dd) if dd is not None else None, None, 0, _l(n)))
        w = 1 if kind == PG else 2
        out = np.zeros(max(int(n[0]), 1) * w, dtype=np.int32)
        self._check(L.abd_export_candidates(
            self.h, kind, _d(dd) if dd is not None else None, _i(out),
            int(n[0]), _l(n)))
        out = out[: int(n[0]) * w]
        return out.reshape(-1, 2) if w == 2 else out

    def eval(self, q=None):
        qq = _f64(q, (-1, 12)) if q is not None else None
        E = np.zeros(1)
        g = np.zeros((self.B, 12))
        Hd = np.zeros((self.B, 12, 12))
        n = np.zeros(1, dtype=np.int64)
        na = np.zeros(1, dtype=np.int64)
        L = lib()
        qp = _d(qq) if qq is not None else None
        self._check(L.abd_eval(self.h, qp, _d(E), _d(g), _d(Hd), 0, _l(n),
                               None, None, _l(na)))
        cap = max(int(n[0]), 1)
        ij = np.zeros((cap, 2), dtype=np.int32)
        Ho = np.zeros((cap, 12, 12))
        self._check(L.abd_eval(self.h, qp, _d(E), _d(g), _d(Hd), cap, _l(n),
                               _i(ij), _d(Ho), _l(na)))
        k = int(n[0])
        return dict(E=float(E[0]), g=g, Hdiag=Hd, off_ij=ij[:k], Hoff=Ho[:k],
                    n_active=int(na[0]))

    def direction(self):
        dq = np.zeros((self.B, 12))
        it = np.zeros(1, dtype=np.int32)
        self._check(lib().abd_direction(self.h, _d(dq), _i(it)))
        return dq, int(it[0])

    def ccd(self, dq, per_pair=False):
        """alpha_max of the step dq; with per_pair, also each swept
        candidate's TOI (PT, EE, PG pairs in the order of candidates())."""
        dd = _f64(dq, (-1, 12))
        a = np.zeros(1)
        n = np.zeros(1, dtype=np.int64)
        if not per_pair:
            self._check(lib().abd_ccd(self.h, _d(dd), _d(a), None, 0, None))
            return float(a[0])
        self._check(lib().abd_ccd(self.h, _d(dd), _d(a), None, 0, _l(n)))
        toi = np.zeros(max(1, int(n[0])))
        self._check(lib().abd_ccd(self.h, _d(dd), _d(a), _d(toi), len(toi),
                                  _l(n)))
        return float(a[0]), toi[:int(n[0])]

    def energy_delta(self, dq, alpha):
        dd = _f64(dq, (-1, 12))
        e = np.zeros(1)
        self._check(lib().abd_energy_delta(self.h, _d(dd), float(alpha),
                                           _d(e)))
        return float(e[0])

    # ---- launch tuning ----
    def tuning(self):
        t = Tuning()
        self._check(lib().abd_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning(**{**self.tuning(), **kw})
        self._check(lib().abd_set_tuning(self.h, C.byref(t)))

    def autotune(self):
        t = Tuning()
        self._check(lib().abd_autotune(self.h, C.byref(t)))
        return t.as_dict()

    # ---- timing ----
    def set_timing(self, on):
        self._check(lib().abd_set_timing(self.h, int(on)))

    def reset_timing(self):
        self._check(lib().abd_reset_timing(self.h))

    def timing(self):
        out = {}
        for s, name in enumerate(STAGES):
            ms = np.zeros(1)
            n = np.zeros(1, dtype=np.int64)
            by = np.zeros(1)
            self._check(lib().abd_get_timing(self.h, s, _d(ms), _l(n), _d(by)))
            fl = np.zeros(1)
            self._check(lib().abd_get_timing_flops(self.h, s, _d(fl)))
            out[name] = dict(ms=float(ms[0]), launches=int(n[0]),
                             bytes=float(by[0]), flops=float(fl[0]))
        return out

    def check_penetration(self):
        """(edge-triangle crossings, smallest candidate distance) of the
        current state; penetration free iff (0, > 0)."""
        nc = np.zeros(1, dtype=np.int64)
        md = np.zeros(1)
        self._check(lib().abd_check_penetration(self.h, _l(nc), _d(md)))
        return int(nc[0]), float(md[0])


class Batch:
    """Several Solver contexts solved together in the same launches."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.h for s in self.solvers])
        h = C.c_void_p()
        rc = lib().abd_batch_create(arr, len(self.solvers), C.byref(h))
        if rc != OK:
            raise AbdError(rc, "abd_batch_create: " + self.solvers[0].error())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().abd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def local_solve(self, check=True):
        st = (Stats * len(self.solvers))()
        rc = lib().abd_batch_run(self.h, st)
        if check and rc != OK:
            bad = [i for i in range(len(self.solvers)) if st[i].status != OK]
            raise AbdError(rc, f"batch solve: problems {bad} failed")
        return [s.as_dict() for s in st]

    def step(self):
        for s in self.solvers:
            s.begin_step()
        out = self.local_solve()
        for s in self.solvers:
            s.end_step()
        return out


def batch_solve(solvers, check=True):
    """One-call batched local solve of several Solver contexts (the merged
    scene is kept by the first context between calls)."""
    arr = (C.c_void_p * len(solvers))(*[s.h for s in solvers])
    st = (Stats * len(solvers))()
    rc = lib().abd_batch_solve(arr, len(solvers), st)
    if check and rc != OK:
        raise AbdError(rc, "abd_batch_solve: " + solvers[0].error())
    return [s.as_dict() for s in st]


class Consensus:
    """Device consensus ADMM over the problems of a Batch (subdomains of one
    scene); the replica table is a scenes.Split's."""

    def __init__(self, batch, rep_prob, rep_body, rep_group, n_groups,
                 beta=1.0, rho_fixed=0.0, tau=2.0, mu=5.0, sigma_min=1e-3,
                 sigma_max=1e3, scale=0.0, adapt_rho=True, merge_check=True,
                 max_iters=50):
        self.batch = batch
        self.rp = np.ascontiguousarray(rep_prob, dtype=np.int32)
        self.rb = np.ascontiguousarray(rep_body, dtype=np.int32)
        self.rg = np.ascontiguousarray(rep_group, dtype=np.int32)
        self.n_rep, self.n_groups = len(self.rp), int(n_groups)
        self._ap = AdmmParams(beta, rho_fixed, tau, mu, sigma_min, sigma_max,
                              scale, int(adapt_rho), int(merge_check),
                              max_iters)
        h = C.c_void_p()
        rc = lib().abd_consensus_create(batch.h, _i(self.rp), _i(self.rb),
                                        _i(self.rg), self.n_rep,
                                        self.n_groups, C.byref(self._ap),
                                        C.byref(h))
        if rc != OK:
            raise AbdError(rc, "abd_consensus_create: " +
                           batch.solvers[0].error())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().abd_consensus_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise AbdError(rc, "consensus call failed")

    def begin(self):
        self._check(lib().abd_consensus_begin(self.h))

    def update(self):
        r = AdmmReport()
        self._check(lib().abd_consensus_update(self.h, C.byref(r)))
        return r.as_dict()

    def adapt(self):
        self._check(lib().abd_consensus_adapt(self.h))

    def merge(self):
        self._check(lib().abd_consensus_merge(self.h))

    def get(self):
        z = np.zeros((self.n_groups, 12))
        u = np.zeros((self.n_rep, 12))
        rho = np.zeros(self.n_rep)
        self._check(lib().abd_consensus_get(self.h, _d(z), _d(u), _d(rho)))
        return z, u, rho

    def admm_step(self, check=True):
        r = AdmmReport()
        rc = lib().abd_admm_step(self.h, C.byref(r))
        if check and rc != OK:
            raise AbdError(rc, "abd_admm_step: " + self.batch.solvers[0].error())
        return r.as_dict()


class Balance:
    """PD controller of the plane between two workers (libabd host code):
    update(t1, t2) takes the frame times of workers 1 and 2 and returns the
    shift of the plane along its normal (from worker 1 to worker 2)."""

    def __init__(self, k_p, k_d, smooth=1.0):
        self.st = BalanceState(k_p=k_p, k_d=k_d, smooth=smooth)

    def update(self, t1, t2):
        dp = C.c_double()
        rc = lib().abd_balance_update(C.byref(self.st), float(t1), float(t2),
                                      C.byref(dp))
        if rc != OK:
            raise AbdError(rc, "abd_balance_update: bad gains or times")
        return dp.value
