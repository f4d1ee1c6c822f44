"""Thin ctypes binding of libmpap (include/mpap.h), same names as the C ABI.

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  If the library is not built, or no gfx950 device is present, calls
fail loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpap.so")

MPAP_OK = 0
MPAP_ERR_INVAL = 1
MPAP_ERR_NOGOAL = 2
MPAP_ERR_NOMEM = 3
MPAP_ERR_HIP = 4
MPAP_ERR_OVERFLOW = 5
MPAP_ERR_NOCONVERGE = 6
MPAP_ERR_CAPACITY = 7
MPAP_ERR_DEVICE = 8
MPAP_PLAN_ANALYTIC = 1


class MpapError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"mpap status {status}: {message}")
        self.status = status


class mpap_env(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("pos", ctypes.c_void_p), ("n_boxes", ctypes.c_int32),
                ("box_lo", ctypes.c_void_p), ("box_hi", ctypes.c_void_p),
                ("n_blobs", ctypes.c_int32), ("blob_mu", ctypes.c_void_p),
                ("blob_sigma", ctypes.c_void_p), ("blob_amp", ctypes.c_void_p),
                ("goal", ctypes.c_float * 3), ("goal_radius", ctypes.c_float),
                ("vel", ctypes.c_void_p)]


class mpap_graph_params(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_float), ("check_step", ctypes.c_float),
                ("reset_q", ctypes.c_float), ("k_out", ctypes.c_int32),
                ("horizon", ctypes.c_float), ("traj_steps", ctypes.c_int32),
                ("near_grid", ctypes.c_int32)]


class mpap_search_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_float), ("lambda_", ctypes.c_float),
                ("radius", ctypes.c_float), ("n_obj", ctypes.c_int32),
                ("init_node", ctypes.c_int32), ("max_waves", ctypes.c_int32),
                ("near_scan", ctypes.c_int32), ("stage_cap", ctypes.c_int32),
                ("heuristic", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("wave_min_targets", ctypes.c_int32), ("skip", ctypes.c_int32),
                ("early_stop", ctypes.c_int32), ("merge_halves", ctypes.c_int32)]


class mpap_stats(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("retries", ctypes.c_int32),
                ("labels_expanded", ctypes.c_int64), ("front_labels", ctypes.c_int64),
                ("merges", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("relaxations", ctypes.c_int64), ("gpu_ms", ctypes.c_float),
                ("lds_front_cap", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("max_front", ctypes.c_int32), ("wave_build", ctypes.c_int32),
                ("judged_failed", ctypes.c_int32), ("fallback_ms", ctypes.c_float),
                ("half_front_cap", ctypes.c_int32), ("build_objectives", ctypes.c_int32),
                ("half_merges", ctypes.c_int64), ("half_backouts", ctypes.c_int64)]


class mpap_mc_params(ctypes.Structure):
    _fields_ = [("rollouts", ctypes.c_int32), ("dt", ctypes.c_float), ("speed", ctypes.c_float),
                ("sigma_w", ctypes.c_float), ("sigma_a", ctypes.c_float),
                ("sigma_v", ctypes.c_float), ("q_min", ctypes.c_float),
                ("sigma0", ctypes.c_float), ("err_bound", ctypes.c_float),
                ("q_p", ctypes.c_float), ("q_v", ctypes.c_float), ("r_u", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class mpap_mc_stats(ctypes.Structure):
    _fields_ = [("rollouts", ctypes.c_int64), ("within_bound", ctypes.c_int64),
                ("collision_free", ctypes.c_int64), ("success", ctypes.c_int64),
                ("steps", ctypes.c_int32), ("duration", ctypes.c_double),
                ("mean_max_err", ctypes.c_double), ("max_max_err", ctypes.c_double),
                ("gain_p", ctypes.c_double), ("gain_v", ctypes.c_double),
                ("gpu_ms", ctypes.c_float)]


SYMBOLS = [
    "mpap_build_graph", "mpap_graph_from_csr", "mpap_graph_info", "mpap_graph_export",
    "mpap_graph_free", "mpap_search", "mpap_goal_front", "mpap_node_front",
    "mpap_label_path", "mpap_result_stats", "mpap_result_free", "mpap_status_string",
    "mpap_last_error", "mpap_wave_trace", "mpap_graph_concat", "mpap_graph_queries",
    "mpap_search_batch", "mpap_query_goal_front", "mpap_query_info",
    "mpap_surrogate_create", "mpap_surrogate_free", "mpap_surrogate_set_params",
    "mpap_surrogate_get_params", "mpap_surrogate_init", "mpap_edge_features",
    "mpap_surrogate_forward", "mpap_surrogate_gradient", "mpap_surrogate_train",
    "mpap_surrogate_score", "mpap_graph_drift", "mpap_rescore_front", "mpap_analytic_drift",
    "mpap_plan_create", "mpap_plan_run", "mpap_plan_info", "mpap_plan_free",
    "mpap_judge", "mpap_surrogate_save", "mpap_surrogate_load", "mpap_search_noalloc",
    "mpap_query_stop", "mpap_refine_front", "mpap_graph_add_boxes", "mpap_search_update",
    "mpap_mc_verify",
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libmpap.so.  torch (if installed) is imported first so that the
    library binds to the same HIP runtime as torch in this process."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built (run __graft_entry__.build())")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.mpap_build_graph.argtypes = [ctypes.POINTER(mpap_env), ctypes.POINTER(mpap_graph_params),
                                     P, ctypes.POINTER(P)]
    lib.mpap_graph_from_csr.argtypes = [I32, P, P, P, P, P, P, P, ctypes.POINTER(P)]
    lib.mpap_graph_info.argtypes = [P, P, P, P]
    lib.mpap_graph_export.argtypes = [P, P, P, P, P, P, P]
    lib.mpap_graph_free.argtypes = [P]
    lib.mpap_graph_free.restype = None
    lib.mpap_search.argtypes = [P, ctypes.POINTER(mpap_search_params), P, ctypes.POINTER(P)]
    lib.mpap_goal_front.argtypes = [P, P, P, P, P, P, I32, P]
    lib.mpap_node_front.argtypes = [P, I32, P, P, P, P, I32, P]
    lib.mpap_label_path.argtypes = [P, I32, P, I32, P]
    lib.mpap_result_stats.argtypes = [P, ctypes.POINTER(mpap_stats)]
    lib.mpap_wave_trace.argtypes = [P, P, I32, P]
    lib.mpap_graph_concat.argtypes = [P, I32, P, ctypes.POINTER(P)]
    lib.mpap_graph_queries.argtypes = [P, P, P]
    lib.mpap_search_batch.argtypes = [P, P, I32, P, ctypes.POINTER(P)]
    lib.mpap_query_goal_front.argtypes = [P, I32, P, P, P, P, P, I32, P]
    lib.mpap_query_info.argtypes = [P, I32, P, P]
    lib.mpap_surrogate_create.argtypes = [ctypes.POINTER(P)]
    lib.mpap_surrogate_free.argtypes = [P]
    lib.mpap_surrogate_free.restype = None
    lib.mpap_surrogate_set_params.argtypes = [P, P, I32]
    lib.mpap_surrogate_get_params.argtypes = [P, P, I32, P]
    lib.mpap_surrogate_init.argtypes = [P, ctypes.c_uint64]
    lib.mpap_edge_features.argtypes = [P, P, P, I64, P]
    lib.mpap_surrogate_forward.argtypes = [P, P, I64, P]
    lib.mpap_surrogate_gradient.argtypes = [P, P, P, I32, P, P]
    lib.mpap_surrogate_train.argtypes = [P, P, P, I64, I32, I32, ctypes.c_float, P, P]
    lib.mpap_surrogate_score.argtypes = [P, P, P, P]
    lib.mpap_graph_drift.argtypes = [P, I32, P]
    lib.mpap_analytic_drift.argtypes = [P, P, P]
    lib.mpap_rescore_front.argtypes = [P, I32, P, P, P, P, I32, P]
    lib.mpap_plan_create.argtypes = [P, P, I32, P, P, I32, I32, P, ctypes.POINTER(P)]
    lib.mpap_plan_run.argtypes = [P, P, ctypes.POINTER(P)]
    lib.mpap_plan_info.argtypes = [P, P, P, P]
    lib.mpap_judge.argtypes = [P, ctypes.c_float, I32, P, P, P]
    lib.mpap_surrogate_save.argtypes = [P, ctypes.c_char_p]
    lib.mpap_surrogate_load.argtypes = [P, ctypes.c_char_p]
    lib.mpap_search_noalloc.argtypes = [P, ctypes.POINTER(mpap_search_params), P, P, P, P, P,
                                        I32, P]
    lib.mpap_query_stop.argtypes = [P, I32, P]
    lib.mpap_mc_verify.argtypes = [P, P, I32, ctypes.POINTER(mpap_mc_params), P, P, P,
                                   ctypes.POINTER(mpap_mc_stats)]
    lib.mpap_graph_add_boxes.argtypes = [P, I32, P, P, P, ctypes.POINTER(P)]
    lib.mpap_search_update.argtypes = [P, P, ctypes.POINTER(mpap_search_params), P,
                                       ctypes.POINTER(P)]
    lib.mpap_refine_front.argtypes = [P, I32, ctypes.c_float, I32, P, P, P, P, P, I32, P]
    lib.mpap_plan_free.argtypes = [P]
    lib.mpap_plan_free.restype = None
    lib.mpap_result_free.argtypes = [P]
    lib.mpap_result_free.restype = None
    lib.mpap_status_string.argtypes = [ctypes.c_int]
    lib.mpap_status_string.restype = ctypes.c_char_p
    lib.mpap_last_error.argtypes = []
    lib.mpap_last_error.restype = ctypes.c_char_p
    for name in ("mpap_build_graph", "mpap_graph_from_csr", "mpap_graph_info",
                 "mpap_graph_export", "mpap_search", "mpap_goal_front", "mpap_node_front",
                 "mpap_label_path", "mpap_result_stats", "mpap_wave_trace",
                 "mpap_graph_concat", "mpap_graph_queries", "mpap_search_batch",
                 "mpap_query_goal_front", "mpap_query_info", "mpap_surrogate_create",
                 "mpap_surrogate_set_params", "mpap_surrogate_get_params",
                 "mpap_surrogate_init", "mpap_edge_features", "mpap_surrogate_forward",
                 "mpap_surrogate_gradient", "mpap_surrogate_train", "mpap_surrogate_score",
                 "mpap_graph_drift", "mpap_rescore_front", "mpap_analytic_drift",
                 "mpap_judge", "mpap_surrogate_save", "mpap_surrogate_load",
                 "mpap_search_noalloc", "mpap_query_stop", "mpap_refine_front",
                 "mpap_graph_add_boxes", "mpap_search_update", "mpap_mc_verify"):
        getattr(lib, name).restype = ctypes.c_int
    _ = I64
    _lib = lib
    return lib


def _check(status: int):
    if status != MPAP_OK:
        msg = _lib.mpap_last_error().decode(errors="replace")
        raise MpapError(status, msg)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(int(stream.cuda_stream))  # torch.cuda.Stream


class Graph:
    """Owner of an mpap_graph handle."""

    def __init__(self, handle):
        self.handle = handle

    def info(self):
        n = ctypes.c_int32()
        e = ctypes.c_int64()
        g = ctypes.c_int32()
        _check(load().mpap_graph_info(self.handle, ctypes.byref(n), ctypes.byref(e),
                                      ctypes.byref(g)))
        return dict(n=n.value, e=e.value, n_goal=g.value)

    def export(self) -> dict:
        inf = self.info()
        n, e = inf["n"], inf["e"]
        out = dict(row_ptr=np.empty(n + 1, np.int32), col=np.empty(e, np.int32),
                   cost=np.empty(e, np.float32), drift=np.empty(e, np.float32),
                   reset=np.empty(n, np.uint8), goal=np.empty(n, np.uint8))
        _check(load().mpap_graph_export(self.handle, _p(out["row_ptr"]), _p(out["col"]),
                                        _p(out["cost"]), _p(out["drift"]), _p(out["reset"]),
                                        _p(out["goal"])))
        return out

    def close(self):
        if self.handle:
            load().mpap_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mpap_graph_from_csr(row_ptr, col, cost, drift, reset, goal, stream=None) -> Graph:
    lib = load()
    rp = np.ascontiguousarray(row_ptr, np.int32)
    cl = np.ascontiguousarray(col, np.int32)
    co = np.ascontiguousarray(cost, np.float32)
    dr = np.ascontiguousarray(drift, np.float32)
    rs = np.ascontiguousarray(reset, np.uint8)
    go = np.ascontiguousarray(goal, np.uint8)
    h = ctypes.c_void_p()
    _check(lib.mpap_graph_from_csr(rp.shape[0] - 1, _p(rp), _p(cl), _p(co), _p(dr), _p(rs),
                                   _p(go), _stream(stream), ctypes.byref(h)))
    return Graph(h)


def mpap_build_graph(env, radius=None, check_step=None, reset_q=None, stream=None,
                     near_grid: int = 0) -> Graph:
    """Build the roadmap of an environment (synth.Env or alike) on the GPU.
    near_grid: 0 lets the library choose how Near finds candidates, 1 a
    uniform grid, -1 all pairs (the same edges either way)."""
    lib = load()
    pos = np.ascontiguousarray(env.pos, np.float32)
    lo = np.ascontiguousarray(env.box_lo, np.float32)
    hi = np.ascontiguousarray(env.box_hi, np.float32)
    mu = np.ascontiguousarray(env.blob_mu, np.float32)
    sg = np.ascontiguousarray(env.blob_sigma, np.float32)
    am = np.ascontiguousarray(env.blob_amp, np.float32)
    e = mpap_env()
    e.dim = env.dim
    e.n_nodes = pos.shape[0]
    e.pos = _p(pos).value
    e.n_boxes = lo.shape[0]
    e.box_lo = _p(lo).value
    e.box_hi = _p(hi).value
    e.n_blobs = mu.shape[0]
    e.blob_mu = _p(mu).value
    e.blob_sigma = _p(sg).value
    e.blob_amp = _p(am).value
    wdim = 3 if env.dim == 6 else env.dim
    gl = np.zeros(3, np.float32)
    gl[:wdim] = env.goal
    for k in range(3):
        e.goal[k] = float(gl[k])
    e.goal_radius = float(env.goal_radius)
    vel = None
    if env.dim == 6:
        vel = np.ascontiguousarray(env.vel, np.float32)
        e.vel = _p(vel).value
    gp = mpap_graph_params(float(env.radius if radius is None else radius),
                           float(env.check_step if check_step is None else check_step),
                           float(env.reset_q if reset_q is None else reset_q),
                           int(getattr(env, "k_out", 0)), float(getattr(env, "horizon", 0.0)),
                           int(getattr(env, "traj_steps", 0)), int(near_grid))
    h = ctypes.c_void_p()
    _check(lib.mpap_build_graph(ctypes.byref(e), ctypes.byref(gp), _stream(stream),
                                ctypes.byref(h)))
    return Graph(h)


@dataclasses.dataclass
class Front:
    vecs: np.ndarray      # float32 [k, 3] (cost, drift, max drift)
    goal_node: np.ndarray  # int32 [k]
    label: np.ndarray      # int32 [k]


class Result:
    """Owner of an mpap_result handle.  Free results before their graph."""

    def __init__(self, handle, graph: Graph):
        self.handle = handle
        self.graph = graph

    def goal_front(self, query: int = 0) -> Front:
        return mpap_query_goal_front(self, query)

    def query_info(self, query: int) -> dict:
        return mpap_query_info(self, query)

    def node_front(self, node: int, with_ids: bool = False):
        return mpap_node_front(self, node, with_ids)

    def path(self, label: int) -> list[int]:
        return mpap_label_path(self, label)

    def stats(self) -> dict:
        return mpap_result_stats(self)

    def wave_trace(self) -> np.ndarray:
        return mpap_wave_trace(self)

    def judge(self, tol: float = 1e-2, fallback: bool = True, stream=None) -> np.ndarray:
        return mpap_judge(self, tol, fallback, stream)

    def stop(self, query: int = 0) -> int:
        return mpap_query_stop(self, query)

    def refine(self, beta_prime: float, n_obj_out: int = 2, query: int = 0) -> Front:
        return mpap_refine_front(self, query, beta_prime, n_obj_out)

    def close(self):
        if self.handle:
            load().mpap_result_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def search_params(beta: float, n_obj: int, radius: float, lam: float = 0.5,
                  init_node: int = 0, max_waves: int = 0, near_scan: int = 0,
                  stage_cap: int = 0, heuristic: int = 0, block_threads: int = 0,
                  wave_min_targets: int = 0, skip: int = 0, early_stop: int = 0,
                  merge_halves: int = 0):
    return mpap_search_params(float(beta), float(lam), float(radius), int(n_obj),
                              int(init_node), int(max_waves), int(near_scan), int(stage_cap),
                              int(heuristic), int(block_threads), int(wave_min_targets),
                              int(skip), int(early_stop), int(merge_halves))


def mpap_search(graph: Graph, beta: float, n_obj: int, radius: float, lam: float = 0.5,
                init_node: int = 0, max_waves: int = 0, near_scan: int = 0,
                stage_cap: int = 0, heuristic: int = 0, stream=None,
                block_threads: int = 0, wave_min_targets: int = 0,
                early_stop: int = 0, merge_halves: int = 0) -> Result:
    lib = load()
    sp = search_params(beta, n_obj, radius, lam, init_node, max_waves, near_scan, stage_cap,
                       heuristic, block_threads, wave_min_targets, early_stop=early_stop,
                       merge_halves=merge_halves)
    h = ctypes.c_void_p()
    _check(lib.mpap_search(graph.handle, ctypes.byref(sp), _stream(stream), ctypes.byref(h)))
    return Result(h, graph)


def mpap_search_noalloc(graph: Graph, beta: float, n_obj: int, radius: float,
                        lam: float = 0.5, capacity: int = 4096, stream=None, **kw) -> Front:
    """The search and goal front of mpap_search with no device allocation
    (the library's fixed per-device scratch).  Returns the goal front (label
    ids are not kept: -1)."""
    lib = load()
    sp = search_params(beta, n_obj, radius, lam, **kw)
    c = np.empty(capacity, np.float32)
    d = np.empty(capacity, np.float32)
    m = np.empty(capacity, np.float32)
    gn = np.empty(capacity, np.int32)
    k = ctypes.c_int32()
    _check(lib.mpap_search_noalloc(graph.handle, ctypes.byref(sp), _stream(stream), _p(c), _p(d),
                                   _p(m), _p(gn), capacity, ctypes.byref(k)))
    k = k.value
    return Front(np.stack([c[:k], d[:k], m[:k]], axis=1), gn[:k].copy(),
                 np.full(k, -1, np.int32))


def mpap_graph_add_boxes(graph: Graph, box_lo, box_hi, stream=None) -> Graph:
    """A new roadmap without the edges that collide with the added boxes."""
    lo = np.ascontiguousarray(box_lo, np.float32)
    hi = np.ascontiguousarray(box_hi, np.float32)
    h = ctypes.c_void_p()
    _check(load().mpap_graph_add_boxes(graph.handle, lo.shape[0], _p(lo), _p(hi),
                                       _stream(stream), ctypes.byref(h)))
    return Graph(h)


def mpap_search_update(prev: Result, graph: Graph, beta: float, n_obj: int, radius: float,
                       lam: float = 0.5, stream=None, **kw) -> Result:
    """The search of ``graph`` continued from the earlier result ``prev``."""
    sp = search_params(beta, n_obj, radius, lam, **kw)
    h = ctypes.c_void_p()
    _check(load().mpap_search_update(prev.handle, graph.handle, ctypes.byref(sp),
                                     _stream(stream), ctypes.byref(h)))
    return Result(h, graph)


MC_DEFAULTS = dict(rollouts=4096, dt=0.005, speed=0.5, sigma_w=0.1, sigma_a=0.1, sigma_v=0.005,
                   q_min=0.8, sigma0=0.002, err_bound=0.05, q_p=100.0, q_v=20.0, r_u=1.0,
                   seed=1)


def mpap_mc_verify(graph: Graph, nodes, with_samples: bool = True, stream=None, **kw):
    """Monte Carlo verification of the plan through ``nodes`` (root first).
    Keyword arguments override MC_DEFAULTS.  Returns (stats dict, max_err
    float64 [R] or None, collided bool [R] or None)."""
    path = np.ascontiguousarray(nodes, np.int32)
    p = dict(MC_DEFAULTS, **kw)
    mp = mpap_mc_params(int(p["rollouts"]), *(float(p[k]) for k in (
        "dt", "speed", "sigma_w", "sigma_a", "sigma_v", "q_min", "sigma0", "err_bound", "q_p",
        "q_v", "r_u")), int(p["seed"]))
    R = mp.rollouts
    me = np.empty(R, np.float64) if with_samples else None
    co = np.empty(R, np.uint8) if with_samples else None
    st = mpap_mc_stats()
    _check(load().mpap_mc_verify(graph.handle, _p(path), path.shape[0], ctypes.byref(mp),
                                 _stream(stream),
                                 _p(me) if with_samples else None,
                                 _p(co) if with_samples else None, ctypes.byref(st)))
    stats = {f: getattr(st, f) for f, _ in mpap_mc_stats._fields_}
    return stats, me, (co.astype(bool) if with_samples else None)


def mpap_query_stop(res: Result, query: int = 0) -> int:
    """Groups expanded before the early stop ended the query's loop, or -1."""
    g = ctypes.c_int32()
    _check(load().mpap_query_stop(res.handle, int(query), ctypes.byref(g)))
    return g.value


def mpap_refine_front(res: Result, query: int, beta_prime: float, n_obj_out: int = 2) -> Front:
    """Goal front under the bound beta_prime from a three-objective search."""
    lib = load()
    cnt = ctypes.c_int32()
    st = lib.mpap_refine_front(res.handle, int(query), ctypes.c_float(beta_prime),
                               int(n_obj_out), None, None, None, None, None, 0,
                               ctypes.byref(cnt))
    if st not in (MPAP_OK, MPAP_ERR_CAPACITY):
        _check(st)
    k = cnt.value
    c = np.empty(k, np.float32)
    d = np.empty(k, np.float32)
    m = np.empty(k, np.float32)
    gn = np.empty(k, np.int32)
    ids = np.empty(k, np.int32)
    _check(lib.mpap_refine_front(res.handle, int(query), ctypes.c_float(beta_prime),
                                 int(n_obj_out), _p(c), _p(d), _p(m), _p(gn), _p(ids), k,
                                 ctypes.byref(cnt)))
    return Front(np.stack([c, d, m], axis=1).reshape(k, 3), gn, ids)


def mpap_graph_concat(parts, stream=None) -> Graph:
    lib = load()
    arr = (ctypes.c_void_p * len(parts))(*[p.handle.value if isinstance(p.handle, ctypes.c_void_p)
                                           else p.handle for p in parts])
    h = ctypes.c_void_p()
    _check(lib.mpap_graph_concat(arr, len(parts), _stream(stream), ctypes.byref(h)))
    return Graph(h)


def mpap_graph_queries(graph: Graph) -> np.ndarray:
    """Node offsets of the queries, int32 [nq + 1]."""
    lib = load()
    nq = ctypes.c_int32()
    _check(lib.mpap_graph_queries(graph.handle, ctypes.byref(nq), None))
    off = np.empty(nq.value + 1, np.int32)
    _check(lib.mpap_graph_queries(graph.handle, ctypes.byref(nq), _p(off)))
    return off


def mpap_search_batch(graph: Graph, params, stream=None) -> Result:
    """params: one mpap_search_params (applied to all queries) or a list, one
    per query (see search_params)."""
    lib = load()
    if isinstance(params, mpap_search_params):
        params = [params]
    arr = (mpap_search_params * len(params))(*params)
    h = ctypes.c_void_p()
    _check(lib.mpap_search_batch(graph.handle, arr, len(params), _stream(stream),
                                 ctypes.byref(h)))
    return Result(h, graph)


def mpap_query_goal_front(res: Result, query: int) -> Front:
    lib = load()
    cnt = ctypes.c_int32()
    st = lib.mpap_query_goal_front(res.handle, int(query), None, None, None, None, None, 0,
                                   ctypes.byref(cnt))
    if st not in (MPAP_OK, MPAP_ERR_CAPACITY):
        _check(st)
    k = cnt.value
    c = np.empty(k, np.float32)
    d = np.empty(k, np.float32)
    m = np.empty(k, np.float32)
    gn = np.empty(k, np.int32)
    lb = np.empty(k, np.int32)
    _check(lib.mpap_query_goal_front(res.handle, int(query), _p(c), _p(d), _p(m), _p(gn),
                                     _p(lb), k, ctypes.byref(cnt)))
    return Front(np.stack([c, d, m], axis=1).reshape(k, 3), gn, lb)


def mpap_goal_front(res: Result) -> Front:
    return mpap_query_goal_front(res, 0)


def mpap_query_info(res: Result, query: int) -> dict:
    lib = load()
    ms = ctypes.c_float()
    lw = ctypes.c_int32()
    _check(lib.mpap_query_info(res.handle, int(query), ctypes.byref(ms), ctypes.byref(lw)))
    return dict(latency_ms=ms.value, last_wave=lw.value)


def mpap_node_front(res: Result, node: int, with_ids: bool = False):
    """Labels of P(node) in storage order: float32 [k, 3] (and int32 ids)."""
    lib = load()
    cnt = ctypes.c_int32()
    st = lib.mpap_node_front(res.handle, int(node), None, None, None, None, 0,
                             ctypes.byref(cnt))
    if st not in (MPAP_OK, MPAP_ERR_CAPACITY):
        _check(st)
    k = cnt.value
    c = np.empty(k, np.float32)
    d = np.empty(k, np.float32)
    m = np.empty(k, np.float32)
    ids = np.empty(k, np.int32)
    _check(lib.mpap_node_front(res.handle, int(node), _p(c), _p(d), _p(m), _p(ids), k,
                               ctypes.byref(cnt)))
    v = np.stack([c, d, m], axis=1).reshape(k, 3)
    return (v, ids) if with_ids else v


def mpap_label_path(res: Result, label: int) -> list[int]:
    lib = load()
    ln = ctypes.c_int32()
    st = lib.mpap_label_path(res.handle, int(label), None, 0, ctypes.byref(ln))
    if st not in (MPAP_OK, MPAP_ERR_CAPACITY):
        _check(st)
    buf = np.empty(ln.value, np.int32)
    _check(lib.mpap_label_path(res.handle, int(label), _p(buf), ln.value, ctypes.byref(ln)))
    return buf.tolist()


def mpap_result_stats(res: Result) -> dict:
    lib = load()
    s = mpap_stats()
    _check(lib.mpap_result_stats(res.handle, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in mpap_stats._fields_}


def mpap_wave_trace(res: Result) -> np.ndarray:
    """int64 [waves, 10] per-iteration trace (see include/mpap.h)."""
    lib = load()
    w = ctypes.c_int32()
    st = lib.mpap_wave_trace(res.handle, None, 0, ctypes.byref(w))
    if st not in (MPAP_OK, MPAP_ERR_CAPACITY):
        _check(st)
    out = np.zeros((w.value, 10), np.int64)
    _check(lib.mpap_wave_trace(res.handle, _p(out), w.value, ctypes.byref(w)))
    return out


N_PARAMS = 5313


class Surrogate:
    """Owner of an mpap_surrogate handle (the learned per-edge drift model)."""

    def __init__(self, seed=None):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.mpap_surrogate_create(ctypes.byref(h)))
        self.handle = h
        if seed is not None:
            _check(lib.mpap_surrogate_init(self.handle, ctypes.c_uint64(int(seed))))

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32).reshape(-1)
        _check(load().mpap_surrogate_set_params(self.handle, _p(p), p.shape[0]))

    def get_params(self) -> np.ndarray:
        out = np.empty(N_PARAMS, np.float32)
        cnt = ctypes.c_int32()
        _check(load().mpap_surrogate_get_params(self.handle, _p(out), N_PARAMS, ctypes.byref(cnt)))
        return out

    def forward(self, X_bits) -> np.ndarray:
        X = np.ascontiguousarray(X_bits, np.uint16).reshape(-1, 16)
        y = np.empty(X.shape[0], np.float32)
        _check(load().mpap_surrogate_forward(self.handle, _p(X), X.shape[0], _p(y)))
        return y

    def gradient(self, X_bits, t):
        X = np.ascontiguousarray(X_bits, np.uint16).reshape(-1, 16)
        tt = np.ascontiguousarray(t, np.float32)
        g = np.empty(N_PARAMS, np.float32)
        y = np.empty(X.shape[0], np.float32)
        _check(load().mpap_surrogate_gradient(self.handle, _p(X), _p(tt), X.shape[0], _p(g), _p(y)))
        return g, y

    def train(self, graph: Graph, edges, epochs: int, batch: int, lr: float, stream=None):
        e = np.ascontiguousarray(edges, np.int64)
        loss = np.zeros(max(epochs, 1), np.float32)
        _check(load().mpap_surrogate_train(self.handle, graph.handle, _p(e), e.shape[0],
                                           int(epochs), int(batch), ctypes.c_float(lr),
                                           _stream(stream), _p(loss)))
        return loss[:epochs]

    def save(self, path: str):
        _check(load().mpap_surrogate_save(self.handle, os.fsencode(path)))

    def load(self, path: str):
        _check(load().mpap_surrogate_load(self.handle, os.fsencode(path)))

    def score(self, graph: Graph, stream=None) -> float:
        ms = ctypes.c_float()
        _check(load().mpap_surrogate_score(self.handle, graph.handle, _stream(stream),
                                           ctypes.byref(ms)))
        return ms.value

    def close(self):
        if self.handle:
            load().mpap_surrogate_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mpap_edge_features(graph: Graph, with_base: bool = False):
    """[e, 16] bfloat16 bit patterns (and, with_base, the float32 8-point base)."""
    e = graph.info()["e"]
    out = np.empty((e, 16), np.uint16)
    base = np.empty(e, np.float32)
    _check(load().mpap_edge_features(graph.handle, None, _p(out), out.size, _p(base)))
    return (out, base) if with_base else out


def mpap_analytic_drift(graph: Graph, stream=None) -> float:
    """Recompute the analytic edge drift on the device; returns kernel ms."""
    ms = ctypes.c_float()
    _check(load().mpap_analytic_drift(graph.handle, _stream(stream), ctypes.byref(ms)))
    return ms.value


def mpap_graph_drift(graph: Graph, which: int) -> np.ndarray:
    out = np.empty(graph.info()["e"], np.float32)
    _check(load().mpap_graph_drift(graph.handle, int(which), _p(out)))
    return out


def mpap_rescore_front(res: Result, query: int = 0) -> dict:
    lib = load()
    cnt = ctypes.c_int32()
    st = lib.mpap_rescore_front(res.handle, int(query), None, None, None, None, 0,
                                ctypes.byref(cnt))
    if st not in (MPAP_OK, MPAP_ERR_CAPACITY):
        _check(st)
    k = cnt.value
    c = np.empty(k, np.float32)
    d = np.empty(k, np.float32)
    m = np.empty(k, np.float32)
    f = np.empty(k, np.uint8)
    _check(lib.mpap_rescore_front(res.handle, int(query), _p(c), _p(d), _p(m), _p(f), k,
                                  ctypes.byref(cnt)))
    return dict(cost=c, drift=d, maxdrift=m, feasible=f.astype(bool))


def mpap_judge(res: Result, tol: float = 1e-2, fallback: bool = True, stream=None) -> np.ndarray:
    """The library's judge of a search on the learned drift (and, with
    fallback, the analytic re-search of the rejected queries); returns the
    per-query rejection flags (bool [nq])."""
    nq = ctypes.c_int32()
    _check(load().mpap_graph_queries(res.graph.handle, ctypes.byref(nq), None))
    failed = np.zeros(nq.value, np.uint8)
    nf = ctypes.c_int32()
    _check(load().mpap_judge(res.handle, ctypes.c_float(tol), int(bool(fallback)),
                             _stream(stream), _p(failed), ctypes.byref(nf)))
    return failed.astype(bool)


class Plan:
    """A fixed batch recorded as one HIP graph (mpap_plan_*): scoring of the
    parts by their surrogates (optional), the search of every query and the
    goal fronts, launched with run().  A result of run() reads the plan's
    workspace for per-node queries until the next run()."""

    def __init__(self, graph: Graph, params, parts=None, models=None, stream=None,
                 analytic: bool = False):
        lib = load()
        if isinstance(params, mpap_search_params):
            params = [params]
        arr = (mpap_search_params * len(params))(*params)
        n = 0
        pa = ma = None
        if parts is not None:
            n = len(parts)
            models = list(models) if models is not None else [None] * n
            pa = (ctypes.c_void_p * n)(*[p.handle for p in parts])
            ma = (ctypes.c_void_p * n)(*[(m.handle if m is not None else None) for m in models])
        self.graph, self.parts, self.models = graph, parts, models
        h = ctypes.c_void_p()
        _check(lib.mpap_plan_create(graph.handle, arr, len(params), pa, ma, n,
                                    MPAP_PLAN_ANALYTIC if analytic else 0, _stream(stream),
                                    ctypes.byref(h)))
        self.handle = h

    def run(self, stream=None) -> Result:
        h = ctypes.c_void_p()
        _check(load().mpap_plan_run(self.handle, _stream(stream), ctypes.byref(h)))
        return Result(h, self.graph)

    def info(self) -> dict:
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().mpap_plan_info(self.handle, ctypes.byref(a), ctypes.byref(b),
                                     ctypes.byref(c)))
        return {"launches": a.value, "records": b.value, "fallbacks": c.value}

    def close(self):
        if self.handle:
            load().mpap_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
