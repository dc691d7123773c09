"""Python binding of libmqo (ctypes).  Argument marshalling only: every step
of the path runs in the HIP library; torch provides device memory and the
current stream.  Importing this module raises if libmqo.so is missing.
The environment variable MQO_LIBRARY, when set, names another build of the
same library to load instead (for comparing kernel variants).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MQO_LIBRARY") or os.path.join(_HERE, "libmqo.so")

MIS = 0
MAXCUT = 1
MAXCUT_FL, MAXCUT_FP, MAXCUT_FA = 2, 3, 4  # Eq. (4), (5), (6); MAXCUT is f_B, Eq. (7)
_KIND = {"mis": MIS, "maxcut": MAXCUT, "maxcut_fl": MAXCUT_FL, "maxcut_fp": MAXCUT_FP, "maxcut_fa": MAXCUT_FA,
         MIS: MIS, MAXCUT: MAXCUT, MAXCUT_FL: MAXCUT_FL, MAXCUT_FP: MAXCUT_FP, MAXCUT_FA: MAXCUT_FA}
PLANS = {"auto": 0, "plain": 1, "batched": 2, "persistent": 3}
PLAN_NAMES = {v: k for k, v in PLANS.items()}
INIT = {"uniform": 0, "degree": 1}
RESET = {"zero": 0, "flip": 1}


class MqoError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib.mqo_status_string(status).decode()} ({status}): "
                         f"{_lib.mqo_last_error().decode()}")


class _Graph(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("vtx_offset", ctypes.POINTER(ctypes.c_int64)),
                ("n_total", ctypes.c_int64), ("nnz_total", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("hub_min_degree", ctypes.c_int32),
                ("hub_offset", ctypes.POINTER(ctypes.c_int64)), ("hub_rows", ctypes.c_void_p),
                ("max_degree", ctypes.c_int32), ("local_rows", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("batch", ctypes.c_int32), ("steps_per_round", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("check_every", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("momentum", ctypes.c_float), ("gamma", ctypes.c_float), ("lam", ctypes.c_float),
                ("rho", ctypes.c_double), ("init_sigma", ctypes.c_float), ("init_mode", ctypes.c_int32),
                ("reset_mode", ctypes.c_int32), ("local_search", ctypes.c_int32), ("plan", ctypes.c_int32),
                ("tile_cols", ctypes.c_int32), ("tile_threads", ctypes.c_int32), ("tile_vec", ctypes.c_int32),
                ("tile_csr", ctypes.c_int32), ("tile_reg", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("time_budget_s", ctypes.c_double), ("maxcut_objective", ctypes.c_int32),
                ("final_search", ctypes.c_int32), ("pool_k", ctypes.c_int32),
                ("restart_every", ctypes.c_int32), ("traj_count", ctypes.c_int32),
                ("traj_ids", ctypes.POINTER(ctypes.c_int64)), ("step_vec", ctypes.c_int32),
                ("step_lanes", ctypes.c_int32), ("tile_sb", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("best_x", ctypes.c_void_p), ("best_value", ctypes.c_void_p), ("traj_best_value", ctypes.c_void_p),
                ("traj_best_x", ctypes.c_void_p), ("edge_updates", ctypes.c_int64),
                ("steps_executed", ctypes.c_int64), ("rounds_executed", ctypes.c_int32),
                ("plan_used", ctypes.c_int32), ("tile_cols_used", ctypes.c_int32),
                ("tile_threads_used", ctypes.c_int32), ("tile_vec_used", ctypes.c_int32),
                ("tile_csr_lds_used", ctypes.c_int32), ("tile_reg_degree_used", ctypes.c_int32),
                ("ls_iterations", ctypes.c_int64),
                ("step_kernel_ms", ctypes.c_double), ("step_kernel_launches", ctypes.c_int64),
                ("final_search_alternations", ctypes.c_int64), ("pool_x", ctypes.c_void_p),
                ("pool_value", ctypes.c_void_p), ("step_vec_used", ctypes.c_int32),
                ("step_lanes_used", ctypes.c_int32), ("tile_single_buffer_used", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2605_06921_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, G, R = ctypes.POINTER(_Params), ctypes.POINTER(_Graph), ctypes.POINTER(_Result)
    vp, i32, i64, u64, f32, f64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_float, ctypes.c_double, ctypes.c_size_t)
    sig = {
        "mqo_params_default": (None, [P]),
        "mqo_workspace_size": (sz, [G, P, i32]),
        "mqo_solve_mis": (i32, [G, P, vp, R, vp, sz, vp]),
        "mqo_solve_maxcut": (i32, [G, P, vp, R, vp, sz, vp]),
        "mqo_objective_workspace_size": (sz, [G, i32]),
        "mqo_objective_grad": (i32, [G, i32, f32, vp, i32, vp, vp, vp, vp, sz, vp]),
        "mqo_objective_grad_static": (i32, [G, i32, f32, vp, i32, vp, vp, vp, vp]),
        "mqo_unrolled_workspace_size": (sz, [G, i32, i32]),
        "mqo_pga_unrolled_forward": (i32, [G, i32, f32, f32, i32, i32, vp, vp, vp, i32, vp, sz, vp]),
        "mqo_pga_unrolled_backward": (i32, [G, i32, f32, f32, i32, i32, vp, vp, vp, vp, vp, i32, vp, sz, vp]),
        "mqo_init_iterate": (i32, [G, i32, P, vp, vp, sz, vp]),
        "mqo_pga_steps": (i32, [G, i32, P, vp, vp, vp, i32, vp]),
        "mqo_round_evaluate": (i32, [G, i32, vp, i32, vp, vp, vp, vp, vp, sz, vp]),
        "mqo_local_search": (i32, [G, i32, i32, u64, i32, vp, ctypes.POINTER(i64), vp, sz, vp]),
        "mqo_toy_reset": (i32, [u64, i32, ctypes.c_float, ctypes.c_float, i32, i32, i32, i32, vp, vp, vp]),
        "mqo_pair_search": (i32, [G, i32, i32, u64, i32, vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                  vp, sz, vp]),
        "mqo_reset": (i32, [G, i32, i32, u64, i32, f64, i32, vp, vp, vp, vp, sz, vp]),
        "mqo_validate_graph_host": (i32, [i64, i64, vp, vp, vp]),
        "mqo_validate_graph": (i32, [G, vp]),
        "mqo_status_string": (ctypes.c_char_p, [i32]),
        "mqo_last_error": (ctypes.c_char_p, []),
        "mqo_version": (i32, []),
        "mqo_clear_caches": (None, []),
        "mqo_tune_cache_load": (i32, [ctypes.c_char_p]),
        "mqo_tune_cache_save": (i32, [ctypes.c_char_p]),
        "mqo_tune_cache_size": (i64, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib, sig


_lib, SIGNATURES = _load()


def lib():
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise MqoError(status, where)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def version() -> int:
    return _lib.mqo_version()


def tune_cache_load(path: str) -> None:
    _check(_lib.mqo_tune_cache_load(os.fsencode(path)), "mqo_tune_cache_load")


def tune_cache_save(path: str) -> None:
    _check(_lib.mqo_tune_cache_save(os.fsencode(path)), "mqo_tune_cache_save")


def tune_cache_size() -> int:
    return _lib.mqo_tune_cache_size()


# --------------------------------------------------------------------------
# graphs
# --------------------------------------------------------------------------

def _local_rows(graph, vtx_offset):
    """1 when every graph's mean distance |u - v| in the vertex order over its
    stored entries is below n_g / 64, else 0."""
    rp = np.asarray(graph.row_ptr, dtype=np.int64)
    ci = np.asarray(graph.col_idx, dtype=np.int64)
    if len(ci) == 0:
        return 0
    rows = np.repeat(np.arange(len(rp) - 1, dtype=np.int64), np.diff(rp))
    dist = np.abs(ci - rows).astype(np.float64)
    for i in range(len(vtx_offset) - 1):
        lo, hi = int(vtx_offset[i]), int(vtx_offset[i + 1])
        a, b = int(rp[lo]), int(rp[hi])
        if b > a and dist[a:b].mean() * 64 >= hi - lo:
            return 0
    return 1


class DeviceGraph:
    """A canonical CSR (or a block-diagonal batch) resident on the GPU.

    ``graph`` needs attributes n, row_ptr, col_idx, weight (or None) and
    vtx_offset (int64[G+1]) as numpy arrays.  Rows of degree above
    ``hub_min_degree`` are listed as hubs (their sparse products get
    workgroups of their own); "auto" takes max(128, 8 x mean degree), None
    lists none.  ``local_rows``: 1 when neighbours are close in the vertex
    order (rows sharing neighbours then share an XCD's L2), 0 if not, "auto"
    measures it: 1 when every graph's mean |u - v| over its stored entries
    is below n_g / 64.  Results depend on neither."""

    def __init__(self, graph, device="cuda", hub_min_degree="auto", local_rows="auto"):
        self.device = torch.device(device)
        self.n = int(graph.n)
        self.vtx_offset = np.ascontiguousarray(graph.vtx_offset, dtype=np.int64)
        self.num_graphs = len(self.vtx_offset) - 1
        self.row_ptr = torch.from_numpy(np.ascontiguousarray(graph.row_ptr, dtype=np.int32)).to(self.device)
        ci = np.ascontiguousarray(graph.col_idx, dtype=np.int32)
        self.nnz = int(len(ci))
        self.col_idx = torch.from_numpy(ci if len(ci) else np.zeros(1, np.int32)).to(self.device)
        self.weight = None
        if graph.weight is not None:
            self.weight = torch.from_numpy(np.ascontiguousarray(graph.weight, dtype=np.int32)).to(self.device)
        self.hub_min_degree = hub_min_degree
        self.hub_offset = None
        self.hub_rows = None
        deg = np.diff(np.asarray(graph.row_ptr, dtype=np.int64))
        self.max_degree = int(deg.max()) if len(deg) else 0
        if hub_min_degree is not None:
            if hub_min_degree == "auto":
                hub_min_degree = max(128, 8 * int(np.ceil(deg.mean()))) if len(deg) else 128
            self.hub_min_degree = hub_min_degree
            hubs = np.nonzero(deg > hub_min_degree)[0]
            if len(hubs):
                self.hub_offset = np.searchsorted(hubs, self.vtx_offset).astype(np.int64)
                self.hub_rows = torch.from_numpy(hubs.astype(np.int32)).to(self.device)
        if local_rows == "auto":
            local_rows = _local_rows(graph, self.vtx_offset)
        self.local_rows = int(local_rows)
        self._struct = _Graph(self.num_graphs,
                              self.vtx_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                              None if self.weight is None else self.weight.data_ptr(),
                              0 if self.hub_offset is None else int(hub_min_degree),
                              None if self.hub_offset is None else
                              self.hub_offset.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              None if self.hub_rows is None else self.hub_rows.data_ptr(), self.max_degree,
                              self.local_rows)

    @property
    def num_hubs(self):
        return 0 if self.hub_offset is None else int(self.hub_offset[-1])

    @property
    def struct(self):
        return ctypes.byref(self._struct)

    def validate(self):
        _check(_lib.mqo_validate_graph(self.struct, _stream(self.device)), "mqo_validate_graph")


def validate_graph_host(n, row_ptr, col_idx, weight=None) -> int:
    """Canonical-form check on host arrays; returns the mqo_status (0 = ok)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    w = None if weight is None else np.ascontiguousarray(weight, dtype=np.int32)
    return _lib.mqo_validate_graph_host(int(n), int(len(ci)), rp.ctypes.data_as(ctypes.c_void_p),
                                        ci.ctypes.data_as(ctypes.c_void_p),
                                        None if w is None else w.ctypes.data_as(ctypes.c_void_p))


def last_error() -> str:
    return _lib.mqo_last_error().decode()


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------

def make_params(batch=1, steps_per_round=200, rounds=1, alpha=0.01, momentum=0.0, gamma=2.0, lam=1e-3,
                rho=0.05, init_sigma=0.0, init_mode="uniform", reset_mode="zero", local_search=True,
                plan="auto", seed=0, time_budget_s=0.0, tile_cols=0, tile_threads=0, tile_vec=0, tile_csr=0,
                tile_reg=0, check_every=0, final_search=False, pool_k=0, restart_every=0, step_vec=0,
                step_lanes=0, tile_sb=0) -> _Params:
    p = _Params()
    _lib.mqo_params_default(ctypes.byref(p))
    p.batch, p.steps_per_round, p.rounds, p.check_every = batch, steps_per_round, rounds, check_every
    p.alpha, p.momentum, p.gamma, p.lam = alpha, momentum, gamma, lam
    p.rho, p.init_sigma = rho, init_sigma
    p.init_mode, p.reset_mode = INIT[init_mode], RESET[reset_mode]
    p.local_search = 1 if local_search else 0
    p.plan = PLANS[plan]
    p.tile_cols, p.tile_threads, p.tile_vec, p.tile_csr = tile_cols, tile_threads, tile_vec, tile_csr
    p.tile_reg = tile_reg
    p.seed, p.time_budget_s = seed, time_budget_s
    p.final_search = 1 if final_search else 0
    p.pool_k = pool_k
    p.restart_every = restart_every
    p.step_vec, p.step_lanes = step_vec, step_lanes
    p.tile_sb = tile_sb
    return p


# --------------------------------------------------------------------------
# the solve
# --------------------------------------------------------------------------

class Workspace:
    """A device byte buffer reused across calls (grows on demand)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws = {}


def _ws_for(device, ws: Optional[Workspace]) -> Workspace:
    """The caller's workspace, else the default one of (device, current
    stream): calls queued on different streams never share scratch, and each
    default buffer is allocated while its stream is current."""
    if ws is not None:
        return ws
    dev = torch.device(device)
    key = (str(dev), torch.cuda.current_stream(dev).cuda_stream)
    if key not in _default_ws:
        _default_ws[key] = Workspace(dev)
    return _default_ws[key]


def solve(kind, dg: DeviceGraph, x0: Optional[torch.Tensor] = None, workspace: Optional[Workspace] = None,
          want_traj: bool = True, trajectories=None, **params):
    """Batched mutation-guided search (mqo_solve_mis / mqo_solve_maxcut).
    ``trajectories`` (plain plan): ascending ids g * batch + b of the only
    trajectories to run.  Returns a dict of device tensors and host counters."""
    k = _KIND[kind]
    p = make_params(**params)
    ids = None
    if trajectories is not None:
        ids = np.ascontiguousarray(np.asarray(trajectories, dtype=np.int64))
        p.traj_count = len(ids)
        p.traj_ids = ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    if k != MIS:
        p.maxcut_objective = k  # the formulation of the MaxCut steps
    B, G = p.batch, dg.num_graphs
    nbytes = _lib.mqo_workspace_size(dg.struct, ctypes.byref(p), k)
    if nbytes == 0:
        raise MqoError(-1, "mqo_workspace_size")
    ws = _ws_for(dg.device, workspace).get(nbytes)
    dev = dg.device
    best_x = torch.empty(dg.n, dtype=torch.int8, device=dev)
    best_value = torch.empty(G, dtype=torch.int64, device=dev)
    traj_v = torch.empty(G * B, dtype=torch.int64, device=dev) if want_traj else None
    traj_x = torch.empty(dg.n * B, dtype=torch.int8, device=dev) if want_traj else None
    if x0 is not None:
        if x0.dtype != torch.float32 or x0.numel() != dg.n * B or x0.device != dev:
            raise ValueError("x0 must be a float32 [n_total * B] tensor on the graph's device")
        x0 = x0.contiguous()
    r = _Result(best_x.data_ptr(), best_value.data_ptr(), None if traj_v is None else traj_v.data_ptr(),
                None if traj_x is None else traj_x.data_ptr())
    K = p.pool_k
    pool_x = torch.empty(dg.n * K, dtype=torch.int8, device=dev) if K else None
    pool_v = torch.empty(G * K, dtype=torch.int64, device=dev) if K else None
    if K:
        r.pool_x, r.pool_value = pool_x.data_ptr(), pool_v.data_ptr()
    fn = _lib.mqo_solve_mis if k == MIS else _lib.mqo_solve_maxcut
    _check(fn(dg.struct, ctypes.byref(p), _ptr(x0), ctypes.byref(r), ctypes.c_void_p(ws.data_ptr()), nbytes,
              _stream(dev)), "mqo_solve")
    out = dict(best_x=best_x, best_value=best_value, edge_updates=r.edge_updates, steps_executed=r.steps_executed,
               rounds_executed=r.rounds_executed, plan=PLAN_NAMES[r.plan_used], tile_cols=r.tile_cols_used,
               tile_threads=r.tile_threads_used, tile_vec=r.tile_vec_used, tile_csr_lds=r.tile_csr_lds_used,
               tile_reg_degree=r.tile_reg_degree_used,
               ls_iterations=r.ls_iterations,
               step_kernel_ms=r.step_kernel_ms, step_kernel_launches=r.step_kernel_launches,
               final_search_alternations=r.final_search_alternations, step_vec=r.step_vec_used,
               step_lanes=r.step_lanes_used, tile_sb=r.tile_single_buffer_used)
    if want_traj:
        out["traj_best_value"] = traj_v
        out["traj_best_x"] = traj_x.view(dg.n, B)
    if K:
        out["pool_value"] = pool_v
        out["pool_x"] = pool_x.view(dg.n, K)
    return out


def solve_mis(dg, **kw):
    return solve(MIS, dg, **kw)


def solve_maxcut(dg, **kw):
    return solve(MAXCUT, dg, **kw)


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _solve_ws(dg, kind, B, workspace=None):
    p = make_params(batch=B)
    nbytes = _lib.mqo_workspace_size(dg.struct, ctypes.byref(p), _KIND[kind])
    return _ws_for(dg.device, workspace).get(nbytes), nbytes


INIT_WORKSPACE_BYTES = 256  # MQO_INIT_WORKSPACE_BYTES


def init_iterate(kind, dg: DeviceGraph, batch: int, seed: int, init_mode="uniform", init_sigma=0.0,
                 workspace=None):
    p = make_params(batch=batch, seed=seed, init_mode=init_mode, init_sigma=init_sigma)
    X = torch.empty(dg.n * batch, dtype=torch.float32, device=dg.device)
    ws = _ws_for(dg.device, workspace).get(INIT_WORKSPACE_BYTES)
    _check(_lib.mqo_init_iterate(dg.struct, _KIND[kind], ctypes.byref(p), _ptr(X), ctypes.c_void_p(ws.data_ptr()),
                                 INIT_WORKSPACE_BYTES, _stream(dg.device)), "mqo_init_iterate")
    return X.view(dg.n, batch)


def pga_steps(kind, dg: DeviceGraph, X: torch.Tensor, nsteps: int, alpha=0.01, gamma=2.0, lam=1e-3,
              momentum=0.0, V: Optional[torch.Tensor] = None):
    """In-place PGA steps on X [n][B] (and V when momentum != 0)."""
    B = X.shape[1]
    p = make_params(batch=B, alpha=alpha, gamma=gamma, lam=lam, momentum=momentum)
    tmp = torch.empty_like(X)
    _check(_lib.mqo_pga_steps(dg.struct, _KIND[kind], ctypes.byref(p), _ptr(X), _ptr(V), _ptr(tmp), nsteps,
                              _stream(dg.device)), "mqo_pga_steps")
    return X


def round_evaluate(kind, dg: DeviceGraph, X: torch.Tensor, workspace=None):
    B = X.shape[1]
    ws, nbytes = _solve_ws(dg, kind, B, workspace)
    G = dg.num_graphs
    Z = torch.empty(dg.n, B, dtype=torch.int8, device=dg.device)
    value = torch.empty(G * B, dtype=torch.int64, device=dg.device)
    conf = torch.empty(G * B, dtype=torch.int64, device=dg.device)
    fixed = torch.empty(G * B, dtype=torch.int8, device=dg.device)
    _check(_lib.mqo_round_evaluate(dg.struct, _KIND[kind], _ptr(X), B, _ptr(Z), _ptr(value), _ptr(conf),
                                   _ptr(fixed), ctypes.c_void_p(ws.data_ptr()), nbytes, _stream(dg.device)),
           "mqo_round_evaluate")
    return Z, value, conf, fixed


def local_search(kind, dg: DeviceGraph, Z: torch.Tensor, seed: int, rnd: int, workspace=None):
    """In-place 1-flip local search on Z [n][B] (int8); returns iterations."""
    B = Z.shape[1]
    ws, nbytes = _solve_ws(dg, kind, B, workspace)
    it = ctypes.c_int64(0)
    _check(_lib.mqo_local_search(dg.struct, _KIND[kind], B, seed, rnd, _ptr(Z), ctypes.byref(it),
                                 ctypes.c_void_p(ws.data_ptr()), nbytes, _stream(dg.device)), "mqo_local_search")
    return it.value


def pair_search(kind, dg: DeviceGraph, Z: torch.Tensor, seed: int, rnd: int, workspace=None, timing=None):
    """In-place OneTwoSwap (MIS) / OneTwoFlip (MaxCut) on Z [n][B] (int8);
    returns the pair iterations that applied a move.  ``timing`` (a dict)
    receives candidate_kernel_ms, the HIP-event time of the candidate
    launches."""
    B = Z.shape[1]
    ws, nbytes = _solve_ws(dg, kind, B, workspace)
    alt = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(_lib.mqo_pair_search(dg.struct, _KIND[kind], B, seed, rnd, _ptr(Z), ctypes.byref(alt),
                                ctypes.byref(ms) if timing is not None else None,
                                ctypes.c_void_p(ws.data_ptr()), nbytes, _stream(dg.device)), "mqo_pair_search")
    if timing is not None:
        timing["candidate_kernel_ms"] = ms.value
    return alt.value


def toy_reset(seed: int, n: int, trials: int, attempts: int, mode="global", alpha=0.5, beta=0.5, steps=128,
              device="cuda", want_x=True):
    """Prop. 4.1's toy (mqo_toy_reset) on the current stream of ``device``:
    returns (first_hit int32[trials], final points [trials][n] or None)."""
    dev = torch.device(device)
    first = torch.empty(trials, dtype=torch.int32, device=dev)
    x = torch.empty(trials, n, dtype=torch.float32, device=dev) if (want_x and mode == "global") else None
    m = 0 if mode == "global" else 1
    _check(_lib.mqo_toy_reset(seed, n, alpha, beta, steps, attempts, trials, m, _ptr(first), _ptr(x), _stream(dev)),
           "mqo_toy_reset")
    return first, x


def reset(kind, dg: DeviceGraph, Zbest: torch.Tensor, seed: int, rnd: int, rho: float, mode="zero",
          keys: Optional[torch.Tensor] = None, workspace=None):
    B = Zbest.shape[1]
    ws, nbytes = _solve_ws(dg, kind, B, workspace)
    X = torch.empty(dg.n, B, dtype=torch.float32, device=dg.device)
    if keys is not None:
        keys = keys.contiguous()
        if keys.dtype != torch.int32 or keys.shape != Zbest.shape:
            raise ValueError("keys must be an int32 tensor (bit pattern of uint32) shaped like Zbest")
    _check(_lib.mqo_reset(dg.struct, _KIND[kind], B, seed, rnd, float(rho), RESET[mode], _ptr(Zbest), _ptr(keys),
                          _ptr(X), ctypes.c_void_p(ws.data_ptr()), nbytes, _stream(dg.device)), "mqo_reset")
    return X


# --------------------------------------------------------------------------
# differentiation
# --------------------------------------------------------------------------

def objective_grad(kind, dg: DeviceGraph, X: torch.Tensor, param: float, scale: Optional[torch.Tensor] = None,
                   want_f=True, want_grad=True, workspace=None):
    B = X.shape[1]
    G = dg.num_graphs
    f = torch.empty(G * B, dtype=torch.float64, device=dg.device) if want_f else None
    grad = torch.empty_like(X) if want_grad else None
    nbytes = _lib.mqo_objective_workspace_size(dg.struct, B)
    ws = _ws_for(dg.device, workspace).get(nbytes) if want_f else None
    if scale is not None:
        scale = scale.to(torch.float32).contiguous()
    _check(_lib.mqo_objective_grad(dg.struct, _KIND[kind], float(param), _ptr(X.contiguous()), B, _ptr(scale),
                                   _ptr(f), _ptr(grad), None if ws is None else ctypes.c_void_p(ws.data_ptr()),
                                   nbytes if want_f else 0, _stream(dg.device)), "mqo_objective_grad")
    return f, grad


STATIC_SCRATCH_BYTES = 16 << 20  # MQO_STATIC_SCRATCH_BYTES


def objective_grad_static(kind, dg: DeviceGraph, X: torch.Tensor, param: float, f: Optional[torch.Tensor] = None,
                          grad: Optional[torch.Tensor] = None, scale: Optional[torch.Tensor] = None):
    """mqo_objective_grad_static: the objective into ``f`` ([G*B] float64)
    and the gradient into ``grad`` (like X), either may be None; both are
    the caller's.  The library allocates nothing: its partial sums go to its
    own device scratch, shared by every call on the GPU (calls that overlap
    on one GPU race)."""
    B = X.shape[1]
    _check(_lib.mqo_objective_grad_static(dg.struct, _KIND[kind], float(param), _ptr(X), B, _ptr(scale), _ptr(f),
                                          _ptr(grad), _stream(dg.device)), "mqo_objective_grad_static")
    return f, grad


class Objective(torch.autograd.Function):
    """f(X) per trajectory (h of Eq. (3) or f_B of Eq. (7)); the backward is
    the hand-written SpMM gradient kernel: dL/dX = dL/df_b * (c + H x)."""

    @staticmethod
    def forward(ctx, X, dg, kind, param):
        f, _ = objective_grad(kind, dg, X, param, want_grad=False)
        ctx.save_for_backward(X)
        ctx.dg, ctx.kind, ctx.param = dg, kind, param
        return f

    @staticmethod
    def backward(ctx, grad_f):
        (X,) = ctx.saved_tensors
        _, grad = objective_grad(ctx.kind, ctx.dg, X, ctx.param, scale=grad_f, want_f=False)
        return grad, None, None, None


def objective(X, dg, kind, param):
    return Objective.apply(X, dg, kind, param)


def unrolled_forward(kind, dg: DeviceGraph, X0: torch.Tensor, alpha: float, K: int, ckpt_every: int, param: float,
                     workspace=None):
    B = X0.shape[1]
    nseg = K // ckpt_every
    ckpt = torch.empty(nseg, dg.n, B, dtype=torch.float32, device=dg.device)
    XK = torch.empty_like(X0)
    nbytes = _lib.mqo_unrolled_workspace_size(dg.struct, B, ckpt_every)
    ws = _ws_for(dg.device, workspace).get(nbytes)
    _check(_lib.mqo_pga_unrolled_forward(dg.struct, _KIND[kind], float(param), float(alpha), K, ckpt_every,
                                         _ptr(X0.contiguous()), _ptr(ckpt), _ptr(XK), B,
                                         ctypes.c_void_p(ws.data_ptr()), nbytes, _stream(dg.device)),
           "mqo_pga_unrolled_forward")
    return XK, ckpt


def unrolled_backward(kind, dg: DeviceGraph, ckpt: torch.Tensor, dL_dXK: torch.Tensor, alpha: float, K: int,
                      ckpt_every: int, param: float, workspace=None, want_sum=False):
    """dL/dx_0 [n][B] and dL/dalpha per trajectory [G*B] (float64); with
    ``want_sum`` also their sum over all trajectories (a 0-d float64 tensor)."""
    B = dL_dXK.shape[1]
    dX0 = torch.empty_like(dL_dXK)
    dalpha = torch.empty(dg.num_graphs * B, dtype=torch.float64, device=dg.device)
    dsum = torch.empty((), dtype=torch.float64, device=dg.device) if want_sum else None
    nbytes = _lib.mqo_unrolled_workspace_size(dg.struct, B, ckpt_every)
    ws = _ws_for(dg.device, workspace).get(nbytes)
    _check(_lib.mqo_pga_unrolled_backward(dg.struct, _KIND[kind], float(param), float(alpha), K, ckpt_every,
                                          _ptr(ckpt), _ptr(dL_dXK.contiguous()), _ptr(dX0), _ptr(dalpha),
                                          _ptr(dsum), B, ctypes.c_void_p(ws.data_ptr()), nbytes,
                                          _stream(dg.device)), "mqo_pga_unrolled_backward")
    return (dX0, dalpha, dsum) if want_sum else (dX0, dalpha)


class UnrolledPGA(torch.autograd.Function):
    """x_K of K unrolled PGA steps from x_0, differentiable in x_0 and in the
    step size alpha (a 0-d tensor), checkpointing every ``ckpt_every`` steps."""

    @staticmethod
    def forward(ctx, X0, alpha, dg, kind, param, K, ckpt_every):
        XK, ckpt = unrolled_forward(kind, dg, X0, float(alpha), K, ckpt_every, param)
        ctx.save_for_backward(ckpt)
        ctx.meta = (dg, kind, param, float(alpha), K, ckpt_every, alpha.dtype, alpha.device)
        return XK

    @staticmethod
    def backward(ctx, grad_XK):
        (ckpt,) = ctx.saved_tensors
        dg, kind, param, alpha, K, c, adt, adev = ctx.meta
        dX0, _, dsum = unrolled_backward(kind, dg, ckpt, grad_XK.contiguous(), alpha, K, c, param, want_sum=True)
        return dX0, dsum.to(adt).to(adev), None, None, None, None, None


def unrolled_pga(X0, alpha, dg, kind, param, K=20, ckpt_every=5):
    return UnrolledPGA.apply(X0, alpha, dg, kind, param, K, ckpt_every)
