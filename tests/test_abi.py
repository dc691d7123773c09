"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and rejects invalid graphs and parameters on the host
before any GPU call.  No compute is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth import graphs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mqo.h")


@pytest.fixture(scope="module")
def m():
    from paper_2605_06921_amd import mqo
    return mqo


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mqo_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(m):
    names = _declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(m.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares a signature for each of them
    assert set(names) == set(m.SIGNATURES)


def test_version_status_and_params(m):
    assert m.version() == 110
    L = m.lib()
    assert L.mqo_status_string(0) == b"ok"
    assert L.mqo_status_string(-2) == b"invalid graph"
    p = m.make_params(batch=7, rho=0.3)
    assert p.struct_size == ctypes.sizeof(m._Params)
    assert p.batch == 7 and abs(p.rho - 0.3) < 1e-15 and p.local_search == 1


def _valid():
    g = graphs.with_weights(graphs.erdos_renyi(40, 0.2, 3), 4)
    return g


def test_validate_graph_host_accepts_canonical(m):
    g = _valid()
    assert m.validate_graph_host(g.n, g.row_ptr, g.col_idx, g.weight) == 0
    assert m.validate_graph_host(5, np.zeros(6, np.int32), np.zeros(0, np.int32)) == 0


@pytest.mark.parametrize("breakage", ["asym", "self", "unsorted", "dup", "range", "rowptr", "weight"])
def test_validate_graph_host_rejects(m, breakage):
    g = _valid()
    rp, ci, w = g.row_ptr.copy(), g.col_idx.copy(), g.weight.copy()
    v = int(np.argmax(np.diff(rp) >= 2))  # a row with at least two entries
    a = rp[v]
    if breakage == "asym":
        ci[a] = [c for c in range(g.n) if c != v and c not in ci[rp[v]:rp[v + 1]]][0]
        ci[rp[v]:rp[v + 1]] = np.sort(ci[rp[v]:rp[v + 1]])
    elif breakage == "self":
        ci[a] = v
        ci[rp[v]:rp[v + 1]] = np.sort(ci[rp[v]:rp[v + 1]])
    elif breakage == "unsorted":
        ci[a], ci[a + 1] = ci[a + 1], ci[a]
    elif breakage == "dup":
        ci[a + 1] = ci[a]
    elif breakage == "range":
        ci[a] = g.n + 3
    elif breakage == "rowptr":
        rp[v + 1] = rp[v] - 1
    elif breakage == "weight":
        w[a] = w[a] + 7
    assert m.validate_graph_host(g.n, rp, ci, w) == -2
    assert m.last_error()


def _struct(m, n=10, G=1, offsets=None, weight=False):
    off = np.array(offsets if offsets is not None else [0, n], dtype=np.int64)
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    s = m._Graph(G, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(off[-1]), 4, dummy, dummy,
                 dummy if weight else None)
    return s, off


@pytest.mark.parametrize("field,value,status", [
    ("batch", 0, -1), ("rounds", 0, -1), ("alpha", -0.1, -1), ("gamma", 1.0, -1), ("rho", 1.0, -1),
    ("momentum", 1.0, -1), ("check_every", -1, -1), ("plan", 9, -1), ("tile_cols", 3, -1),
    ("tile_threads", 100, -1), ("steps_per_round", -1, -1), ("init_mode", 4, -1),
])
def test_solve_rejects_parameters_on_host(m, field, value, status):
    s, off = _struct(m)
    p = m.make_params(batch=2)
    setattr(p, field, value)
    r = m._Result()
    st = m.lib().mqo_solve_mis(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None)
    assert st == status, m.last_error()


def test_solve_rejects_graph_arguments_on_host(m):
    L = m.lib()
    p = m.make_params(batch=2, lam=1e-3)
    r = m._Result()
    s, off = _struct(m, weight=True)
    assert L.mqo_solve_mis(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None) == -1
    p2 = m.make_params(batch=2, lam=2.0)
    s, off = _struct(m)
    assert L.mqo_solve_maxcut(ctypes.byref(s), ctypes.byref(p2), None, ctypes.byref(r), None, 0, None) == -1
    s, off = _struct(m, G=2, offsets=[0, 5, 5])  # an empty graph in the batch
    assert L.mqo_solve_maxcut(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None) == -2
    s, off = _struct(m, G=1, offsets=[1, 5])
    assert L.mqo_solve_maxcut(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None) == -2
    # missing outputs
    s, off = _struct(m)
    assert L.mqo_solve_maxcut(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None) == -1


def test_hub_list_rejected_on_host(m):
    L = m.lib()
    p = m.make_params(batch=2)
    r = m._Result()
    for hoff, mindeg, rows, status in [([1, 1], 8, True, -2), ([0, 11], 8, True, -2), ([0, 2], 8, False, -1),
                                       ([0, 2], -1, True, -1)]:
        s, off = _struct(m)
        ho = np.array(hoff, dtype=np.int64)
        s.hub_offset = ho.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        s.hub_min_degree = mindeg
        s.hub_rows = 0x1000 if rows else None
        assert L.mqo_solve_mis(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None) == status
    # the objective's partial rows grow by one per hub of the largest graph
    s, off = _struct(m, n=1000)
    base = L.mqo_objective_workspace_size(ctypes.byref(s), 64)
    ho = np.array([0, 40], dtype=np.int64)
    s.hub_offset = ho.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    s.hub_min_degree = 8
    s.hub_rows = 0x1000
    assert L.mqo_objective_workspace_size(ctypes.byref(s), 64) >= base + 40 * 64 * 8


def test_negative_degree_hint_rejected(m):
    s, off = _struct(m)
    s.max_degree = -1
    p = m.make_params(batch=2)
    r = m._Result()
    assert m.lib().mqo_solve_mis(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None) == -1


def test_workspace_sizes(m):
    L = m.lib()
    s, off = _struct(m, n=1000)
    p = m.make_params(batch=64)
    ws = L.mqo_workspace_size(ctypes.byref(s), ctypes.byref(p), 1)
    assert ws >= 1000 * 64 * (4 * 5 + 3)
    p.batch = 0
    assert L.mqo_workspace_size(ctypes.byref(s), ctypes.byref(p), 1) == 0
    assert L.mqo_unrolled_workspace_size(ctypes.byref(s), 64, 5) >= 8 * 1000 * 64 * 4
    assert L.mqo_objective_workspace_size(ctypes.byref(s), 64) > 0


def test_async_entry_points_reject_bad_arguments(m):
    L = m.lib()
    s, off = _struct(m)
    assert L.mqo_objective_grad(ctypes.byref(s), 0, 0.5, ctypes.c_void_p(0x1000), 4, None, None, None, None, 0,
                                None) == -1  # gamma <= 1
    assert L.mqo_pga_unrolled_forward(ctypes.byref(s), 1, 1e-3, 0.01, 7, 5, ctypes.c_void_p(0x1000),
                                      ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), 4, None, 0, None) == -1
    assert L.mqo_reset(ctypes.byref(s), 0, 4, 0, 1, 1.5, 0, ctypes.c_void_p(0x1000), None, ctypes.c_void_p(0x1000),
                       None, 0, None) == -1


def test_degree_init_needs_its_scratch(m):
    """The degree initialisation measures the largest degree into caller
    scratch (so calls on different streams never share it): without it the
    call is refused before anything runs."""
    L = m.lib()
    s, off = _struct(m)
    p = m.make_params(batch=4, init_mode="degree")
    X = ctypes.c_void_p(0x1000)
    assert L.mqo_init_iterate(ctypes.byref(s), 0, ctypes.byref(p), X, None, 0, None) == -3
    assert L.mqo_init_iterate(ctypes.byref(s), 0, ctypes.byref(p), X, ctypes.c_void_p(0x1000),
                              m.INIT_WORKSPACE_BYTES - 1, None) == -3


def test_trajectory_subset_checked_on_host(m):
    L = m.lib()
    s, off = _struct(m)  # one graph
    r = m._Result(0x1000, 0x1000)  # output pointers, never written: the call stops first
    for ids, plan, status in [([0, 2], "batched", -5), ([2, 1], "plain", -1), ([0, 4], "plain", -1),
                              ([1, 1], "plain", -1), ([-1], "plain", -1), ([0, 3], "plain", -3)]:
        p = m.make_params(batch=4, plan=plan)
        arr = np.array(ids, dtype=np.int64)
        p.traj_count = len(arr)
        p.traj_ids = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        # no workspace: a valid subset gets as far as the workspace check
        assert L.mqo_solve_mis(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), ctypes.c_void_p(0x1000),
                               0, None) == status, (ids, plan, m.last_error())
    p = m.make_params(batch=4, plan="plain")
    p.traj_count = 2
    assert L.mqo_solve_mis(ctypes.byref(s), ctypes.byref(p), None, ctypes.byref(r), None, 0, None) == -1


def test_static_scratch_variant_checks_its_limit_on_host(m):
    """The no-allocation objective entry point refuses, before anything is
    enqueued, a batch whose partial sums exceed its static scratch."""
    L = m.lib()
    n = 200_000
    s, off = _struct(m, n=n)
    B = 256
    need = L.mqo_objective_workspace_size(ctypes.byref(s), B)
    assert need > m.STATIC_SCRATCH_BYTES
    X = ctypes.c_void_p(0x1000)
    assert L.mqo_objective_grad_static(ctypes.byref(s), 0, 2.0, X, B, None, ctypes.c_void_p(0x1000), None,
                                       None) == -3
    assert "static scratch" in m.last_error()
    assert L.mqo_objective_grad_static(ctypes.byref(s), 0, 0.5, X, B, None, None, None, None) == -1  # gamma <= 1


def test_tuning_cache_file_round_trip(m, tmp_path):
    """The autotuner cache is host data: load merges a file's entries, save
    writes every entry back, malformed files are refused whole."""
    L = m.lib()
    L.mqo_clear_caches()
    src = tmp_path / "in.txt"
    src.write_text("# comment\nstep|gfx950x256|0|0|0|14|13|32|32|0|0\t4 3 0.051200\n\n"
                   "tile|gfx950x256|0|0|0|800|15|512|128|1|0|0|0|0|0|16\t8 1024 1 0 0 0 0.120000\n"
                   "plan|gfx950x256|0|0|0|800|15|512|128|1\tpersistent 0.12 0.90\n")
    m.tune_cache_load(str(src))
    assert m.tune_cache_size() == 3
    out = tmp_path / "out.txt"
    m.tune_cache_save(str(out))
    lines = [ln for ln in out.read_text().splitlines() if ln and not ln.startswith("#")]
    want = [ln for ln in src.read_text().splitlines() if ln and not ln.startswith("#")]
    assert sorted(lines) == sorted(want)
    L.mqo_clear_caches()
    m.tune_cache_load(str(out))
    assert m.tune_cache_size() == 3
    bad = tmp_path / "bad.txt"
    bad.write_text("step|x\t1 2 3\nno tab here\n")
    with pytest.raises(m.MqoError):
        m.tune_cache_load(str(bad))
    assert m.tune_cache_size() == 3  # nothing of the malformed file merged
    with pytest.raises(m.MqoError):
        m.tune_cache_load(str(tmp_path / "missing.txt"))
    L.mqo_clear_caches()
    assert m.tune_cache_size() == 0


def test_local_rows_measured_from_the_vertex_order(m):
    """The binding's locality hint: a torus (neighbours at +-1 and +-side)
    is local, a random graph and a star are not."""
    torus = graphs.torus_pm1(200, 5)
    er = graphs.erdos_renyi(400, 0.02, 6)
    star = graphs.star(300)
    assert m._local_rows(torus, np.asarray(torus.vtx_offset)) == 1
    assert m._local_rows(er, np.asarray(er.vtx_offset)) == 0
    assert m._local_rows(star, np.asarray(star.vtx_offset)) == 0
    both = graphs.concat([graphs.with_weights(er, 7), torus])
    assert m._local_rows(both, np.asarray(both.vtx_offset)) == 0
