"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Bit-exact: initial iterates, float32 steps (against the oracle's float32
replay), rounding, evaluation, checker, local search, reset sets and whole
solves under every launch plan.  Tolerances: one step and the gradient
against float64 within 1e-5 relative; objective values, adjoints as stated
per test."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import graphs, arrays  # noqa: E402
from oracle import objectives as obj, pga, discrete, solver  # noqa: E402


@pytest.fixture(scope="module")
def mqo():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_06921_amd import mqo as m
    return m


DEV = "cuda:0"


def _graph_cases():
    # ragged sizes, isolated vertices, a batch of graphs, weighted torus
    return {
        "er300": ("mis", graphs.erdos_renyi(300, 0.03, 11)),
        "er_batch": ("mis", graphs.concat([graphs.erdos_renyi(97, 0.08, 12), graphs.empty(3),
                                           graphs.erdos_renyi(180, 0.05, 13), graphs.star(40)])),
        "reg3": ("maxcut", graphs.random_regular(250, 3, 14)),
        "torus": ("maxcut", graphs.torus_pm1(13, 15)),
        "cut_batch": ("maxcut", graphs.concat([graphs.erdos_renyi(120, 0.05, 16), graphs.cycle(33),
                                               graphs.path(2)])),
    }


CASES = _graph_cases()


def _x(kind, n, B, seed):
    lo, hi = obj.box(kind)
    return arrays.uniform((n, B), lo, hi, seed)


# --------------------------------------------------------------------------
# a2 init, a3-a5 step
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("B", [1, 3, 8, 64])
def test_init_uniform_bit_exact(mqo, name, B):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    X = mqo.init_iterate(kind, dg, B, seed=123).cpu().numpy()
    for gi in range(g.num_graphs):
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        ref = pga.init_uniform(kind, hi - lo, gi * B + np.arange(B), 123)
        assert np.array_equal(X[lo:hi], ref)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("B", [1, 2, 5, 16, 32, 100, 256])
def test_one_step_bit_exact_and_within_1e5_of_fp64(mqo, name, B):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    X0 = _x(kind, g.n, B, 21 + B)
    param = 2.0 if kind == "mis" else 1e-3
    X = torch.from_numpy(X0).to(DEV)
    mqo.pga_steps(kind, dg, X, 1, alpha=0.01, gamma=2.0, lam=1e-3)
    got = X.cpu().numpy()
    ref32, _ = pga.step32(g, X0, kind, 0.01, param)
    assert np.array_equal(got, ref32)
    ref64, _ = pga.step64(X0.astype(np.float64), obj.adjacency(g), kind, 0.01, param)
    assert np.abs(got - ref64).max() / max(1.0, np.abs(ref64).max()) <= 1e-5


@pytest.mark.parametrize("name", ["er300", "torus", "cut_batch"])
def test_many_steps_with_momentum_bit_exact(mqo, name):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    B = 12
    X0 = _x(kind, g.n, B, 31)
    param = 2.0 if kind == "mis" else 1e-3
    for mu in (0.0, 0.6):
        X = torch.from_numpy(X0).to(DEV)
        V = torch.zeros_like(X)
        mqo.pga_steps(kind, dg, X, 37, alpha=0.02, gamma=2.0, lam=1e-3, momentum=mu, V=V)
        ref, Vr = X0, None
        for _ in range(37):
            ref, Vr = pga.step32(g, ref, kind, 0.02, param, mu, Vr)
        assert np.array_equal(X.cpu().numpy(), ref)
        if mu:
            assert np.array_equal(V.cpu().numpy(), Vr)


# --------------------------------------------------------------------------
# a6 rounding, a7 evaluation and checker
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("B", [1, 7, 64])
def test_round_evaluate_bit_exact(mqo, name, B):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    X0 = _x(kind, g.n, B, 41)
    # include the thresholds themselves
    X0[::7, 0] = 0.5 if kind == "mis" else 0.0
    Z, value, conf, fixed = mqo.round_evaluate(kind, dg, torch.from_numpy(X0).to(DEV))
    Zr = discrete.round_x(kind, X0)
    assert np.array_equal(Z.cpu().numpy(), Zr)
    for gi in range(g.num_graphs):
        sub = g.subgraph(gi)
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        zg = Zr[lo:hi]
        assert np.array_equal(value.cpu().numpy()[gi * B:(gi + 1) * B], discrete.value(kind, sub, zg))
        if kind == "mis":
            _, c = discrete.evaluate_mis(sub, zg)
            assert np.array_equal(conf.cpu().numpy()[gi * B:(gi + 1) * B], c)
            fx = discrete.is_pga_fixed_mis(sub, zg, 2.0, 0.01)
            assert np.array_equal(fixed.cpu().numpy()[gi * B:(gi + 1) * B].astype(bool), fx)


def test_checker_on_maximal_sets(mqo):
    g = graphs.erdos_renyi(60, 0.1, 51)
    Z0 = arrays.binary01((60, 16), 52)
    Zm, _ = discrete.local_search("mis", g, Z0, 3, np.arange(16), 0)  # maximal independent sets
    Zmix = np.concatenate([Zm, Z0], axis=1).astype(np.float32)
    dg = mqo.DeviceGraph(g, DEV)
    _, value, conf, fixed = mqo.round_evaluate("mis", dg, torch.from_numpy(Zmix).to(DEV))
    fx = fixed.cpu().numpy().astype(bool)
    assert fx[:16].all()
    assert np.array_equal(fx, discrete.is_pga_fixed_mis(g, Zmix.astype(np.int8), 2.0, 0.01))


# --------------------------------------------------------------------------
# a8 local search
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("B", [1, 9, 64])
def test_local_search_bit_exact(mqo, name, B):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    Z0 = arrays.binary01((g.n, B), 61) if kind == "mis" else arrays.spins((g.n, B), 61)
    Z = torch.from_numpy(Z0.copy()).to(DEV)
    it = mqo.local_search(kind, dg, Z, seed=99, rnd=4)
    got = Z.cpu().numpy()
    its = []
    for gi in range(g.num_graphs):
        sub = g.subgraph(gi)
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        ref, i = discrete.local_search(kind, sub, Z0[lo:hi], 99, gi * B + np.arange(B), 4)
        assert np.array_equal(got[lo:hi], ref)
        its.append(i)
    assert it == max(its)


DENSE_LS_CASES = {
    # mean degree >= 24: one wavefront per (row, 64 columns); random starts
    # move many columns of a row at first (each lane walks the row) and few
    # later (lanes over the neighbours)
    "mis_dense": ("mis", graphs.concat([graphs.erdos_renyi(150, 0.3, 4904), graphs.erdos_renyi(90, 0.5, 4905),
                                        graphs.complete(5)])),
    "cut_dense": ("maxcut", graphs.concat([graphs.erdos_renyi(130, 0.35, 4906), graphs.complete(7)])),
    "cut_dense_weighted": ("maxcut", graphs.with_weights(graphs.erdos_renyi(140, 0.3, 4907), 4908,
                                                         values=(-2, -1, 1, 3))),
}


@pytest.mark.parametrize("name", list(DENSE_LS_CASES))
@pytest.mark.parametrize("B", [1, 5, 64, 130])
def test_local_search_dense_rows_bit_exact(mqo, name, B):
    kind, g = DENSE_LS_CASES[name]
    assert g.nnz / g.n >= 24
    dg = mqo.DeviceGraph(g, DEV)
    Z0 = arrays.binary01((g.n, B), 62) if kind == "mis" else arrays.spins((g.n, B), 62)
    Z = torch.from_numpy(Z0.copy()).to(DEV)
    it = mqo.local_search(kind, dg, Z, seed=98, rnd=2)
    got = Z.cpu().numpy()
    its = []
    for gi in range(g.num_graphs):
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        ref, i = discrete.local_search(kind, g.subgraph(gi), Z0[lo:hi], 98, gi * B + np.arange(B), 2)
        assert np.array_equal(got[lo:hi], ref)
        its.append(i)
    assert it == max(its)


# --------------------------------------------------------------------------
# a10 reset
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("B", [1, 6, 64])
@pytest.mark.parametrize("mode", ["zero", "flip"])
def test_reset_bit_exact(mqo, name, B, mode):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    Zb = arrays.binary01((g.n, B), 71) if kind == "mis" else arrays.spins((g.n, B), 71)
    for rho in (0.0, 0.05, 0.37):
        X = mqo.reset(kind, dg, torch.from_numpy(Zb).to(DEV), seed=5, rnd=3, rho=rho, mode=mode).cpu().numpy()
        for gi in range(g.num_graphs):
            lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
            n = hi - lo
            mask = discrete.reset_set(n, discrete.reset_count(rho, n), 5, gi * B + np.arange(B), 3)
            ref = discrete.reset_apply(kind, Zb[lo:hi], mask, mode)
            assert np.array_equal(X[lo:hi], ref), (gi, rho)


def test_reset_ties_with_given_keys(mqo):
    g = graphs.erdos_renyi(700, 0.01, 81)
    dg = mqo.DeviceGraph(g, DEV)
    B = 5
    keys = arrays.integers((700, B), 0, 6, 82)  # heavy ties
    keys[:, 4] = 3  # every key equal
    Zb = arrays.binary01((700, B), 83)
    X = mqo.reset("mis", dg, torch.from_numpy(Zb).to(DEV), seed=0, rnd=1, rho=0.1,
                  keys=torch.from_numpy(keys.astype(np.int32)).to(DEV)).cpu().numpy()
    mask = discrete.reset_set(700, 70, 0, np.arange(B), 1, keys=keys)
    assert np.array_equal(X, discrete.reset_apply("mis", Zb, mask, "zero"))


# --------------------------------------------------------------------------
# a9, a11, a12 whole solves under every plan
# --------------------------------------------------------------------------

SOLVE_CASES = [
    ("mis", "er300", dict(batch=6, steps_per_round=40, rounds=4, alpha=0.01, rho=0.05)),
    ("mis", "er_batch", dict(batch=5, steps_per_round=30, rounds=3, alpha=0.02, rho=0.1)),
    ("maxcut", "reg3", dict(batch=10, steps_per_round=50, rounds=4, alpha=0.01, rho=0.05)),
    ("maxcut", "torus", dict(batch=4, steps_per_round=40, rounds=3, alpha=0.02, rho=0.2, reset_mode="flip")),
    ("maxcut", "cut_batch", dict(batch=3, steps_per_round=25, rounds=3, alpha=0.03, rho=0.3, momentum=0.5)),
    ("mis", "er300", dict(batch=4, steps_per_round=20, rounds=2, alpha=0.05, rho=0.0, local_search=False)),
    ("mis", "er_batch", dict(batch=2, steps_per_round=0, rounds=2, alpha=0.05, rho=0.2)),
]


def _oracle_solve(kind, g, kw, x0=None):
    p = solver.Params(batch=kw["batch"], steps_per_round=kw["steps_per_round"], rounds=kw["rounds"],
                      alpha=kw["alpha"], seed=kw.get("seed", 17), mu=kw.get("momentum", 0.0), rho=kw["rho"],
                      reset_mode=kw.get("reset_mode", "zero"), local_search=kw.get("local_search", True))
    return solver.solve(kind, g, p, x0=x0)


@pytest.mark.parametrize("ci", range(len(SOLVE_CASES)))
@pytest.mark.parametrize("plan", ["persistent", "batched", "plain"])
def test_solve_bit_exact_every_plan(mqo, ci, plan):
    kind, name, kw = SOLVE_CASES[ci]
    g = CASES[name][1]
    kw = dict(kw, seed=17)
    dg = mqo.DeviceGraph(g, DEV)
    out = mqo.solve(kind, dg, plan=plan, **kw)
    ref = _oracle_solve(kind, g, kw)
    assert out["plan"] == plan
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])
    assert np.array_equal(out["best_value"].cpu().numpy(), ref["best_value"])
    assert np.array_equal(out["best_x"].cpu().numpy(), ref["best_x"])
    assert out["edge_updates"] == g.nnz * kw["batch"] * kw["steps_per_round"] * kw["rounds"]


@pytest.mark.parametrize("T", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("threads", [256, 1024])
@pytest.mark.parametrize("vec", [1, 2, 4])
@pytest.mark.parametrize("csr", [1, 2])
@pytest.mark.parametrize("name", ["reg3", "torus"])
def test_persistent_tile_shapes_agree(mqo, name, T, threads, vec, csr):
    if vec > T:
        pytest.skip("a lane cannot own more trajectories than the tile has")
    kind, g = CASES[name]
    kw = dict(batch=37, steps_per_round=30, rounds=3, alpha=0.01, rho=0.05, seed=3, momentum=0.3)
    dg = mqo.DeviceGraph(g, DEV)
    ref = mqo.solve(kind, dg, plan="batched", **kw)
    out = mqo.solve(kind, dg, plan="persistent", tile_cols=T, tile_threads=threads, tile_vec=vec, tile_csr=csr, **kw)
    assert (out["tile_cols"], out["tile_threads"], out["tile_vec"], out["tile_csr_lds"]) == (T, threads, vec, csr - 1)
    assert torch.equal(out["traj_best_value"], ref["traj_best_value"])
    assert torch.equal(out["traj_best_x"], ref["traj_best_x"])


def test_solve_with_given_x0_degree_init(mqo):
    g = graphs.erdos_renyi(150, 0.06, 91)
    B = 8
    x0 = pga.init_degree("mis", g.degrees(), np.arange(B), 4, 0.1).astype(np.float32)
    kw = dict(batch=B, steps_per_round=30, rounds=3, alpha=0.02, rho=0.1, seed=4)
    dg = mqo.DeviceGraph(g, DEV)
    ref = _oracle_solve("mis", g, kw, x0=x0)
    for plan in ("persistent", "batched", "plain"):
        out = mqo.solve("mis", dg, x0=torch.from_numpy(x0.ravel()).to(DEV), plan=plan, **kw)
        assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
        assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])


def test_degree_init_close_to_oracle(mqo):
    g = graphs.barabasi_albert(500, 3, 92)
    dg = mqo.DeviceGraph(g, DEV)
    for kind in ("mis", "maxcut"):
        X = mqo.init_iterate(kind, dg, 16, seed=8, init_mode="degree", init_sigma=0.2).cpu().numpy()
        ref = pga.init_degree(kind, g.degrees(), np.arange(16), 8, 0.2)
        assert np.abs(X - ref).max() < 1e-5


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
def test_plain_trajectory_subset(mqo, kind):
    """The plain plan on a subset of trajectory ids runs each of them exactly
    as the full batched solve does; the others hold no incumbent."""
    g = CASES["er_batch"][1] if kind == "mis" else CASES["cut_batch"][1]
    dg = mqo.DeviceGraph(g, DEV)
    B = 8
    kw = dict(batch=B, steps_per_round=20, rounds=3, alpha=0.05, rho=0.15, seed=81, final_search=True)
    ids = np.array([1, 6, B + 0, 2 * B + 3, (g.num_graphs - 1) * B + 7])
    full = mqo.solve(kind, dg, plan="batched", **kw)
    sub = mqo.solve(kind, dg, plan="plain", trajectories=ids, **kw)
    tv, tx = sub["traj_best_value"].cpu().numpy(), sub["traj_best_x"].cpu().numpy()
    assert np.array_equal(tv[ids], full["traj_best_value"].cpu().numpy()[ids])
    fx = full["traj_best_x"].cpu().numpy()
    ran = np.zeros_like(tx, dtype=bool)
    for t in ids:
        gi, b = divmod(int(t), B)
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        assert np.array_equal(tx[lo:hi, b], fx[lo:hi, b])
        ran[lo:hi, b] = True
    assert np.all(tx[~ran] == 0)
    rest = np.setdiff1d(np.arange(g.num_graphs * B), ids)
    assert np.all(tv[rest] == np.iinfo(np.int64).min)
    nnz = np.diff(g.row_ptr[g.vtx_offset])
    assert sub["edge_updates"] == sum(int(nnz[t // B]) for t in ids) * 20 * 3
    ref = solver.solve(kind, g, solver.Params(**kw))
    assert np.array_equal(tv[ids], ref["traj_best_value"][ids])


def test_trace_reports_every_phase(mqo, tmp_path, monkeypatch):
    """MQO_TRACE=<file>: one JSON line per solve with HIP-event totals per
    phase; unset: nothing is written."""
    import json
    kind, g = CASES["er_batch"]
    dg = mqo.DeviceGraph(g, DEV)
    path = tmp_path / "trace.jsonl"
    monkeypatch.setenv("MQO_TRACE", str(path))
    kw = dict(batch=8, steps_per_round=20, rounds=3, alpha=0.05, rho=0.15, seed=3)
    mqo.solve(kind, dg, plan="batched", final_search=True, **kw)
    mqo.solve(kind, dg, plan="persistent", **kw)
    monkeypatch.setenv("MQO_TRACE", "0")
    mqo.solve(kind, dg, plan="batched", **kw)
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(lines) == 2
    b, t = lines
    assert b["plan"] == "batched" and t["plan"] == "persistent" and b["rounds_executed"] == 3
    G = g.num_graphs
    # one step launch per round over the whole batch of graphs
    assert b["phases"]["steps"]["count"] == 3 and b["phases"]["reset"]["count"] == 2 * G
    assert b["phases"]["local_search"]["count"] == 3 * G and b["phases"]["evaluate"]["count"] == 3 * G
    assert b["phases"]["pair_search"]["count"] == 1
    assert all(v["ms"] >= 0 for v in b["phases"].values())
    assert t["phases"]["persistent_rounds"]["count"] >= 1 and "steps" not in t["phases"]


def _step_shapes(B):
    out = []
    for vec in (1, 2, 4):
        if vec > 1 and (B % vec or B < 2 * vec):
            continue
        groups = -(-B // vec)
        lanes = 1
        while True:
            out.append((vec, lanes))
            if lanes >= groups or lanes == 64:
                break
            lanes *= 2
    return out


_SHAPE_REF = {}


@pytest.mark.parametrize("kind,B,vec,lanes", [(k, B, v, l) for k in ("mis", "maxcut") for B in (8, 13)
                                              for v, l in _step_shapes(B)])
def test_forced_step_shapes_bit_exact(mqo, kind, B, vec, lanes):
    """Every launch shape of the streaming step kernel (columns per lane x
    lanes per row, more columns than lanes x vec in further column slices)
    on the batched plan, over a ragged batch with a hub row (MIS) or a
    weighted batch (MaxCut), equals the oracle bit for bit."""
    g = graphs.concat([graphs.erdos_renyi(150, 0.05, 31), graphs.star(200), graphs.path(3)]) if kind == "mis" else \
        graphs.concat([graphs.torus_pm1(9, 32), graphs.with_weights(graphs.erdos_renyi(80, 0.1, 33), 34)])
    dg = mqo.DeviceGraph(g, DEV, hub_min_degree=64)
    kw = dict(batch=B, steps_per_round=20, rounds=2, alpha=0.05, rho=0.15, seed=35)
    out = mqo.solve(kind, dg, plan="batched", step_vec=vec, step_lanes=lanes, **kw)
    assert (out["step_vec"], out["step_lanes"]) == (vec, lanes)
    if (kind, B) not in _SHAPE_REF:
        _SHAPE_REF[(kind, B)] = solver.solve(kind, g, solver.Params(**kw))
    ref = _SHAPE_REF[(kind, B)]
    for key in ("traj_best_value", "traj_best_x", "best_value"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


def test_step_shape_rejected_when_it_does_not_fit(mqo):
    dg = mqo.DeviceGraph(CASES["reg3"][1], DEV)
    with pytest.raises(mqo.MqoError) as e:
        mqo.solve("maxcut", dg, plan="batched", batch=6, steps_per_round=4, step_vec=4)
    assert e.value.status == -1
    with pytest.raises(mqo.MqoError):
        mqo.solve("maxcut", dg, plan="batched", batch=6, steps_per_round=4, step_lanes=3)


def test_auto_plan_is_tuned_and_cached(mqo, tmp_path, monkeypatch):
    """MQO_PLAN_AUTO times the persistent and streaming shapes once per shape
    key; the choice is in the cache file, reused by the next solve, and
    either plan gives the same result."""
    kind, g = CASES["er_batch"]
    dg = mqo.DeviceGraph(g, DEV)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MQO_TUNE_CACHE", str(path))
    mqo.lib().mqo_clear_caches()
    kw = dict(batch=16, steps_per_round=20, rounds=2, alpha=0.05, rho=0.15, seed=36)
    a = mqo.solve(kind, dg, **kw)
    assert a["plan"] in ("persistent", "batched")
    keys = [ln.split("\t")[0] for ln in path.read_text().splitlines() if ln and not ln.startswith("#")]
    assert any(k.startswith("plan|") for k in keys) and any(k.startswith("tile|") for k in keys)
    n = mqo.tune_cache_size()
    b = mqo.solve(kind, dg, **kw)
    assert b["plan"] == a["plan"] and mqo.tune_cache_size() == n  # nothing timed again
    other = "batched" if a["plan"] == "persistent" else "persistent"
    c = mqo.solve(kind, dg, plan=other, **kw)
    for key in ("traj_best_value", "traj_best_x", "best_value", "best_x"):
        assert torch.equal(a[key], c[key]), key
    mqo.lib().mqo_clear_caches()


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
def test_auto_plan_trial_leaves_no_trace(mqo, kind):
    """When the per-step timings are within a factor of two, AUTO times both
    plans on up to eight rounds of the solve before it runs; the solve that follows
    reports the same answer and counters as the same plan forced (the
    trial's writes are all written again), with and without the tuning."""
    g = graphs.concat([graphs.erdos_renyi(120, 0.1, 61), graphs.erdos_renyi(90, 0.12, 62)])
    dg = mqo.DeviceGraph(g, DEV)
    mqo.lib().mqo_clear_caches()
    kw = dict(batch=24, steps_per_round=30, rounds=3, alpha=0.03, rho=0.1, seed=63, momentum=0.3, check_every=5,
              final_search=True)
    first = mqo.solve(kind, dg, **kw)
    again = mqo.solve(kind, dg, **kw)
    forced = mqo.solve(kind, dg, plan=first["plan"], **kw)
    assert again["plan"] == first["plan"]
    for out in (again, forced):
        for key in ("traj_best_value", "traj_best_x", "best_value", "best_x"):
            assert torch.equal(first[key], out[key]), key
        for key in ("edge_updates", "steps_executed", "rounds_executed", "ls_iterations",
                    "final_search_alternations"):
            assert first[key] == out[key], key
    mqo.lib().mqo_clear_caches()


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("plan", ["batched", "plain"])
def test_paper_hyperparameters_bit_exact(mqo, kind, plan):
    """The paper's own settings (its ER tables): MIS alpha 0.8, momentum
    0.3, rho 0.6; MaxCut alpha 0.0025, momentum 0.8, rho 0.8; a degree-based
    start (the oracle's, given to both sides: its Gaussian uses log and cos),
    PGA until a fixed point checked every 10 steps, reset rounds, and the
    pair search closing the run."""
    if kind == "mis":
        g = graphs.erdos_renyi(300, 30.0 / 299, 37)
        kw = dict(alpha=0.8, mu=0.3, rho=0.6)
    else:
        g = graphs.erdos_renyi(200, 20.0 / 199, 38)
        kw = dict(alpha=0.0025, mu=0.8, rho=0.8)
    B = 8
    x0 = pga.init_degree(kind, g.degrees(), np.arange(B), 39, 0.1).astype(np.float32)
    common = dict(batch=B, steps_per_round=60, rounds=5, seed=39, check_every=10, final_search=True)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), x0=torch.from_numpy(x0).to(DEV).reshape(-1), plan=plan,
                    momentum=kw["mu"], alpha=kw["alpha"], rho=kw["rho"], **common)
    ref = solver.solve(kind, g, solver.Params(**kw, **common), x0=x0)
    for key in ("traj_best_value", "traj_best_x", "best_value", "best_x"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
    nnz = g.nnz
    assert out["edge_updates"] == int(ref["traj_steps"].sum()) * nnz


@pytest.mark.parametrize("name", ["torus", "er300", "cut_batch"])
def test_local_rows_hint_keeps_results(mqo, name):
    """The XCD row-range order (local_rows = 1) and the launch order (0)
    give the same steps, objective, gradient, adjoint and solves."""
    kind, g = CASES[name]
    B = 8
    X0 = torch.from_numpy(_x(kind, g.n, B, 41)).to(DEV)
    param = 2.0 if kind == "mis" else 1e-3
    res = []
    for lr in (0, 1):
        dg = mqo.DeviceGraph(g, DEV, local_rows=lr, hub_min_degree=4)
        X = X0.clone()
        mqo.pga_steps(kind, dg, X, 3, alpha=0.05)
        f, gr = mqo.objective_grad(kind, dg, X0, param)
        XK, ck = mqo.unrolled_forward(kind, dg, X0, 0.05, 4, 2, param)
        dX, da = mqo.unrolled_backward(kind, dg, ck, torch.ones_like(X0), 0.05, 4, 2, param)
        out = mqo.solve(kind, dg, plan="batched", batch=B, steps_per_round=10, rounds=2, alpha=0.05, seed=42)
        res.append([X, f, gr, XK, dX, da, out["traj_best_value"], out["traj_best_x"]])
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_two_streams_at_once(mqo):
    """Degree initialisation and objective + gradient queued on two streams
    at the same time, each with its default workspace (one per stream):
    both results equal the oracle's."""
    g = graphs.barabasi_albert(3000, 3, 97)
    dg = mqo.DeviceGraph(g, DEV)
    B = 16
    Xm = torch.from_numpy(_x("mis", g.n, B, 98)).to(DEV)
    Xc = torch.from_numpy(_x("maxcut", g.n, B, 99)).to(DEV)
    main = torch.cuda.current_stream()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(main)
    s2.wait_stream(main)
    with torch.cuda.stream(s1):
        Ia = mqo.init_iterate("mis", dg, B, seed=8, init_mode="degree", init_sigma=0.2)
        fa, ga = mqo.objective_grad("mis", dg, Xm, 2.0)
    with torch.cuda.stream(s2):
        Ib = mqo.init_iterate("maxcut", dg, B, seed=9, init_mode="degree", init_sigma=0.3)
        fb, gb = mqo.objective_grad("maxcut", dg, Xc, 1e-3)
    torch.cuda.synchronize()
    deg = g.degrees()
    assert np.abs(Ia.cpu().numpy() - pga.init_degree("mis", deg, np.arange(B), 8, 0.2)).max() < 1e-5
    assert np.abs(Ib.cpu().numpy() - pga.init_degree("maxcut", deg, np.arange(B), 9, 0.3)).max() < 1e-5
    for kind, X, param, f, gr in (("mis", Xm, 2.0, fa, ga), ("maxcut", Xc, 1e-3, fb, gb)):
        X0 = X.cpu().numpy()
        fr, grr = pga.objective_and_grad(g, kind, param, X0.astype(np.float64))
        assert np.allclose(f.cpu().numpy(), fr, rtol=1e-5, atol=1e-5 * np.abs(X0).sum())
        assert np.abs(gr.cpu().numpy() - grr).max() / max(1.0, np.abs(grr).max()) <= 1e-5


@pytest.mark.parametrize("plan,pool", [("persistent", 0), ("batched", 0), ("plain", 0), ("batched", 2)])
@pytest.mark.parametrize("kind", ["mis", "maxcut"])
def test_time_budget_stops_after_round_0(mqo, plan, pool, kind):
    # a budget that has run out before round 1: every trajectory runs round 0
    # (the plain plan too, one trajectory after the other), and the pass the
    # budget cut short ends with the pair search (round index = rounds)
    g = CASES["er_batch"][1] if kind == "mis" else CASES["cut_batch"][1]
    dg = mqo.DeviceGraph(g, DEV)
    kw = dict(batch=4, steps_per_round=10, rounds=1000, alpha=0.01, rho=0.1, seed=1, final_search=True, pool_k=pool)
    out = mqo.solve(kind, dg, plan=plan, time_budget_s=1e-9, **kw)
    assert out["plan"] == plan
    assert out["rounds_executed"] == 1
    assert out["steps_executed"] == 10
    ref = solver.solve(kind, g, solver.Params(rounds_run=1, **kw))
    for key in ("traj_best_value", "traj_best_x", "best_value", "best_x") + (("pool_value", "pool_x") if pool else ()):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


def test_invalid_graph_rejected_before_launch(mqo):
    g = graphs.erdos_renyi(50, 0.1, 94)
    bad = graphs.Graph(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[0] = (bad.col_idx[0] + 1) % 50  # breaks symmetry or ordering
    dg = mqo.DeviceGraph(bad, DEV)
    with pytest.raises(mqo.MqoError) as e:
        mqo.solve("mis", dg, batch=2, steps_per_round=5, rounds=1)
    assert e.value.status == -2
    with pytest.raises(mqo.MqoError):
        dg.validate()
    mqo.DeviceGraph(g, DEV).validate()
    with pytest.raises(mqo.MqoError) as e:
        mqo.solve("maxcut", mqo.DeviceGraph(g, DEV), batch=2, lam=2.5)
    assert e.value.status == -1


# --------------------------------------------------------------------------
# a13 objective and SpMM-gradient backward, a14 unrolled adjoint
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("B", [1, 4, 64])
def test_objective_and_gradient(mqo, name, B):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    param = 2.0 if kind == "mis" else 1e-3
    X0 = _x(kind, g.n, B, 101)
    scale = arrays.uniform((g.num_graphs * B,), -2, 2, 102)
    f, grad = mqo.objective_grad(kind, dg, torch.from_numpy(X0).to(DEV), param,
                                 scale=torch.from_numpy(scale).to(DEV))
    f = f.cpu().numpy()
    grad = grad.cpu().numpy()
    for gi in range(g.num_graphs):
        sub = g.subgraph(gi)
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        fr, gr = pga.objective_and_grad(sub, kind, param, X0[lo:hi].astype(np.float64), scale[gi * B:(gi + 1) * B])
        # f: float32 neighbour sums (relative error <= deg * 2^-24), float64 accumulation
        assert np.allclose(f[gi * B:(gi + 1) * B], fr, rtol=1e-5, atol=1e-5 * np.abs(X0[lo:hi]).sum())
        assert np.abs(grad[lo:hi] - gr).max() / max(1.0, np.abs(gr).max()) <= 1e-5


def test_autograd_objective_backward_matches_closed_form(mqo):
    kind, g = CASES["torus"]
    dg = mqo.DeviceGraph(g, DEV)
    X0 = _x(kind, g.n, 8, 111)
    X = torch.from_numpy(X0).to(DEV).requires_grad_(True)
    f = mqo.objective(X, dg, kind, 1e-3)
    wn = np.linspace(-1, 1, f.numel())
    w = torch.from_numpy(wn).to(DEV)
    (f * w).sum().backward()
    _, gr = pga.objective_and_grad(g, kind, 1e-3, X0.astype(np.float64), wn)
    got = X.grad.cpu().numpy()
    assert np.abs(got - gr).max() / max(1.0, np.abs(gr).max()) <= 1e-5


@pytest.mark.parametrize("name", ["er300", "reg3", "torus"])
def test_unrolled_forward_bit_exact_and_adjoint(mqo, name):
    kind, g = CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    param = 2.0 if kind == "mis" else 1e-3
    B, K, c, alpha = 6, 20, 5, 0.01
    X0 = _x(kind, g.n, B, 121)
    XK, ckpt = mqo.unrolled_forward(kind, dg, torch.from_numpy(X0).to(DEV), alpha, K, c, param)
    xs = pga.unrolled_forward(g, kind, param, alpha, K, X0, precision="fp32")
    assert np.array_equal(XK.cpu().numpy(), xs[K])
    for j in range(K // c):
        assert np.array_equal(ckpt[j].cpu().numpy(), xs[j * c])
    dL = obj.gradient(kind, xs[K].astype(np.float64), obj.adjacency(g), param)
    dX0, da = mqo.unrolled_backward(kind, dg, ckpt, torch.from_numpy(dL.astype(np.float32)).to(DEV), alpha, K, c,
                                    param)
    rX0, ra = pga.unrolled_backward(g, kind, param, alpha, K, X0, dL.astype(np.float32).astype(np.float64),
                                    precision="fp32")
    got = dX0.cpu().numpy()
    # float32 adjoint recursion over K steps against float64: relative 1e-4
    assert np.abs(got - rX0).max() / max(1.0, np.abs(rX0).max()) <= 1e-4
    assert np.allclose(da.cpu().numpy(), ra, rtol=1e-4, atol=1e-4 * np.abs(ra).max())


def test_unrolled_autograd_function(mqo):
    kind, g = CASES["reg3"]
    dg = mqo.DeviceGraph(g, DEV)
    X0 = torch.from_numpy(_x(kind, g.n, 4, 131)).to(DEV).requires_grad_(True)
    alpha = torch.tensor(0.01, dtype=torch.float64, device=DEV, requires_grad=True)
    XK = mqo.unrolled_pga(X0, alpha, dg, kind, 1e-3, K=10, ckpt_every=5)
    loss = mqo.objective(XK, dg, kind, 1e-3).sum()
    loss.backward()
    x0 = X0.detach().cpu().numpy()
    xs = pga.unrolled_forward(g, kind, 1e-3, 0.01, 10, x0, precision="fp32")
    dL = obj.gradient(kind, xs[10].astype(np.float64), obj.adjacency(g), 1e-3)
    rX0, ra = pga.unrolled_backward(g, kind, 1e-3, 0.01, 10, x0, dL, precision="fp32")
    assert np.abs(X0.grad.cpu().numpy() - rX0).max() / max(1.0, np.abs(rX0).max()) <= 1e-4
    assert abs(float(alpha.grad) - ra.sum()) <= 1e-4 * max(1.0, abs(ra.sum()))


# --------------------------------------------------------------------------
# rows of very high degree (hubs) in the streaming kernels
# --------------------------------------------------------------------------

HUB_CASES = {
    "ba_star": ("mis", graphs.concat([graphs.barabasi_albert(1500, 3, 131), graphs.star(700)])),
    "ba_weighted": ("maxcut", graphs.with_weights(graphs.barabasi_albert(3000, 5, 132), 133)),
}


@pytest.mark.parametrize("name", list(HUB_CASES))
@pytest.mark.parametrize("B", [1, 3, 16, 64, 130])
@pytest.mark.parametrize("hub_min_degree", [None, 8, 128])
def test_hub_rows_steps_objective_adjoint(mqo, name, B, hub_min_degree):
    kind, g = HUB_CASES[name]
    assert g.degrees().max() > 128
    dg = mqo.DeviceGraph(g, DEV, hub_min_degree=hub_min_degree)
    assert (dg.num_hubs > 0) == (hub_min_degree is not None)
    param = 2.0 if kind == "mis" else 1e-3
    X0 = _x(kind, g.n, B, 141 + B)
    X = torch.from_numpy(X0).to(DEV)
    mqo.pga_steps(kind, dg, X, 3, alpha=0.02, gamma=2.0, lam=1e-3)
    ref = X0
    for _ in range(3):
        ref, _ = pga.step32(g, ref, kind, 0.02, param)
    assert np.array_equal(X.cpu().numpy(), ref)

    f, grad = mqo.objective_grad(kind, dg, torch.from_numpy(X0).to(DEV), param)
    for gi in range(g.num_graphs):
        sub = g.subgraph(gi)
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        fr, gr = pga.objective_and_grad(sub, kind, param, X0[lo:hi].astype(np.float64), np.ones(B))
        assert np.allclose(f.cpu().numpy()[gi * B:(gi + 1) * B], fr, rtol=1e-5,
                           atol=1e-5 * np.abs(X0[lo:hi]).sum())
        assert np.abs(grad.cpu().numpy()[lo:hi] - gr).max() / max(1.0, np.abs(gr).max()) <= 1e-5

    if g.num_graphs == 1 and B in (3, 64):
        K, c, alpha = 10, 5, 0.01
        XK, ckpt = mqo.unrolled_forward(kind, dg, torch.from_numpy(X0).to(DEV), alpha, K, c, param)
        xs = pga.unrolled_forward(g, kind, param, alpha, K, X0, precision="fp32")
        assert np.array_equal(XK.cpu().numpy(), xs[K])
        dL = obj.gradient(kind, xs[K].astype(np.float64), obj.adjacency(g), param).astype(np.float32)
        dX0, da = mqo.unrolled_backward(kind, dg, ckpt, torch.from_numpy(dL).to(DEV), alpha, K, c, param)
        rX0, ra = pga.unrolled_backward(g, kind, param, alpha, K, X0, dL.astype(np.float64), precision="fp32")
        assert np.abs(dX0.cpu().numpy() - rX0).max() / max(1.0, np.abs(rX0).max()) <= 1e-4
        assert np.allclose(da.cpu().numpy(), ra, rtol=1e-4, atol=1e-4 * np.abs(ra).max())


@pytest.mark.parametrize("plan", ["batched", "plain"])
@pytest.mark.parametrize("hub_min_degree", [8, 128])
def test_hub_rows_solve_bit_exact(mqo, plan, hub_min_degree):
    kind, g = HUB_CASES["ba_star"]
    kw = dict(batch=5, steps_per_round=20, rounds=2, alpha=0.02, rho=0.1, seed=17)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV, hub_min_degree=hub_min_degree), plan=plan, **kw)
    ref = _oracle_solve(kind, g, kw)
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])


def test_hub_list_checked_on_device(mqo):
    kind, g = HUB_CASES["ba_star"]
    dg = mqo.DeviceGraph(g, DEV, hub_min_degree=8)
    dg.validate()
    kw = dict(batch=2, steps_per_round=2, rounds=1)
    # drop one hub from the list: the count no longer matches
    rows = dg.hub_rows.clone()
    dg.hub_rows[-1] = rows[-2]
    with pytest.raises(mqo.MqoError) as e:
        mqo.solve(kind, dg, **kw)
    assert e.value.status == -2
    dg.hub_rows.copy_(rows)
    # a listed row below the threshold
    light = int(np.nonzero(g.degrees() <= 8)[0][0])
    dg.hub_rows[0] = light
    with pytest.raises(mqo.MqoError):
        dg.validate()
    dg.hub_rows.copy_(rows)
    mqo.solve(kind, dg, **kw)


# --------------------------------------------------------------------------
# lane groups taking rows in pairs (chosen for near-regular graphs); forced
# here through the max_degree hint on irregular graphs so that both the
# lockstep and the one-after-the-other paths run
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["er300", "cut_batch", "ba_star"])
@pytest.mark.parametrize("B", [16, 64, 100])
def test_row_pairs_forced(mqo, name, B):
    kind, g = HUB_CASES[name] if name in HUB_CASES else CASES[name]
    dg = mqo.DeviceGraph(g, DEV, hub_min_degree=8 if name == "ba_star" else "auto")
    dg._struct.max_degree = 1  # hint: "near-regular" -> pairs
    param = 2.0 if kind == "mis" else 1e-3
    X0 = _x(kind, g.n, B, 161 + B)
    X = torch.from_numpy(X0).to(DEV)
    mqo.pga_steps(kind, dg, X, 3, alpha=0.02, gamma=2.0, lam=1e-3)
    ref = X0
    for _ in range(3):
        ref, _ = pga.step32(g, ref, kind, 0.02, param)
    assert np.array_equal(X.cpu().numpy(), ref)
    f, grad = mqo.objective_grad(kind, dg, torch.from_numpy(X0).to(DEV), param)
    for gi in range(g.num_graphs):
        sub = g.subgraph(gi)
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        fr, gr = pga.objective_and_grad(sub, kind, param, X0[lo:hi].astype(np.float64), np.ones(B))
        assert np.allclose(f.cpu().numpy()[gi * B:(gi + 1) * B], fr, rtol=1e-5,
                           atol=1e-5 * np.abs(X0[lo:hi]).sum())
        assert np.abs(grad.cpu().numpy()[lo:hi] - gr).max() / max(1.0, np.abs(gr).max()) <= 1e-5
    if g.num_graphs == 1:
        K, c, alpha = 10, 5, 0.01
        XK, ckpt = mqo.unrolled_forward(kind, dg, torch.from_numpy(X0).to(DEV), alpha, K, c, param)
        xs = pga.unrolled_forward(g, kind, param, alpha, K, X0, precision="fp32")
        assert np.array_equal(XK.cpu().numpy(), xs[K])
        dL = obj.gradient(kind, xs[K].astype(np.float64), obj.adjacency(g), param).astype(np.float32)
        dX0, da = mqo.unrolled_backward(kind, dg, ckpt, torch.from_numpy(dL).to(DEV), alpha, K, c, param)
        rX0, ra = pga.unrolled_backward(g, kind, param, alpha, K, X0, dL.astype(np.float64), precision="fp32")
        assert np.abs(dX0.cpu().numpy() - rX0).max() / max(1.0, np.abs(rX0).max()) <= 1e-4
        assert np.allclose(da.cpu().numpy(), ra, rtol=1e-4, atol=1e-4 * np.abs(ra).max())


# --------------------------------------------------------------------------
# a11: optional early exit of a round at fixed points of the projected step
# --------------------------------------------------------------------------

EXIT_CASES = [
    ("mis", "er300", dict(batch=6, steps_per_round=60, rounds=3, alpha=0.05, rho=0.1)),
    ("mis", "er_batch", dict(batch=5, steps_per_round=45, rounds=2, alpha=0.05, rho=0.1)),
    ("maxcut", "reg3", dict(batch=10, steps_per_round=80, rounds=3, alpha=0.2, rho=0.05)),
    ("maxcut", "torus", dict(batch=4, steps_per_round=50, rounds=2, alpha=0.2, rho=0.2, reset_mode="flip")),
    ("maxcut", "cut_batch", dict(batch=3, steps_per_round=40, rounds=2, alpha=0.2, rho=0.3, momentum=0.5)),
]


@pytest.mark.parametrize("ci", range(len(EXIT_CASES)))
@pytest.mark.parametrize("check", [1, 7, 200])
@pytest.mark.parametrize("plan,tile", [("persistent", {}), ("persistent", dict(tile_cols=4, tile_reg=1)),
                                       ("batched", {}), ("plain", {})])
def test_early_exit_bit_exact(mqo, ci, check, plan, tile):
    kind, name, kw = EXIT_CASES[ci]
    g = CASES[name][1]
    kw = dict(kw, seed=23, check_every=check)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), plan=plan, **tile, **kw)
    p = solver.Params(batch=kw["batch"], steps_per_round=kw["steps_per_round"], rounds=kw["rounds"],
                      alpha=kw["alpha"], seed=23, mu=kw.get("momentum", 0.0), rho=kw["rho"],
                      reset_mode=kw.get("reset_mode", "zero"), check_every=check)
    ref = solver.solve(kind, g, p)
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])
    nnz_g = np.diff(g.row_ptr[g.vtx_offset])
    eu = int((ref["traj_steps"].reshape(g.num_graphs, -1) * nnz_g[:, None]).sum())
    assert out["edge_updates"] == eu


# --------------------------------------------------------------------------
# the other MaxCut formulations: f_L (Eq. (4)), f_P (Eq. (5)), f_A (Eq. (6))
# --------------------------------------------------------------------------

FORMS = ["maxcut_fl", "maxcut_fp", "maxcut_fa"]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name", ["er300", "torus", "cut_batch"])
@pytest.mark.parametrize("B", [1, 5, 32])
def test_formulation_steps_objective_adjoint(mqo, form, name, B):
    g = CASES[name][1]
    dg = mqo.DeviceGraph(g, DEV)
    lam = 0.3
    X0 = _x("maxcut", g.n, B, 171 + B)
    for mu in (0.0, 0.5):
        X = torch.from_numpy(X0).to(DEV)
        V = torch.zeros_like(X)
        mqo.pga_steps(form, dg, X, 6, alpha=0.05, lam=lam, momentum=mu, V=V)
        ref, Vr = X0, None
        for _ in range(6):
            ref, Vr = pga.step32(g, ref, form, 0.05, lam, mu, Vr)
        assert np.array_equal(X.cpu().numpy(), ref)
    f, grad = mqo.objective_grad(form, dg, torch.from_numpy(X0).to(DEV), lam)
    for gi in range(g.num_graphs):
        sub = g.subgraph(gi)
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        fr, gr = pga.objective_and_grad(sub, form, lam, X0[lo:hi].astype(np.float64), np.ones(B))
        assert np.allclose(f.cpu().numpy()[gi * B:(gi + 1) * B], fr, rtol=1e-5,
                           atol=1e-5 * (np.abs(X0[lo:hi]).sum() + 1))
        assert np.abs(grad.cpu().numpy()[lo:hi] - gr).max() / max(1.0, np.abs(gr).max()) <= 1e-5
    if g.num_graphs == 1:
        K, c, alpha = 10, 5, 0.02
        XK, ckpt = mqo.unrolled_forward(form, dg, torch.from_numpy(X0).to(DEV), alpha, K, c, lam)
        xs = pga.unrolled_forward(g, form, lam, alpha, K, X0, precision="fp32")
        assert np.array_equal(XK.cpu().numpy(), xs[K])
        dL = obj.gradient(form, xs[K].astype(np.float64), obj.adjacency(g), lam).astype(np.float32)
        dX0, da = mqo.unrolled_backward(form, dg, ckpt, torch.from_numpy(dL).to(DEV), alpha, K, c, lam)
        rX0, ra = pga.unrolled_backward(g, form, lam, alpha, K, X0, dL.astype(np.float64), precision="fp32")
        assert np.abs(dX0.cpu().numpy() - rX0).max() / max(1.0, np.abs(rX0).max()) <= 1e-4
        assert np.allclose(da.cpu().numpy(), ra, rtol=1e-4, atol=1e-4 * max(1.0, np.abs(ra).max()))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("plan", ["auto", "batched", "plain"])
def test_formulation_solves_bit_exact(mqo, form, plan):
    g = CASES["cut_batch"][1]
    kw = dict(batch=4, steps_per_round=30, rounds=3, alpha=0.05, rho=0.2, seed=29, lam=0.3)
    out = mqo.solve(form, mqo.DeviceGraph(g, DEV), plan=plan, **kw)
    assert out["plan"] in ("batched", "plain")
    p = solver.Params(batch=4, steps_per_round=30, rounds=3, alpha=0.05, seed=29, lam=0.3, rho=0.2)
    ref = solver.solve(form, g, p)
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])


def test_formulations_rejected_where_not_offered(mqo):
    dg = mqo.DeviceGraph(CASES["reg3"][1], DEV)
    with pytest.raises(mqo.MqoError) as e:
        mqo.solve("maxcut_fl", dg, batch=2, steps_per_round=4, plan="persistent")
    assert e.value.status == -5
    with pytest.raises(mqo.MqoError) as e:
        mqo.solve("maxcut_fa", dg, batch=2, steps_per_round=4, check_every=2)
    assert e.value.status == -5
    with pytest.raises(mqo.MqoError) as e:
        mqo.objective_grad("maxcut_fp", dg, torch.zeros(dg.n, 2, device=DEV), 0.0)
    assert e.value.status == -1


# Appendix B's escapability set-up: ten ER graphs n = 100, p = 0.66, step
# 0.1, lambda 1e-3, no local search and no reset.  What the propositions
# fix is checked exactly: c*1 is stationary for f_L (Prop. 3.2) and not for
# f_P, f_B; every binary point is PGA-fixed under f_L and f_P (Prop. 3.2,
# Thm. 3.3); a 1-flip repairable point is not PGA-fixed under f_A (Prop. 3.4)
# nor f_B (Thm. 3.6).  Dyadic c keeps every sum exact in float32.

def _appendix_b_graphs():
    return graphs.concat([graphs.erdos_renyi(100, 0.66, 700 + i) for i in range(10)])


def _one_flip_repairable(g, X):
    A = obj.adjacency(g)
    return np.array([bool(np.any(X[:, j] * (A @ X[:, j]) > 0)) for j in range(X.shape[1])])


@pytest.mark.parametrize("form", ["maxcut_fl", "maxcut_fp", "maxcut"])
def test_escapability_of_laplacian_stationary_points(mqo, form):
    g = _appendix_b_graphs()
    dg = mqo.DeviceGraph(g, DEV)
    cs = np.array([-0.75, -0.25, 0.375, 0.5, -0.5, 0.125], dtype=np.float32)
    X0 = np.tile(cs, (g.n, 1))
    X = torch.from_numpy(X0).to(DEV)
    mqo.pga_steps(form, dg, X, 1, alpha=0.1, lam=1e-3)
    moved = ~np.all(X.cpu().numpy() == X0, axis=0)
    assert np.all(moved == (form != "maxcut_fl"))
    X = torch.from_numpy(X0).to(DEV)
    mqo.pga_steps(form, dg, X, 200, alpha=0.1, lam=1e-3)
    ref = X0
    for _ in range(200):
        ref, _v = pga.step32(g, ref, form, 0.1, 1e-3, 0.0, None)
    assert np.array_equal(X.cpu().numpy(), ref)
    if form == "maxcut_fl":
        _, value, _, _ = mqo.round_evaluate(form, dg, X)
        assert np.all(value.cpu().numpy() == 0)


@pytest.mark.parametrize("form", ["maxcut_fl", "maxcut_fp", "maxcut_fa", "maxcut"])
def test_escapability_of_one_flip_repairable_points(mqo, form):
    g = _appendix_b_graphs()
    dg = mqo.DeviceGraph(g, DEV)
    rng = np.random.default_rng(31)
    X0 = np.where(rng.random((g.n, 24)) < 0.5, -1.0, 1.0).astype(np.float32)
    for gi in range(g.num_graphs):
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        assert _one_flip_repairable(g.subgraph(gi), X0[lo:hi]).all()
    X = torch.from_numpy(X0).to(DEV)
    mqo.pga_steps(form, dg, X, 1, alpha=0.1, lam=1e-3)
    X1 = X.cpu().numpy()
    for gi in range(g.num_graphs):
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        fixed = np.all(X1[lo:hi] == X0[lo:hi], axis=0)
        assert np.all(fixed == (form in ("maxcut_fl", "maxcut_fp")))
    ref, _v = pga.step32(g, X0, form, 0.1, 1e-3, 0.0, None)
    assert np.array_equal(X1, ref)


def test_formulation_comparison_ordering(mqo):
    """Appendix B's comparison on synthetic ER graphs (n = 100, mean degree
    50; three graphs, eight common starts, step 0.01, no search, no reset):
    the GPU trajectories equal the oracle's bit for bit, and the adjacency
    formulations end at larger cuts than the Laplacian ones."""
    g = graphs.concat([graphs.erdos_renyi(100, 50 / 99, 900 + i) for i in range(3)])
    dg = mqo.DeviceGraph(g, DEV)
    X0 = arrays.uniform((g.n, 8), -1.0, 1.0, 77)
    mean_cut = {}
    for form in ["maxcut_fl", "maxcut_fp", "maxcut_fa", "maxcut"]:
        X = torch.from_numpy(X0).to(DEV)
        mqo.pga_steps(form, dg, X, 300, alpha=0.01, lam=1e-3)
        ref = X0
        for _ in range(300):
            ref, _v = pga.step32(g, ref, form, 0.01, 1e-3, 0.0, None)
        assert np.array_equal(X.cpu().numpy(), ref)
        _, value, _, _ = mqo.round_evaluate(form, dg, X)
        cuts = value.cpu().numpy()
        for gi in range(g.num_graphs):
            lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
            S = np.where(ref[lo:hi] > 0, 1, -1).astype(np.int8)
            assert np.array_equal(cuts[gi * 8:(gi + 1) * 8], discrete.evaluate_cut(g.subgraph(gi), S))
        mean_cut[form] = cuts.mean()
    assert min(mean_cut["maxcut_fa"], mean_cut["maxcut"]) > 1.05 * max(mean_cut["maxcut_fl"], mean_cut["maxcut_fp"])


# --------------------------------------------------------------------------
# the paper's own searches: OneTwoSwap (Def. 2.3), OneTwoFlip (Def. 2.5)
# --------------------------------------------------------------------------

PAIR_CASES = {
    "mis_er300": ("mis", CASES["er300"][1]),
    "mis_batch": ("mis", graphs.concat([CASES["er_batch"][1], graphs.star(7), graphs.path(3), graphs.path(2)])),
    # mean degree >= 24: proposals by one wavefront per row
    "mis_dense": ("mis", graphs.concat([graphs.erdos_renyi(150, 0.3, 4904), graphs.erdos_renyi(90, 0.5, 4905),
                                        graphs.complete(5)])),
    "cut_reg4": ("maxcut", graphs.random_regular(240, 4, 4900)),
    "cut_torus": ("maxcut", CASES["torus"][1]),
    "cut_batch": ("maxcut", graphs.concat([CASES["cut_batch"][1], graphs.cycle(4), graphs.empty(2)])),
    "cut_weighted": ("maxcut", graphs.with_weights(graphs.erdos_renyi(150, 0.06, 4901), 4902, values=(-2, -1, 1, 3))),
}


def _pair_ref(kind, g, Z, seed, rnd, B):
    out = np.empty_like(Z)
    for gi in range(g.num_graphs):
        lo, hi = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        out[lo:hi], _ = discrete.pair_search(kind, g.subgraph(gi), Z[lo:hi], seed, gi * B + np.arange(B), rnd)
    return out


@pytest.mark.parametrize("name", list(PAIR_CASES))
@pytest.mark.parametrize("B", [1, 5, 64])
def test_pair_search_bit_exact(mqo, name, B):
    kind, g = PAIR_CASES[name]
    dg = mqo.DeviceGraph(g, DEV)
    Z0 = discrete.round_x(kind, _x(kind, g.n, B, 311 + B))
    if kind == "mis":
        Z0 = (arrays.uniform((g.n, B), 0.0, 1.0, 312 + B) < 0.25).astype(np.int8)  # infeasible starts too
    Z = torch.from_numpy(Z0).to(DEV)
    alt = mqo.pair_search(kind, dg, Z, 41, 7)
    ref = _pair_ref(kind, g, Z0, 41, 7, B)
    assert np.array_equal(Z.cpu().numpy(), ref)
    ls = np.empty_like(Z0)
    for gi in range(g.num_graphs):
        r0, r1 = g.vtx_offset[gi], g.vtx_offset[gi + 1]
        ls[r0:r1], _ = discrete.local_search(kind, g.subgraph(gi), Z0[r0:r1], 41, gi * B + np.arange(B), 7)
    moved = not np.array_equal(ls, ref)
    assert (alt > 0) == moved
    if name in ("mis_er300", "cut_reg4", "cut_weighted"):
        assert moved


@pytest.mark.parametrize("B", [65, 130])
def test_pair_search_dense_column_chunks(mqo, B):
    """Several 64-column chunks, the last one partial."""
    kind, g = PAIR_CASES["mis_dense"]
    dg = mqo.DeviceGraph(g, DEV)
    Z0 = (arrays.uniform((g.n, B), 0.0, 1.0, 313 + B) < 0.2).astype(np.int8)
    Z = torch.from_numpy(Z0).to(DEV)
    mqo.pair_search(kind, dg, Z, 42, 3)
    assert np.array_equal(Z.cpu().numpy(), _pair_ref(kind, g, Z0, 42, 3, B))


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("plan", ["persistent", "batched", "plain"])
def test_solve_final_search_bit_exact(mqo, kind, plan):
    g = CASES["er_batch"][1] if kind == "mis" else graphs.concat([graphs.random_regular(120, 4, 4903),
                                                                  CASES["cut_batch"][1]])
    kw = dict(batch=8, steps_per_round=30, rounds=3, alpha=0.05, rho=0.1, seed=43)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), plan=plan, final_search=True, **kw)
    assert out["plan"] == plan
    ref = solver.solve(kind, g, solver.Params(final_search=True, **kw))
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])
    assert np.array_equal(out["best_value"].cpu().numpy(), ref["best_value"])
    base = solver.solve(kind, g, solver.Params(**kw))
    assert np.all(ref["traj_best_value"] >= base["traj_best_value"])


# --------------------------------------------------------------------------
# the pmQO pool (Alg. 3 / Alg. 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("K,B,final", [(1, 4, False), (3, 8, True), (8, 8, False), (5, 33, True)])
def test_pool_solve_bit_exact(mqo, kind, K, B, final):
    g = CASES["er_batch"][1] if kind == "mis" else CASES["cut_batch"][1]
    kw = dict(batch=B, steps_per_round=25, rounds=4, alpha=0.05, rho=0.15, seed=61 + K, pool_k=K,
              final_search=final, reset_mode="flip" if K == 3 else "zero")
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), plan="batched", **kw)
    assert out["plan"] == "batched"
    ref = solver.solve(kind, g, solver.Params(**kw))
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])
    assert np.array_equal(out["pool_value"].cpu().numpy(), ref["pool_value"])
    assert np.array_equal(out["pool_x"].cpu().numpy(), ref["pool_x"])
    assert np.array_equal(out["best_value"].cpu().numpy(), ref["best_value"])
    assert np.array_equal(out["best_x"].cpu().numpy(), ref["best_x"])


def test_pool_rejected_where_not_offered(mqo):
    dg = mqo.DeviceGraph(CASES["reg3"][1], DEV)
    with pytest.raises(mqo.MqoError) as e:
        mqo.solve("maxcut", dg, batch=4, steps_per_round=4, pool_k=2, plan="plain")
    assert e.value.status == -5
    with pytest.raises(mqo.MqoError):
        mqo.solve("maxcut", dg, batch=4, steps_per_round=4, pool_k=5)


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("K,B,final,restart,budget", [(3, 8, False, 0, 0.0), (3, 8, True, 3, 0.0),
                                                     (8, 8, True, 0, 0.0), (5, 33, True, 2, 0.0),
                                                     (2, 6, True, 0, 1e-9)])
def test_pool_on_the_persistent_plan(mqo, kind, K, B, final, restart, budget):
    """pmQO on the persistent plan: a launch per round writes every
    trajectory's candidate; the pool, its best set and the pass searches run
    between launches; bases of the next round's resets come from the pool."""
    g = CASES["er_batch"][1] if kind == "mis" else CASES["cut_batch"][1]
    kw = dict(batch=B, steps_per_round=25, rounds=6, alpha=0.05, rho=0.15, seed=91 + K, pool_k=K,
              final_search=final, restart_every=restart)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), plan="persistent", time_budget_s=budget, **kw)
    assert out["plan"] == "persistent"
    ref = solver.solve(kind, g, solver.Params(rounds_run=1 if budget else None, **kw))
    for key in ("traj_best_value", "traj_best_x", "pool_value", "pool_x", "best_value", "best_x"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


# --------------------------------------------------------------------------
# the outer loop of Alg. 1-4: fresh starts every restart_every rounds
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("plan,pool", [("batched", 0), ("plain", 0), ("batched", 3)])
def test_restarts_bit_exact(mqo, kind, plan, pool):
    g = CASES["er_batch"][1] if kind == "mis" else CASES["cut_batch"][1]
    kw = dict(batch=6, steps_per_round=20, rounds=7, alpha=0.05, rho=0.15, seed=71, restart_every=3, pool_k=pool)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), plan=plan, **kw)
    assert out["plan"] == plan
    ref = solver.solve(kind, g, solver.Params(**kw))
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), ref["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), ref["traj_best_x"])
    assert np.array_equal(out["best_value"].cpu().numpy(), ref["best_value"])


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("plan,pool", [("batched", 0), ("plain", 0), ("batched", 3), ("batched", 6)])
def test_restarts_with_pass_searches_bit_exact(mqo, kind, plan, pool):
    # the pair search closes every pass of the outer loop (rounds 2, 5 and the
    # last, 6): Alg. 1 / 2 reset the next pass from the searched incumbents,
    # Alg. 3 searches I_sol, Alg. 4 every pool member into S_sol
    g = CASES["er_batch"][1] if kind == "mis" else CASES["cut_batch"][1]
    kw = dict(batch=6, steps_per_round=20, rounds=7, alpha=0.05, rho=0.15, seed=75, restart_every=3, pool_k=pool,
              final_search=True)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), plan=plan, **kw)
    assert out["plan"] == plan
    ref = solver.solve(kind, g, solver.Params(**kw))
    for key in ("traj_best_value", "traj_best_x", "best_value", "best_x") + (("pool_value", "pool_x") if pool else ()):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
    assert out["final_search_alternations"] >= 0


@pytest.mark.parametrize("kind", ["mis", "maxcut"])
@pytest.mark.parametrize("search,budget", [(False, 0.0), (True, 0.0), (True, 1e-9)])
def test_restarts_on_the_persistent_plan(mqo, kind, search, budget):
    """Fresh starts every R rounds on the persistent plan: one launch per
    pass of the outer loop, its start written into x0; with final_search the
    pair search closes each pass between launches; a budget that runs out
    before round 1 leaves round 0 and the search of its pass."""
    g = CASES["er_batch"][1] if kind == "mis" else CASES["cut_batch"][1]
    kw = dict(batch=6, steps_per_round=20, rounds=7, alpha=0.05, rho=0.15, seed=77, restart_every=3,
              final_search=search)
    out = mqo.solve(kind, mqo.DeviceGraph(g, DEV), plan="persistent", time_budget_s=budget, **kw)
    assert out["plan"] == "persistent"
    ref = solver.solve(kind, g, solver.Params(rounds_run=1 if budget else None, **kw))
    for key in ("traj_best_value", "traj_best_x", "best_value", "best_x"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
