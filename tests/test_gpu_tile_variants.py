"""The persistent plan's register-adjacency step loop (unweighted graphs of
degree <= 16, a single graph or a ragged batch of graphs) forced on
(tile_reg = 2) against the batched plan and the oracle, for every tile
shape it supports; shapes that do not fit are rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synth import graphs  # noqa: E402
from oracle import solver  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def mqo():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_06921_amd import mqo as m
    return m


CASES = {
    # degree 3 -> padded 4; degree <= 8; degree <= 16 over a ragged batch
    "reg3": ("maxcut", graphs.random_regular(300, 3, 21)),
    "reg7_mis": ("mis", graphs.random_regular(200, 7, 22)),
    "er_batch": ("mis", graphs.concat([graphs.erdos_renyi(150, 0.05, 23), graphs.cycle(17),
                                       graphs.erdos_renyi(90, 0.08, 24)])),
}

_oracle = {}


def _oracle_solve(name, kind, g, momentum, kw):
    key = (name, momentum)
    if key not in _oracle:
        _oracle[key] = solver.solve(kind, g, solver.Params(mu=momentum, **{k: v for k, v in kw.items()
                                                                          if k != "momentum"}))
    return _oracle[key]


def test_cases_fit_the_register_path():
    for kind, g in CASES.values():
        assert g.degrees().max() <= 16


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("T", [1, 2, 8, 64])
@pytest.mark.parametrize("threads", [256, 1024])
@pytest.mark.parametrize("momentum", [0.0, 0.4])
def test_register_adjacency_agrees(mqo, name, T, threads, momentum):
    kind, g = CASES[name]
    B = 23
    kw = dict(batch=B, steps_per_round=25, rounds=3, alpha=0.02, rho=0.1, seed=5, momentum=momentum)
    dg = mqo.DeviceGraph(g, DEV)
    dmax = g.degrees().max()
    rows_per_lane = 1 if dmax > 8 else (4 if threads <= 512 else 2)
    if max(np.diff(g.vtx_offset)) * T > rows_per_lane * threads:  # no register shape
        with pytest.raises(mqo.MqoError):
            mqo.solve(kind, dg, plan="persistent", tile_cols=T, tile_threads=threads, tile_reg=2, **kw)
        return
    out = mqo.solve(kind, dg, plan="persistent", tile_cols=T, tile_threads=threads, tile_reg=2, **kw)
    assert out["tile_reg_degree"] in (3, 4, 8, 16)
    ref = mqo.solve(kind, dg, plan="batched", **kw)
    assert torch.equal(out["traj_best_value"], ref["traj_best_value"])
    assert torch.equal(out["traj_best_x"], ref["traj_best_x"])
    o = _oracle_solve(name, kind, g, momentum, kw)
    assert np.array_equal(out["traj_best_value"].cpu().numpy(), o["traj_best_value"])
    assert np.array_equal(out["traj_best_x"].cpu().numpy(), o["traj_best_x"])
    assert np.array_equal(out["best_value"].cpu().numpy(), o["best_value"])


def test_register_adjacency_rejected_when_degree_too_high(mqo):
    g = graphs.star(40)
    dg = mqo.DeviceGraph(g, DEV)
    with pytest.raises(mqo.MqoError):
        mqo.solve("mis", dg, batch=4, steps_per_round=5, rounds=1, plan="persistent", tile_reg=2)


SB_CASES = {
    "er_dense": ("mis", graphs.concat([graphs.erdos_renyi(120, 0.2, 25), graphs.erdos_renyi(77, 0.3, 26)])),
    "cut_w": ("maxcut", graphs.concat([graphs.with_weights(graphs.erdos_renyi(100, 0.15, 27), 28),
                                       graphs.with_weights(graphs.cycle(40), 29)])),
}


@pytest.mark.parametrize("name", list(SB_CASES))
@pytest.mark.parametrize("T,vec,csr", [(32, 4, 1), (32, 4, 2), (16, 2, 1), (64, 4, 1), (8, 1, 2)])
@pytest.mark.parametrize("momentum,check", [(0.0, 0), (0.4, 7)])
def test_single_buffer_tile_agrees(mqo, name, T, vec, csr, momentum, check):
    """The single-buffered step (one iterate buffer in LDS, gathers into
    registers, then in place) forced on: bit-exact against the oracle,
    with weights, momentum and early exit."""
    kind, g = SB_CASES[name]
    B = 40
    kw = dict(batch=B, steps_per_round=25, rounds=3, alpha=0.02, rho=0.1, seed=6, momentum=momentum,
              check_every=check)
    dg = mqo.DeviceGraph(g, DEV)
    out = mqo.solve(kind, dg, plan="persistent", tile_cols=T, tile_vec=vec, tile_csr=csr, tile_reg=1, tile_sb=2,
                    **kw)
    assert out["tile_sb"] == 1 and out["tile_cols"] == T
    o = solver.solve(kind, g, solver.Params(batch=B, steps_per_round=25, rounds=3, alpha=0.02, rho=0.1, seed=6,
                                            mu=momentum, check_every=check))
    for key in ("traj_best_value", "traj_best_x", "best_value"):
        assert np.array_equal(out[key].cpu().numpy(), o[key]), key
    nnz_g = np.diff(g.row_ptr[g.vtx_offset])
    assert out["edge_updates"] == int((o["traj_steps"].reshape(g.num_graphs, -1) * nnz_g[:, None]).sum())


def test_graph_launch_order_and_row_order(mqo):
    """A batch of 16 graphs of unequal size (a multiple of 8, so the graphs
    are dealt to the XCDs' ranges in snake order, largest first) on the
    general step loop (rows walked in descending degree order), single- and
    double-buffered: bit-exact against the oracle and the batched plan."""
    rng = np.random.default_rng(71)
    gs = [graphs.erdos_renyi(int(n), float(p), 200 + i)
          for i, (n, p) in enumerate(zip(rng.integers(20, 90, 16), rng.uniform(0.05, 0.3, 16)))]
    g = graphs.concat(gs)
    assert g.num_graphs == 16
    dg = mqo.DeviceGraph(g, DEV)
    kw = dict(batch=16, steps_per_round=20, rounds=3, alpha=0.03, rho=0.1, seed=72)
    o = solver.solve("mis", g, solver.Params(**kw))
    ref = mqo.solve("mis", dg, plan="batched", **kw)
    for sb in (1, 2):
        out = mqo.solve("mis", dg, plan="persistent", tile_cols=8, tile_vec=4, tile_reg=1, tile_sb=sb, **kw)
        assert out["plan"] == "persistent" and out["tile_reg_degree"] == 0 and out["tile_sb"] == sb - 1
        for key in ("traj_best_value", "traj_best_x", "best_value", "best_x"):
            assert np.array_equal(out[key].cpu().numpy(), o[key]), key
            assert torch.equal(out[key], ref[key]), key
