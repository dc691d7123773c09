"""Named synthetic workloads: graph recipe, seeds and run parameters.

Graph seed for workload k is ``1000*k + i`` (i = instance); the run seed
is ``graph seed + 10**6``.  Parameters the workload statements leave open
take the defaults documented next to each entry (step 0.01, gamma 2,
lambda 1e-3, 200-step rounds, rho 0.05, plain gradient ascent).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict

from . import graphs


@dataclasses.dataclass
class Workload:
    name: str
    problem: str  # "mis" or "maxcut"
    make_graph: Callable[[], graphs.Graph]
    batch: int
    steps_per_round: int
    rounds: int
    alpha: float
    seed: int
    gamma: float = 2.0
    lam: float = 1e-3
    rho: float = 0.05
    reset_mode: str = "zero"
    local_search: bool = True
    momentum: float = 0.0
    check_every: int = 0
    init_mode: str = "uniform"
    init_sigma: float = 0.0
    final_search: bool = False
    description: str = ""

    @property
    def steps(self) -> int:
        return self.steps_per_round * self.rounds


def _c1():
    return graphs.erdos_renyi(100, 0.1, 1000)


def _c2():
    return graphs.random_regular(2000, 3, 2000)


def _c3():
    return graphs.er_batch(128, 700, 800, 0.15, 3000)


def _c4_ba():
    return graphs.barabasi_albert(100_000, 4, 4000)


def _c4_reg():
    return graphs.random_regular(100_000, 5, 4001)


def _c5_er():
    n = 1_000_000
    return graphs.erdos_renyi(n, 10.0 / (n - 1), 5000)


def _c5_torus():
    return graphs.torus_pm1(1000, 5001)


def _paper_mis():
    return graphs.erdos_renyi(3000, 100.0 / 2999, 6000)


def _paper_maxcut():
    return graphs.erdos_renyi(1000, 100.0 / 999, 6001)


WORKLOADS: Dict[str, Workload] = {
    "er100_mis": Workload(
        "er100_mis", "mis", _c1, batch=1, steps_per_round=1000, rounds=1,
        alpha=0.01, seed=1000 + 10**6,
        description="ER G(100,0.1), MIS h with gamma=2, one trajectory, "
                    "1000 steps of 0.01, round at 0.5, repair + 1-flip search"),
    "reg3_maxcut": Workload(
        "reg3_maxcut", "maxcut", _c2, batch=256, steps_per_round=200, rounds=10,
        alpha=0.01, seed=2000 + 10**6, reset_mode="flip",
        description="random 3-regular n=2000, MaxCut f_B (lambda=1e-3), 256 restarts, "
                    "2000 steps in 10 rounds of 200, flip 5% of the incumbent's spins, "
                    "1-flip search, int64 cuts"),
    "er_batch_mis": Workload(
        "er_batch_mis", "mis", _c3, batch=512, steps_per_round=200, rounds=10,
        alpha=0.01, seed=3000 + 10**6,
        description="128 ER graphs, n uniform in [700,800], p=0.15, 512 trajectories each, "
                    "MIS h, 2000 steps in 10 rounds of 200, reset 5%, 1-flip search"),
    "ba100k_mis": Workload(
        "ba100k_mis", "mis", _c4_ba, batch=64, steps_per_round=20, rounds=1,
        alpha=0.01, seed=4000 + 10**6,
        description="Barabasi-Albert n=100000 m=4, MIS h, batch 64 (differentiation)"),
    "reg5_100k_maxcut": Workload(
        "reg5_100k_maxcut", "maxcut", _c4_reg, batch=64, steps_per_round=20, rounds=1,
        alpha=0.01, seed=4001 + 10**6,
        description="random 5-regular n=100000, MaxCut f_B, batch 64 (differentiation)"),
    "er1m_mis": Workload(
        "er1m_mis", "mis", _c5_er, batch=32, steps_per_round=200, rounds=25,
        alpha=0.01, seed=5000 + 10**6,
        description="ER n=1e6 mean degree 10, MIS h, 32 restarts, 5000 steps in 25 rounds"),
    "torus1m_maxcut": Workload(
        "torus1m_maxcut", "maxcut", _c5_torus, batch=32, steps_per_round=200, rounds=25,
        alpha=0.01, seed=5001 + 10**6,
        description="1000x1000 torus with +-1 weights, MaxCut f_B, 32 restarts, "
                    "5000 steps in 25 rounds"),
    # the paper's own hyper-parameters (its ER tables: alpha, momentum, rho,
    # T_gs) with its algorithm's pieces: degree-based start, momentum, PGA
    # until a fixed point (checked every 10 steps, at most 200 per round),
    # T_gs reset rounds, the pair search closing the run; 64 independent chains
    "er3000_paper_mis": Workload(
        "er3000_paper_mis", "mis", _paper_mis, batch=64, steps_per_round=200, rounds=61,
        alpha=0.8, seed=6000 + 10**6, rho=0.6, momentum=0.3, check_every=10, init_mode="degree",
        init_sigma=0.1, final_search=True,
        description="ER (n, d) = (3000, 100), MIS h, the paper's alpha 0.8, momentum 0.3, rho 0.6, "
                    "T_gs = 60, degree start, OneTwoSwap at the end, 64 chains"),
    "er1000_paper_maxcut": Workload(
        "er1000_paper_maxcut", "maxcut", _paper_maxcut, batch=64, steps_per_round=200, rounds=91,
        alpha=0.0025, seed=6001 + 10**6, rho=0.8, momentum=0.8, check_every=10, init_mode="degree",
        init_sigma=0.1, final_search=True,
        description="ER (n, d) = (1000, 100), MaxCut f_B, the paper's alpha 0.0025, momentum 0.8, rho 0.8, "
                    "T_gs = 90, degree start, OneTwoFlip at the end, 64 chains"),
}
