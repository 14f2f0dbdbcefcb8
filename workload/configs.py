"""Named model and workload configurations.

Sizes are those of the benchmark workloads of this project (the paper itself gives no
architecture: Sec. 2.2 defers it to earlier work). ``ModelCfg`` mirrors the C struct
``fmd_model_config`` of ``include/fmd.h``.
"""

from dataclasses import dataclass, field, replace

F_FEAT = 9          # [ln(pT/10 GeV), eta, phi, onehot5(class), charge]
T_EMBED = 32        # sinusoidal time-embedding width
MLP_RATIO = 4

EULER, RK4, MIDPOINT = 0, 1, 2
FP32, BF16, FP8 = 0, 1, 2


@dataclass(frozen=True)
class ModelCfg:
    d_model: int
    n_blocks: int
    n_heads: int
    mlp_ratio: int = MLP_RATIO
    t_embed_dim: int = T_EMBED
    f_truth: int = F_FEAT
    f_reco: int = F_FEAT
    n_max: int = 1000
    precision: int = FP32

    @property
    def d_head(self) -> int:
        return self.d_model // self.n_heads

    def with_precision(self, precision: int) -> "ModelCfg":
        return replace(self, precision=precision)


@dataclass(frozen=True)
class Schedule:
    scheme: int = EULER
    n_steps: int = 50        # default number of integration steps (App. C, generator block)
    t0: float = 0.0
    t1: float = 1.0

    @property
    def stages(self) -> int:
        return {EULER: 1, MIDPOINT: 2}.get(self.scheme, 4)

    @property
    def evals(self) -> int:
        return self.stages * self.n_steps


@dataclass(frozen=True)
class Workload:
    name: str
    n_events: int
    mult: tuple              # ("uniform", lo, hi) or ("lognormal", median, sigma, lo, hi)
    model: ModelCfg
    schedule: Schedule
    truth_seed: int = 2
    weight_seed: int = 0
    noise_seed: int = 1
    parity_events: int = 0   # size of the leading subset compared against the oracle
    extra: dict = field(default_factory=dict)


SMALL_MODEL = ModelCfg(d_model=64, n_blocks=2, n_heads=4, n_max=64)
BASE_MODEL = ModelCfg(d_model=256, n_blocks=6, n_heads=8, n_max=1000)

# 64 events, N ~ U{8..48}, d=64, 2 blocks, 4 heads, Euler 20, all events checked.
SMALL = Workload("small-fp32-euler20", 64, ("uniform", 8, 48), SMALL_MODEL,
                 Schedule(EULER, 20), parity_events=64)
# 4096 events, N ~ U{20..200}, d=256, 6 blocks, 8 heads, RK4 16; oracle on 128 events.
BASE_FP32 = Workload("base-fp32-rk4x16", 4096, ("uniform", 20, 200), BASE_MODEL,
                     Schedule(RK4, 16), parity_events=128)
# The same events, net and schedule with BF16 GEMM/attention inputs; oracle on 256 events.
BASE_BF16 = Workload("base-bf16-rk4x16", 4096, ("uniform", 20, 200), BASE_MODEL.with_precision(BF16),
                     Schedule(RK4, 16), parity_events=256)
# 65536 events, heavy-tailed multiplicity (log-normal, median 60, sigma 0.8, clipped [1,1000]).
BATCH_BF16 = Workload("batch-bf16-rk4x16", 65536, ("lognormal", 60.0, 0.8, 1, 1000),
                      BASE_MODEL.with_precision(BF16), Schedule(RK4, 16))
# Serving: Poisson arrivals, 1..512 events per request, multiplicities as BATCH_BF16.
SERVE_BF16 = Workload("serve-bf16", 0, ("lognormal", 60.0, 0.8, 1, 1000),
                      BASE_MODEL.with_precision(BF16), Schedule(RK4, 16),
                      extra={"rates": (1000, 2000, 5000, 10000, 20000, 50000),
                             "events_per_request": (1, 512), "hbm_budget_bytes": 64 << 30,
                             "arrival_seed": 3})

ALL = {w.name: w for w in (SMALL, BASE_FP32, BASE_BF16, BATCH_BF16, SERVE_BF16)}
