"""Workload definitions (shapes, distributions, hyper-parameters, seeds).

c0  order-3 100^3, 10,000 uniform distinct nonzeros, planted J=R=4 model
    (entries N(0, 0.5^2)) + N(0, 0.01^2) noise; J=R=4, M=512, lr 0.01,
    lambda 1e-3, 5 alternating epochs. The parity workload.
c1  order-3 rating tensor 20,000 x 20,000 x 1,000, 10M nonzeros, Zipf(1.1)
    indices per mode, integer ratings 1..5 from a rounded, clamped planted
    J=R=16 model + N(0, 0.3^2) noise; J=R=16, M=65,536, FP32, 20 epochs,
    per-row mean steps; lr_A 0.02, lr_B 1.0 (the core matrices take one
    full-batch step per epoch), lambda 1e-3, N(0, 0.3^2) initial entries.
    From a 30-epoch trace of test RMSE over lr_A in {0.005 .. 0.03} and
    lr_B in {0.1 .. 3}: at 0.03 / 3.0 the FP32 curve itself rises and falls
    from epoch to epoch (the edge of stability) and the FP8 run drifts 11%
    away; at 0.02 / 1.0 all three contractions descend together. Stands in
    for the Netflix / Yahoo!Music rating tensors of Table 5.
c2  order-4 1,000,000 x 500,000 x 1,000 x 100, 100M nonzeros, Zipf(1.2),
    real values from a planted J=R=32 model + N(0, 0.1^2); M=262,144;
    lr_A = lr_B = 0.01 from 32-epoch runs on the full tensor (0.02 diverges
    after epoch 12; at 0.01 the test RMSE leaves the zero predictor's 1.046
    around epoch 20 and reaches 0.946 at epoch 32; at 0.005 it stays there).
c3  order-5 200,000 x 200,000 x 50,000 x 1,000 x 24, 200M nonzeros,
    Zipf(1.1), planted J=R=32 + N(0, 0.1^2); M=262,144; lr_A 0.003,
    lr_B 0.5 from 32-epoch runs on the full tensor: a factor step is stable
    only while lr_A |B d|^2 < 2 (single-sample steps on the tensor's outlier
    values), and |B d|^2 grows with B during training, so every larger pair
    tried (lr_A 0.005-0.01 with lr_B 0.2-2) diverged between epochs 14 and
    32; this one stays finite and still improving at epoch 32.
c4  differentiation instance: 30^3, 500 nonzeros, J=R=3.
90/10 train/test split everywhere. Seeds: data 1000+k, init 2000+k,
order 3000+k.
"""
from dataclasses import dataclass, replace


@dataclass(frozen=True)
class Workload:
    name: str
    dims: tuple
    nnz: int
    J: int
    R: int
    M: int
    epochs: int
    lr_A: float
    lr_B: float
    lam_A: float
    lam_B: float
    row_mean: bool
    index_dist: str = "uniform"    # "uniform" | "zipf"
    zipf_s: float = 1.1
    values: str = "real"           # "real" | "rating"
    rating_offset: float = 3.0
    noise_std: float = 0.01
    planted_rank: int = 4
    planted_a_std: float = 0.5
    planted_b_std: float = 0.5
    planted_scale: float = 1.0
    test_frac: float = 0.1
    init_dist: str = "normal"
    init_a_std: float = 0.5
    init_b_std: float = 0.5
    data_seed: int = 1000
    init_seed: int = 2000
    order_seed: int = 3000

    @property
    def order(self):
        return len(self.dims)

    @property
    def nnz_train(self):
        return self.nnz - int(round(self.nnz * self.test_frac))


CONFIGS = {
    "c0": Workload(
        name="c0-order3-100^3-10k-uniform-J4R4", dims=(100, 100, 100),
        nnz=10_000, J=4, R=4, M=512, epochs=5, lr_A=0.01, lr_B=0.01,
        lam_A=1e-3, lam_B=1e-3, row_mean=False, index_dist="uniform",
        noise_std=0.01, planted_rank=4, planted_a_std=0.5, planted_b_std=0.5,
        init_a_std=0.5, init_b_std=0.5, data_seed=1000, init_seed=2000,
        order_seed=3000),
    "c1": Workload(
        name="c1-order3-20000x20000x1000-10M-zipf1.1-rating-J16R16",
        dims=(20_000, 20_000, 1_000), nnz=10_000_000, J=16, R=16, M=65_536,
        epochs=20, lr_A=0.02, lr_B=1.0, lam_A=1e-3, lam_B=1e-3,
        row_mean=True, index_dist="zipf", zipf_s=1.1, values="rating",
        rating_offset=3.0, noise_std=0.3, planted_rank=16, planted_a_std=1.0,
        planted_b_std=0.25, planted_scale=0.25, init_dist="normal",
        init_a_std=0.3, init_b_std=0.3, data_seed=1001, init_seed=2001,
        order_seed=3001),
    "c2": Workload(
        name="c2-order4-1e6x5e5x1000x100-100M-zipf1.2-J32R32",
        dims=(1_000_000, 500_000, 1_000, 100), nnz=100_000_000, J=32, R=32,
        M=262_144, epochs=10, lr_A=0.01, lr_B=0.01, lam_A=1e-3, lam_B=1e-3,
        row_mean=True, index_dist="zipf", zipf_s=1.2, noise_std=0.1,
        planted_rank=32, planted_a_std=1.0, planted_b_std=32 ** -0.5,
        planted_scale=32 ** -0.5, init_a_std=0.3, init_b_std=0.3,
        data_seed=1002, init_seed=2002, order_seed=3002),
    "c3": Workload(
        name="c3-order5-2e5x2e5x5e4x1000x24-200M-zipf1.1-J32R32",
        dims=(200_000, 200_000, 50_000, 1_000, 24), nnz=200_000_000, J=32,
        R=32, M=262_144, epochs=10, lr_A=0.003, lr_B=0.5, lam_A=1e-3,
        lam_B=1e-3, row_mean=True, index_dist="zipf", zipf_s=1.1,
        noise_std=0.1, planted_rank=32, planted_a_std=1.0,
        planted_b_std=32 ** -0.5, planted_scale=32 ** -0.5, init_a_std=0.3,
        init_b_std=0.3, data_seed=1003, init_seed=2003, order_seed=3003),
    "c4": Workload(
        name="c4-fd-order3-30^3-500-J3R3", dims=(30, 30, 30), nnz=500, J=3,
        R=3, M=500, epochs=1, lr_A=0.01, lr_B=0.01, lam_A=1e-3, lam_B=1e-3,
        row_mean=False, index_dist="uniform", noise_std=0.01, planted_rank=3,
        test_frac=0.0, data_seed=1004, init_seed=2004, order_seed=3004),
}


# Order and rank sweep of the paper's synthetic study (Table 5, Fig. 2):
# I_n = 10,000 in every mode, |Omega| = 1e8, ratings 1..5 (from a planted
# model, uniform indices; the paper gives no value distribution), orders
# 3..10 at J = R = 16 (the paper's setting), and J = R = 32 at orders 3..5
# for the rank comparison. M = 65,536. Throughput workloads: the step sizes
# are not tuned for them.
for _n in range(3, 11):
    for _r in ((16, 32) if _n <= 5 else (16,)):
        CONFIGS[f"sweep-N{_n}-R{_r}"] = Workload(
            name=f"sweep-order{_n}-1e4^{_n}-100M-uniform-rating-J{_r}R{_r}",
            dims=(10_000,) * _n, nnz=100_000_000, J=_r, R=_r, M=65_536,
            epochs=5, lr_A=0.01, lr_B=0.1, lam_A=1e-3, lam_B=1e-3,
            row_mean=True, index_dist="uniform", values="rating",
            rating_offset=3.0, noise_std=0.3, planted_rank=_r,
            planted_a_std=1.0, planted_b_std=_r ** -0.5,
            planted_scale=_r ** -0.5, init_dist="normal",
            init_a_std=0.3, init_b_std=0.3, data_seed=1100 + 10 * _n + _r,
            init_seed=2100 + 10 * _n + _r, order_seed=3100 + 10 * _n + _r)


def get(key, **overrides):
    w = CONFIGS[key]
    return replace(w, **overrides) if overrides else w
