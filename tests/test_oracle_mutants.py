"""The oracle's pins catch plausible mistakes: each mutant below is a copy of
ft_oracle.c with one planted error (on the CPU, in a temporary build); at
least one pin check must fail for every mutant, while all pass on the
unmodified oracle."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.lib_path()), "ft_oracle.c")

MUTANTS = {
    "regulariser dropped":
        ("gr[j] += r * bd + lamA * a[j];", "gr[j] += r * bd;"),
    "residual sign flipped":
        ("double r = sample_xhat(N, R, c) - vals[s];\n        loss += 0.5 * r * r;\n        for (int n = 0; n < N; ++n) {\n            const double *a = A[n] + rows[n] * (int64_t)J[n];\n            double *gr",
         "double r = vals[s] - sample_xhat(N, R, c);\n        loss += 0.5 * r * r;\n        for (int n = 0; n < N; ++n) {\n            const double *a = A[n] + rows[n] * (int64_t)J[n];\n            double *gr"),
    "B read transposed in c":
        ("acc += a[j] * B[n][(int64_t)j * R + r];",
         "acc += a[j] * B[n][(int64_t)(r % J[n]) * R + (j % R)];"),
    "leave-one-out keeps own mode":
        ("if (k != n) p *= c[k * R + r];", "p *= c[k * R + r];"),
    "row mean ignored":
        ("double scale = row_mean ? 1.0 / (double)cnt[n][i] : 1.0;",
         "double scale = 1.0;"),
    "core gradient without residual":
        ("Grad[n][(int64_t)j * R + q] += r * a[j] * d[n * R + q];",
         "Grad[n][(int64_t)j * R + q] += a[j] * d[n * R + q];"),
    "core step not divided by |Omega|":
        ("B[n][e] -= lrB * (Grad[n][e] / (double)nnz + lamB * B[n][e]);",
         "B[n][e] -= lrB * (Grad[n][e] + lamB * B[n][e]);"),
    "factor step sign flipped":
        ("a[j] -= lrA * (gr[j] * scale);", "a[j] += lrA * (gr[j] * scale);"),
    "regulariser of Eq. (4) on mode 0 only":
        ("na += A[n][e] * A[n][e];", "na += n == 0 ? A[n][e] * A[n][e] : 0.0;"),
    "tail minibatch of the factor epoch dropped":
        ("for (int64_t first = 0; first < nnz; first += M, ++b) {",
         "for (int64_t first = 0; first + M <= nnz; first += M, ++b) {"),
    "per-minibatch core step divided by M instead of the slice size":
        ("B[n][e] -= lrB * (Grad[n][e] / (double)m + lamB * B[n][e]);",
         "B[n][e] -= lrB * (Grad[n][e] / (double)M + lamB * B[n][e]);"),
    "B held fixed across the per-minibatch core steps":
        ("loss += orc_core_grad(N, J, R, A, B, m, bidx, bvals, Grad);",
         "static double *Bs[ORC_MAX_ORDER];\n"
         "            if (first == 0)\n"
         "                for (int n = 0; n < N; ++n) {\n"
         "                    Bs[n] = malloc(sizeof(double) * J[n] * (size_t)R);\n"
         "                    memcpy(Bs[n], B[n], sizeof(double) * J[n] * (size_t)R);\n"
         "                }\n"
         "            loss += orc_core_grad(N, J, R, A, Bs, m, bidx, bvals, Grad);"),
    "A held fixed across the factor minibatches":
        ("double l = orc_factor_minibatch(N, dims, J, R, A, B, m, bidx, bvals,\n"
         "                                        lrA, lamA, row_mean, 1, NULL, NULL);",
         "static double *As[ORC_MAX_ORDER];\n"
         "        if (first == 0)\n"
         "            for (int n = 0; n < N; ++n) {\n"
         "                As[n] = malloc(sizeof(double) * dims[n] * J[n]);\n"
         "                memcpy(As[n], A[n], sizeof(double) * dims[n] * J[n]);\n"
         "            }\n"
         "        double l = orc_factor_minibatch(N, dims, J, R, As, B, m, bidx, bvals,\n"
         "                                        lrA, lamA, row_mean, 0, NULL, NULL);\n"
         "        {\n"
         "            double *Gd[ORC_MAX_ORDER]; int64_t *Kd[ORC_MAX_ORDER];\n"
         "            for (int n = 0; n < N; ++n) {\n"
         "                Gd[n] = calloc((size_t)(dims[n] * J[n]), sizeof(double));\n"
         "                Kd[n] = calloc((size_t)dims[n], sizeof(int64_t));\n"
         "            }\n"
         "            orc_factor_minibatch(N, dims, J, R, As, B, m, bidx, bvals,\n"
         "                                 lrA, lamA, row_mean, 0, Gd, Kd);\n"
         "            for (int n = 0; n < N; ++n)\n"
         "                for (int64_t i = 0; i < dims[n]; ++i)\n"
         "                    for (int32_t j = 0; j < J[n]; ++j)\n"
         "                        if (Kd[n][i]) A[n][i * J[n] + j] -= lrA * Gd[n][i * J[n] + j]\n"
         "                            / (row_mean ? (double)Kd[n][i] : 1.0);\n"
         "        }"),
    "Gauss-Seidel rows within the minibatch":
        ("gr[j] += r * bd + lamA * a[j];",
         "gr[j] += r * bd + lamA * a[j];\n                if (apply) ((double *)a)[j] -= lrA * (r * bd + lamA * a[j]);"),
}


def run_pins():
    """Pin checks from test_oracle_pins; returns the names that fail."""
    failed = []
    checks = {
        "P1": lambda: pins.test_p1_dense_tucker_brute_force(
            oracle, (4, 5, 6), (2, 3, 4), 3),
        "P2": lambda: pins.test_p2_factor_and_core_gradients_vs_autograd(
            oracle, (6, 7, 5), (2, 3, 4), 3, 60, 1),
        "P4s": lambda: pins.test_p4_residual_free_decay(oracle, False),
        "P4m": lambda: pins.test_p4_residual_free_decay(oracle, True),
        "P5": lambda: pins.test_p5_jacobi_minibatch_matches_autograd_step(
            oracle),
        "P6": lambda: pins.test_p6_matrix_factorisation_special_case(oracle),
        "loss": lambda: pins.test_loss_and_residual_stats_definitions(oracle),
        "core": lambda: pins.test_core_epoch_step_matches_autograd(oracle),
        "P8": lambda: pins.test_p8_core_epoch_order_invariance(oracle),
        "split-sum": lambda:
            pins.test_factor_epoch_splits_into_minibatches_with_tail(
                oracle, False),
        "split-mean": lambda:
            pins.test_factor_epoch_splits_into_minibatches_with_tail(
                oracle, True),
        "core-split": lambda:
            pins.test_core_epoch_per_minibatch_steps_with_tail(oracle),
    }
    for name, fn in checks.items():
        try:
            fn()
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(name)
    return failed


@pytest.fixture(scope="module")
def tmpdir_mod():
    with tempfile.TemporaryDirectory() as d:
        yield d


def test_unmodified_oracle_passes_every_check():
    oracle.use_library(None)
    assert run_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmpdir_mod):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mutant = os.path.join(tmpdir_mod, f"m{abs(hash(name))}.c")
    lib = mutant[:-2] + ".so"
    open(mutant, "w").write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                           "-ffp-contract=off", mutant, "-o", lib, "-lm"])
    try:
        oracle.use_library(lib)
        with np.errstate(all="ignore"):
            failed = run_pins()
    finally:
        oracle.use_library(None)
    assert failed, f"no pin catches: {name}"
