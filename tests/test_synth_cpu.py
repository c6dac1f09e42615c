"""The input generators' C kernels against their plain numpy definitions:
the Zipf inverse-CDF lookup (searchsorted), first-occurrence duplicate
removal (np.unique), and the planted tensor's values."""
import numpy as np

import synth
from synth import gen


def test_zipf_lookup_equals_searchsorted():
    rng = np.random.Generator(np.random.PCG64(5))
    for I, s in ((1, 1.1), (24, 1.1), (1000, 1.2), (50_000, 1.1)):
        z = gen._Zipf(rng, I, s)
        u = rng.random(200_000)
        # edges and the values right at the cdf's steps
        u[:I] = z.cdf[:200_000][:I]
        u[I:2 * I] = np.nextafter(z.cdf[:I], 0.0)
        u[-1] = 0.0
        k = np.minimum(np.searchsorted(z.cdf, u, side="right"), I - 1)
        want = z.label[k]
        got = np.empty_like(want)
        lib = gen._load()
        assert lib.syn_zipf_lookup(gen._p(z.cdf), I, gen._p(z.label),
                                   gen._p(u), u.size, gen._p(got)) == 0
        np.testing.assert_array_equal(got, want)


def test_first_distinct_equals_unique_first_index():
    rng = np.random.Generator(np.random.PCG64(9))
    for N, hi, n in ((1, 50, 1000), (3, 7, 5000), (5, 4, 20_000),
                     (2, 100_000, 300_000)):
        idx = rng.integers(0, hi, size=(N, n), dtype=np.int32)
        got = gen._first_distinct(idx, [hi] * N)
        _, first = np.unique(idx.T, axis=0, return_index=True)
        np.testing.assert_array_equal(got, np.sort(first))


def test_planted_values_definition():
    rng = np.random.Generator(np.random.PCG64(3))
    dims = (30, 20, 10, 5)
    idx = np.stack([rng.integers(0, d, size=500, dtype=np.int32)
                    for d in dims])
    got = synth.planted_values(11, dims, idx, 3, 4, 1.0, 0.5, scale=0.7)
    r = np.random.Generator(np.random.PCG64(11))
    U = []
    for d in dims:
        P = r.normal(0.0, 1.0, size=(d, 3))
        Q = r.normal(0.0, 0.5, size=(3, 4))
        U.append(P @ Q)
    want = np.zeros(500)
    for s in range(500):
        want[s] = 0.7 * sum(np.prod([U[n][idx[n, s], q] for n in range(4)])
                            for q in range(4))
    np.testing.assert_allclose(got, want, rtol=1e-13)


def test_split_is_disjoint_and_complete():
    w = synth.get("c0", nnz=5000, dims=(40, 40, 40))
    T = synth.make_tensor(w)
    assert T.train_idx.shape[1] == 4500 and T.test_idx.shape[1] == 500
    keys = {tuple(c) for c in T.train_idx.T} | {tuple(c) for c in T.test_idx.T}
    assert len(keys) == 5000
