"""CPU checks of the seeded input generators against their stated recipes
(structure, value distributions, determinism, the batched order mix).  The
same generators feed the oracle, the GPU tests and bench.py."""
import numpy as np
import pytest

from paper_1710_08538_amd import inputs


@pytest.mark.parametrize("n", [1, 7, 64])
def test_random_pencil_recipe(n):
    A, B = inputs.random_pencil(n, seed=11)
    assert A.shape == B.shape == (n, n)
    assert A.flags.f_contiguous and B.flags.f_contiguous
    assert np.count_nonzero(np.tril(B, -1)) == 0  # upper triangular
    # B is the R factor of a Gaussian matrix drawn right after A: R^T R = G^T G
    rng = np.random.default_rng(11)
    A2 = rng.standard_normal((n, n))
    G = rng.standard_normal((n, n))
    np.testing.assert_array_equal(A, A2)
    np.testing.assert_allclose(B.T @ B, G.T @ G, rtol=0, atol=1e-10 * max(n, 1))


def test_random_pencil_is_deterministic_per_seed():
    a = inputs.random_pencil(20, seed=5)
    b = inputs.random_pencil(20, seed=5)
    c = inputs.random_pencil(20, seed=6)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], c[0])


def test_illcond_pencil_recipe():
    n = 400
    A, B = inputs.illcond_pencil(n, seed=2)
    assert np.count_nonzero(np.tril(B, -1)) == 0
    d = np.diag(B)
    mags = np.log10(np.abs(d))
    # diagonal magnitudes log-uniform in [1e-8, 1], random signs
    assert mags.min() >= -8.0 and mags.max() <= 0.0
    assert abs(mags.mean() + 4.0) < 0.4 and abs(mags.std() - 8.0 / np.sqrt(12.0)) < 0.3
    assert 0.4 < np.mean(d > 0) < 0.6
    # strictly upper entries and A: iid N(0, 1)
    up = B[np.triu_indices(n, 1)]
    assert abs(up.mean()) < 0.02 and abs(up.std() - 1.0) < 0.02
    assert abs(A.mean()) < 0.02 and abs(A.std() - 1.0) < 0.02


def test_batched_workload_mix():
    sizes = inputs.batch_sizes(2048, seed=4)
    assert len(sizes) == 2048 and sizes.min() >= 32 and sizes.max() <= 512
    np.testing.assert_array_equal(sizes, inputs.batch_sizes(2048, seed=4))
    assert abs(sizes.mean() - 272.0) < 8.0  # uniform on 32..512
    # pencil i comes from child seed i, independent of the other pencils
    P = inputs.batch_pencils(6, seed=4)
    s6 = inputs.batch_sizes(6, seed=4)
    for i in (0, 5):
        A, B = inputs.batch_pencil(i, s6[i], 6, seed=4)
        assert A.shape[0] == s6[i]
        assert np.array_equal(A, P[i][0]) and np.array_equal(B, P[i][1])


def test_named_workloads():
    A, B = inputs.workload("n256")
    A0, B0 = inputs.random_pencil(256, seed=0)
    assert np.array_equal(A, A0) and np.array_equal(B, B0)
    # the order override keeps the generator and seed
    A, B = inputs.workload("n16384", n=50)
    A1, B1 = inputs.illcond_pencil(50, seed=2)
    assert np.array_equal(A, A1) and np.array_equal(B, B1)
    assert inputs.WORKLOADS["n4096"] == ("random", 4096, 1)
    assert inputs.WORKLOADS["n16384"] == ("illcond", 16384, 2)
