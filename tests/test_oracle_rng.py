"""Pins of the oracle's seeded start vector (oracle/rng.py): Philox4x64-10.

Pinned against the generator's published known-answer block (counter 0, key 0,
from the Random123 distribution of Salmon et al., SC 2011), against numpy's own
Philox bit generator (an independent implementation whose counter is advanced
before each block), and against the moments of U(-1, 1).
"""
import numpy as np

from oracle import rng


def test_known_answer_block():
    out = rng.philox4x64_10(np.zeros((1, 4), np.uint64), (0, 0))[0]
    assert [int(v) for v in out] == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC,
                                     0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_stream_equals_numpy_philox():
    for seed in (0, 1, 105, 2**32 + 3, 2**63 + 5, 2**64 - 1):
        words = rng.philox_words(4099, seed)
        ref = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64)).random_raw(4099)
        assert np.array_equal(words, ref), seed


def test_high_counter_words_equal_numpy():
    # a counter whose low word carries: numpy's block after counter c is block c + 1
    c = np.array([2**64 - 1, 5, 0, 0], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([9, 0], dtype=np.uint64), counter=c)
    ref = bg.random_raw(4)
    out = rng.philox4x64_10(np.array([[0, 6, 0, 0]], np.uint64), (9, 0))[0]
    assert np.array_equal(out, ref)


def test_uniform_pm1_mapping_and_moments():
    n = 1 << 20
    u = rng.uniform_pm1(n, 0)
    w = rng.philox_words(n, 0)
    # the mapping is exact: 2 k 2^-53 - 1 with k = w >> 11
    k = (w >> np.uint64(11)).astype(np.int64)
    assert np.array_equal(u, (k - 2**52) * 2.0**-52)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 5 * np.sqrt(1 / 3 / n)
    assert abs(u.var() - 1 / 3) < 5 * np.sqrt(4 / 45 / n)
    # different seeds give unrelated vectors
    assert abs(np.corrcoef(u[:4096], rng.uniform_pm1(4096, 1))[0, 1]) < 0.1


def test_oracle_solve_without_v0_uses_the_seeded_vector():
    from oracle import gmres
    from paper_1907_00072_amd import workloads as W
    P = W.config(1, N=24)
    A = P.A.to_scipy()
    for seed in (0, 3):
        x0, s0 = gmres.pp_gmres(A, P.b, 20, 1e-10, d=5, v0_seed=seed)
        x1, s1 = gmres.pp_gmres(A, P.b, 20, 1e-10, d=5, v0=rng.uniform_pm1(P.A.n, seed))
        assert s0.iters == s1.iters and np.array_equal(x0, x1)


def test_seeded_vector_on_the_section5_laplacian():
    # Section V: a random U(-1, 1) start vector gives a good polynomial for the
    # 201 x 201 Laplacian (alpha p(alpha) near 1 on the bulk of the spectrum)
    # and GMRES(50) with 6 roots converges in about 148 iterations
    from oracle import gmres
    from paper_1907_00072_amd import workloads as W
    A = W.laplacian5(201).to_scipy()
    b = np.ones(A.shape[0])
    x, st = gmres.pp_gmres(A, b, 50, 1e-8, d=6, v0_seed=0, max_iters=400)
    assert st.converged and 145 <= st.iters <= 152, st.iters
    al = np.linspace(0.5, 8.0, 20001)
    vals = 1.0 - np.prod([1.0 - al / t for t in st.roots], axis=0).real
    assert vals.min() >= 0.8 and vals.max() <= 1.2
