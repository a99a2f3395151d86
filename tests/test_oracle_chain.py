"""Pins of the sequential-chain shape of the hierarchical multinomial
(tree = 1; Sec. 6 draws the multinomial "hierarchically" from binomials
without fixing the shape; the balanced binary tree is the default).

Node i draws bin i's facets out of those that reach it with p_i / S_i, S_i
the suffix sum of the probabilities.  Pinned by: expected counts N_P p_k;
a single facet lands in bin k with probability exactly p_k (each node's
dual gate at N = 1 is an exact Bernoulli draw, so the chain is an exact
categorical draw); K = 2 equals the balanced tree; a zero-probability
suffix sends nothing past it; conservation for integer counts that never
pass through a real Gaussian count below 2.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from tests.test_oracle_shade import env_products, flat_gbuf, luts
import synth

P8 = np.array([0.0118, 0.1343, 0.2137, 0.3402, 0.2175, 0.0706, 0.01175, 1.87e-5])
P8 = P8 / P8.sum()


def test_single_facet_is_an_exact_categorical_draw():
    n = 40000
    hits = np.zeros(8)
    for a in range(n):
        M, codes, fl = oracle.multinomial(0, 1.0, P8, 3, 5, 0, a, 17, tree=1)
        assert M.sum() == 1.0 and np.all((M == 0) | (M == 1)), M
        hits += M
    expect = n * P8
    sel = expect > 5
    chi2 = ((hits[sel] - expect[sel]) ** 2 / expect[sel]).sum()
    assert chi2 < stats.chi2.ppf(0.999, sel.sum() - 1), (hits, expect)


def test_two_bins_equal_the_balanced_tree():
    p = np.array([0.3, 0.7])
    for a in range(500):
        for NP in (0.4, 1.0, 1.7, 2.0, 37.5, 1e6):
            A = oracle.multinomial(0, NP, p, 1, 2, 3, a, 4, tree=0)
            B = oracle.multinomial(0, NP, p, 1, 2, 3, a, 4, tree=1)
            assert np.array_equal(A[0], B[0]) and np.array_equal(A[1], B[1]) and A[2] == B[2]


def test_zero_suffix_sends_nothing_on():
    """p = (0.5, 0.5, 0, 0): the chain's node 1 sees S_1 = 0.5 and p = 1:
    every facet that reaches it stays in bin 1; nodes 2, 3 see nothing."""
    p = np.array([0.5, 0.5, 0.0, 0.0])
    for a in range(300):
        M, codes, fl = oracle.multinomial(0, 1000.0, p, 1, 2, 3, a, 4, tree=1)
        assert M[2] == 0.0 and M[3] == 0.0
        assert M[0] + M[1] == pytest.approx(1000.0, rel=1e-12)


def test_chain_expected_counts_follow_probabilities():
    """Mean chain counts over independent lattice vertices -> N_P p_k, on a
    shaded frame (probabilities from the filtered map)."""
    R, K, M = 32, 8, 6
    env = synth.make_env(R, 1)
    levels, ind, rgb = env_products(env, K, M)
    S_lut, E_lut = luts()
    rng = np.random.default_rng(2)
    P = 6000
    NP = 800.0
    v = np.array([0.3, 0.5, 0.81]); v /= np.linalg.norm(v)
    n = np.array([0.0, 0.2, 1.0]); n /= np.linalg.norm(n)
    g = flat_gbuf(P, n, v, 1e-4, 0.2, NP / 1e-4, rng)
    out = oracle.shade(g, ind, rgb, levels, S_lut, E_lut, R, K, M, seed=9, tree=1)
    base = oracle.shade(g, ind, rgb, levels, S_lut, E_lut, R, K, M, seed=9, tree=0)
    np.testing.assert_array_equal(out["probs"], base["probs"])
    p = out["probs"][0]
    Np = float(np.float32(1e-4)) * float(np.float32(NP / 1e-4))
    counts = out["counts"][:, 0, :]
    dev = np.abs(counts.sum(1) - Np)
    assert np.mean(dev < 1e-9) > 0.5 and dev.max() < K
    mean = counts.mean(0)
    sd = np.sqrt(Np * p * (1 - p) / P)
    assert np.all(np.abs(mean - Np * p) <= 4 * sd + 3.0), (mean, Np * p)
    # another shape, another draw: the chain is not the tree in disguise
    assert not np.array_equal(out["counts"], base["counts"])
    assert out["flags"].mean() < 5e-3


def test_chain_counts_for_large_N_are_gaussian_per_node():
    """N_P = 1e6: node 0 is a Gaussian draw of mean 1 + (N-2) p_0 and the
    remainder is N - n exactly (no gate passes at these N p)."""
    p = np.array([0.25, 0.25, 0.25, 0.25])
    firsts = []
    for a in range(3000):
        M, codes, fl = oracle.multinomial(0, 1e6, p, 7, 1, 2, a, 9, tree=1)
        assert np.all(codes == 16)
        assert M.sum() == pytest.approx(1e6, rel=1e-12)
        firsts.append(M[0])
    firsts = np.array(firsts)
    mu, sd = 1 + (1e6 - 2) * 0.25, np.sqrt((1e6 - 2) * 0.25 * 0.75)
    assert abs(firsts.mean() - mu) < 4 * sd / np.sqrt(len(firsts))
    assert firsts.std() == pytest.approx(sd, rel=0.06)
