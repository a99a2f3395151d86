"""Pins of the oracle's sampling pieces against what the paper and mathematics fix.

Covers Sec. 6 (dual-gated Gaussian, Alg. "Dual-gated Gaussian", Fig.
"gatingdiagram", paragraph "Numeric Gating Issues", Fig. "smallp"), App. B,
the inverse normal CDF (AS 241) and the per-footprint hash.
"""
import math
import os

import numpy as np
import pytest
from scipy import special, stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# exact float32 grid of xi1 values covering (0,1)
XI_BITS = 16
XI = ((np.arange(2 ** XI_BITS) + 0.5) / 2 ** XI_BITS).astype(np.float32)


def outcome_distribution(N, p, xi2=0.5):
    """Empirical outcome frequencies of the oracle's sampler over a uniform xi1 grid."""
    out = {}
    for x in XI:
        n, nb, _ = oracle.dual_gated(N, p, float(x), xi2)
        key = (n, nb)
        out[key] = out.get(key, 0) + 1
    return {k: v / len(XI) for k, v in out.items()}


def load_diagram():
    rows = []
    with open(os.path.join(GOLDEN, "gatingdiagram_outcomes.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            regime, outcome, prob = [c.strip() for c in line.split("|")]
            rows.append((regime, outcome, prob))
    return rows


def eval_prob(expr, p, f, N=None):
    env = {"p1": p, "p2": 1.0 - p, "f": f, "N": N}
    return eval(expr.replace("^", "**"), {"__builtins__": {}}, env)


@pytest.mark.parametrize("p", [0.07, 0.3, 0.5, 0.81])
@pytest.mark.parametrize("N", [0.0, 1.0, 2.0, 0.25, 0.6, 1.3, 1.75])
def test_small_N_outcomes_match_gating_diagram(N, p):
    """N in {0,1,2}: exactly binomial; fractional N: the figure's interpolated table."""
    rows = load_diagram()
    if N in (0.0, 1.0, 2.0):
        regime = "N=%d" % int(N)
    elif N < 1:
        regime = "0<N<1"
    else:
        regime = "1<N<2"
    f = N - math.floor(N)
    expected = {}
    for reg, outcome, prob in rows:
        if reg != regime:
            continue
        key = tuple(float(v) for v in outcome.strip("()").split(","))
        expected[key] = eval_prob(prob, p, f)
    got = outcome_distribution(N, p)
    tol = 3.0 / len(XI)
    for key, prob in expected.items():
        assert abs(got.get(key, 0.0) - prob) <= tol, (N, p, key, got, expected)
    assert abs(sum(got.get(k, 0.0) for k in expected) - 1.0) <= tol
    if N in (0.0, 1.0, 2.0):  # cross-check with the binomial pmf itself
        for k in range(int(N) + 1):
            assert abs(got.get((float(k), float(N - k)), 0.0) - stats.binom.pmf(k, int(N), p)) <= tol


@pytest.mark.parametrize("N,p", [(3.0, 0.3), (7.5, 0.6), (40.0, 0.05), (1e4, 0.999), (123.25, 0.5)])
def test_large_N_cases(N, p):
    """N > 2: all-positive with p^N, all-negative with (1-p)^N, else Gaussian in
    [1, N-1]; n + nbar = N (no dithering above 2)."""
    got_allpos = got_allneg = got_gauss = 0
    for x in XI[::4]:
        n, nb, code = oracle.dual_gated(N, p, float(x), 0.37)
        assert abs((n + nb) - N) <= 4 * np.spacing(N), (n, nb, N)
        if n == N:
            got_allpos += 1
        elif nb == N:
            got_allneg += 1
        else:
            got_gauss += 1
            assert 1.0 <= n <= N - 1.0
            assert code & 16
    m = len(XI[::4])
    tol = 3.0 / m + 1e-4  # the all-negative probability carries the biased-power error
    assert abs(got_allpos / m - p ** N) <= tol
    assert abs(got_allneg / m - (1 - p) ** N) <= tol


def test_gaussian_branch_moments():
    """Gaussian branch: mean 1 + (N-2)p and variance (N-2)p(1-p) before clamping,
    i.e. one known positive and one known negative sample (Sec. 6)."""
    N, p = 5000.0, 0.3
    # xi1 in the middle of (P(n=N)+P(n=1), 1-P(nb=N)-P(nb=1)) selects the Gaussian
    xs = (np.arange(4096) + 0.5) / 4096
    vals = np.array([oracle.dual_gated(N, p, 0.5, float(np.float32(x)))[0] for x in xs])
    mu = 1 + (N - 2) * p
    sd = math.sqrt((N - 2) * p * (1 - p))
    assert abs(vals.mean() - mu) < 0.02 * sd
    assert abs(vals.std() - sd) < 0.02 * sd


def test_dual_gated_mean_bias_bound():
    """Exact expectation of the sampler (xi1 grid x xi2 grid) versus N p.  For
    N > 2 the two gates fix one positive and one negative sample; the mean
    deviates from N p by at most |1 - 2p| facets (before clamping)."""
    xs2 = ((np.arange(32) + 0.5) / 32).astype(np.float32)  # symmetric about 1/2
    for N, p in [(3.0, 0.2), (10.0, 0.5), (25.0, 0.1), (64.0, 0.9)]:
        tot = 0.0
        for x1 in XI[::64]:
            for x2 in xs2:
                tot += oracle.dual_gated(N, p, float(x1), float(x2))[0]
        mean = tot / (len(XI[::64]) * len(xs2))
        assert abs(mean - N * p) <= abs(1 - 2 * p) + 0.05 + 3 * math.sqrt(N * p * (1 - p)) / 64, (N, p, mean)


def test_appendix_b_single_gating_probability():
    """App. B: min(N p, 1-(1-p)^N) equals N p for N <= 1 and 1-(1-p)^N for N >= 1;
    the dual-gated sampler's P(n >= 1) for N <= 1 is N p (consistent)."""
    Ns = np.concatenate([np.linspace(0, 1, 41), np.linspace(1, 8, 57)])
    ps = np.linspace(0, 1, 41)
    for N in Ns:
        for p in ps:
            any_hit = 1 - (1 - p) ** N
            m = min(N * p, any_hit)
            if N <= 1:
                assert m == pytest.approx(N * p, abs=1e-12)
            else:
                assert m == pytest.approx(any_hit, abs=1e-12)
    for N in [0.2, 0.5, 0.9, 1.0]:
        for p in [0.1, 0.5, 0.8]:
            P = oracle.gate_probs(N, p)
            assert float(P[0]) + float(P[1]) == pytest.approx(N * p, rel=1e-6)


def _read_numeric_constants():
    vals = {}
    with open(os.path.join(GOLDEN, "numeric_gating.txt")) as f:
        for line in f:
            if line.startswith("#") or "=" not in line:
                continue
            k, v = [c.strip() for c in line.split("=")]
            vals[k] = [float(x) for x in v.split()]
    return vals


def test_naive_fp32_power_fails_below_threshold():
    """Sec. 6: in FP32, 1 - p rounds to 1 for p below 10^-7.525 (= 2^-25), so a
    naive (1-p)^N evaluates to 1 although the true value tends to 0."""
    c = _read_numeric_constants()
    thr = 10.0 ** c["naive_failure_p_log10"][0]
    assert thr == pytest.approx(2.0 ** -25, rel=2e-3)
    for p in [10 ** -7.6, 10 ** -8, 10 ** -10]:
        one = np.float32(1) - np.float32(p)
        assert one == np.float32(1)
        N = np.float32(10.0 / p)
        assert np.power(one, N) == np.float32(1)  # wrong; true value ~ e^-10
    for p in [10 ** -7.4, 10 ** -7]:
        assert np.float32(1) - np.float32(p) != np.float32(1)


def test_biased_power_error_map():
    """Fig. "smallp": with c = max(1, eps/p), eps = 10^-3.54, the float32
    evaluation of (1-cp)^(N/c) stays within ~1e-4 of (1-p)^N over
    (N, p) in [1, 1e16] x [1e-16, 1]; the oracle's gating uses this form."""
    c = _read_numeric_constants()
    assert 10.0 ** c["eps_log10"][0] == pytest.approx(2.8840315031266055e-04, rel=1e-12)
    worst = 0.0
    for lN in np.linspace(0.31, 16, 64):  # N >= 2 so that clamp(N-1) = 1
        for lp in np.linspace(-16, 0, 64):
            N, p = 10.0 ** lN, 10.0 ** lp
            Nf, pf = float(np.float32(N)), float(np.float32(p))
            got = float(oracle.gate_probs(Nf, pf)[2])
            exact = math.exp(Nf * math.log1p(-pf)) if pf < 1 else 0.0
            worst = max(worst, abs(got - exact))
    assert worst <= c["biased_error_scale"][0], worst


def test_ppnd16_matches_library_inverse_normal():
    ps = np.concatenate([10.0 ** -np.arange(1, 300, 7.0), np.linspace(0.001, 0.999, 997),
                         1 - 10.0 ** -np.arange(1, 16, 0.5)])
    for p in ps:
        a = oracle.ppnd16(float(p))
        b = float(special.ndtri(p))
        assert abs(a - b) <= 4e-15 * max(1.0, abs(b)), (p, a, b)


def test_hash_uniformity_and_exactness():
    """xi = ((h >> 9) + 1/2) 2^-23 is an exact float in (0,1); chi^2 uniformity of
    xi1, xi2 over consecutive lattice vertices and nodes."""
    vals1, vals2 = [], []
    for a in range(64):
        for node in range(16):
            x1, x2 = oracle.hash_xi(1, 2, -7, a, a * 3 + 1, node)
            vals1.append(x1)
            vals2.append(x2)
    for vals in (np.array(vals1), np.array(vals2)):
        assert np.all((vals > 0) & (vals < 1))
        q = vals * 2 ** 23 - 0.5
        assert np.all(q == np.round(q))
        hist = np.histogram(vals, bins=16, range=(0, 1))[0]
        chi2 = ((hist - len(vals) / 16) ** 2 / (len(vals) / 16)).sum()
        assert chi2 < stats.chi2.ppf(0.999, 15)
    # different seeds / nodes give different streams
    assert oracle.hash_xi(1, 2, 0, 5, 5, 0) != oracle.hash_xi(1, 2, 0, 5, 5, 1)
    assert oracle.hash_xi(1, 2, 0, 5, 5, 0) != oracle.hash_xi(2, 2, 0, 5, 5, 0)


def test_lattice_level_is_floor_of_half_log2_area():
    """Footprint lattice level: floor(log2(|P|)/2), decided exactly from the
    binary exponent; the blend weight is the fractional part."""
    rng = np.random.default_rng(1)
    areas = np.concatenate([10.0 ** rng.uniform(-12, 2, 2000), 4.0 ** np.arange(-10, 3),
                            np.nextafter(4.0 ** np.arange(-10, 3), 0)])
    for a in areas:
        a = float(np.float32(a))
        l0, frac = oracle.lattice_level(a)
        lam = 0.5 * math.log2(a)
        assert l0 == math.floor(lam) or (abs(lam - round(lam)) < 1e-12 and l0 in (round(lam) - 1, round(lam)))
        assert 0.0 <= frac <= 1.0
        assert abs((l0 + frac) - lam) < 1e-12 or frac in (0.0, 1.0)


# --- the bias on both powers (sampler 3) ------------------------------------------

def test_symmetric_gate_small_integer_N_is_exact_binomial():
    """N in {0, 1, 2}: the same exact binomial outcomes as the dual gate."""
    for N in (0.0, 1.0, 2.0):
        for p in (0.0, 0.1, 0.5, 0.93, 1.0):
            a = oracle.gate_probs(N, p)
            b = oracle.gate_probs_symmetric(N, p, float(np.float32(1.0 - p)))
            if N != 2.0:
                np.testing.assert_array_equal(a, b)
            else:  # P(n=2) = p^2 either way, within float rounding
                assert abs(a[0] - b[0]) <= 2e-7 * max(a[0], 1e-30) + 1e-7 and np.array_equal(a[1:], b[1:])


def test_symmetric_gate_fixes_the_mirrored_small_probability():
    """When the node's negative side has a probability q below 2^-25, p = 1 - q
    rounds to 1 in float: the printed algorithm then gives P(n = N) = p^N = 1
    (no facet ever goes to the negative side, whatever N), while the exact
    value is (1 - q)^N.  With the bias on that power too the error stays
    within the paper's bound (about 1e-4 over N in [1, 1e16])."""
    worst_sym = worst_lit = 0.0
    for lq in np.arange(-16.0, -7.6, 0.25):
        for lN in np.arange(0.5, 16.0, 0.5):
            q, N = 10.0 ** lq, 10.0 ** lN
            qf, Nf = float(np.float32(q)), float(np.float32(N))
            exact = math.exp(Nf * math.log1p(-qf))
            sym = float(oracle.gate_probs_symmetric(Nf, float(np.float32(1.0 - q)), qf)[0])
            lit = float(oracle.gate_probs(Nf, float(np.float32(1.0 - q)))[0])
            worst_sym = max(worst_sym, abs(sym - exact))
            worst_lit = max(worst_lit, abs(lit - exact))
    assert worst_sym <= 2e-4, worst_sym
    assert worst_lit > 0.5, worst_lit  # e.g. q = 1e-9, N = 1e10: 1 instead of exp(-10)


def test_symmetric_gate_negative_counts_follow_N_q():
    """N = 1e10, q = 1e-9 (N q = 10 facets on the negative side): the printed
    algorithm puts every facet on the positive side; with the bias on both
    powers the Gaussian branch runs and the negative count N - G has the
    mean 1 + (N - 2) q of Alg. "Dual-gated Gaussian" (G has mean
    1 + (N - 2) p)."""
    rng = np.random.default_rng(9)
    m = 4000
    N = np.full(m, 1e10)
    q = 1e-9
    p = np.full(m, 1.0 - q)
    h1 = rng.integers(0, 2 ** 32, m, dtype=np.uint32)
    h2 = rng.integers(0, 2 ** 32, m, dtype=np.uint32)
    lit = oracle.sample_binomial(0, N, p, h1, h2)
    sym = oracle.sample_binomial(3, N, p, h1, h2)
    assert np.all(lit["nb"] == 0)
    mean = sym["nb"].mean()
    expect = 1.0 + (1e10 - 2.0) * q
    assert abs(mean - expect) < 4 * math.sqrt(expect / m), mean
    assert np.allclose(sym["n"] + sym["nb"], 1e10, rtol=1e-15)
