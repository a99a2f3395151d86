"""Quality pins of the per-footprint hash (pcg4d, Jarzynski & Olano, JCGT
2020) that supplies the random numbers of Sec. 3.3 ("random seeds stored at
the grid vertices") and the two uniforms of each node of Alg. "Dual-gated
Gaussian".  No published output values of the hash are at hand, so its
definition is pinned by the properties the method relies on and that a
plausible slip in the definition breaks:

* avalanche: one flipped input bit flips each of the upper 16 bits of every
  output word with probability near 1/2 (a dropped xorshift, a dropped
  second multiply-add round or a swapped multiplier fails);
* the carry structure of multiply-add plus one xorshift by 16: output bit k
  depends on input bits <= k + 16 only, and on every one of them;
* joint uniformity (2-D chi^2) of the node's (xi1, xi2), of the two nodes
  that share one hash (2i takes outputs x, y; 2i+1 takes z, w), and of
  neighbouring lattice vertices.
"""
import numpy as np
from scipy import stats

import oracle

RNG = np.random.default_rng(20250702)


def _flip_rates(n=8192):
    x = RNG.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    h = oracle.pcg4d(x)
    rates = np.zeros((128, 4, 32))
    shifts = np.arange(32, dtype=np.uint32)
    for ib in range(128):
        y = x.copy()
        y[:, ib // 32] ^= np.uint32(1 << (ib % 32))
        d = h ^ oracle.pcg4d(y)
        rates[ib] = ((d[:, :, None] >> shifts) & 1).mean(0)
    return rates


RATES = None


def rates():
    global RATES
    if RATES is None:
        RATES = _flip_rates()
    return RATES


def test_pcg4d_is_deterministic_and_word_wise():
    x = RNG.integers(0, 2 ** 32, size=(64, 4), dtype=np.uint64).astype(np.uint32)
    a = oracle.pcg4d(x)
    assert np.array_equal(a, oracle.pcg4d(x))
    assert np.array_equal(a[7], oracle.pcg4d(x[7:8])[0])
    assert len({tuple(r) for r in a}) == len(a)


def test_pcg4d_avalanche_upper_bits():
    """Measured on 8192 random inputs: per (input bit, output word, upper
    output bit) flip rate 0.33..0.64, per (input bit, output word) mean over
    the upper 16 bits 0.37..0.51.  The bounds below leave about 5 sigma."""
    r = rates()[:, :, 16:]
    assert r.min() > 0.30 and r.max() < 0.70, (r.min(), r.max())
    m = r.mean(axis=2)
    assert m.min() > 0.35 and m.max() < 0.55, (m.min(), m.max())


def test_pcg4d_carry_structure():
    """Multiply-add carries only upwards; the one xorshift by 16 brings bits
    down by 16.  So output bit k of every word ignores input bits above
    k + 16 and depends on all others."""
    r = rates()
    j = np.arange(128) % 32
    for k in range(32):
        dep = r[:, :, k].max(axis=1)  # any output word
        expected_zero = j > k + 16
        assert np.all(dep[expected_zero] == 0.0), k
        assert np.all(dep[~expected_zero] > 0.05), k


def _chi2_2d(u, v, bins=16):
    h, _, _ = np.histogram2d(u, v, bins=bins, range=[[0, 1], [0, 1]])
    e = len(u) / bins ** 2
    return ((h - e) ** 2 / e).sum(), bins * bins - 1


def _xi_grid(node, n_side=256, seed=3, surf=11, level=-5, da=0, db=0):
    out = np.empty((n_side * n_side, 2))
    i = 0
    for a in range(n_side):
        for b in range(n_side):
            out[i] = oracle.hash_xi(seed, surf, level, a + da, b + db, node)
            i += 1
    return out


XI = {}


def xi(node, **kw):
    key = (node, tuple(sorted(kw.items())))
    if key not in XI:
        XI[key] = _xi_grid(node, **kw)
    return XI[key]


def test_node_uniforms_jointly_uniform():
    """(xi1, xi2) of one node over a 256 x 256 block of lattice vertices."""
    for node in (0, 1, 2):
        u = xi(node)
        c, dof = _chi2_2d(u[:, 0], u[:, 1])
        assert c < stats.chi2.ppf(0.9999, dof), (node, c)


def test_nodes_sharing_one_hash_are_independent():
    """Nodes 2i and 2i+1 take (x, y) and (z, w) of the same pcg4d call: every
    pair of their uniforms is jointly uniform."""
    a, b = xi(0), xi(1)
    for i in range(2):
        for j in range(2):
            c, dof = _chi2_2d(a[:, i], b[:, j])
            assert c < stats.chi2.ppf(0.9999, dof), (i, j, c)
    # and the next pair of nodes (another call) against the first
    d = xi(2)
    c, dof = _chi2_2d(a[:, 0], d[:, 0])
    assert c < stats.chi2.ppf(0.9999, dof), c


def test_neighbouring_vertices_are_independent():
    """Draws at lattice vertex (a, b) and at (a+1, b), (a, b+1)."""
    base = xi(0)
    for da, db in ((1, 0), (0, 1)):
        nb = xi(0, da=da, db=db)
        c, dof = _chi2_2d(base[:, 0], nb[:, 0])
        assert c < stats.chi2.ppf(0.9999, dof), (da, db, c)
        c, dof = _chi2_2d(base[:, 1], nb[:, 1])
        assert c < stats.chi2.ppf(0.9999, dof), (da, db, c)


def test_slipped_definitions_fail_these_pins():
    """The pins above are strong enough to reject plausible slips in the
    definition: each variant (written here only to plant the mistake)
    fails the avalanche bounds or the carry structure."""
    M = np.uint64(0xFFFFFFFF)

    def variant(v, drop_xorshift=False, swap=False, drop_round2=False, shift=16):
        v = (v.astype(np.uint64) * np.uint64(1664525) + np.uint64(1013904223)) & M
        x, y, z, w = (v[:, i].copy() for i in range(4))
        x = (x + y * (z if swap else w)) & M
        y = (y + z * x) & M
        z = (z + x * y) & M
        w = (w + y * z) & M
        if not drop_xorshift:
            x ^= x >> np.uint64(shift); y ^= y >> np.uint64(shift)
            z ^= z >> np.uint64(shift); w ^= w >> np.uint64(shift)
        if not drop_round2:
            x = (x + y * w) & M
            y = (y + z * x) & M
            z = (z + x * y) & M
            w = (w + y * z) & M
        return np.stack([x, y, z, w], 1).astype(np.uint32)

    x = RNG.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(variant(x), oracle.pcg4d(x))  # the planted-mistake harness is faithful

    def passes(fn):
        h = fn(x)
        r = np.zeros((128, 4, 32))
        for ib in range(128):
            y = x.copy()
            y[:, ib // 32] ^= np.uint32(1 << (ib % 32))
            d = h ^ fn(y)
            r[ib] = ((d[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(0)
        up = r[:, :, 16:]
        ok_av = up.min() > 0.30 and up.max() < 0.70 and up.mean(2).min() > 0.35
        j = np.arange(128) % 32
        ok_carry = all(np.all(r[:, :, k].max(1)[j > k + 16] == 0) and np.all(r[:, :, k].max(1)[j <= k + 16] > 0.05)
                       for k in range(32))
        return ok_av and ok_carry

    assert passes(variant)
    for kw in (dict(drop_xorshift=True), dict(swap=True), dict(drop_round2=True), dict(shift=15),
               dict(shift=17)):
        assert not passes(lambda v, kw=kw: variant(v, **kw)), kw
