"""Pins of the oracle's footprint grid (vertices = 12: Sec. 3.3, the pixel
footprint by length, anisotropy and orientation, its facets distributed
over a tetrahedral cell of that space, a uv triangle grid per cell vertex;
the layout is the library's, see include/glint.h)."""
import math

import numpy as np
import pytest

import oracle
import synth


def jac(smaj, A, theta):
    """uv Jacobian whose footprint ellipse has major axis smaj along theta
    and minor axis smaj / A."""
    c, s = math.cos(theta), math.sin(theta)
    Rm = np.array([[c, -s], [s, c]])
    return Rm @ np.diag([smaj, smaj / A])


def grid(u, v, J):
    return oracle.footprint_grid(u, v, J[0, 0], J[0, 1], J[1, 0], J[1, 1])


def unpack(key):
    l = np.int8((key >> 24) & 0xFF)
    return int(l), int((key >> 20) & 0xF), int((key >> 16) & 0xF)


def test_weights_form_a_partition_of_unity():
    rng = np.random.default_rng(1)
    for _ in range(500):
        J = rng.normal(size=(2, 2)) * 10.0 ** rng.uniform(-5, -1)
        g = grid(*rng.uniform(-50, 50, 2), J)
        assert g is not None
        assert np.all(g["w"] >= -1e-15)
        assert abs(g["w"].sum() - 1) < 1e-12


def test_cell_vertices_bracket_the_footprint():
    """The 4 cell vertices (l, a, o) surround the footprint's continuous grid
    coordinates, and the weighted mean of the vertex coordinates is the
    footprint's own (barycentric interpolation)."""
    rng = np.random.default_rng(2)
    for _ in range(300):
        smaj, A, th = 10.0 ** rng.uniform(-4, -1), 2.0 ** rng.uniform(0, 3.9), rng.uniform(0, math.pi)
        g = grid(0.37, -1.3, jac(smaj, A, th))
        w4 = g["w"].reshape(4, 3).sum(1)
        verts = np.array([unpack(k) for k in g["key"][::3]], np.float64)
        want = np.array([math.log2(smaj), math.log2(A), th * 8 / math.pi])
        # orientation is periodic: unwrap the vertices next to the base
        verts[:, 2] = np.where(verts[:, 2] < np.floor(want[2]) - 4, verts[:, 2] + 8, verts[:, 2])
        verts[:, 2] = np.where(verts[:, 2] > np.floor(want[2]) + 4, verts[:, 2] - 8, verts[:, 2])
        np.testing.assert_allclose((w4[:, None] * verts).sum(0), want, atol=1e-9)


def test_count_ratio_is_vertex_area_over_pixel_area():
    smaj, A, th = 3e-3, 4.0, 0.4
    g = grid(0.1, 0.2, jac(smaj, A, th))
    for k, r in zip(g["key"], g["r"]):
        l, a, o = unpack(k)
        np.testing.assert_allclose(r, (4.0 ** l / 2.0 ** a) / (smaj * smaj / A), rtol=1e-12)


def test_orientation_is_periodic_and_sign_free():
    """J and -J (and a turn by pi) describe the same footprint."""
    J = jac(2e-3, 3.0, 1.1)
    a, b = grid(0.2, 0.9, J), grid(0.2, 0.9, -J)
    c = grid(0.2, 0.9, jac(2e-3, 3.0, 1.1 + math.pi))
    for o in (b, c):
        np.testing.assert_allclose(o["w"], a["w"], atol=1e-12)
        assert np.array_equal(o["key"], a["key"]) and np.array_equal(o["a"], a["a"])


def test_anisotropy_is_clamped_and_degenerate_footprints_draw_nothing():
    g = grid(0.1, 0.1, np.array([[1e-3, 0.0], [0.0, 0.0]]))  # rank one: A = 16
    assert g is not None and max(unpack(k)[1] for k in g["key"]) <= 5
    assert grid(0.1, 0.1, np.zeros((2, 2))) is None


def test_draws_are_fixed_by_the_vertex_not_the_pixel():
    """Temporal stability: a footprint that changes slightly (rotation,
    scale, the area scaled alike) keeps its cell, lattice vertices and the
    vertices' counts; only the weights move."""
    J0 = jac(2.0e-3, 2.5, 0.7)
    a = grid(0.31, 0.77, J0)
    b = grid(0.31, 0.77, jac(2.0e-3 * 1.001, 2.5, 0.7005))
    assert np.array_equal(a["key"], b["key"]) and np.array_equal(a["a"], b["a"]) and np.array_equal(a["b"], b["b"])
    # N_i = N_P r_i with N_P proportional to the footprint area: unchanged
    na = a["r"] * 1.0
    nb = b["r"] * (1.001 ** 2)
    np.testing.assert_allclose(nb, na, rtol=1e-12)
    assert not np.allclose(a["w"], b["w"], atol=1e-6)


@pytest.fixture(scope="module")
def frame():
    R, K, M = 16, 8, 5
    env = synth.make_env(R, 6)
    levels, ij, it = oracle.partition(env, K)
    chain = oracle.mipchain(env, ij, it, K, M)
    ind, rgb = oracle.split_pyramid(oracle.prefilter(env, ij, it, chain, K, M, 64), K)
    S, E = oracle.lut_tables()
    W, H = 128, 72
    g = synth.scene_frame(W, H, seed=3, density_decades=(3.0, 7.0))
    g["dudx"], g["dudy"], g["dvdx"], g["dvdy"] = synth.uv_jacobian(g, W, H)
    hit = np.nonzero(g["surf_id"] != synth.NO_SURFACE)[0]
    return dict(R=R, K=K, M=M, levels=levels, ind=ind, rgb=rgb, S=S, E=E, g=g, hit=hit)


def run(f, V, g=None):
    g = f["g"] if g is None else g
    return oracle.shade(g, f["ind"], f["rgb"], f["levels"], f["S"], f["E"], f["R"], f["K"], f["M"], 5, V,
                        pixels=f["hit"])


def test_grid_shading_is_unbiased_against_one_vertex(frame):
    """Normalised by the weighted vertex count, the grid's glints average to
    the same frame radiance as the single-vertex draw (both estimate the
    smooth radiance)."""
    a, b = run(frame, 1), run(frame, 12)
    ratio = b["radiance"].sum() / a["radiance"].sum()
    assert abs(ratio - 1) < 0.03, ratio
    assert b["counts"].shape[1] == 12
    assert ((b["flags"] & 16) != 0).mean() < 0.01


def test_grid_requires_the_jacobian(frame):
    g = {k: v for k, v in frame["g"].items() if k not in ("dudx", "dudy", "dvdx", "dvdy")}
    with pytest.raises(ValueError):
        run(frame, 12, g)
