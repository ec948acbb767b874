"""The asteroid's graded point set (Sec. 5.4): the spacing the paper states at its four places, the
quadtree's leaves against that spacing, the edge rule, and the properties the solver relies on (every
point inside the domain, supports covering every place, touching leaves at most 2:1 apart)."""
import math

import numpy as np
import pytest

import workloads as W


def _tree(coarsen):
    a = W.asteroid(0.1)
    x, R, L = W.asteroid_graded_points(a, coarsen)
    return a, x, R, L


def test_spacing_at_the_papers_places():
    # Sec. 5.4 in the paper's units: 0.2 on the shell's inner surface, 0.1 on its outer surface,
    # 1.0 halfway between the source and the asteroid, 0.1 at the source
    a = W.asteroid(1.0)
    assert a.radius == 35.0 and a.thickness == 2.0
    src = np.asarray(a.src)
    assert np.linalg.norm(src) - a.radius == pytest.approx(70.0)
    pts = np.array([[a.radius - a.thickness, 0.0], [0.0, -a.radius], [src[0] / 2 - a.radius / 2, 0.0], src])
    h = W.asteroid_spacing(a, pts)
    assert h == pytest.approx([0.2, 0.1, 1.0, 0.1], abs=1e-12)
    # the scaled workload keeps the same spacing relative to its lengths; coarsening multiplies it
    b = W.asteroid(0.1)
    assert W.asteroid_spacing(b, pts * 0.1) == pytest.approx(0.1 * h, abs=1e-13)
    assert W.asteroid_spacing(b, pts * 0.1, 4.0) == pytest.approx(0.4 * h, abs=1e-13)
    # never coarser than 1.0 anywhere, finest on the shell's outer surface and at the source
    far = np.array([[40.0, 40.0], [-110.0, -40.0], [0.0, 0.0]])
    assert np.all(W.asteroid_spacing(a, far) <= 1.0 + 1e-12)


@pytest.mark.parametrize("coarsen", [10.0, 1.0])
def test_leaves_follow_the_spacing(coarsen):
    a, x, R, L = _tree(coarsen)
    lo, hi = np.asarray(a.lo), np.asarray(a.hi)
    assert np.all(x > lo) and np.all(x < hi)
    np.testing.assert_array_equal(R, 2.0 * L)
    # each point is its leaf's centre moved by at most 0.2 leaf sides, so h at the point is within
    # sqrt(2) of the leaf size up to the spacing's change over that distance (slope 0.9/35, or 0.05
    # across the shell), except where the edge rule split a leaf further
    h = W.asteroid_spacing(a, x, coarsen)
    ratio = L / h
    assert ratio.max() <= math.sqrt(2.0) * 1.06
    edge = np.any((x - lo < L[:, None]) | (hi - x < L[:, None]), axis=1)
    assert ratio[~edge].min() >= 1.0 / math.sqrt(2.0) / 2.0 / 1.06
    # the leaves tile the domain: their areas add up to it
    assert float(np.sum(L * L)) == pytest.approx(float(np.prod(hi - lo)), rel=1e-12)


def test_touching_leaves_and_edge_rows():
    a, x, R, L = _tree(10.0)
    lo, hi = np.asarray(a.lo), np.asarray(a.hi)
    from scipy.spatial import cKDTree
    t = cKDTree(x)
    # two points closer than 0.9 of the larger leaf's size sit in touching leaves (a jittered point
    # stays 0.3 of its leaf's size inside it): their sizes differ by at most 2:1
    pairs = t.query_pairs(float(R.max()), output_type="ndarray")
    d = np.linalg.norm(x[pairs[:, 0]] - x[pairs[:, 1]], axis=1)
    big = np.maximum(L[pairs[:, 0]], L[pairs[:, 1]])
    close = d <= 0.9 * big
    r = L[pairs[close, 0]] / L[pairs[close, 1]]
    assert max(r.max(), (1.0 / r).max()) <= 2.0 + 1e-12
    # every quadrature place near the domain's edge lies in the supports of two rows of points:
    # sample the edges densely and count the supports that reach each sample
    s = np.linspace(0.0, 1.0, 2001)[1:-1]
    edges = np.concatenate([
        np.stack([lo[0] + s * (hi[0] - lo[0]), np.full_like(s, lo[1])], 1),
        np.stack([lo[0] + s * (hi[0] - lo[0]), np.full_like(s, hi[1])], 1),
        np.stack([np.full_like(s, lo[0]), lo[1] + s * (hi[1] - lo[1])], 1),
        np.stack([np.full_like(s, hi[0]), lo[1] + s * (hi[1] - lo[1])], 1)])
    for y in edges[::7]:
        js = t.query_ball_point(y, float(R.max()))
        js = np.asarray(js)
        cover = js[np.linalg.norm(x[js] - y, axis=1) < R[js]]
        # the covering points do not all sit in one row parallel to the edge
        n = np.array([0.0, 1.0]) if (abs(y[1] - lo[1]) < 1e-12 or abs(y[1] - hi[1]) < 1e-12) else np.array([1.0, 0.0])
        depth = np.abs((x[cover] - y) @ n)
        assert cover.size >= 3          # as at the corners of a uniform lattice with R = 2 dx
        assert depth.max() - depth.min() >= 0.5 * L[cover].min(), y


def test_seeded_and_ordered():
    a, x, R, L = _tree(4.0)
    x2, R2, L2 = W.asteroid_graded_points(a, 4.0)
    np.testing.assert_array_equal(x, x2)
    np.testing.assert_array_equal(L, L2)
    x3, _, _ = W.asteroid_graded_points(a, 4.0, seed=W.SEED_BASE + 11)
    assert not np.array_equal(x, x3)
    # Morton order: consecutive points are near each other (median step about one spacing)
    step = np.linalg.norm(np.diff(x, axis=0), axis=1)
    assert np.median(step / L[1:]) < 1.6


def test_step_absorption_in_the_exact_flux():
    a = W.asteroid(0.1)
    a0 = W.asteroid_step_inv_c_dt(a)
    assert 1.0 / a0 == pytest.approx(100.0 * math.hypot(15.0, 8.0))
    x = np.array([[-7.0, 0.0], [-5.0, 1.0], [2.0, 2.0]])
    r = np.linalg.norm(x - np.asarray(a.src), axis=1)
    np.testing.assert_allclose(W.asteroid_optical_depth(a, x, a0) - W.asteroid_optical_depth(a, x), a0 * r,
                               rtol=1e-12)
    # with one polar level of cosine 0 (in-plane rays) the flux is S/(4 pi r) 2 w e^-omega
    phi = W.asteroid_phi_ordinates(a, x[:1], np.array([0.0]), np.array([1.0]), a0)
    om = a.sigma_back * r[0] + a0 * r[0]
    assert phi[0] == pytest.approx(a.strength / (4 * math.pi * r[0]) * 2.0 * math.exp(-om), rel=1e-12)
