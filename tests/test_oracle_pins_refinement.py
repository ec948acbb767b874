"""Pins of the oracle's angular refinement (Alg. 2, Sec. 4.3) on the azimuthal hierarchy.

Checked against the definitions: the weights keep the full solid angle; with
nothing hit the result is the coarse product rule and with everything hit
the goal rule; the kept goal ordinates are exactly those whose rays meet the
disk, decided here by the ray-circle intercepts of the paper's appendix; the
kept sectors tile each polar level's circle once; and the asteroid setting
of Sec. 5.4 (4096 goal ordinates) refines to a few hundred ordinates.
"""
import math

import numpy as np
import pytest

import oracle


def _sector_of(om, w):
    """(polar level, level, index) of every ordinate from its weight and azimuth."""
    xg, wg = np.polynomial.legendre.leggauss(4)
    wp = wg[xg > 0]
    out = []
    for o, wt in zip(om, w):
        # the polar level from the in-plane length, then the sector width 2 pi / A_L from the weight
        st = math.hypot(o[0], o[1])
        p = int(np.argmin(np.abs(np.sqrt(1.0 - (xg[xg > 0]) ** 2) - st)))
        na = 2.0 * wp[p] * 2.0 * math.pi / wt
        L = int(round(math.log2(na / 4.0)))
        phi = math.atan2(o[1], o[0]) % (2.0 * math.pi)
        k = int(round(phi * (4 * 2 ** L) / (2.0 * math.pi) - 0.5))
        out.append((p, L, k))
    return out


def _hits_by_intercepts(src, center, radius, phi, far=1e6):
    """Ray-circle test by the parametric intercepts s = (-l1 +- sqrt(l1^2 - l0 l2)) / l2 of the appendix."""
    xs = np.asarray(src, float) - np.asarray(center, float)
    xe = xs + far * np.array([math.cos(phi), math.sin(phi)])
    l0 = xs @ xs - radius * radius
    l1 = xs @ (xe - xs)
    l2 = (xe - xs) @ (xe - xs)
    disc = l1 * l1 - l0 * l2
    if l0 <= 0.0:
        return True
    if disc < 0.0:
        return False
    s_far = (-l1 + math.sqrt(disc)) / l2
    return s_far > 0.0


@pytest.mark.parametrize("lmin,lgoal", [(0, 5), (1, 7), (2, 9), (3, 3)])
def test_weights_keep_the_solid_angle(lmin, lgoal):
    om, w = oracle.refined_quadrature(lmin, lgoal, (-3.0, 0.4), (1.0, 0.0), 0.7)
    assert abs(w.sum() - 4.0 * math.pi) <= 1e-13
    assert np.all(w > 0)


def test_nothing_hit_gives_the_coarse_rule_and_everything_hit_the_goal_rule():
    om, w = oracle.refined_quadrature(2, 6, (0.0, 0.0), (1.0, 0.0), 0.0)     # aim between midpoints
    om_c, w_c = oracle.angular_quadrature(2, 2 * 4 * 2 ** 2)
    assert np.abs(om - om_c).max() <= 1e-15 and np.abs(w - w_c).max() <= 1e-15
    om, w = oracle.refined_quadrature(2, 6, (0.3, 0.1), (0.0, 0.0), 1.0)     # source inside the disk
    om_g, w_g = oracle.angular_quadrature(2, 2 * 4 * 2 ** 6)
    assert np.abs(om - om_g).max() <= 1e-15 and np.abs(w - w_g).max() <= 1e-15


@pytest.mark.parametrize("src,center,radius", [((-105.0, 0.0), (0.0, 0.0), 35.0),
                                               ((0.5, -2.0), (0.2, 1.0), 0.4),
                                               ((2.0, 2.0), (-1.0, -1.5), 1.0)])
def test_kept_goal_ordinates_are_exactly_the_hits(src, center, radius):
    lmin, lgoal = 1, 8
    om, w = oracle.refined_quadrature(lmin, lgoal, src, center, radius)
    secs = _sector_of(om, w)
    ng = 4 * 2 ** lgoal
    for p in range(2):
        kept_goal = {k for (q, L, k) in secs if q == p and L == lgoal}
        hits = {c for c in range(ng) if _hits_by_intercepts(src, center, radius, 2.0 * math.pi * (c + 0.5) / ng)}
        assert hits <= kept_goal
        # a goal sector is kept without hitting only when its sibling subtree hits (it cannot merge)
        for c in kept_goal - hits:
            sib = c ^ 1
            assert sib in hits or any(s in hits for s in range(ng) if s // 2 == sib // 2)


@pytest.mark.parametrize("src,center,radius", [((-105.0, 0.0), (0.0, 0.0), 35.0), ((0.5, -2.0), (0.2, 1.0), 0.4)])
def test_kept_sectors_tile_each_circle_once(src, center, radius):
    lmin, lgoal = 0, 9
    om, w = oracle.refined_quadrature(lmin, lgoal, src, center, radius)
    ng = 4 * 2 ** lgoal
    for p in range(2):
        spans = sorted((k << (lgoal - L), (k + 1) << (lgoal - L)) for (q, L, k) in _sector_of(om, w) if q == p)
        assert spans[0][0] == 0 and spans[-1][1] == ng
        assert all(a[1] == b[0] for a, b in zip(spans, spans[1:]))


def test_asteroid_setting_refines_4096_goal_ordinates_to_a_few_hundred():
    """Sec. 5.4: a source 70 from the surface of a radius-35 disk; 4096 goal ordinates."""
    om, w = oracle.refined_quadrature(0, 9, (-105.0, 0.0), (0.0, 0.0), 35.0)
    assert 2 * 4 * 2 ** 9 == 4096
    hits = sum(_hits_by_intercepts((-105.0, 0.0), (0.0, 0.0), 35.0, math.atan2(o[1], o[0])) for o in om)
    # the hit ordinates are those of the goal rule inside the disk's angular width 2 asin(35/105)
    assert abs(hits - 2 * 4096 / 2 * 2 * math.asin(35.0 / 105.0) / (2 * math.pi)) <= 4
    assert hits < om.shape[0] < 600
