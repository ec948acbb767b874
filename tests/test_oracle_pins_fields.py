"""Pins of the oracle's spatially varying materials and of the paper's manufactured problems.

Material fields move the weight ``a + b prod_alpha cos(k y_alpha + phase)`` of
every volume quadrature point from material 0 to another material, which
represents the sinusoidal opacities of Sec. 5.1.  The pins:
- a constant field splits the blocks in a fixed ratio (exact identity);
- the block sums equal closed-form integrals of the field, through the RK
  reproducing conditions of Sec. 2.2 (partition of unity and linear
  reproduction turn sums over i, j into integrals of the field);
- the sinusoidal (varying opacities) and outgoing-wave manufactured problems
  of Sec. 5.1 converge at second order in space for linear RK.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_orders.json")))
LO2, HI2 = (-1.0, -1.0), (1.0, 1.0)


def _geom(n, d=2, jitter=0.2, seed=9):
    lo, hi = (-1.0,) * d, (1.0,) * d
    x, dx = W.jittered_lattice((n,) * d, lo, hi, jitter, seed)
    R = np.full(x.shape[0], (2.0 if d == 2 else 2.5) * dx)
    return x, dx, oracle.geometry(x, R, lo, hi)


def _cos_int(k, ph):
    """int_{-1}^{1} cos(k y + ph) dy"""
    return (math.sin(k + ph) - math.sin(-k + ph)) / k


def _ycos_int(k, ph):
    """int_{-1}^{1} y cos(k y + ph) dy"""
    F = lambda y: y * math.sin(k * y + ph) / k + math.cos(k * y + ph) / (k * k)
    return F(1.0) - F(-1.0)


@pytest.mark.parametrize("d", [2, 3])
def test_constant_field_splits_blocks(d):
    x, dx, g = _geom(6 if d == 2 else 4, d)
    ref = oracle.integrate(g, 1)
    it = oracle.integrate(g, 1, n_mat=2, fields=((0.3, 0.0, 1.7, 0.2, 1),))
    nv = 1 + d
    for b in range(nv):
        scale = np.abs(ref.blocks[b]).max()
        assert np.abs(it.blocks[nv + b] - 0.3 * ref.blocks[b]).max() <= 1e-13 * scale, b
        assert np.abs(it.blocks[b] - 0.7 * ref.blocks[b]).max() <= 1e-13 * scale, b
    # the direction-only blocks (K, surface) do not see the material
    assert np.array_equal(it.blocks[2 * nv:], ref.blocks[nv:])


def test_field_block_sums_are_field_integrals():
    """sum_ij Mass_g = int f_g,  sum_ij Mass_g x_j^a = int f_g y_a,  sum_ij x_i^a D^a_g = int f_g."""
    a, b, k, ph = 0.4, 0.5, 2.3, 0.7
    x, dx, g = _geom(12)
    it = oracle.integrate(g, 1, n_mat=2, fields=((a, b, k, ph, 1),))
    nnz = it.blocks.shape[1]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_off))
    cols = g.col
    mass1 = it.blocks[3]
    I0 = 4.0 * a + b * _cos_int(k, ph) ** 2
    I1 = b * _ycos_int(k, ph) * _cos_int(k, ph)            # int f y_a (the a-term integrates to 0)
    assert abs(mass1.sum() - I0) <= 1e-10 * abs(I0)
    for al in range(2):
        assert abs(np.sum(mass1 * x[cols, al]) - I1) <= 1e-10 * abs(I0), al
        d1 = it.blocks[4 + al]
        assert abs(np.sum(x[rows, al] * d1) - I0) <= 1e-10 * abs(I0), al
    # material 0 holds the rest of the unit fraction
    mass0 = it.blocks[0]
    assert abs(mass0.sum() - (4.0 - I0)) <= 1e-10 * 4.0
    assert nnz == g.row_off[-1]


def test_mms_cos_fields_reproduce_opacity_integrals():
    """The sinusoidal opacities as fields: sum_ij of sum_g sigma_g Mass_g = int sigma over [-1, 1]^2."""
    x, dx, g = _geom(12)
    it = oracle.integrate(g, 1, n_mat=3, fields=W.MMS_COS_FIELDS)
    mass = [it.blocks[3 * gm] for gm in range(3)]
    st = sum(s * m for s, m in zip(W.MMS_COS_SIGMA_T, mass)).sum()
    ss = sum(s * m for s, m in zip(W.MMS_COS_SIGMA_S, mass)).sum()
    # sigma_a = 1 + (2/3) cos(3x) cos(3y); sigma_s = 1 + (3/4) sin(2x) sin(2y) (odd: integrates to 0)
    int_sa = 4.0 + (2.0 / 3.0) * (2.0 * math.sin(3.0) / 3.0) ** 2
    int_ss = 4.0
    assert abs(ss - int_ss) <= 1e-10 * int_ss
    assert abs(st - (int_sa + int_ss)) <= 1e-10 * (int_sa + int_ss)
    assert abs(sum(mass).sum() - 4.0) <= 1e-12 * 4.0


def _mms_error(n, kind, M=8):
    x, dx, g = _geom(n, jitter=0.0)
    if kind == "cos":
        it = oracle.integrate(g, 1, n_mat=3, fields=W.MMS_COS_FIELDS)
        st, ss, t = W.MMS_COS_SIGMA_T, W.MMS_COS_SIGMA_S, 0.0
        psi_f, src = W.mms_cos_psi, W.mms_cos_source
    else:
        it = oracle.integrate(g, 1)
        st, ss, t = W.MMS_WAVE_SIGMA_A + W.MMS_WAVE_SIGMA_S, W.MMS_WAVE_SIGMA_S, 0.5
        psi_f, src = W.mms_wave_psi, W.mms_wave_source
    om, wq = oracle.angular_quadrature(2, M)
    tr = oracle.Transport(it, om, wq, st, ss, 0.0, dx)
    pb = np.repeat(psi_f(it.bq_y, t)[:, None], M, axis=1)
    psi, phi, info = tr.step(None, src(x, om, t, 0.0), pb)
    assert info["outer_res"] <= 1e-10
    ex = 4.0 * np.pi * psi_f(x, t)
    # relative error of the scalar flux at the centres, Sec. 5 (sum of absolute differences)
    return np.abs(tr.point_values(phi) - ex).sum() / ex.sum(), dx


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["cos", "wave"])
def test_paper_mms_spatial_order_two(kind):
    """Both manufactured problems of Sec. 5.1 (steady, uniform lattice on [-1, 1]^2) converge at second order."""
    errs, hs = zip(*[_mms_error(n, kind) for n in (8, 16, 32)])
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert abs(slope - GOLD["mms_spatial_order_linear_rk"]) <= GOLD["order_tolerance"], (errs, slope)


# --------------------------------------------------------------------- shells
def test_shells_cover_everything_or_nothing():
    """A shell containing the whole domain moves every block to its material; one outside changes nothing."""
    x, dx, g = _geom(8)
    ref = oracle.integrate(g, 1, n_mat=2)
    full = oracle.integrate(g, 1, n_mat=2, shells=(((0.1, -0.2), 0.0, 10.0, 1),))
    none = oracle.integrate(g, 1, n_mat=2, shells=(((0.1, -0.2), 5.0, 10.0, 1),))
    assert np.array_equal(full.blocks[3:6], ref.blocks[0:3]) and not np.any(full.blocks[0:3])
    assert np.array_equal(none.blocks, ref.blocks)


def test_shell_area_converges_and_boxes_come_first():
    """sum_ij Mass_g over an annulus tends to its area; a shell overrides a box that covers the domain."""
    c, r0, r1 = (0.13, -0.07), 0.35, 0.8
    exact = math.pi * (r1 * r1 - r0 * r0)
    errs = []
    for n in (8, 16, 32):
        x, dx, g = _geom(n)
        it = oracle.integrate(g, 1, n_mat=2, regions=(((-1.0, -1.0), (1.0, 1.0), 1),), shells=((c, r0, r1, 0),))
        errs.append(abs(it.blocks[0].sum() - exact) / exact)
        assert abs(it.blocks[0].sum() + it.blocks[3].sum() - 4.0) <= 1e-12
    assert errs[2] < errs[1] < errs[0] and errs[2] <= 2e-3, errs
