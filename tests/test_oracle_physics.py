"""Pins of the oracle's physics pieces against closed forms: the
Henyey-Greenstein inverse CDF, the scattering rotation, and the Fresnel
reflectance."""
import math

import numpy as np
import pytest

GS = [0.0, 0.01, 0.5, 0.9, -0.5, 0.99]


def hg_cdf(g, mu):
    """P(cos theta <= mu) for the Henyey-Greenstein phase function."""
    if g == 0:
        return (mu + 1) / 2
    return (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * mu) ** -0.5 - 1 / (1 + g))


@pytest.mark.parametrize("g", GS)
def test_hg_inverts_closed_form_cdf(oracle_mod, g):
    rng = np.random.default_rng(3)
    for u in list(rng.random(400)) + [2.0**-24, 0.5, 1 - 2.0**-24]:
        c = oracle_mod.hg_cos(g, u)
        assert -1.0 <= c <= 1.0
        assert abs(hg_cdf(g, c) - u) < 1e-11 * max(1.0, 1 / max(1e-300, 1 - abs(g))) , (g, u, c)


@pytest.mark.parametrize("g", GS)
def test_hg_moments(oracle_mod, g):
    # Midpoint rule over u: E[cos] = g and E[P2(cos)] = g^2 for HG.
    n = 20000
    u = (np.arange(n) + 0.5) / n
    c = np.array([oracle_mod.hg_cos(g, x) for x in u])
    assert abs(c.mean() - g) < 2e-4
    p2 = (3 * c * c - 1) / 2
    assert abs(p2.mean() - g * g) < 2e-3


def test_hg_isotropic_is_linear(oracle_mod):
    for u in [0.1, 0.25, 0.5, 0.8]:
        assert oracle_mod.hg_cos(0.0, u) == pytest.approx(2 * u - 1, abs=1e-15)


DIRS = [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0, -1, 0), (0.6, 0.0, 0.8), (0.48, -0.6, 0.64),
        (-0.36, 0.48, -0.8), (1e-9, 0.6, -0.8)]


@pytest.mark.parametrize("v", DIRS)
def test_rotation_invariants(oracle_mod, v):
    v = np.array(v, float)
    v /= np.linalg.norm(v)
    for ct in [-1.0, -0.3, 0.0, 0.5, 0.9999, 1.0]:
        for up in [0.0, 0.1, 0.37, 0.5, 0.99]:
            w = oracle_mod.scatter_dir(v, ct, up)
            assert abs(np.linalg.norm(w) - 1) < 1e-12
            assert abs(w @ v - ct) < 1e-12


@pytest.mark.parametrize("v", DIRS)
def test_rotation_azimuth_uniform(oracle_mod, v):
    # Over a uniform azimuth the perpendicular part averages to zero, and
    # azimuths half a turn apart are mirror images about v.
    v = np.array(v, float)
    v /= np.linalg.norm(v)
    ct = 0.3
    ws = np.array([oracle_mod.scatter_dir(v, ct, (i + 0.5) / 64) for i in range(64)])
    assert np.allclose(ws.mean(axis=0), ct * v, atol=1e-12)
    a = oracle_mod.scatter_dir(v, ct, 0.2)
    b = oracle_mod.scatter_dir(v, ct, 0.7)
    assert np.allclose(a + b, 2 * ct * v, atol=1e-12)
    # quarter turns are orthogonal in the plane normal to v
    p0 = oracle_mod.scatter_dir(v, 0.0, 0.0)
    p1 = oracle_mod.scatter_dir(v, 0.0, 0.25)
    assert abs(p0 @ p1) < 1e-12


def test_rotation_basis_at_pole(oracle_mod):
    # For v = +z the basis is (x, y): azimuth 0 tilts toward +x.
    w = oracle_mod.scatter_dir([0, 0, 1], 0.0, 0.0)
    assert np.allclose(w, [1, 0, 0], atol=1e-15)
    w = oracle_mod.scatter_dir([0, 0, 1], 0.0, 0.25)
    assert np.allclose(w, [0, 1, 0], atol=1e-15)


def test_fresnel_normal_incidence(oracle_mod):
    for n1, n2 in [(1.37, 1.0), (1.0, 1.37), (1.5, 1.33)]:
        assert oracle_mod.fresnel(n1, n2, 1.0) == pytest.approx(((n1 - n2) / (n1 + n2)) ** 2,
                                                                 rel=1e-14)
    assert oracle_mod.fresnel(1.37, 1.0, 1.0) == pytest.approx(0.024373, abs=5e-7)


def test_fresnel_total_internal_reflection(oracle_mod):
    n1, n2 = 1.37, 1.0
    crit = math.asin(n2 / n1)
    assert math.degrees(crit) == pytest.approx(46.88, abs=0.01)
    assert oracle_mod.fresnel(n1, n2, math.cos(crit + 1e-6)) == 1.0
    assert oracle_mod.fresnel(n1, n2, math.cos(crit - 1e-3)) < 1.0
    # into the denser medium there is no total reflection, but R -> 1 at grazing
    assert oracle_mod.fresnel(n2, n1, 1e-9) > 0.999999


def test_fresnel_reciprocity_and_brewster(oracle_mod):
    n1, n2 = 1.37, 1.0
    for ti in np.linspace(0.01, math.asin(n2 / n1) - 0.01, 12):
        tt = math.asin(n1 / n2 * math.sin(ti))
        assert oracle_mod.fresnel(n1, n2, math.cos(ti)) == pytest.approx(
            oracle_mod.fresnel(n2, n1, math.cos(tt)), rel=1e-12)
    # At Brewster's angle the p wave vanishes: R = rs^2 / 2 with
    # rs = (n1^2 - n2^2) / (n1^2 + n2^2).
    for a, b in [(1.0, 1.37), (1.37, 1.0)]:
        tb = math.atan(b / a)
        rs = (a * a - b * b) / (a * a + b * b)
        assert oracle_mod.fresnel(a, b, math.cos(tb)) == pytest.approx(rs * rs / 2, rel=1e-12)
