"""Pins for the mechanical laws (Appendix B) and the TL cofactor (Appendix A).

Closed forms derived by hand from the law definitions:
  * linear elasticity under uniaxial strain e: sigma = diag((2mu+lam) e, lam e, lam e);
  * neo-Hookean uniaxial stretch F = diag(s,1,1) and simple shear F = I + g e_x(x)e_y;
  * objectivity: a rigid rotation F = Q gives zero Cauchy stress;
  * small-strain limit: d sigma_NH / d(grad u) at grad u = 0 is the linear law.
"""

import numpy as np
import pytest

import meshgen as mg
from oracle.fv import material_constants, stress_linear_elastic, neo_hookean, cofactor


def _consts(law="neo_hookean", E=1e6, nu=0.45):
    return material_constants(mg.Material(law, E, nu))


def test_material_constants():
    c = _consts(E=1e6, nu=0.45)
    assert np.isclose(c["mu"], 1e6 / 2.9)
    assert np.isclose(c["lam"], 1e6 * 0.45 / (1.45 * 0.1))
    assert np.isclose(c["kappa"], 1e6 / (3 * 0.1))
    # K_bar = 4/3 mu + kappa = 2 mu + lambda (Section 2.3.3)
    assert np.isclose(c["Kbar"], 4.0 / 3.0 * c["mu"] + c["kappa"])


def test_linear_elastic_uniaxial():
    c = _consts("linear_elastic", 200e9, 0.3)
    e = 1e-4
    g = np.zeros((1, 3, 3))
    g[0, 0, 0] = e
    s = stress_linear_elastic(g, c)[0]
    assert np.allclose(np.diag(s), [(2 * c["mu"] + c["lam"]) * e, c["lam"] * e, c["lam"] * e])
    assert np.allclose(s - np.diag(np.diag(s)), 0.0)


@pytest.mark.parametrize("s", [0.7, 1.0, 1.3, 2.0])
def test_neo_hookean_uniaxial_stretch(s):
    c = _consts()
    mu, kap = c["mu"], c["kappa"]
    g = np.zeros((1, 3, 3))
    g[0, 0, 0] = s - 1.0
    sig, cof = neo_hookean(g, c)
    sxx = mu / s * s ** (-2.0 / 3.0) * 2.0 * (s * s - 1.0) / 3.0 + 0.5 * kap * (s * s - 1.0) / s
    syy = -mu / s * s ** (-2.0 / 3.0) * (s * s - 1.0) / 3.0 + 0.5 * kap * (s * s - 1.0) / s
    assert np.allclose(np.diag(sig[0]), [sxx, syy, syy], rtol=1e-13, atol=1e-9 * mu)
    assert np.allclose(cof[0], np.diag([1.0, s, s]))


@pytest.mark.parametrize("gam", [0.1, 0.5, 1.5])
def test_neo_hookean_simple_shear(gam):
    c = _consts()
    mu = c["mu"]
    g = np.zeros((1, 3, 3))
    g[0, 1, 0] = gam          # u_x = gam * y  ->  d u_x / d y = gam
    sig = neo_hookean(g, c)[0][0]
    expect = mu * np.array([[2 * gam ** 2 / 3, gam, 0], [gam, -gam ** 2 / 3, 0], [0, 0, -gam ** 2 / 3]])
    assert np.allclose(sig, expect, rtol=1e-13, atol=1e-12 * mu)


def test_neo_hookean_objective_under_rotation():
    c = _consts()
    rng = np.random.default_rng(3)
    for _ in range(5):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] *= -1
        g = (Q - np.eye(3)).T[None]
        sig = neo_hookean(g, c)[0]
        assert np.abs(sig).max() < 1e-9 * c["mu"]
        # the linear law is not objective: it gives a nonzero stress (control)
        assert np.abs(stress_linear_elastic(g, c)).max() > 1e-3 * c["mu"]


def test_cofactor_against_library_inverse():
    rng = np.random.default_rng(4)
    F = np.eye(3) + 0.3 * rng.standard_normal((6, 3, 3))
    cof = cofactor(F)
    for k in range(6):
        assert np.allclose(cof[k], np.linalg.det(F[k]) * np.linalg.inv(F[k]).T, rtol=1e-13, atol=1e-14)


def test_neo_hookean_small_strain_limit():
    """Appendix B: for small deformations the neo-Hookean law reduces to linear elasticity."""
    c = _consts()
    rng = np.random.default_rng(5)
    H = rng.standard_normal((1, 3, 3))
    h = 1e-30
    dsig = neo_hookean(1j * h * H, c)[0].imag / h
    assert np.allclose(dsig, stress_linear_elastic(H, c), rtol=1e-13, atol=1e-13 * c["mu"])


def test_plane_strain_embedding():
    """2-D neo-Hookean uses F_zz = 1: out-of-plane stress from the 3x3 law."""
    c = _consts()
    g2 = np.array([[[0.1, 0.02], [0.03, -0.05]]])
    g3 = np.zeros((1, 3, 3))
    g3[0, :2, :2] = g2[0]
    s2 = neo_hookean(g2, c)[0]
    s3 = neo_hookean(g3, c)[0]
    assert np.allclose(s2, s3)


# ---------------------------------------------------------------- St. Venant-Kirchhoff
from oracle.fv import st_venant_kirchhoff, traction  # noqa: E402


@pytest.mark.parametrize("s", [0.8, 1.0, 1.25, 1.6])
def test_st_venant_kirchhoff_uniaxial_stretch(s):
    """F = diag(s, 1, 1): E = diag((s^2 - 1)/2, 0, 0), S = 2 mu E + lam tr E I,
    sigma = F S F^T / J = diag(s S11, S22 / s, S33 / s) with J = s."""
    c = _consts("st_venant_kirchhoff", 5.6e6, 0.4)
    g = np.zeros((1, 3, 3))
    g[0, 0, 0] = s - 1.0
    sig, _ = st_venant_kirchhoff(g, c)
    E11 = 0.5 * (s * s - 1.0)
    S11 = (2 * c["mu"] + c["lam"]) * E11
    S22 = c["lam"] * E11
    assert np.allclose(np.diag(sig[0]), [s * S11, S22 / s, S22 / s], rtol=1e-13, atol=1e-6)
    assert np.allclose(sig[0] - np.diag(np.diag(sig[0])), 0.0, atol=1e-6)
    # the face force on the reference face with normal e_x is F S Gamma
    G = np.array([[2.0, 0.0, 0.0]])
    t = traction(g, G, c)[0]
    assert np.allclose(t, [s * S11 * 2.0, 0.0, 0.0], rtol=1e-13, atol=1e-6)


def test_st_venant_kirchhoff_objective_under_rotation():
    c = _consts("st_venant_kirchhoff", 5.6e6, 0.4)
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    g = (Q - np.eye(3)).T[None]       # F = I + g^T = Q
    sig, _ = st_venant_kirchhoff(g, c)
    assert np.abs(sig).max() <= 1e-9 * c["mu"]


def test_st_venant_kirchhoff_small_strain_limit():
    """d sigma / d(grad u) at grad u = 0 is Hooke's law (complex step)."""
    c = _consts("st_venant_kirchhoff", 5.6e6, 0.4)
    rng = np.random.default_rng(4)
    d = rng.standard_normal((1, 3, 3))
    h = 1e-30
    sig, _ = st_venant_kirchhoff(1j * h * d, c)
    lin = stress_linear_elastic(d, c)
    assert np.allclose(sig.imag / h, lin, rtol=1e-13, atol=1e-13 * np.abs(lin).max())
