"""Closed-form stress and displacement around a spherical cavity of radius a
in an infinite linear-elastic solid under remote uniaxial tension T along z
(Appendix G: the stress in cylindrical coordinates, rotated to Cartesian;
the displacement in spherical coordinates plus the uniform uniaxial field).
Test helper: the reference for the spherical-cavity verification."""

import numpy as np


def stress(x, T, nu, a):
    """Cartesian stress [n, 3, 3] at points x [n, 3]."""
    x = np.asarray(x, dtype=np.float64)
    r2 = x[:, 0] ** 2 + x[:, 1] ** 2
    R2 = r2 + x[:, 2] ** 2
    R = np.sqrt(R2)
    r = np.sqrt(r2)
    q = a * a / R2                   # a^2 / R^2
    s = r2 / R2                      # r^2 / R^2
    k = T / (14.0 - 10.0 * nu) * (a / R) ** 3
    srr = k * (9 - 15 * nu - 12 * q - s * (72 - 15 * nu - 105 * q) + 15 * s * s * (5 - 7 * q))
    stt = k * (9 - 15 * nu - 12 * q - 15 * s * (1 - 2 * nu - q))
    szz = T - k * (38 - 10 * nu - 24 * q - s * (117 - 15 * nu - 120 * q) + 15 * s * s * (5 - 7 * q))
    szr = T / (14.0 - 10.0 * nu) * a ** 3 * x[:, 2] * r / R ** 5 * \
        (-3 * (19 - 5 * nu) + 60 * q + 15 * s * (5 - 7 * q))
    th = np.arctan2(x[:, 1], x[:, 0])
    c, sn = np.cos(th), np.sin(th)
    out = np.zeros((x.shape[0], 3, 3))
    out[:, 0, 0] = srr * c * c + stt * sn * sn
    out[:, 1, 1] = srr * sn * sn + stt * c * c
    out[:, 0, 1] = out[:, 1, 0] = (srr - stt) * sn * c
    out[:, 0, 2] = out[:, 2, 0] = szr * c
    out[:, 1, 2] = out[:, 2, 1] = szr * sn
    out[:, 2, 2] = szz
    return out


def displacement(x, T, E, nu, a):
    """Cartesian displacement [n, 3] at points x [n, 3]."""
    x = np.asarray(x, dtype=np.float64)
    mu = E / (2.0 * (1.0 + nu))
    A = -a ** 3 * T / (8 * mu) * (13 - 10 * nu) / (7 - 5 * nu)
    B = a ** 5 * T / (8 * mu) / (7 - 5 * nu)
    C = a ** 3 * T / (8 * mu) * 5 * (1 - 2 * nu) / (7 - 5 * nu)
    R = np.linalg.norm(x, axis=1)
    th = np.arccos(np.clip(x[:, 2] / R, -1.0, 1.0))      # polar angle from z
    ph = np.arctan2(x[:, 1], x[:, 0])
    uR = -A / R ** 2 - 3 * B / R ** 4 + ((5 - 4 * nu) / (1 - 2 * nu) * C / R ** 2 - 9 * B / R ** 4) * np.cos(2 * th)
    ut = -(2 * C / R ** 2 + 6 * B / R ** 4) * np.sin(2 * th)
    u = np.zeros_like(x)
    u[:, 0] = uR * np.sin(th) * np.cos(ph) + ut * np.cos(th) * np.cos(ph)
    u[:, 1] = uR * np.sin(th) * np.sin(ph) + ut * np.cos(th) * np.sin(ph)
    u[:, 2] = uR * np.cos(th) - ut * np.sin(th)
    u[:, 0] += -nu * T / E * x[:, 0]
    u[:, 1] += -nu * T / E * x[:, 1]
    u[:, 2] += T / E * x[:, 2]
    return u
