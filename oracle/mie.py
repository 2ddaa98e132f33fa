"""Mie series for a homogeneous dielectric sphere (textbook closed form,
Bohren & Huffman 1983, ch. 4), used to pin the whole MoM chain.

The textbook uses e^{-iwt}; the paper e^{jwt}.  A lossy eps_r = e' - j e''
of the paper is the refractive index m = conj(sqrt(eps_r)) in the textbook.
Scattering angle is measured from the propagation direction.  For an
incident wave polarised along x, the bistatic RCS in the E-plane
(containing the polarisation) is 4 pi |S2|^2 / k^2 and in the H-plane
4 pi |S1|^2 / k^2.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def _psi(n, z):
    return z * spherical_jn(n, z)


def _dpsi(n, z):
    return spherical_jn(n, z) + z * spherical_jn(n, z, derivative=True)


def coefficients(x, m, nmax=None):
    """a_n, b_n (n = 1..nmax) for size parameter x = k a and relative index m
    (mu = 1)."""
    if nmax is None:
        nmax = int(np.ceil(x + 4 * x ** (1 / 3) + 2))
    n = np.arange(1, nmax + 1)
    mx = m * x
    psi_x, dpsi_x = _psi(n, x), _dpsi(n, x)
    xi_x = x * (spherical_jn(n, x) + 1j * spherical_yn(n, x))
    dxi_x = (spherical_jn(n, x) + 1j * spherical_yn(n, x)) + x * (
        spherical_jn(n, x, derivative=True) + 1j * spherical_yn(n, x, derivative=True))
    psi_m, dpsi_m = _psi(n, mx), _dpsi(n, mx)
    a = (m * psi_m * dpsi_x - psi_x * dpsi_m) / (m * psi_m * dxi_x - xi_x * dpsi_m)
    b = (psi_m * dpsi_x - m * psi_x * dpsi_m) / (psi_m * dxi_x - m * xi_x * dpsi_m)
    return a, b


def amplitudes(x, m, theta):
    """Scattering amplitudes S1, S2 at scattering angles ``theta`` (rad)."""
    a, b = coefficients(x, m)
    nmax = len(a)
    mu = np.cos(np.atleast_1d(theta))
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    S1 = np.zeros(mu.shape, dtype=np.complex128)
    S2 = np.zeros(mu.shape, dtype=np.complex128)
    for n in range(1, nmax + 1):
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        c = (2 * n + 1) / (n * (n + 1))
        S1 += c * (a[n - 1] * pi_cur + b[n - 1] * tau)
        S2 += c * (a[n - 1] * tau + b[n - 1] * pi_cur)
        pi_prev, pi_cur = pi_cur, ((2 * n + 1) * mu * pi_cur - (n + 1) * pi_prev) / n
    return S1, S2


def bistatic_rcs(radius, k0, eps_r, theta_s):
    """(sigma_E, sigma_H) in wavelength^2 units (k0 = 2 pi / lambda0) for the
    E-plane and H-plane cuts at scattering angles ``theta_s``."""
    m = np.conj(np.sqrt(complex(eps_r)))
    S1, S2 = amplitudes(k0 * radius, m, theta_s)
    return 4 * np.pi * np.abs(S2) ** 2 / k0 ** 2, 4 * np.pi * np.abs(S1) ** 2 / k0 ** 2
