"""Mie series far field of a perfectly conducting sphere.

Independent of the paper; it pins the discretised EFIE (Sec. 2) against the
exact solution.  Written for incidence x-polarised along +z, unit amplitude,
in the exp(+i w t) convention used by the Green's function of Sec. 2 (fields are
complex conjugates of the exp(-i w t) textbook forms, e.g. Bohren & Huffman).

Far field: e_s(r) ~ F(rhat) exp(-ikr)/r with
  F = (-i/k) [cos(phi) conj(S2) theta_hat - sin(phi) conj(S1) phi_hat],
  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
  S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n),
  a_n = psi_n'(x)/xi_n'(x), b_n = psi_n(x)/xi_n(x) (PEC limit),
  psi_n = x j_n(x), xi_n = x h_n^(1)(x), x = k a,
truncated at n_max = x + 4 x^(1/3) + 2 (Wiscombe 1980).
"""
import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def coefficients(x):
    nmax = int(math.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    n = np.arange(1, nmax + 1)
    jn = spherical_jn(n, x)
    jnp = spherical_jn(n, x, derivative=True)
    yn = spherical_yn(n, x)
    ynp = spherical_yn(n, x, derivative=True)
    hn = jn + 1j * yn
    hnp = jnp + 1j * ynp
    psi = x * jn
    psip = jn + x * jnp
    xi = x * hn
    xip = hn + x * hnp
    return n, psip / xip, psi / xi


def amplitudes(theta, x):
    """S1(theta), S2(theta) for a PEC sphere of size parameter x."""
    n, a, b = coefficients(x)
    mu = np.cos(theta)
    S1 = np.zeros(len(mu), dtype=np.complex128)
    S2 = np.zeros(len(mu), dtype=np.complex128)
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    for i, nn in enumerate(n):
        if nn > 1:
            pi_new = ((2 * nn - 1) / (nn - 1)) * mu * pi_cur - (nn / (nn - 1)) * pi_prev
            pi_prev, pi_cur = pi_cur, pi_new
        tau = nn * mu * pi_cur - (nn + 1) * pi_prev
        f = (2 * nn + 1) / (nn * (nn + 1))
        S1 += f * (a[i] * pi_cur + b[i] * tau)
        S2 += f * (a[i] * tau + b[i] * pi_cur)
    return S1, S2


def far_field(theta, phi, radius, k=2.0 * math.pi):
    """Cartesian far-field vectors F at directions (theta, phi): [n, 3]."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    phi = np.broadcast_to(np.asarray(phi, dtype=np.float64), theta.shape)
    S1, S2 = amplitudes(theta, k * radius)
    th_hat = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], 1)
    ph_hat = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], 1)
    Fth = (-1j / k) * np.cos(phi) * np.conj(S2)
    Fph = (-1j / k) * (-np.sin(phi)) * np.conj(S1)
    return Fth[:, None] * th_hat + Fph[:, None] * ph_hat
