"""Series solution for a TE plane wave on a homogeneous circular cylinder.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper checks its discretisation against "the analytical solution for a
homogeneous circular cylinder" (Section 4, grid rule) without writing it out.
This is the textbook separation-of-variables series in the paper's setting:
time factor exp(-i omega t), so H^(1) is outgoing (eq. GreenFunction);
TE Maxwell equations (eq. MaxwellTE) with J = 0 give

    E1 = -d2 H3 / (i omega eps),   E2 = d1 H3 / (i omega eps).

Incident H3 = exp(i k (x cos psi + y sin psi)) = sum_n i^n J_n(k r) e^{i n (phi - psi)}.
Outside: H3 = sum_n i^n [J_n(k r) + a_n H_n(k r)] e^{i n (phi - psi)};
inside:  H3 = sum_n i^n c_n J_n(k1 r) e^{i n (phi - psi)},  k1 = k sqrt(eps).
Continuity of H3 and of (1/eps) dH3/dr (tangential E) at r = R fixes a_n, c_n.
Units: eps_b = mu_b = 1, k = omega.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import jv, jvp, hankel1, h1vp


def coefficients(k: float, radius: float, eps: complex, nmax: int):
    """(n, a_n, c_n) for n = -nmax..nmax (Cramer's rule on the two interface conditions)."""
    n = np.arange(-nmax, nmax + 1)
    s = np.sqrt(complex(eps))
    k1 = k * s
    x, x1 = k * radius, k1 * radius
    J, Jp = jv(n, x), jvp(n, x)
    H, Hp = hankel1(n, x), h1vp(n, x)
    J1, J1p = jv(n, x1), jvp(n, x1)
    # H a - J1 c = -J ;  H' a - (J1'/s) c = -J'
    det = J1 * Hp - H * J1p / s
    a = (J * J1p / s - J1 * Jp) / det
    c = (J * Hp - H * Jp) / det
    return n, a, c


def _grad_cyl(n, coef, Zm1, Zp1, kap, phi, psi):
    """Gradient of sum_n coef_n Z_n(kap r) e^{i n (phi - psi)} via the recurrences
    (d1 + i d2)[Z_n e^{i n phi}] = -kap Z_{n+1} e^{i (n+1) phi},
    (d1 - i d2)[Z_n e^{i n phi}] =  kap Z_{n-1} e^{i (n-1) phi}."""
    e = np.exp(-1j * n * psi)[:, None]
    plus = -kap * (coef[:, None] * e * Zp1 * np.exp(1j * (n[:, None] + 1) * phi[None, :])).sum(0)
    minus = kap * (coef[:, None] * e * Zm1 * np.exp(1j * (n[:, None] - 1) * phi[None, :])).sum(0)
    d1 = 0.5 * (plus + minus)
    d2 = (plus - minus) / 2j
    return d1, d2


def total_field(x: np.ndarray, y: np.ndarray, k: float, radius: float, eps: complex,
                psi: float = 0.0, nmax: int | None = None) -> np.ndarray:
    """Total in-plane E (shape [2, *x.shape]) at the points (x, y)."""
    if nmax is None:
        nmax = int(math.ceil(k * abs(np.sqrt(complex(eps))) * radius)) + 20
    n, a, c = coefficients(k, radius, eps, nmax)
    shape = np.shape(x)
    xf, yf = np.ravel(x), np.ravel(y)
    r = np.hypot(xf, yf)
    phi = np.arctan2(yf, xf)
    inside = r <= radius
    E = np.zeros((2, xf.size), dtype=np.complex128)
    pref = (1j ** n).astype(np.complex128)
    omega = k
    if np.any(~inside):
        ro, po = r[~inside], phi[~inside]
        z = k * ro
        ns = n[:, None]
        Jm1, Jp1 = jv(ns - 1, z[None]), jv(ns + 1, z[None])
        Hm1, Hp1 = hankel1(ns - 1, z[None]), hankel1(ns + 1, z[None])
        g1a, g2a = _grad_cyl(n, pref, Jm1, Jp1, k, po, psi)
        g1b, g2b = _grad_cyl(n, pref * a, Hm1, Hp1, k, po, psi)
        d1, d2 = g1a + g1b, g2a + g2b
        E[0, ~inside] = -d2 / (1j * omega * 1.0)
        E[1, ~inside] = d1 / (1j * omega * 1.0)
    if np.any(inside):
        ri, pi_ = r[inside], phi[inside]
        k1 = k * np.sqrt(complex(eps))
        z = k1 * ri
        ns = n[:, None]
        Jm1, Jp1 = jv(ns - 1, z[None]), jv(ns + 1, z[None])
        d1, d2 = _grad_cyl(n, pref * c, Jm1, Jp1, k1, pi_, psi)
        E[0, inside] = -d2 / (1j * omega * eps)
        E[1, inside] = d1 / (1j * omega * eps)
    return E.reshape((2,) + shape)


def incident_field(x, y, k: float, psi: float = 0.0) -> np.ndarray:
    """Incident E from its own series (same recurrences, no scatterer): checks the
    series machinery against the closed-form plane wave."""
    nmax = int(math.ceil(k * float(np.max(np.hypot(x, y))))) + 25
    n = np.arange(-nmax, nmax + 1)
    xf, yf = np.ravel(x), np.ravel(y)
    r = np.hypot(xf, yf)
    phi = np.arctan2(yf, xf)
    z = k * r
    ns = n[:, None]
    d1, d2 = _grad_cyl(n, (1j ** n).astype(np.complex128), jv(ns - 1, z[None]), jv(ns + 1, z[None]), k, phi, psi)
    E = np.stack([-d2 / (1j * k), d1 / (1j * k)])
    return E.reshape((2,) + np.shape(x))


# ---------------------------------------------------------------- generalisations
# Magnetic contrast (TE, eq. MaxwellTE with mu != mu_b) and the TM polarisation
# (eq. MaxwellTM).  With k1 = k sqrt(eps mu) inside:
#   TE: H3 continuous, (1/eps) dH3/dr continuous (tangential E);
#   TM: E3 continuous, (1/mu) dE3/dr continuous (tangential H).
# Both are "field continuous, (1/p) d/dr field continuous" with p = eps (TE) or mu (TM).


def coefficients_general(k: float, radius: float, eps: complex, mu: complex, nmax: int, pol: str):
    """(n, a_n, c_n) of the field F = H3 (pol 'te') or E3 (pol 'tm'):
    outside sum i^n [J_n(k r) + a_n H_n(k r)] e^{i n (phi - psi)}, inside sum i^n c_n J_n(k1 r) ..."""
    n = np.arange(-nmax, nmax + 1)
    k1 = k * np.sqrt(complex(eps) * complex(mu))
    p = complex(eps) if pol == "te" else complex(mu)
    f = (k1 / k) / p  # (1/p) d/dr of J_n(k1 r) relative to d/dr of the outside terms
    x, x1 = k * radius, k1 * radius
    J, Jp = jv(n, x), jvp(n, x)
    H, Hp = hankel1(n, x), h1vp(n, x)
    J1, J1p = jv(n, x1), jvp(n, x1)
    # H a - J1 c = -J ;  H' a - f J1' c = -J'
    det = J1 * Hp - H * J1p * f
    a = (J * J1p * f - J1 * Jp) / det
    c = (J * Hp - H * Jp) / det
    return n, a, c


def _series(x, y, k, radius, eps, mu, psi, pol, nmax):
    if nmax is None:
        nmax = int(math.ceil(k * abs(np.sqrt(complex(eps) * complex(mu))) * radius)) + 20
    n, a, c = coefficients_general(k, radius, eps, mu, nmax, pol)
    xf, yf = np.ravel(x), np.ravel(y)
    r = np.hypot(xf, yf)
    phi = np.arctan2(yf, xf)
    inside = r <= radius
    k1 = k * np.sqrt(complex(eps) * complex(mu))
    pref = (1j ** n).astype(np.complex128)
    F = np.zeros(xf.size, dtype=np.complex128)
    d1 = np.zeros(xf.size, dtype=np.complex128)
    d2 = np.zeros(xf.size, dtype=np.complex128)
    ns = n[:, None]
    e = np.exp(1j * n[:, None] * (phi[None, :] - psi))
    if np.any(~inside):
        ro, po = r[~inside], phi[~inside]
        z = k * ro
        F[~inside] = (pref[:, None] * (jv(ns, z[None]) + a[:, None] * hankel1(ns, z[None])) * e[:, ~inside]).sum(0)
        g1a, g2a = _grad_cyl(n, pref, jv(ns - 1, z[None]), jv(ns + 1, z[None]), k, po, psi)
        g1b, g2b = _grad_cyl(n, pref * a, hankel1(ns - 1, z[None]), hankel1(ns + 1, z[None]), k, po, psi)
        d1[~inside], d2[~inside] = g1a + g1b, g2a + g2b
    if np.any(inside):
        ri, pi_ = r[inside], phi[inside]
        z = k1 * ri
        F[inside] = (pref[:, None] * c[:, None] * jv(ns, z[None]) * e[:, inside]).sum(0)
        d1[inside], d2[inside] = _grad_cyl(n, pref * c, jv(ns - 1, z[None]), jv(ns + 1, z[None]), k1, pi_, psi)
    return F, d1, d2, inside


def te_fields(x, y, k: float, radius: float, eps: complex, mu: complex = 1.0, psi: float = 0.0,
              nmax: int | None = None) -> np.ndarray:
    """[E1, E2, H3] (shape [3, *x.shape]) for the TE plane wave H3_in = exp(i k (x cos psi + y sin psi))
    on a homogeneous magneto-dielectric cylinder: E1 = -d2 H3 / (i omega eps), E2 = d1 H3 / (i omega eps)
    with the local eps (eq. MaxwellTE with J = 0, omega = k)."""
    H3, d1, d2, inside = _series(x, y, k, radius, eps, mu, psi, "te", nmax)
    epsl = np.where(inside, complex(eps), 1.0)
    out = np.stack([-d2 / (1j * k * epsl), d1 / (1j * k * epsl), H3])
    return out.reshape((3,) + np.shape(x))


def tm_field(x, y, k: float, radius: float, eps: complex, mu: complex = 1.0, psi: float = 0.0,
             nmax: int | None = None) -> np.ndarray:
    """E3 for the TM plane wave E3_in = exp(i k (x cos psi + y sin psi)) on a homogeneous cylinder."""
    E3, _, _, _ = _series(x, y, k, radius, eps, mu, psi, "tm", nmax)
    return E3.reshape(np.shape(x))


def interface_jumps(k: float, radius: float, eps: complex, mu: complex, psi: float, pol: str, m: int = 64):
    """Largest jumps, across r = radius, of the field and of (1/p) dF/dr (p = eps for TE, mu for TM),
    evaluated from the series just inside and just outside (central differences in r)."""
    phi = np.linspace(0, 2 * np.pi, m, endpoint=False)
    d = 1e-6 * radius

    def field(r):
        x, y = r * np.cos(phi), r * np.sin(phi)
        F, _, _, _ = _series(x, y, k, radius, eps, mu, psi, pol, None)
        return F

    p = complex(eps) if pol == "te" else complex(mu)
    Fo, Fi = field(radius * (1 + 1e-12) + d), field(radius * (1 - 1e-12) - d)
    dFo = (field(radius + 2 * d) - field(radius + d)) / d
    dFi = (field(radius - d) - field(radius - 2 * d)) / d / p
    return float(np.max(np.abs(Fo - Fi)) / np.max(np.abs(Fo))), float(np.max(np.abs(dFo - dFi)) / np.max(np.abs(dFo)))
