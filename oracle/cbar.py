"""Closed-form envelope-speed bound of Sec. 4.1 (TEST INFRASTRUCTURE ONLY).

Sec. 4.1 reduces the constant-sensitivity system (eq. velo-system) with
n + b = n0 (eq. mass-conser) to a Fisher-type scalar equation with effective
diffusivity D~(b) = n0 b (1 - b/n0)(1 + chi0 b) (eq. D-tilde) and reaction
g(b) = n0 b (1 - b/n0) (eq. reac-term).  The Malaguti-Marcelli threshold is
bounded by

    cbar(n0, chi0) = 2 sqrt( sup_b  sigma0 D~(b) g(b) / b )
                   = 2 n0 sqrt(sigma0) sqrt( max_{0<=b<=n0} psi(b) ),
    psi(b) = b (1 - b/n0)^2 (1 + chi0 b),

maximised at the root b* of psi'(b) = 0 in (0, n0) (eq. c-bar-chi0); for
chi0 = 0 the maximiser is n0/3 and cbar = 4/(3 sqrt 3) n0^(3/2) sigma0^(1/2)
(eq. c-bar-0).

Reading taken: the printed expression for b* is algebraically the positive
root of 4 chi0 b^2 + (3 - 2 chi0 n0) b - n0 = 0 (the quadratic factor of
psi'); it is evaluated here in the cancellation-free form
b* = 2 n0 / (p + sqrt(p^2 + 16 chi0 n0)), p = 3 - 2 chi0 n0, which is the
same number and reduces to n0/3 at chi0 = 0.  The paper's "psi(b*)" in
eq. c-bar-chi0 is read as psi~(b*) (the chi0-dependent function), and the
sigma^(1/2) of eq. c-bar-0 as sigma0^(1/2).
"""
import math


def psi(b, n0, chi):
    """psi~(b) = b (1 - b/n0)^2 (1 + chi b)."""
    return b * (1.0 - b / n0) ** 2 * (1.0 + chi * b)


def bstar(n0, chi):
    """Maximiser of psi~ on [0, n0]."""
    p = 3.0 - 2.0 * chi * n0
    return 2.0 * n0 / (p + math.sqrt(p * p + 16.0 * chi * n0))


def cbar(n0, chi, sigma0=1.0):
    """Speed bound cbar(n0, chi0) of eq. c-bar-chi0 (eq. c-bar-0 when chi0 = 0)."""
    return 2.0 * n0 * math.sqrt(sigma0) * math.sqrt(psi(bstar(n0, chi), n0, chi))
