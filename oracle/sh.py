"""Real spherical harmonics in FP64 (torch, differentiable) -- TEST INFRASTRUCTURE ONLY.

View-dependent colour uses spherical harmonics (Sec. II, scene
representations).  The basis is the orthonormal real SH basis written from its
definition, with the Condon-Shortley phase kept in the associated Legendre
functions:

  Y_l0  = K_l^0 P_l^0(cos t)
  Y_lm  = sqrt(2) K_l^m P_l^m(cos t) cos(m p)      (m > 0)
  Y_l-m = sqrt(2) K_l^m P_l^m(cos t) sin(m p)      (m > 0)
  K_l^m = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!)

for a unit direction (x, y, z) = (sin t cos p, sin t sin p, cos t).  Using
P_l^m(z) = (-1)^m (1-z^2)^(m/2) d^m P_l/dz^m and
sin^m t (cos mp, sin mp) = (Re, Im) (x + i y)^m, each term is a polynomial in
(x, y, z), which keeps the derivative finite at the poles.  Basis index
k = l^2 + l + m; colour = max(0, sum_k c_k Y_k(d) + 1/2).
"""
from __future__ import annotations

import math

import torch


def _dfact(n: int) -> int:
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def _K(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def _legendre_derivs(z: torch.Tensor, L: int):
    """Q[l][m](z) = d^m P_l / dz^m for 0 <= m <= l <= L, by the standard recurrences.

    Q_mm = (2m-1)!!, Q_{m+1,m} = (2m+1) z Q_mm,
    (l-m) Q_lm = (2l-1) z Q_{l-1,m} - (l+m-1) Q_{l-2,m}.
    """
    Q = [[None] * (L + 1) for _ in range(L + 1)]
    one = torch.ones_like(z)
    for m in range(L + 1):
        Q[m][m] = one * float(_dfact(2 * m - 1))
        if m + 1 <= L:
            Q[m + 1][m] = (2 * m + 1) * z * Q[m][m]
        for l in range(m + 2, L + 1):
            Q[l][m] = ((2 * l - 1) * z * Q[l - 1][m] - (l + m - 1) * Q[l - 2][m]) / (l - m)
    return Q


def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Real SH basis [(degree+1)^2, N] for unit directions d [3, N]."""
    x, y, z = d[0], d[1], d[2]
    Q = _legendre_derivs(z, degree)
    A = [torch.ones_like(x)]
    B = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        A.append(x * A[m - 1] - y * B[m - 1])
        B.append(x * B[m - 1] + y * A[m - 1])
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            p = ((-1) ** am) * Q[l][am]
            if m == 0:
                out.append(_K(l, 0) * p)
            elif m > 0:
                out.append(math.sqrt(2.0) * _K(l, am) * p * A[am])
            else:
                out.append(math.sqrt(2.0) * _K(l, am) * p * B[am])
    return torch.stack(out)


def sh_colour(coeffs: torch.Tensor, d: torch.Tensor, degree: int) -> torch.Tensor:
    """RGB [3, N] = max(0, sum_k c[k*3+ch] Y_k(d) + 0.5); coeffs [(degree+1)^2 * 3, N]."""
    nb = (degree + 1) ** 2
    Y = sh_basis(d, degree)  # [nb, N]
    c = coeffs[: nb * 3].reshape(nb, 3, -1)
    raw = (c * Y[:, None, :]).sum(0) + 0.5
    return torch.clamp(raw, min=0.0)
