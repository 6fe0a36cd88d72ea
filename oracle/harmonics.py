"""Real spherical harmonics in Cartesian form (paper, Appendix B) and the
addition-theorem coefficients C_lm used by the 3-body descriptor (Eq. 7).

TEST INFRASTRUCTURE ONLY: this package is the FP64 reference that the GPU
library is checked against.  Only tests, the smoke check and the CPU-baseline
leg of the benchmark may import it.

b_lm(x, y, z) is the table of Appendix B (B1.1-B8.17), written with
r2 = x^2 + y^2 + z^2.  The descriptor uses B_lm = b_lm / r^l (B9.1), a
function of the direction only.
"""
from __future__ import annotations

import math

import numpy as np

# Appendix B, one entry per (l, m), m = 0..2l, in the paper's order.
B_TABLE = {
    1: [
        lambda x, y, z, r2: z,                                   # B1.1
        lambda x, y, z, r2: x,                                   # B1.2
        lambda x, y, z, r2: y,                                   # B1.3
    ],
    2: [
        lambda x, y, z, r2: 3 * z * z - r2,                      # B2.1
        lambda x, y, z, r2: x * z,                               # B2.2
        lambda x, y, z, r2: y * z,                               # B2.3
        lambda x, y, z, r2: x * x - y * y,                       # B2.4
        lambda x, y, z, r2: 2 * x * y,                           # B2.5
    ],
    3: [
        lambda x, y, z, r2: 5 * z ** 3 - 3 * z * r2,             # B3.1
        lambda x, y, z, r2: (5 * z * z - r2) * x,                # B3.2
        lambda x, y, z, r2: (5 * z * z - r2) * y,                # B3.3
        lambda x, y, z, r2: (x * x - y * y) * z,                 # B3.4
        lambda x, y, z, r2: 2 * x * y * z,                       # B3.5
        lambda x, y, z, r2: (x * x - 3 * y * y) * x,             # B3.6
        lambda x, y, z, r2: (3 * x * x - y * y) * y,             # B3.7
    ],
    4: [
        lambda x, y, z, r2: 35 * z ** 4 - 30 * z * z * r2 + 3 * r2 * r2,          # B4.1
        lambda x, y, z, r2: (7 * z ** 3 - 3 * z * r2) * x,                        # B4.2
        lambda x, y, z, r2: (7 * z ** 3 - 3 * z * r2) * y,                        # B4.3
        lambda x, y, z, r2: (7 * z * z - r2) * (x * x - y * y),                   # B4.4
        lambda x, y, z, r2: (7 * z * z - r2) * 2 * x * y,                         # B4.5
        lambda x, y, z, r2: (x ** 3 - 3 * x * y * y) * z,                         # B4.6
        lambda x, y, z, r2: (3 * x * x * y - y ** 3) * z,                         # B4.7
        lambda x, y, z, r2: x ** 4 - 6 * x * x * y * y + y ** 4,                  # B4.8
        lambda x, y, z, r2: 4 * x ** 3 * y - 4 * x * y ** 3,                      # B4.9
    ],
    5: [
        lambda x, y, z, r2: 63 * z ** 5 - 70 * z ** 3 * r2 + 15 * z * r2 * r2,                   # B5.1
        lambda x, y, z, r2: (21 * z ** 4 - 14 * z * z * r2 + r2 * r2) * x,                       # B5.2
        lambda x, y, z, r2: (21 * z ** 4 - 14 * z * z * r2 + r2 * r2) * y,                       # B5.3
        lambda x, y, z, r2: (3 * z ** 3 - z * r2) * (x * x - y * y),                             # B5.4
        lambda x, y, z, r2: (3 * z ** 3 - z * r2) * 2 * x * y,                                   # B5.5
        lambda x, y, z, r2: (9 * z * z - r2) * (x ** 3 - 3 * x * y * y),                         # B5.6
        lambda x, y, z, r2: (9 * z * z - r2) * (3 * x * x * y - y ** 3),                         # B5.7
        lambda x, y, z, r2: z * (x ** 4 - 6 * x * x * y * y + y ** 4),                           # B5.8
        lambda x, y, z, r2: z * (4 * x ** 3 * y - 4 * x * y ** 3),                               # B5.9
        lambda x, y, z, r2: x ** 5 - 10 * x ** 3 * y * y + 5 * x * y ** 4,                       # B5.10
        lambda x, y, z, r2: 5 * x ** 4 * y - 10 * x * x * y ** 3 + y ** 5,                       # B5.11
    ],
    6: [
        lambda x, y, z, r2: 231 * z ** 6 - 315 * z ** 4 * r2 + 105 * z * z * r2 ** 2 - 5 * r2 ** 3,   # B6.1
        lambda x, y, z, r2: (33 * z ** 5 - 30 * z ** 3 * r2 + 5 * z * r2 ** 2) * x,                  # B6.2
        lambda x, y, z, r2: (33 * z ** 5 - 30 * z ** 3 * r2 + 5 * z * r2 ** 2) * y,                  # B6.3
        lambda x, y, z, r2: (33 * z ** 4 - 18 * z * z * r2 + r2 ** 2) * (x * x - y * y),             # B6.4
        lambda x, y, z, r2: (33 * z ** 4 - 18 * z * z * r2 + r2 ** 2) * 2 * x * y,                   # B6.5
        lambda x, y, z, r2: (11 * z ** 3 - 3 * z * r2) * (x ** 3 - 3 * x * y * y),                   # B6.6
        lambda x, y, z, r2: (11 * z ** 3 - 3 * z * r2) * (3 * x * x * y - y ** 3),                   # B6.7
        lambda x, y, z, r2: (11 * z * z - r2) * (x ** 4 - 6 * x * x * y * y + y ** 4),               # B6.8
        lambda x, y, z, r2: (11 * z * z - r2) * (4 * x ** 3 * y - 4 * x * y ** 3),                   # B6.9
        lambda x, y, z, r2: z * (x ** 5 - 10 * x ** 3 * y * y + 5 * x * y ** 4),                     # B6.10
        lambda x, y, z, r2: z * (5 * x ** 4 * y - 10 * x * x * y ** 3 + y ** 5),                     # B6.11
        lambda x, y, z, r2: x ** 6 - 15 * x ** 4 * y * y + 15 * x * x * y ** 4 - y ** 6,             # B6.12
        lambda x, y, z, r2: 6 * x ** 5 * y - 20 * x ** 3 * y ** 3 + 6 * x * y ** 5,                  # B6.13
    ],
    7: [
        lambda x, y, z, r2: 429 * z ** 7 - 693 * z ** 5 * r2 + 315 * z ** 3 * r2 ** 2 - 35 * z * r2 ** 3,    # B7.1
        lambda x, y, z, r2: (429 * z ** 6 - 495 * z ** 4 * r2 + 135 * z * z * r2 ** 2 - 5 * r2 ** 3) * x,   # B7.2
        lambda x, y, z, r2: (429 * z ** 6 - 495 * z ** 4 * r2 + 135 * z * z * r2 ** 2 - 5 * r2 ** 3) * y,   # B7.3
        lambda x, y, z, r2: (143 * z ** 5 - 110 * z ** 3 * r2 + 15 * z * r2 ** 2) * (x * x - y * y),        # B7.4
        lambda x, y, z, r2: (143 * z ** 5 - 110 * z ** 3 * r2 + 15 * z * r2 ** 2) * 2 * x * y,              # B7.5
        lambda x, y, z, r2: (143 * z ** 4 - 66 * z * z * r2 + 3 * r2 ** 2) * (x ** 3 - 3 * x * y * y),      # B7.6
        lambda x, y, z, r2: (143 * z ** 4 - 66 * z * z * r2 + 3 * r2 ** 2) * (3 * x * x * y - y ** 3),      # B7.7
        lambda x, y, z, r2: (13 * z ** 3 - 3 * z * r2) * (x ** 4 - 6 * x * x * y * y + y ** 4),             # B7.8
        lambda x, y, z, r2: (13 * z ** 3 - 3 * z * r2) * (4 * x ** 3 * y - 4 * x * y ** 3),                 # B7.9
        lambda x, y, z, r2: (13 * z * z - r2) * (x ** 5 - 10 * x ** 3 * y * y + 5 * x * y ** 4),            # B7.10
        lambda x, y, z, r2: (13 * z * z - r2) * (5 * x ** 4 * y - 10 * x * x * y ** 3 + y ** 5),            # B7.11
        lambda x, y, z, r2: z * (x ** 6 - 15 * x ** 4 * y * y + 15 * x * x * y ** 4 - y ** 6),              # B7.12
        lambda x, y, z, r2: z * (6 * x ** 5 * y - 20 * x ** 3 * y ** 3 + 6 * x * y ** 5),                   # B7.13
        lambda x, y, z, r2: x ** 7 - 21 * x ** 5 * y * y + 35 * x ** 3 * y ** 4 - 7 * x * y ** 6,           # B7.14
        lambda x, y, z, r2: 7 * x ** 6 * y - 35 * x ** 4 * y ** 3 + 21 * x * x * y ** 5 - y ** 7,           # B7.15
    ],
    8: [
        lambda x, y, z, r2: (6435 * z ** 8 - 12012 * z ** 6 * r2 + 6930 * z ** 4 * r2 ** 2
                             - 1260 * z * z * r2 ** 3 + 35 * r2 ** 4),                                       # B8.1
        lambda x, y, z, r2: (715 * z ** 7 - 1001 * z ** 5 * r2 + 385 * z ** 3 * r2 ** 2 - 35 * z * r2 ** 3) * x,  # B8.2
        lambda x, y, z, r2: (715 * z ** 7 - 1001 * z ** 5 * r2 + 385 * z ** 3 * r2 ** 2 - 35 * z * r2 ** 3) * y,  # B8.3
        lambda x, y, z, r2: (143 * z ** 6 - 143 * z ** 4 * r2 + 33 * z * z * r2 ** 2 - r2 ** 3) * (x * x - y * y),  # B8.4
        lambda x, y, z, r2: (143 * z ** 6 - 143 * z ** 4 * r2 + 33 * z * z * r2 ** 2 - r2 ** 3) * 2 * x * y,        # B8.5
        lambda x, y, z, r2: (39 * z ** 5 - 26 * z ** 3 * r2 + 3 * z * r2 ** 2) * (x ** 3 - 3 * x * y * y),          # B8.6
        lambda x, y, z, r2: (39 * z ** 5 - 26 * z ** 3 * r2 + 3 * z * r2 ** 2) * (3 * x * x * y - y ** 3),          # B8.7
        lambda x, y, z, r2: (65 * z ** 4 - 26 * z * z * r2 + r2 ** 2) * (x ** 4 - 6 * x * x * y * y + y ** 4),      # B8.8
        lambda x, y, z, r2: (65 * z ** 4 - 26 * z * z * r2 + r2 ** 2) * (4 * x ** 3 * y - 4 * x * y ** 3),          # B8.9
        lambda x, y, z, r2: (5 * z ** 3 - z * r2) * (x ** 5 - 10 * x ** 3 * y * y + 5 * x * y ** 4),                # B8.10
        lambda x, y, z, r2: (5 * z ** 3 - z * r2) * (5 * x ** 4 * y - 10 * x * x * y ** 3 + y ** 5),                # B8.11
        lambda x, y, z, r2: (15 * z * z - r2) * (x ** 6 - 15 * x ** 4 * y * y + 15 * x * x * y ** 4 - y ** 6),     # B8.12
        lambda x, y, z, r2: (15 * z * z - r2) * (6 * x ** 5 * y - 20 * x ** 3 * y ** 3 + 6 * x * y ** 5),          # B8.13
        lambda x, y, z, r2: z * (x ** 7 - 21 * x ** 5 * y * y + 35 * x ** 3 * y ** 4 - 7 * x * y ** 6),             # B8.14
        lambda x, y, z, r2: z * (7 * x ** 6 * y - 35 * x ** 4 * y ** 3 + 21 * x * x * y ** 5 - y ** 7),             # B8.15
        lambda x, y, z, r2: x ** 8 - 28 * x ** 6 * y * y + 70 * x ** 4 * y ** 4 - 28 * x * x * y ** 6 + y ** 8,     # B8.16
        lambda x, y, z, r2: 8 * x ** 7 * y - 56 * x ** 5 * y ** 3 + 56 * x ** 3 * y ** 5 - 8 * x * y ** 7,         # B8.17
    ],
}

LMAX_TABLE = 8


def n_harmonics(lmax: int) -> int:
    """Number of (l, m) with 1 <= l <= lmax."""
    return lmax * (lmax + 2)


def harmonic_index(l: int, m: int) -> int:
    """Position of (l, m) in the flattened l-major list (l from 1)."""
    return (l - 1) * (l + 1) + m


def b_poly(l: int, m: int, x, y, z):
    """b_lm evaluated on arrays/tensors x, y, z (Appendix B)."""
    return B_TABLE[l][m](x, y, z, x * x + y * y + z * z)


def B_dir(lmax: int, d):
    """B_lm = b_lm(d) / |d|^l for 1 <= l <= lmax (B9.1), stacked on the last
    axis in l-major order.  `d` is a torch tensor [..., 3]."""
    import torch
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    r2 = x * x + y * y + z * z
    r = torch.sqrt(r2)
    out = []
    for l in range(1, lmax + 1):
        rl = r ** l
        for m in range(2 * l + 1):
            out.append(B_TABLE[l][m](x, y, z, r2) / rl)
    return torch.stack(out, -1)


def _sphere_quadrature(n_theta: int = 24, n_phi: int = 48):
    """Gauss-Legendre in cos(theta) times the trapezoid rule in phi: exact for
    polynomials in (x, y, z) of total degree < min(2*n_theta, n_phi)."""
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1 - ct * ct)
    x = (st[:, None] * np.cos(phi)[None]).ravel()
    y = (st[:, None] * np.sin(phi)[None]).ravel()
    z = np.repeat(ct, n_phi)
    w = np.repeat(wt, n_phi) * (2 * np.pi / n_phi)
    return x, y, z, w


def clm_table(lmax: int) -> np.ndarray:
    """C_lm of Eq. 7 in l-major order.

    The paper calls them constant coefficients without values.  The reading
    used here makes q_nl the rotation-invariant power spectrum: with
    C_lm = 1 / integral over the unit sphere of b_lm^2, sqrt(C_lm) b_lm are
    orthonormal real spherical harmonics and the addition theorem gives
    sum_m C_lm B_lm(u) B_lm(v) = (2l+1)/(4 pi) P_l(u.v)."""
    x, y, z, w = _sphere_quadrature()
    out = []
    for l in range(1, lmax + 1):
        for m in range(2 * l + 1):
            b = b_poly(l, m, x, y, z)
            out.append(1.0 / float(np.sum(w * b * b)))
    return np.array(out)


def legendre_P(l: int, t):
    c = np.zeros(l + 1)
    c[l] = 1.0
    return np.polynomial.legendre.legval(t, c)


FOUR_PI = 4.0 * math.pi
