"""Pins of the oracle's radial basis and harmonics against closed forms and
library routines (Appendix A, Appendix B)."""
import math

import numpy as np
import pytest
import torch

from oracle import chebyshev, cutoff, harmonics as hm, radial_functions

DT = torch.float64


def test_chebyshev_matches_trig_closed_form_and_numpy():
    xi = np.linspace(-1, 1, 101)
    T = chebyshev(torch.tensor(xi, dtype=DT), 12).numpy()
    for k in range(12):
        np.testing.assert_allclose(T[:, k], np.cos(k * np.arccos(xi)), atol=1e-12)
        c = np.zeros(k + 1)
        c[k] = 1
        np.testing.assert_allclose(T[:, k], np.polynomial.chebyshev.chebval(xi, c), atol=1e-12)


def test_chebyshev_derivative_recursion_A1_5():
    # dT_k/dxi from the paper's recursion (A1.3-A1.5) equals the exact
    # derivative k U_{k-1}(xi) = k sin(k t)/sin(t), xi = cos t
    t = np.linspace(0.1, 3.0, 37)
    xi = np.cos(t)
    K = 11
    T = [np.ones_like(xi), xi]
    dT = [np.zeros_like(xi), np.ones_like(xi)]
    for k in range(2, K):
        T.append(2 * xi * T[k - 1] - T[k - 2])
        dT.append(2 * T[k - 1] + 2 * xi * dT[k - 1] - dT[k - 2])
    for k in range(K):
        np.testing.assert_allclose(dT[k], k * np.sin(k * t) / np.sin(t), atol=1e-9)


def test_cutoff_values_and_smoothness():
    rc = 6.0
    r = torch.tensor([0.0, 3.0, 6.0, 6.5], dtype=DT)
    np.testing.assert_allclose(cutoff(r, rc).numpy(), [1.0, 0.5, 0.0, 0.0], atol=1e-15)
    rr = torch.tensor([1.0, 2.5, 5.9, rc], dtype=DT, requires_grad=True)
    (g,) = torch.autograd.grad(cutoff(rr, rc).sum(), rr)
    exact = -math.pi / (2 * rc) * np.sin(math.pi * rr.detach().numpy() / rc)   # A2.2
    np.testing.assert_allclose(g.numpy(), exact, atol=1e-14)
    assert abs(g.numpy()[-1]) < 1e-15


def test_radial_functions_closed_form_and_C1_at_cutoff():
    rc, K = 4.0, 9
    r = np.linspace(0.05, rc, 50)
    xi = 2 * (r / rc - 1) ** 2 - 1
    exact = 0.5 * (np.cos(np.arange(K)[None] * np.arccos(np.clip(xi, -1, 1))[:, None]) + 1) \
        * (0.5 * (1 + np.cos(np.pi * r / rc)))[:, None]
    f = radial_functions(torch.tensor(r, dtype=DT), rc, K).numpy()
    np.testing.assert_allclose(f, exact, atol=1e-13)
    rr = torch.tensor([rc], dtype=DT, requires_grad=True)
    fk = radial_functions(rr, rc, K)
    for k in range(K):
        (g,) = torch.autograd.grad(fk[0, k], rr, retain_graph=True)
        assert abs(float(g)) < 1e-14 and abs(float(fk[0, k])) < 1e-15


@pytest.mark.parametrize("l", range(1, 9))
def test_harmonics_homogeneous_and_harmonic(l):
    rng = np.random.default_rng(l)
    p = torch.tensor(rng.normal(size=(20, 3)), dtype=DT, requires_grad=True)
    for m in range(2 * l + 1):
        b = hm.b_poly(l, m, p[:, 0], p[:, 1], p[:, 2])
        b2 = hm.b_poly(l, m, 1.7 * p[:, 0], 1.7 * p[:, 1], 1.7 * p[:, 2])
        ref = 1.7 ** l * b.detach().numpy()
        np.testing.assert_allclose(b2.detach().numpy(), ref, atol=1e-12 * max(1.0, np.abs(ref).max()))
        # Laplacian of b_lm vanishes (a typo in a coefficient would break this)
        (g,) = torch.autograd.grad(b.sum(), p, create_graph=True)
        if not g.requires_grad:   # l = 1: linear, the Laplacian is identically zero
            continue
        lap = 0
        for a in range(3):
            (ga,) = torch.autograd.grad(g[:, a].sum(), p, retain_graph=True, allow_unused=True)
            if ga is not None:
                lap = lap + ga[:, a]
        assert float(lap.abs().max()) < 1e-8 * max(1.0, float(b.abs().max()))


def test_clm_textbook_values_l1_l2():
    c = hm.clm_table(2) * 4 * math.pi
    np.testing.assert_allclose(c[:3], [3, 3, 3], rtol=1e-13)
    np.testing.assert_allclose(c[3:8], [5 / 4, 15, 15, 15 / 4, 15 / 4], rtol=1e-13)


@pytest.mark.parametrize("l", range(1, 9))
def test_addition_theorem(l):
    """sum_m C_lm B_lm(u) B_lm(v) = (2l+1)/(4 pi) P_l(u.v)."""
    rng = np.random.default_rng(100 + l)
    u = rng.normal(size=(50, 3))
    v = rng.normal(size=(50, 3))
    Bu = hm.B_dir(l, torch.tensor(u, dtype=DT)).numpy()
    Bv = hm.B_dir(l, torch.tensor(v, dtype=DT)).numpy()
    a, b = hm.harmonic_index(l, 0), hm.harmonic_index(l, 2 * l) + 1
    c = hm.clm_table(l)[a:b]
    lhs = (c * Bu[:, a:b] * Bv[:, a:b]).sum(1)
    cos = (u * v).sum(1) / np.linalg.norm(u, axis=1) / np.linalg.norm(v, axis=1)
    rhs = (2 * l + 1) / (4 * math.pi) * hm.legendre_P(l, cos)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
