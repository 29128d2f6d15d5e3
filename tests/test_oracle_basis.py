"""Pins of the oracle's 1D basis and element operators against mathematics.

P1 Gauss-Legendre nodes/weights: closed forms (n <= 5) and exact quadrature.
P2 interpolation/derivative operators exact on polynomials of degree <= p.
P3 DG correction functions: end values, the Radau orthogonality, and the FR-DG identity
   g_R'(xi_a) = l_a(1)/w_a, g_L'(xi_a) = -l_a(-1)/w_a.
"""
import math

import numpy as np
import pytest

from oracle.basis import Basis1D
from oracle.operators import ElementOperators, monomials

CLOSED_FORM_GL = {
    2: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
    3: ([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    4: (sorted([s * math.sqrt(3 / 7 + t * 2 / 7 * math.sqrt(6 / 5)) for s in (-1, 1) for t in (-1, 1)]),
        None),
    5: (sorted([0.0] + [s * math.sqrt(5 + t * 2 * math.sqrt(10 / 7)) / 3 for s in (-1, 1) for t in (-1, 1)]),
        None),
}


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_gl_closed_form(n):
    b = Basis1D(n - 1)
    x, w = CLOSED_FORM_GL[n]
    assert np.max(np.abs(b.xi - np.array(x))) < 1e-15
    if w is not None:
        assert np.max(np.abs(b.w - np.array(w))) < 1e-15
    if n == 4:
        ww = [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36]
        assert abs(b.w[0] - ww[0]) < 1e-15 and abs(b.w[1] - ww[1]) < 1e-15
    if n == 5:
        assert abs(b.w[2] - 128 / 225) < 1e-15
        assert abs(b.w[0] - (322 - 13 * math.sqrt(70)) / 900) < 1e-15


@pytest.mark.parametrize("p", range(1, 7))
def test_gl_quadrature_exact(p):
    b = Basis1D(p)
    for m in range(2 * p + 2):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(b.w * b.xi ** m) - exact) < 1e-14


@pytest.mark.parametrize("p", range(1, 7))
def test_lagrange_cardinal_and_derivative(p):
    b = Basis1D(p)
    assert np.max(np.abs(b.lagrange(b.xi) - np.eye(p + 1))) < 1e-13
    # interpolation and derivative of monomials of degree <= p are exact
    xs = np.linspace(-1, 1, 7)
    for m in range(p + 1):
        vals = b.xi ** m
        assert np.max(np.abs(b.lagrange(xs) @ vals - xs ** m)) < 1e-13
        dm = m * xs ** (m - 1) if m > 0 else 0 * xs
        assert np.max(np.abs(b.dlagrange(xs) @ vals - dm)) < 1e-12


@pytest.mark.parametrize("p", range(1, 7))
def test_correction_functions(p):
    b = Basis1D(p)
    assert abs(b.g_right(1.0) - 1) < 1e-14 and abs(b.g_right(-1.0)) < 1e-14
    assert abs(b.g_left(-1.0) - 1) < 1e-14 and abs(b.g_left(1.0)) < 1e-14
    # Radau: orthogonal to every polynomial of degree <= p-1 (over-integrated quadrature)
    xq, wq = np.polynomial.legendre.leggauss(p + 4)
    for m in range(p):
        assert abs(np.sum(wq * b.g_right(xq) * xq ** m)) < 1e-14
        assert abs(np.sum(wq * b.g_left(xq) * xq ** m)) < 1e-14
    # FR with DG correction functions == nodal DG: lifting identity
    lp = b.lagrange(1.0)[0]
    lm = b.lagrange(-1.0)[0]
    assert np.max(np.abs(b.dg_right(b.xi) - lp / b.w)) < 1e-12
    assert np.max(np.abs(b.dg_left(b.xi) + lm / b.w)) < 1e-12


@pytest.mark.parametrize("d,p", [(2, 1), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_tensor_operators_exact(d, p):
    ops = ElementOperators(d, p)
    for e in monomials(d, p):
        u = np.prod(ops.upt_ref ** np.array(e), axis=1)
        uf = np.prod(ops.fpt_ref ** np.array(e), axis=1)
        assert np.max(np.abs(ops.M0 @ u - uf)) < 1e-13
        for k in range(d):
            ek = np.array(e)
            if ek[k] == 0:
                du = np.zeros_like(u)
            else:
                e2 = ek.copy()
                e2[k] -= 1
                du = ek[k] * np.prod(ops.upt_ref ** e2, axis=1)
            assert np.max(np.abs(ops.D[k] @ u - du)) < 1e-12
    # quadrature weights integrate the reference element exactly
    assert abs(ops.W.sum() - 2.0 ** d) < 1e-13
    # correction functions: nhat_j'.g_j(x_j') = delta; sensor transform recovers modes
    assert np.max(np.abs(ops.Vt_inv @ ops.Vt - np.eye(ops.nupts))) < 1e-12


def test_face_point_layout():
    ops = ElementOperators(3, 2)
    n = 3
    # face 2 is -xi_1; its tangential dims are (0, 2); first tangential index fastest
    j = 2 * n * n + 1 + n * 2
    assert ops.fpt_ref[j, 1] == -1.0
    assert ops.fpt_ref[j, 0] == ops.b.xi[1] and ops.fpt_ref[j, 2] == ops.b.xi[2]
