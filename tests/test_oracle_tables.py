"""Pins of the oracle's 1-D FDM tables (Sec. 2.2-2.3, 3.2) against closed forms,
the paper's structural statements and an independently produced fixture."""
import os

import numpy as np
import pytest

from oracle.tables1d import Element1D, gauss_legendre, p1_embedding

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_p1_closed_form():
    e = Element1D(1)
    assert np.allclose(e.B, [[2 / 3, 1 / 3], [1 / 3, 2 / 3]], atol=1e-15)
    assert np.allclose(e.A, 0.5 * np.array([[1, -1], [-1, 1]]), atol=1e-15)


def test_p2_closed_form():
    # hand derivation: s_1 = sqrt(15/16)(1 - x^2), lambda_1 = 5/2
    e = Element1D(2)
    x = np.linspace(-1, 1, 7)
    assert np.allclose(e.s(x)[:, 1], np.sqrt(15 / 16) * (1 - x ** 2), atol=1e-14)
    assert abs(e.lam[0] - 2.5) < 1e-14
    assert abs(e.B[0, 0] - 0.25) < 1e-14 and abs(e.B[0, 2] + 1 / 12) < 1e-14
    r15 = np.sqrt(15.0)
    Aex = np.array([[37 / 24, -5 * r15 / 12, 13 / 24],
                    [-5 * r15 / 12, 2.5, -5 * r15 / 12],
                    [13 / 24, -5 * r15 / 12, 37 / 24]])
    assert np.allclose(e.A, Aex, atol=1e-13)
    Dex = np.array([[-2 ** -0.5, 0, 2 ** -0.5],
                    [-5 * np.sqrt(6) / 12, np.sqrt(10) / 2, -5 * np.sqrt(6) / 12]])
    assert np.allclose(e.D_raw, Dex, atol=1e-13)


def test_p3_p4_eigenvalues():
    assert np.allclose(Element1D(3).lam, [2.5, 10.5], atol=1e-12)
    r = np.sqrt(133.0)
    assert np.allclose(Element1D(4).lam, [14 - r, 10.5, 14 + r], atol=1e-11)


def test_appendix_fixture():
    rows = [l.split() for l in open(os.path.join(GOLD, "fdm_tables_appendix.txt")) if l[0] != "#"]
    for row in rows:
        p = int(row[0])
        e = Element1D(p)
        assert abs(e.B[0, 0] - float(row[1])) < 1e-13
        assert abs(e.B[0, p] - float(row[2])) < 1e-13
        lam = np.array([float(v) for v in row[3:]])
        assert np.allclose(e.lam, lam, rtol=2e-10)


@pytest.mark.parametrize("p", range(1, 10))
def test_structure_of_raw_tables(p):
    e = Element1D(p)
    n = p + 1
    # mass near diagonal: only B_0p off the diagonal (Sec. 2.2)
    off = e.B_raw.copy()
    np.fill_diagonal(off, 0.0)
    off[0, p] = off[p, 0] = 0.0
    assert np.abs(off).max() < 1e-13
    # interior stiffness diagonal = lambda (eq. fdmbasis)
    if p >= 2:
        AII = e.A_raw[1:p, 1:p]
        assert np.allclose(AII, np.diag(e.lam), atol=1e-11 * max(1, e.lam.max()))
        assert np.allclose(np.diag(e.D_raw[1:, 1:p]), np.sqrt(e.lam), rtol=1e-12)
    # D row 0 = (-2^-1/2, 0, ..., 0, 2^-1/2) (Sec. 2.3)
    ref = np.zeros(n)
    ref[0], ref[p] = -2 ** -0.5, 2 ** -0.5
    assert np.allclose(e.D_raw[0], ref, atol=1e-13)
    # A = D^T D (r orthonormal basis of DP_{p-1} = d(P_p))
    assert np.allclose(e.A_raw, e.D_raw.T @ e.D_raw, atol=1e-12 * np.abs(e.A_raw).max())
    # r orthonormal
    xq, wq = gauss_legendre(p + 2)
    R = e.r(xq)
    assert np.allclose(R.T @ (wq[:, None] * R), np.eye(p), atol=1e-12)
    # stiffness annihilates constants (coefficients of 1 by the dual DoFs)
    one = e.dof_functionals(lambda x: np.ones_like(x))
    assert np.allclose(e.A @ one, 0.0, atol=1e-11 * np.abs(e.A).max())
    # cleaned tables differ from raw ones only by roundoff
    assert np.abs(e.B - e.B_raw).max() < 1e-13
    assert np.abs(e.A - e.A_raw).max() < 1e-12 * max(1.0, np.abs(e.A).max())


@pytest.mark.parametrize("p", range(2, 10))
def test_sign_rule_and_duality(p):
    e = Element1D(p)
    slope = e.ds(np.array([-1.0]))[0, 1:p]
    assert (slope > 1.0).all()           # s_j'(-1) > 0, well separated from 0
    # duality (eq. unisolvence): the dual DoFs applied to s_j give e_j
    for j in range(p + 1):
        f = lambda x, j=j: e.s(x)[:, j]
        assert np.allclose(e.dof_functionals(f), np.eye(p + 1)[j], atol=1e-12)


def test_ritz_bounds():
    lams = {p: Element1D(p).lam for p in range(2, 11)}
    for p in range(2, 10):
        for j in range(1, p):
            lo = (j * np.pi / 2) ** 2
            assert lams[p][j - 1] >= lams[p + 1][j - 1] - 1e-10
            assert lams[p + 1][j - 1] >= lo - 1e-10


@pytest.mark.parametrize("p", [1, 3, 6])
def test_broken_basis_orthonormal(p):
    e = Element1D(p)
    # broken coefficients c_bar = G c; broken mass = G^{-T} B G^{-1} must be I
    Gi = np.linalg.inv(e.G)
    assert np.allclose(Gi.T @ e.B @ Gi, np.eye(p + 1), atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 5])
def test_p1_embedding_reproduces_hats(p):
    e = Element1D(p)
    E = p1_embedding(e)
    x = np.linspace(-1, 1, 9)
    assert np.allclose(e.s(x) @ E[:, 0], 0.5 * (1 - x), atol=1e-13)
    assert np.allclose(e.s(x) @ E[:, 1], 0.5 * (1 + x), atol=1e-13)
