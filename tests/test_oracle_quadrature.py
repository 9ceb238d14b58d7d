"""Pins of the oracle's quadrature rules, sampled coefficients and cell-averaged
separable weights, against closed forms and invariants of the mathematics."""
import numpy as np
import pytest

import synth
from oracle.lattice import Mesh, Lattice
from oracle import assemble as asm, auxop, matfree, pmg
from oracle.quadrature import (gll_rule, default_points, quadratic_lagrange, sampled_values,
                               averaged_coefficients, sample_function)


@pytest.mark.parametrize("q", [2, 3, 5, 9, 14])
def test_gll_rule_exactness(q):
    x, w = gll_rule(q)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.allclose(x, -x[::-1], atol=1e-15)
    for k in range(0, 2 * q - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13, k
    # degree 2q-2 is not integrated exactly by a q-point Lobatto rule
    k = 2 * q - 2
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-10


def test_default_points():
    # ceil(3(p+1)/2)
    assert [default_points(p) for p in (1, 2, 3, 7, 8)] == [3, 5, 6, 12, 14]


def test_triquadratic_interpolation_reproduces_quadratics():
    t = np.array([-1.0, 0.0, 1.0])
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")

    def f(x, y, z):
        return 1.0 + 2 * x - y * y + 3 * x * y * z * z - 0.5 * x * x * y * y * z * z

    s = f(X, Y, Z).ravel()[None, :]
    xq = np.linspace(-0.9, 0.8, 5)
    v = sampled_values(s, xq).reshape(5, 5, 5)
    Zq, Yq, Xq = np.meshgrid(xq, xq, xq, indexing="ij")
    assert np.abs(v - f(Xq, Yq, Zq)).max() < 1e-13
    assert np.allclose(quadratic_lagrange(xq).sum(1), 1.0)


def test_averaged_coefficients_box_closed_form():
    # box cells, constant alpha, beta: sigma_d = alpha V / (2 h_d^2), mu = beta V / 8
    n = (2, 3, 1)
    xs = [np.array([0.0, 0.3, 1.0]), np.array([0.0, 0.2, 0.7, 1.0]), np.array([0.0, 1.0])]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    m = Mesh(*n, vertices=np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1))
    al, be = 2.5, 0.7
    c = averaged_coefficients(m, np.full((m.ncells, 27), al), np.full((m.ncells, 27), be), 3)
    hs = asm.cell_sizes(m)
    for k in range(m.ncells):
        V = hs[k].prod()
        assert np.allclose(c[k, :3], al * V / (2 * hs[k] ** 2), rtol=1e-14)
        assert np.allclose(c[k, 3:], be * V / 8, rtol=1e-14)


def _perturbed(n, seed=3):
    return Mesh(n, n, n, vertices=synth.perturbed_vertices(n, seed))


def test_sampled_quadrature_paths_agree_on_perturbed_mesh():
    m = _perturbed(2)
    lat = Lattice(m, "grad", 3)
    f = lambda X: np.exp(0.5 * np.sin(2 * np.pi * X[:, 0]) * np.sin(2 * np.pi * X[:, 1]) *
                         np.sin(2 * np.pi * X[:, 2]))
    a = sample_function(m, f)
    b = np.ones((m.ncells, 27))
    q = default_points(3)
    A = asm.quadrature_operator(lat, a, b, q, kind="gll")
    x = np.where(lat.dirichlet_mask(), 0.0, synth.uniform_pm1(5, lat.ndofs))
    y1 = asm.with_dirichlet(lat, A) @ x
    y2 = matfree.apply(lat, x, a, b, q, kind="gll")
    assert np.linalg.norm(y1 - y2) < 1e-12 * np.linalg.norm(y1)
    assert abs(A - A.T).max() < 1e-13


def test_perturbed_mesh_volume_and_linear_energy():
    # constants: stiffness vanishes, 1^T M 1 = volume of the cube = 1 (trilinear cells
    # tile it, det J has degree <= 2 per axis, integrated exactly by GLL q >= 3);
    # u = x_r: int |grad u|^2 = 1 and cross terms vanish
    m = Mesh(2, 2, 2, vertices=synth.perturbed_vertices(2, 3), dirichlet=0)
    for p in (1, 3):
        lat, latc = Lattice(m, "grad", p), Lattice(m, "grad", 1)
        q = default_points(p)
        ones = np.ones((m.ncells, 27))
        zeros = np.zeros((m.ncells, 27))
        M = asm.quadrature_operator(lat, zeros, ones, q, kind="gll")
        K = asm.quadrature_operator(lat, ones, zeros, q, kind="gll")
        Pr = pmg.prolongation(lat, latc)
        one = Pr @ np.ones(latc.ndofs)
        assert abs(one @ (M @ one) - 1.0) < 1e-13
        assert np.abs(K @ one).max() < 1e-12
        U = [Pr @ m.vertices[:, r] for r in range(3)]
        for r in range(3):
            for s in range(3):
                assert abs(U[r] @ (K @ U[s]) - (1.0 if r == s else 0.0)) < 1e-12


def test_averaged_separable_equals_operator_on_boxes():
    # Cartesian cells, constant coefficients: the separable auxiliary built from
    # averaged weights is the operator itself (P = A, Sec. 3.2)
    m = Mesh(2, 2, 2)
    lat = Lattice(m, "grad", 3)
    al = synth.cell_coefficients(8, 1)
    be = synth.cell_coefficients(8, 2)
    a = np.repeat(al[:, None], 27, 1)
    b = np.repeat(be[:, None], 27, 1)
    c = averaged_coefficients(m, a, b, default_points(3))
    P = auxop.separable_operator(lat, c)
    A = asm.cartesian_operator(lat, al, be)
    assert abs(P - A).max() < 1e-12 * abs(A).max()
