"""Pins of the oracle's learned-auxiliary pieces: the separable least-squares fit
to the broken diagonals (factorised vs direct, closed form on boxes), the
features, and the hand-written MLP backward pass (finite differences) and Adam."""
import numpy as np
import pytest

import synth
from oracle.lattice import Mesh
from oracle.auxop import cartesian_coefficients
from oracle.assemble import cell_sizes
from oracle import learned


def _mesh(n=2, seed=3):
    return Mesh(n, n, n, vertices=synth.perturbed_vertices(n, seed))


@pytest.mark.parametrize("p", [1, 3, 6])
def test_targets_factorised_equal_direct(p):
    m = _mesh()
    a = synth.c5_coefficient_samples(m.vertices, 2)
    b = np.repeat(synth.cell_coefficients(m.ncells, 5, 0.5, 2.0)[:, None], 27, 1)
    t1 = learned.diagonal_targets(m, a, b, p)
    t2 = learned.diagonal_targets_direct(m, a, b, p)
    assert np.allclose(t1, t2, rtol=1e-12, atol=0)


def test_targets_on_boxes_are_exact_weights():
    xs = [np.array([0.0, 0.4, 1.0]), np.array([0.0, 0.3, 1.0]), np.array([0.0, 0.5, 1.0])]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    m = Mesh(2, 2, 2, vertices=np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1))
    al, be = 3.0, 0.25
    t = learned.diagonal_targets(m, np.full((8, 27), al), np.full((8, 27), be), 4)
    hs = cell_sizes(m)
    for k in range(8):
        assert np.allclose(t[k], cartesian_coefficients("grad", hs[k], al, be), rtol=1e-13)


def test_features_of_cubes_vanish():
    m = Mesh(3, 3, 3)
    f = learned.features(m, np.full((27, 27), 2.0))
    assert f.shape == (27, 51)
    assert np.abs(f).max() < 1e-14
    g = learned.features(_mesh(3), synth.c5_coefficient_samples(_mesh(3).vertices, 3))
    assert np.abs(g[:, :24]).max() > 1e-3 and np.abs(g[:, 24:].mean(1)).max() < 1e-14


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = learned.init_params(51, 16, 6, 77)
    X = rng.standard_normal((9, 51))
    Y = rng.standard_normal((9, 6))
    _, g = learned.loss_and_grads(P, X, Y)
    for k in range(6):
        for idx in [tuple(rng.integers(0, s) for s in P[k].shape) for _ in range(5)]:
            Pp = [q.copy() for q in P]
            Pm = [q.copy() for q in P]
            Pp[k][idx] += 1e-6
            Pm[k][idx] -= 1e-6
            fd = (learned.loss_and_grads(Pp, X, Y)[0] - learned.loss_and_grads(Pm, X, Y)[0]) / 2e-6
            assert abs(fd - g[k][idx]) < 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_adam_first_step_is_signed_lr():
    P = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    m, v = [np.zeros(3)], [np.zeros(3)]
    learned.adam_step(P, g, m, v, 1, 0.01)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> -lr g/(|g| + eps)
    assert np.allclose(P[0], np.array([1.0, -2.0, 3.0]) - 0.01 * np.sign(g[0]), atol=1e-7)


def test_init_params_glorot_bounds():
    P = learned.init_params(51, 64, 6, 5)
    assert [q.shape for q in P] == [(64, 51), (64,), (64, 64), (64,), (6, 64), (6,)]
    assert np.abs(P[0]).max() <= np.sqrt(6 / 115) and np.abs(P[4]).max() <= np.sqrt(6 / 70)
    assert all(np.all(P[k] == 0) for k in (1, 3, 5))
