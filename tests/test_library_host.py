"""Host-side checks of the C-ABI library (no GPU): the shared library loads and
exports every entry point of include/rz.h; the numbering, the vertex-star
patches, the static-condensation IC pattern and the 1-D tables of a host-only
context match the oracle bit-exactly (integers) or to 1e-13 (tables)."""
import os
import re

import numpy as np
import pytest

from oracle.lattice import Mesh, Lattice
from oracle.tables1d import Element1D, p1_embedding
from oracle import schwarz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rz():
    from paper_2211_14284_amd import rz
    return rz


def test_exports_every_declared_symbol():
    rz = _rz()
    header = open(os.path.join(ROOT, "include", "rz.h")).read()
    names = set(re.findall(r"\b(rz_[a-z_]+)\s*\(", header))
    assert len(names) >= 15
    for name in sorted(names):
        assert hasattr(rz.lib, name), name


def test_host_only_context_refuses_compute():
    rz = _rz()
    ctx = rz.Context(-1)
    pb = rz.Problem(ctx, 2, 3)
    with pytest.raises(rz.RzError) as e:
        pb.apply(1, 2)
    assert e.value.code == -7


@pytest.mark.parametrize("n,p", [((2, 3, 2), 3), ((4, 4, 4), 4), ((2, 2, 2), 7)])
def test_dofmap_bit_exact(n, p):
    rz = _rz()
    pb = rz.Problem(rz.Context(-1), n, p)
    lat = Lattice(Mesh(*n), "grad", p)
    assert np.array_equal(pb.dofmap(), lat.cell_dofs())
    assert pb.ndofs == lat.ndofs
    assert pb.nfree == int((~lat.dirichlet_mask()).sum())


@pytest.mark.parametrize("n,p,dirichlet", [((4, 4, 4), 4, 0x3F), ((3, 2, 3), 3, 0x3F), ((3, 3, 2), 2, 0x15)])
def test_patches_and_ic_pattern_bit_exact(n, p, dirichlet):
    rz = _rz()
    pb = rz.Problem(rz.Context(-1), n, p, dirichlet=dirichlet)
    m = Mesh(*n, dirichlet=dirichlet)
    lat = Lattice(m, "grad", p)
    ref = schwarz.vertex_patches_grad(lat)
    assert pb.npatches == len(ref)
    pat = schwarz.symbolic_schur_pattern_grad(lat)
    for k, (vid, dofs) in enumerate(ref):
        v, d = pb.patch(k)
        assert v == vid
        assert np.array_equal(d, dofs)
        pv = pat[dofs][:, dofs].toarray().astype(bool)
        r, c = np.nonzero(np.tril(pv))
        order = np.lexsort((c, r))
        got = pb.ic_pattern(k)
        assert np.array_equal(got, np.stack([r[order], c[order]], 1))


@pytest.mark.parametrize("p", [1, 2, 4, 7, 9])
def test_tables1d_match_oracle(p):
    rz = _rz()
    pb = rz.Problem(rz.Context(-1), 2, p)
    t = pb.tables1d()
    e = Element1D(p)
    sc = max(1.0, np.abs(e.A).max())
    assert np.allclose(t["lam"], e.lam, rtol=1e-13, atol=0)
    assert np.abs(t["B"] - e.B).max() < 1e-14
    assert np.abs(t["A"] - e.A).max() < 1e-13 * sc
    assert np.abs(t["D"] - e.D).max() < 1e-13 * np.sqrt(sc)
    assert np.abs(t["E"] - p1_embedding(e)).max() < 1e-14


def test_aux_coefficients_cartesian():
    rz = _rz()
    from oracle import auxop
    m = Mesh(3, 2, 2)
    m.vertices[:, 0] *= 1.5
    alpha = np.linspace(0.5, 2, 12)
    beta = np.linspace(3, 1, 12)
    pb = rz.Problem(rz.Context(-1), (3, 2, 2), 3, alpha, beta, vertices=m.vertices)
    ref = auxop.cartesian_coefficient_array(Lattice(m, "grad", 3), alpha, beta)
    assert np.allclose(pb.aux_coefficients(), ref, rtol=1e-14)


@pytest.mark.parametrize("p", [1, 3, 8])
def test_aux_coefficients_trilinear_sampled(p):
    # cell-averaged separable weights on a perturbed mesh with sampled coefficients
    import synth
    from oracle.quadrature import averaged_coefficients, sample_function, default_points
    rz = _rz()
    m = Mesh(3, 2, 2)
    m = Mesh(3, 2, 2, vertices=_perturb(m.vertices, (3, 2, 2), 7))
    f = lambda X: np.exp(0.5 * np.sin(2 * np.pi * X[:, 0]) * np.sin(2 * np.pi * X[:, 1]) *
                         np.sin(2 * np.pi * X[:, 2]))
    a = sample_function(m, f)
    b = sample_function(m, lambda X: 1.0 + X[:, 0] ** 2)
    pb = rz.Problem(rz.Context(-1), (3, 2, 2), p, a, b, vertices=m.vertices)
    ref = averaged_coefficients(m, a, b, default_points(p))
    assert np.allclose(pb.aux_coefficients(), ref, rtol=1e-13, atol=0)


def _perturb(v, n, seed):
    """Move interior vertices by up to 0.15 h per coordinate (seeded)."""
    import synth
    nx, ny, nz = n
    v = v.copy()
    u = synth.uniform_pm1(seed, v.size).reshape(v.shape)
    k = np.arange(v.shape[0])
    ix, iy, iz = k % (nx + 1), (k // (nx + 1)) % (ny + 1), k // ((nx + 1) * (ny + 1))
    inner = (ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz)
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    v[inner] += 0.15 * h * u[inner]
    return v


def test_rejects_inverted_cell():
    rz = _rz()
    m = Mesh(2, 2, 2)
    v = m.vertices.copy()
    v[13] += 0.6          # the centre vertex beyond the opposite corner: det J < 0
    with pytest.raises(rz.RzError) as e:
        rz.Problem(rz.Context(-1), 2, 3, vertices=v)
    assert e.value.code == -1


@pytest.mark.parametrize("p", [2, 5, 8])
def test_aux_fit_targets_and_features(p):
    # least-squares separable fit to the broken diagonals and the MLP features
    import synth
    from oracle import learned
    rz = _rz()
    v = synth.perturbed_vertices(3, 3)
    m = Mesh(3, 3, 3, vertices=v)
    a = synth.c5_coefficient_samples(v, 3)
    b = np.repeat(synth.cell_coefficients(27, 4, 0.5, 2.0)[:, None], 27, 1)
    pb = rz.Problem(rz.Context(-1), 3, p, a, b, vertices=v)
    t, f, base = pb.aux_data()
    assert np.allclose(t, learned.diagonal_targets(m, a, b, p), rtol=1e-12, atol=0)
    assert np.abs(f - learned.features(m, a)).max() < 1e-13
    assert np.array_equal(base, pb.aux_coefficients())


@pytest.mark.parametrize("space", ["curl", "div"])
@pytest.mark.parametrize("n,p,dirichlet", [((2, 3, 2), 3, 0x3F), ((3, 2, 2), 2, 0x15), ((2, 2, 2), 6, 0x3F)])
def test_vector_space_numbering_and_weights(space, n, p, dirichlet):
    from oracle import auxop
    rz = _rz()
    m = Mesh(*n, dirichlet=dirichlet)
    m.vertices[:, 1] *= 0.7
    al = np.linspace(0.5, 2.0, m.ncells)
    be = np.linspace(3.0, 1.0, m.ncells)
    pb = rz.Problem(rz.Context(-1), n, p, al, be, space=space, vertices=m.vertices, dirichlet=dirichlet)
    lat = Lattice(m, space, p)
    assert pb.ndofs == lat.ndofs
    assert pb.nfree == int((~lat.dirichlet_mask()).sum())
    assert np.array_equal(pb.dofmap(), lat.cell_dofs())
    assert np.allclose(pb.aux_coefficients(), auxop.cartesian_coefficient_array(lat, al, be), rtol=1e-14)


def test_vector_space_rejects_relaxation():
    rz = _rz()
    pb = rz.Problem(rz.Context(-1), 2, 3, space="curl")
    with pytest.raises(rz.RzError):
        pb.relax(1, 2)
