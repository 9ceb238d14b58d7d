"""Pin of the order of the interface DoFs inside a vertex patch (nested dissection,
separators last; Sec. 4.5 asks for a nested-dissection order without fixing one).

The reading pinned here, written out by hand from the rule rather than from the
oracle's sort key:
  1. the 12 faces of the star: by normal axis (x, y, z), then by the (-, +) sides
     along the two remaining axes, compared lexicographically with the lower axis
     first; inside a face, lattice order (x fastest, then y, then z);
  2. the 6 edges: by axis (x, y, z), then side (-, +) along the edge axis;
  3. the vertex.
Dirichlet DoFs are left out; the same rule holds for stars truncated by the
boundary.  The library exports its own patch order, which the host tests compare
with the oracle's bit for bit, so this also pins the library.
"""
import numpy as np

from oracle.lattice import Mesh, Lattice
from oracle import schwarz


def _offsets(lat, vid, dofs):
    nvx, nvy = lat.mesh.nx + 1, lat.mesh.ny + 1
    v = (vid % nvx, (vid // nvx) % nvy, vid // (nvx * nvy))
    Ex, Ey, _ = lat.extents[0]
    out = []
    for g in dofs:
        X, Y, Z = g % Ex, (g // Ex) % Ey, g // (Ex * Ey)
        out.append((X - v[0] * lat.p, Y - v[1] * lat.p, Z - v[2] * lat.p))
    return out


def _patch(lat, vid):
    for v, dofs in schwarz.vertex_patches_grad(lat):
        if v == vid:
            return dofs
    raise KeyError(vid)


# the interior p = 2 star: one DoF per face, one per edge, the vertex (19 rows)
P2_INTERIOR = [
    # faces with normal x: sides (y, z) = (-,-), (-,+), (+,-), (+,+)
    (0, -1, -1), (0, -1, 1), (0, 1, -1), (0, 1, 1),
    # normal y: sides (x, z)
    (-1, 0, -1), (-1, 0, 1), (1, 0, -1), (1, 0, 1),
    # normal z: sides (x, y)
    (-1, -1, 0), (-1, 1, 0), (1, -1, 0), (1, 1, 0),
    # edges along x, y, z, each (-, +)
    (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1),
    # the vertex
    (0, 0, 0),
]


def test_interior_p2_star_order():
    lat = Lattice(Mesh(2, 2, 2), "grad", 2)
    vid = 1 + 3 * (1 + 3 * 1)            # the centre vertex of the 2x2x2 mesh
    assert _offsets(lat, vid, _patch(lat, vid)) == P2_INTERIOR


def test_face_interior_is_lattice_ordered_p3():
    # p = 3: each face holds 2 x 2 DoFs; the first face (normal x, sides y-, z-)
    # lists them x fastest, then y, then z: (dy, dz) = (-2,-2), (-1,-2), (-2,-1), (-1,-1)
    lat = Lattice(Mesh(2, 2, 2), "grad", 3)
    vid = 1 + 3 * (1 + 3 * 1)
    off = _offsets(lat, vid, _patch(lat, vid))
    assert len(off) == 1 + 6 * 2 + 12 * 4
    assert off[:4] == [(0, -2, -2), (0, -1, -2), (0, -2, -1), (0, -1, -1)]
    # the last face of the y-normal group is (x+, z+), the first edge block starts
    # after all 12 faces (48 DoFs) with the x-edge on the - side, nearest the vertex last
    assert off[48:50] == [(-2, 0, 0), (-1, 0, 0)]
    assert off[-1] == (0, 0, 0)


def test_truncated_star_on_neumann_bottom():
    # Dirichlet on every face but z = 0: the star of vertex (1, 1, 0) keeps only the
    # cells above z = 0 and its DoFs on the free bottom face (offsets d_z in {0, 1})
    lat = Lattice(Mesh(2, 2, 2, dirichlet=0x3F & ~16), "grad", 2)
    vid = 1 + 3 * (1 + 3 * 0)
    expected = [
        (0, -1, 1), (0, 1, 1),                           # normal x: only z+ sides exist
        (-1, 0, 1), (1, 0, 1),                           # normal y
        (-1, -1, 0), (-1, 1, 0), (1, -1, 0), (1, 1, 0),  # normal z (on the free bottom face)
        (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),    # edges along x and y on the bottom
        (0, 0, 1),                                       # the z-edge above the vertex
        (0, 0, 0),                                       # the vertex
    ]
    assert _offsets(lat, vid, _patch(lat, vid)) == expected


def test_truncated_star_all_dirichlet():
    # the same vertex with Dirichlet on z = 0 too: its bottom-face DoFs are dropped
    lat = Lattice(Mesh(2, 2, 2), "grad", 2)
    vid = 1 + 3 * (1 + 3 * 0)
    expected = [(0, -1, 1), (0, 1, 1), (-1, 0, 1), (1, 0, 1), (0, 0, 1)]
    assert _offsets(lat, vid, _patch(lat, vid)) == expected


def test_misordered_key_would_fail(monkeypatch):
    # a plausible slip -- face sides keyed by the higher remaining axis first -- is
    # caught by the hand-listed order
    def wrong_key(d, g):
        zero = [a for a in range(3) if d[a] == 0]
        side = lambda a: 0 if d[a] < 0 else 1
        if len(zero) == 1:
            a = zero[0]
            rest = [b for b in range(3) if b != a]
            return (0, a, side(rest[1]), side(rest[0]), g)
        if len(zero) == 2:
            a = [b for b in range(3) if d[b] != 0][0]
            return (1, a, side(a), 0, g)
        return (2, 0, 0, 0, g)
    monkeypatch.setattr(schwarz, "_patch_key", wrong_key)
    lat = Lattice(Mesh(2, 2, 2), "grad", 2)
    vid = 1 + 3 * (1 + 3 * 1)
    assert _offsets(lat, vid, _patch(lat, vid)) != P2_INTERIOR
