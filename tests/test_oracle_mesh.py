"""Pins of the oracle's interface meshes (output path, Sec. 3.2: one
marching-cubes triangle mesh per phase).  Each pin is a property that the
surface phi = iso must have whatever case table produced it: exact planes
for fields linear along the edges, closed and consistently wound surfaces
(Euler characteristic 2 for a sphere, 0 for a torus), enclosed volume and
normals pointing out of the phase, and closure across every face of all
256 corner configurations."""
import collections
import itertools

import numpy as np
import pytest

import oracle


def _field(shape, fn):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = np.zeros((4,) + shape)
    phi[1] = fn(x.astype(float), y.astype(float), z.astype(float))
    return phi


def _edges(tris):
    """Directed edges of all triangles, vertices as exact float tuples."""
    out = []
    for t in tris:
        v = [tuple(map(float, p)) for p in t]
        out += [(v[0], v[1]), (v[1], v[2]), (v[2], v[0])]
    return out


def _check_closed(tris, open_z=None, manifold=True):
    """No holes and consistent winding: every directed edge is matched by as
    many reversed ones (edges in an open z plane excepted).  manifold: each
    directed edge appears exactly once.  Faces whose inside corners lie on a
    diagonal can give two sheets that touch along a face line, so the
    exhaustive and random cases check only the first property."""
    d = collections.Counter(_edges(tris))
    if manifold:
        assert max(d.values()) == 1
    for (a, b), k in d.items():
        if open_z is not None and a[2] == b[2] and a[2] in open_z:
            continue
        assert d[(b, a)] == k, (a, b)


def _wrap(tris, nx, ny):
    """Identify the periodic images x = nx and y = ny with x = 0, y = 0."""
    w = tris.copy()
    w[:, :, 0][w[:, :, 0] == nx] = 0.0
    w[:, :, 1][w[:, :, 1] == ny] = 0.0
    return w


def _euler(tris):
    verts = {tuple(map(float, p)) for t in tris for p in t}
    edges = {tuple(sorted(e)) for e in _edges(tris)}
    return len(verts) - len(edges) + len(tris)


def _normals(tris):
    t = tris.astype(np.float64)
    return np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])


def _signed_volume(tris):
    t = tris.astype(np.float64)
    return float(np.sum(np.einsum("ij,ij->i", t[:, 0], np.cross(t[:, 1], t[:, 2])))) / 6.0


def test_plane_is_exact():
    """phi linear in z: linear interpolation puts every vertex on the plane;
    two triangles per crossed cube (periodic in x and y), total area nx ny,
    normals pointing to lower phi."""
    shape = (9, 5, 7)
    nz = shape[0]
    phi = _field(shape, lambda x, y, z: (z + 0.5) / nz)
    m = oracle.mesh_phase(phi, 1, 0.5)
    assert len(m) == 2 * 5 * 7
    assert np.all(m[:, :, 2] == np.float32(nz / 2 - 0.5))
    n = _normals(m)
    assert np.allclose(0.5 * np.linalg.norm(n, axis=1).sum(), 5 * 7)
    assert np.all(n[:, 2] < 0) and np.allclose(n[:, :2], 0)


def test_plane_at_a_fraction_of_the_edge():
    """iso between the cell values: the vertex sits at the interpolated
    fraction t = (iso - a)/(b - a) of the edge."""
    shape = (4, 3, 3)
    phi = _field(shape, lambda x, y, z: 0.1 * z)
    m = oracle.mesh_phase(phi, 1, 0.13)
    assert np.allclose(m[:, :, 2], 1.3) and len(m) == 2 * 3 * 3


def test_empty_and_full_fields_give_no_triangles():
    shape = (5, 4, 6)
    assert len(oracle.mesh_phase(_field(shape, lambda x, y, z: 0 * x), 1)) == 0
    assert len(oracle.mesh_phase(_field(shape, lambda x, y, z: 0 * x + 1), 1)) == 0


@pytest.mark.parametrize("R", [4.0, 7.31])
def test_sphere_closed_outward_and_volume(R):
    shape = (24, 22, 20)
    c = np.array([9.7, 10.2, 11.4])  # x, y, z; well inside, off the lattice

    def fn(x, y, z):
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        return 1.0 - r / (2 * R)
    m = oracle.mesh_phase(_field(shape, fn), 1, 0.5)
    _check_closed(m)
    assert _euler(m) == 2
    cen = m.astype(np.float64).mean(axis=1)
    assert np.all(np.einsum("ij,ij->i", _normals(m), cen - c) > 0)
    vol = _signed_volume(m)
    assert abs(vol / (4.0 / 3.0 * np.pi * R ** 3) - 1.0) < 0.05
    r = np.linalg.norm(m.reshape(-1, 3).astype(np.float64) - c, axis=1)
    assert np.all(np.abs(r - R) < 0.2)


def test_torus_has_euler_characteristic_zero():
    shape = (16, 30, 30)
    c = np.array([14.6, 15.3, 7.8])
    Rm, rm = 8.0, 3.2

    def fn(x, y, z):
        q = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2) - Rm
        return 1.0 - np.sqrt(q ** 2 + (z - c[2]) ** 2) / (2 * rm)
    m = oracle.mesh_phase(_field(shape, fn), 1, 0.5)
    _check_closed(m)
    assert _euler(m) == 0
    vol = _signed_volume(m)
    assert abs(vol / (2 * np.pi ** 2 * Rm * rm ** 2) - 1.0) < 0.06


def test_surface_wraps_periodically_in_x_and_y():
    """A cylinder along z centred on the corner of the periodic box: the
    cubes past the last column close it through the images at nx, ny."""
    shape = (6, 12, 10)

    def fn(x, y, z):
        dx = np.minimum(x, 10 - x)
        dy = np.minimum(y, 12 - y)
        return 1.0 - np.sqrt(dx ** 2 + dy ** 2) / 6.0
    m = oracle.mesh_phase(_field(shape, fn), 1, 0.5)
    assert m[:, :, 0].max() > 9.0 and m[:, :, 1].max() > 11.0  # reaches the images
    w = _wrap(m, 10, 12)
    _check_closed(w, open_z={0.0, 5.0})
    assert _euler(w) == 0  # an open tube


def test_all_corner_configurations_close_across_faces():
    """For each of the 256 inside/outside patterns of one cube's corners,
    the pattern tiled over a periodic 4x4x2 grid: its cubes see the pattern
    and its mirror images, and every face between them must be cut the same
    way from both sides (closed surface apart from the open z planes)."""
    for mask in range(256):
        cell = np.zeros((2, 2, 2))
        for c in range(8):
            cell[(c >> 2) & 1, (c >> 1) & 1, c & 1] = 1.0 if (mask >> c) & 1 else 0.0
        phi = np.zeros((4, 2, 4, 4))
        phi[1] = np.tile(cell, (1, 2, 2))
        m = oracle.mesh_phase(phi, 1, 0.5)
        if mask in (0, 255):
            assert len(m) == 0
            continue
        assert len(m) > 0
        _check_closed(_wrap(m, 4, 4), open_z={0.0, 1.0}, manifold=False)
        # midpoints of the edges only
        frac = np.modf(m.astype(np.float64))[0]
        assert np.all(np.isin(np.round(frac, 6), [0.0, 0.5]))


def test_single_corner_cut_points_away_from_it():
    """One inside cell in the middle of a 3x3x3 grid: each of the eight cubes
    around it sees it at a different corner and cuts it off with one
    triangle whose normal points away from it; together they close."""
    phi = np.zeros((4, 3, 3, 3))
    phi[1, 1, 1, 1] = 1.0
    m = oracle.mesh_phase(phi, 1, 0.5)
    assert len(m) == 8
    cen = m.astype(np.float64).mean(axis=1)
    assert np.all(np.einsum("ij,ij->i", _normals(m), cen - 1.0) > 0)
    _check_closed(m)
    assert _euler(m) == 2


def test_random_field_is_closed_and_phase_complement_reverses():
    """A random field: the surface is closed apart from the open z planes.
    The mesh of the complement field (1 - phi at iso 1 - iso) has the same
    vertices (edges are crossed where the sign changes either way)."""
    rng = np.random.default_rng(5)
    shape = (7, 6, 8)
    phi = np.zeros((4,) + shape)
    phi[2] = rng.random(shape)
    m = oracle.mesh_phase(phi, 2, 0.5)
    _check_closed(_wrap(m, shape[2], shape[1]), open_z={0.0, float(shape[0] - 1)}, manifold=False)
    phc = phi.copy()
    phc[2] = 1.0 - phi[2]
    mc = oracle.mesh_phase(phc, 2, 0.5)
    va = {tuple(map(float, p)) for t in _wrap(m, 8, 6) for p in t}
    vb = {tuple(map(float, p)) for t in _wrap(mc, 8, 6) for p in t}
    assert va == vb


def test_counts_match_brute_force_crossings():
    """Every crossed cube edge carries exactly one vertex: the distinct
    vertices are the sign-changing lattice edges of the cubes."""
    rng = np.random.default_rng(9)
    shape = (5, 4, 6)
    phi = np.zeros((4,) + shape)
    phi[0] = rng.random(shape)
    m = _wrap(oracle.mesh_phase(phi, 0, 0.5), shape[2], shape[1])
    verts = {tuple(map(float, p)) for t in m for p in t}
    f = phi[0] > 0.5
    nz, ny, nx = shape
    cross = 0
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if f[z, y, x] != f[z, y, (x + 1) % nx]:
            cross += 1
        if f[z, y, x] != f[z, (y + 1) % ny, x]:
            cross += 1
        if z + 1 < nz and f[z, y, x] != f[z + 1, y, x]:
            cross += 1
    assert len(verts) == cross
