"""Pins for the oracle's mesh, jitter generator and degree-of-freedom maps."""
import numpy as np
import pytest

from oracle import mesh, dofmap, fe


def test_splitmix64_published_vector():
    # Vigna's reference splitmix64.c seeded with 0 returns these first outputs.
    out = [int(mesh.splitmix64_counter(0, t)) for t in (1, 2, 3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_range():
    u = mesh.uniform01(12345, np.arange(1, 100001, dtype=np.uint64))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005


@pytest.mark.parametrize("dim,N", [(2, 1), (2, 5), (3, 1), (3, 4)])
def test_counts_and_euler(dim, N):
    coords, cells = mesh.structured_mesh(dim, N)
    V, Ed, F, T = mesh.mesh_counts(dim, N)
    assert len(coords) == V and len(cells) == T
    edges, _ = dofmap.entities(cells, 1)
    assert len(edges) == Ed
    if dim == 3:
        faces, _ = dofmap.entities(cells, 2)
        assert len(faces) == F
        assert V - Ed + F - T == 1
    else:
        assert V - Ed + T == 1


@pytest.mark.parametrize("dim,N,jit", [(2, 6, 0.0), (2, 6, 0.2), (3, 4, 0.0), (3, 4, 0.2)])
def test_cells_sorted_and_volume_partition(dim, N, jit):
    coords, cells = mesh.structured_mesh(dim, N, jitter=jit, seed=7)
    assert np.all(np.diff(cells, axis=1) > 0)
    det = np.linalg.det(mesh.jacobians(coords, cells))
    vol = np.abs(det).sum() / (2.0 if dim == 2 else 6.0)
    assert abs(vol - 1.0) < 1e-13
    _, cells0 = mesh.structured_mesh(dim, N)
    coords0, _ = mesh.structured_mesh(dim, N)
    det0 = np.linalg.det(mesh.jacobians(coords0, cells0))
    assert np.all(np.sign(det) == np.sign(det0))
    assert np.all(np.abs(det) > 0)


def test_jitter_bounds_and_boundary_fixed():
    N = 6
    h = 1.0 / N
    c0, _ = mesh.structured_mesh(3, N)
    c1, _ = mesh.structured_mesh(3, N, jitter=0.2, seed=99)
    delta = c1 - c0
    assert np.max(np.abs(delta)) <= 0.2 * h
    onb = np.any((np.abs(c0) < 1e-15) | (np.abs(c0 - 1.0) < 1e-15), axis=1)
    assert np.all(delta[onb] == 0.0)
    assert np.all(np.abs(delta[~onb]) > 0.0)
    c2, _ = mesh.structured_mesh(3, N, jitter=0.2, seed=100)
    assert not np.array_equal(c1, c2)


def _mult_by_entity(family, dim, degree, N):
    ref = fe.reference_element(family, dim, degree)
    coords, cells = mesh.structured_mesh(dim, N)
    pi, n, offs = dofmap.build_dofmap(cells, len(coords), ref.dofs_per_entity)
    d = dofmap.multiplicity(pi, n)
    assert d.sum() == pi.size
    return coords, cells, pi, n, offs, d


def test_fig_P_example_multiplicities_2d():
    # Fig. P_example: interior vertex 6, interior edge 2, cell interior 1.
    coords, cells, pi, n, offs, d = _mult_by_entity("P", 2, 3, 4)
    V = len(coords)
    interior_v = np.all((coords > 1e-12) & (coords < 1 - 1e-12), axis=1)
    assert set(d[:V][interior_v]) == {6}
    edges, _ = dofmap.entities(cells, 1)
    mid = coords[edges].mean(axis=1)
    interior_e = np.all((mid > 1e-12) & (mid < 1 - 1e-12), axis=1)
    de = d[offs[1]:offs[2]].reshape(len(edges), 2)
    assert set(de[interior_e].ravel()) == {2}
    assert set(de[~interior_e].ravel()) == {1}
    assert set(d[offs[2]:]) == {1}


def test_kuhn_multiplicities_3d():
    coords, cells, pi, n, offs, d = _mult_by_entity("P", 3, 3, 4)
    V = len(coords)
    interior_v = np.all((coords > 1e-12) & (coords < 1 - 1e-12), axis=1)
    assert set(d[:V][interior_v]) == {24}
    edges, _ = dofmap.entities(cells, 1)
    mid = coords[edges].mean(axis=1)
    interior_e = np.all((mid > 1e-12) & (mid < 1 - 1e-12), axis=1)
    de = d[offs[1]:offs[2]].reshape(len(edges), 2)[:, 0]
    assert set(de[interior_e]) == {4, 6}
    faces, _ = dofmap.entities(cells, 2)
    fm = coords[faces].mean(axis=1)
    interior_f = np.all((fm > 1e-12) & (fm < 1 - 1e-12), axis=1)
    df = d[offs[2]:offs[3]]
    assert set(df[interior_f]) == {2}
    assert set(df[~interior_f]) == {1}


@pytest.mark.parametrize("family,dim,deg", [("P", 2, 1), ("P", 3, 4), ("N1curl", 3, 2), ("RT", 3, 4), ("RT", 2, 2)])
def test_dofmap_shapes(family, dim, deg):
    ref = fe.reference_element(family, dim, deg)
    N = 3
    coords, cells = mesh.structured_mesh(dim, N)
    pi, n, offs = dofmap.build_dofmap(cells, len(coords), ref.dofs_per_entity)
    assert pi.shape == (len(cells), ref.n_loc)
    for row in pi:
        assert len(set(row.tolist())) == ref.n_loc
    d = dofmap.multiplicity(pi, n)
    assert d.min() >= 1
    V, Ed, F, T = mesh.mesh_counts(dim, N)
    k = ref.dofs_per_entity
    if dim == 3:
        assert n == V * k[0] + Ed * k[1] + F * k[2] + T * k[3]
    else:
        assert n == V * k[0] + Ed * k[1] + T * k[2]
