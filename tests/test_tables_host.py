"""Host-side checks of the mass-solve sweep: the closed-form DOF counts of the
Kuhn meshes agree with the library's DOF numbering, and the chosen meshes have
about 1e6 DOFs (Section 3's solve size)."""
import pytest

from paper_2607_12138_amd import _lib as L
from paper_2607_12138_amd import tables


@pytest.mark.parametrize("family", tables.FAMILIES)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_dof_count_matches_numbering(family, dim, degree):
    for N in (1, 2, 3):
        coords, cells = L.bras_mesh_structured(dim, N, 0.0, 0)
        n, _ = L.bras_dofmap(L.FAMILY[family], dim, degree, len(coords), cells)
        assert tables.dof_count(family, dim, degree, N) == n
        assert len(cells) == tables.entity_counts(dim, N)[-1]


@pytest.mark.parametrize("family", tables.FAMILIES)
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_sweep_meshes_have_about_a_million_dofs(family, dim, degree):
    N = tables.mesh_for(family, dim, degree)
    n = tables.dof_count(family, dim, degree, N)
    assert 0.85e6 < n < 1.15e6
