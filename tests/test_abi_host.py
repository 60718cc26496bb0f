"""C-ABI library: loads, exports what the header declares, and its host helpers
(mesh, numbering, reference tables) agree with the oracle.  CPU only: no
device call is made."""
import ctypes

import numpy as np
import pytest

from paper_2607_12138_amd import _lib as L
from oracle import mesh as omesh, dofmap as odofmap, fe as ofe


def test_library_exports_every_header_symbol():
    lib = L.lib()
    names = L.header_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert set(L._SIGS) | {"bras_last_error"} == set(names)


@pytest.mark.parametrize("dim,N,jit,seed", [(2, 7, 0.0, 0), (2, 9, 0.2, 123), (3, 5, 0.0, 0), (3, 6, 0.2, 99),
                                            (3, 24, 0.2, 0x260712138 + 32)])
def test_mesh_bit_exact(dim, N, jit, seed):
    c1, t1 = L.bras_mesh_structured(dim, N, jit, seed)
    c2, t2 = omesh.structured_mesh(dim, N, jitter=jit, seed=seed)
    assert np.array_equal(t1, t2)
    assert np.array_equal(c1.view(np.uint64), c2.view(np.uint64))


CASES = [("P", 2, 1), ("P", 2, 3), ("P", 3, 1), ("P", 3, 3), ("P", 3, 4), ("N1curl", 3, 1), ("N1curl", 3, 2),
         ("RT", 3, 1), ("RT", 3, 4), ("RT", 2, 2), ("N1curl", 2, 3), ("P", 2, 5), ("B", 2, 3), ("B", 3, 2),
         ("B", 3, 4), ("N2curl", 2, 2), ("N2curl", 3, 1), ("N2curl", 3, 3), ("BDM", 2, 4), ("BDM", 3, 1),
         ("BDM", 3, 3), ("BDM", 3, 4), ("N2curl", 2, 6), ("BDM", 2, 7)]


@pytest.mark.parametrize("family,dim,deg", CASES)
def test_element_info(family, dim, deg):
    nl, counts = L.bras_element_info(L.FAMILY[family], dim, deg)
    ref = ofe.reference_element(family, dim, deg)
    assert nl == ref.n_loc
    assert counts == tuple(ref.dofs_per_entity)


@pytest.mark.parametrize("family,dim,deg", CASES)
def test_dofmap_bit_exact(family, dim, deg):
    coords, cells = omesh.structured_mesh(dim, 3, jitter=0.2, seed=4)
    n1, l2g = L.bras_dofmap(L.FAMILY[family], dim, deg, len(coords), cells)
    ref = ofe.reference_element(family, dim, deg)
    pi, n2, _ = odofmap.build_dofmap(cells, len(coords), ref.dofs_per_entity)
    assert n1 == n2
    assert np.array_equal(l2g, pi.astype(np.int32))


@pytest.mark.parametrize("family,dim,deg", CASES)
def test_reference_mass_matches_oracle(family, dim, deg):
    lib_tab = L.bras_reference_mass(L.FAMILY[family], dim, deg)
    ref = ofe.reference_element(family, dim, deg)
    if family in ("P", "B"):
        expect = ref.mass[None]
        got = lib_tab[None]
    else:
        pairs = [(a, b) for a in range(dim) for b in range(a, dim)]
        expect = np.array([ref.mass[a, a] if a == b else ref.mass[a, b] + ref.mass[b, a] for a, b in pairs])
        got = lib_tab
    scale = np.max(np.abs(expect))
    assert np.max(np.abs(got - expect)) <= 2e-15 * scale * max(1, ref.n_loc / 10)


def test_host_errors_are_reported():
    with pytest.raises(L.BrasError) as e:
        L.bras_mesh_size(4, 3)
    assert e.value.code == L.BRAS_EINVAL and "dim" in str(e.value)
    with pytest.raises(L.BrasError):
        L.bras_element_info(L.HDIV, 3, 9)
    bad = np.array([[0, 2, 1]], dtype=np.int32)          # not ascending
    with pytest.raises(L.BrasError) as e:
        L.bras_dofmap(L.H1, 2, 1, 3, bad)
    assert "ascending" in str(e.value)
    nv = ctypes.c_int64()
    assert L.lib().bras_mesh_size(3, 2, None, ctypes.byref(nv)) == L.BRAS_EINVAL


def test_binding_constants_match_header():
    """Every numeric #define of the header has the same value in the binding."""
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bras.h")
    defs = dict((m.group(1), int(m.group(2)))
                for m in re.finditer(r"^#define (BRAS_\w+)\s+(-?\d+)", open(path).read(), re.M))
    py = {"BRAS_" + k: getattr(L, k) for k in ("H1", "HCURL", "HDIV", "H1_BERNSTEIN", "HCURL2", "HDIV2",
                                               "ELEM_EXPLICIT", "ELEM_SCALED_REF", "ELEM_METRIC_REF",
                                               "FP64", "FP32", "BF16", "PC_NONE", "PC_JACOBI", "PC_BRAS",
                                               "EXPORT_MULT", "EXPORT_ROWPTR", "EXPORT_SLOT", "EXPORT_DIAG",
                                               "OP_MASS", "OP_BRAS", "OP_JACOBI", "OPT_GRAPH_ITERS", "OPT_MAX_RESTART",
                                               "OPT_VARIANT", "OPT_SMALL_CG", "OPT_PATCH", "OPT_FLEXIBLE")}
    py.update({k: getattr(L, k) for k in ("BRAS_OK", "BRAS_EINVAL", "BRAS_ENOTSPD", "BRAS_EHIP", "BRAS_ENOCONV",
                                          "BRAS_EBREAKDOWN", "BRAS_ENOMEM")})
    py.update({"BRAS_INFO_" + k.upper(): v for k, v in L.INFO.items()})
    assert set(py) == set(defs), set(py) ^ set(defs)
    for k, v in defs.items():
        assert py[k] == v, k


def test_setup_and_geometry_reject_bad_arguments():
    """Empty inputs, sizes beyond the documented limits and unsupported form /
    precision pairs are rejected with EINVAL by checks that run before any
    device call (placeholder pointers are never dereferenced)."""
    lib = L.lib()
    P = ctypes.c_void_p(0x1000)   # non-null placeholder, never dereferenced on these paths
    h = ctypes.c_void_p()

    def setup(n=10, E=4, nl=3, l2g=P, form=L.ELEM_SCALED_REF, ref=P, elem=P, nsym=0, prec=L.FP64, rhs=1):
        return lib.bras_setup(ctypes.byref(h), n, E, nl, l2g, form, ref, elem, nsym, prec, rhs, None)

    cases = {
        "empty n": dict(n=0), "empty E": dict(E=0), "n_loc 0": dict(nl=0), "n_loc 121": dict(nl=121),
        "E * n_loc >= 2^31": dict(E=1 << 28, nl=8), "null map": dict(l2g=None), "null elements": dict(elem=None),
        "unknown form": dict(form=7), "metric without nsym": dict(form=L.ELEM_METRIC_REF, nsym=0),
        "missing tables": dict(ref=None), "unknown precision": dict(prec=5),
        "BF16 scaled": dict(prec=L.BF16), "FP32 scaled": dict(prec=L.FP32),
        "max_rhs 0": dict(rhs=0), "max_rhs 257": dict(rhs=257), "block vector >= 4 GiB": dict(n=1 << 28, rhs=2),
    }
    for name, kw in cases.items():
        assert setup(**kw) == L.BRAS_EINVAL, name
        assert h.value is None, name
        assert lib.bras_last_error(), name
    assert lib.bras_setup(None, 10, 4, 3, P, L.ELEM_SCALED_REF, P, P, 0, L.FP64, 1, None) == L.BRAS_EINVAL
    geo = lib.bras_geometry
    assert geo(L.H1, 4, 3, P, 1, P, None, P, None) == L.BRAS_EINVAL          # dim
    assert geo(9, 2, 3, P, 1, P, None, P, None) == L.BRAS_EINVAL             # family
    assert geo(L.H1, 2, 3, None, 1, P, None, P, None) == L.BRAS_EINVAL       # null coordinates
    assert geo(L.H1, 2, 3, P, 0, P, None, P, None) == L.BRAS_EINVAL          # empty mesh
    # calls on a null handle
    for fn in ("bras_apply", "mass_apply", "jacobi_apply"):
        assert getattr(lib, fn)(None, P, P, 1, None) == L.BRAS_EINVAL, fn
    assert lib.pcg_solve(None, L.PC_BRAS, P, P, 1, 1e-8, 10, None, None, None) == L.BRAS_EINVAL


def test_local_gemm_microbenchmark_counts():
    """The BF16 local-GEMM microbenchmark's FLOP count (blocks = 0 launches
    nothing): issued 32x32x16 MFMAs of one element and 32 columns, counted by
    hand from the tile shapes (rows in 32-row tiles, k in 16-deep steps; the
    first product stops at the tile's last row, the second starts at k-step 2t)."""
    from paper_2607_12138_amd import _lib as L
    per_mfma = 2 * 32 * 32 * 16
    for nl, count in ((20, 2 + 2), (36, (2 + 3) + (3 + 1)), (70, (2 + 5) + (4 + 3) + (5 + 1)),
                      (84, (2 + 6) + (4 + 4) + (6 + 2))):
        assert L.bras_bench_bf16_local_gemm(nl, 1, 0) == count * per_mfma, nl
    with pytest.raises(L.BrasError):
        L.bras_bench_bf16_local_gemm(15, 1, 0)
    with pytest.raises(L.BrasError):
        L.bras_bench_bf16_local_gemm(70, -1, 0)
