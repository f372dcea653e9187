"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function that include/blr_tag.h declares; the planner's lists, colours,
tag vectors and aspect ratios match the oracle; invalid input maps to the
documented status codes."""
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blr_tag.h")

lib_mod = pytest.importorskip("paper_2501_05528_amd._lib")


def _lib():
    try:
        return lib_mod.lib()
    except ImportError as e:  # pragma: no cover
        pytest.fail(f"library not built: {e}")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(blr_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding declares the same set
    assert set(names) == set(lib_mod.SIGNATURES), set(names) ^ set(lib_mod.SIGNATURES)


def test_status_strings_and_version():
    L = _lib()
    assert L.blr_status_string(0) == b"BLR_OK"
    assert L.blr_status_string(2) == b"BLR_ERR_GEOMETRY"
    assert b"gfx950" in L.blr_version()


def _plan(geom, k, p, extra, T, aspect=True):
    from paper_2501_05528_amd.api import Plan
    return Plan(geom.box_ptr, geom.lattice, k, T, p=p, extra_tag_cols=extra, aspect_opt=aspect)


@pytest.mark.parametrize("dim,B,q,extra", [(2, 8, 8, 3), (2, 5, 4, 3), (3, 4, 3, 3), (1, 12, 5, 2), (2, 6, 4, 0)])
def test_plan_matches_oracle(dim, B, q, extra):
    from paper_2501_05528_amd.api import tag_columns
    g = W.grid_geometry(dim, B, q)
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, extra)
    assert tag_columns(g.box_ptr, g.lattice, extra) == ell
    T = W.tag_matrix(100 + dim, g.nboxes, ell)
    k = 2
    pl = _plan(g, k, 3, extra, T)
    near_ptr, near_idx, colour, boff = pl.lists()
    assert near_ptr.tolist() == np.cumsum([0] + [len(n) for n in near]).tolist()
    assert near_idx.tolist() == [j for n in near for j in n]
    assert colour.tolist() == O.colours(g.lattice).tolist()
    sizes = g.box_sizes()
    expect_off = np.cumsum([0] + [sizes[i] * sizes[j] for i in range(g.nboxes) for j in near[i]])[:-1]
    assert boff.tolist() == expect_off.tolist()
    z, rho = pl.tags()
    zo, rhoo = O.tag_plan(T, near, far)
    assert np.allclose(rho, rhoo, rtol=1e-9, atol=0)
    assert np.allclose(z, zo, rtol=0, atol=1e-9)
    for i in range(g.nboxes):
        assert np.linalg.norm(T[near[i]] @ z[i]) <= 1e-13 * np.linalg.norm(T)


def test_plan_without_optimisation_matches_oracle():
    g = W.grid_geometry(2, 6, 4)
    near = O.near_lists(g.lattice)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(5, g.nboxes, ell)
    pl = _plan(g, 2, 3, 3, T, aspect=False)
    z, rho = pl.tags()
    zo, rhoo = O.tag_plan(T, near, far, optimise=False)
    assert np.allclose(z, zo, atol=1e-12)
    assert np.allclose(rho, rhoo, rtol=1e-10)


def test_plan_errors():
    from paper_2501_05528_amd.api import BlrError
    g = W.grid_geometry(2, 4, 3)   # m = 9
    ell = O.num_tag_columns(O.near_lists(g.lattice), 3)
    T = W.tag_matrix(1, g.nboxes, ell)
    with pytest.raises(BlrError) as e:
        _plan(g, 5, 10, 3, T)        # k + p = 15 > m = 9
    assert e.value.name == "BLR_ERR_INVALID_ARG"
    g2 = W.grid_geometry(1, 2, 20)  # two touching boxes: empty far field
    ell2 = O.num_tag_columns(O.near_lists(g2.lattice), 3)
    with pytest.raises(BlrError) as e:
        _plan(g2, 2, 2, 3, W.tag_matrix(1, 2, ell2))
    assert e.value.name == "BLR_ERR_GEOMETRY"
    bad = W.grid_geometry(2, 4, 3)
    bad.box_ptr = bad.box_ptr.copy()
    bad.box_ptr[3] = bad.box_ptr[2]          # empty box
    with pytest.raises(BlrError) as e:
        _plan(bad, 2, 2, 3, T)
    assert e.value.name == "BLR_ERR_INVALID_ARG"
    Tn = T.copy()
    Tn[0, 0] = np.nan
    with pytest.raises(BlrError) as e:
        _plan(g, 2, 2, 3, Tn)
    assert e.value.name == "BLR_ERR_INVALID_ARG"
    # rank-deficient tag submatrix: two identical rows of T among neighbours
    Tr = T.copy()
    Tr[1] = Tr[0]
    with pytest.raises(BlrError) as e:
        _plan(g, 2, 2, 3, Tr)
    assert e.value.name == "BLR_ERR_GEOMETRY"


def test_null_outputs_are_rejected():
    import ctypes
    L = _lib()
    g = W.grid_geometry(2, 4, 3)
    from paper_2501_05528_amd.api import _geometry
    geo, keep = _geometry(g.box_ptr, g.lattice)
    assert L.blr_tag_columns(ctypes.byref(geo), 3, None) == 1
    assert L.blr_tag_plan(ctypes.byref(geo), None, None) == 1
    assert b"NULL" in L.blr_last_error_message()


def chebyshev_lists(lattice, radius):
    """Neighbour lists for a wider admissibility: lattice Chebyshev distance <= radius."""
    lat = np.asarray(lattice)
    return [[j for j in range(len(lat)) if int(np.max(np.abs(lat[i] - lat[j]))) <= radius]
            for i in range(len(lat))]


@pytest.mark.parametrize("dim,B,radius", [(2, 7, 2), (1, 12, 1), (3, 5, 1), (2, 6, 1)])
def test_plan_with_explicit_lists_matches_oracle(dim, B, radius):
    from paper_2501_05528_amd.api import Plan, tag_columns
    g = W.grid_geometry(dim, B, 3)
    near = chebyshev_lists(g.lattice, radius)
    far = O.far_lists(near, g.nboxes)
    ell = O.num_tag_columns(near, 3)
    assert tag_columns(g.box_ptr, None, 3, near=near) == ell
    T = W.tag_matrix(300 + dim, g.nboxes, ell)
    pl = Plan(g.box_ptr, None, 2, T, p=1, extra_tag_cols=3, near=near)
    near_ptr, near_idx, colour, _ = pl.lists()
    assert near_idx.tolist() == [j for n in near for j in n]
    assert colour.tolist() == O.greedy_colours(near).tolist()
    assert pl.info["ncolours"] == int(np.max(colour)) + 1
    for i in range(g.nboxes):           # every probe meets at most one neighbour per colour
        assert len({int(colour[j]) for j in near[i]}) == len(near[i])
    z, rho = pl.tags()
    zo, rhoo = O.tag_plan(T, near, far)
    assert np.allclose(rho, rhoo, rtol=1e-9, atol=0)
    assert np.allclose(z, zo, rtol=0, atol=1e-9)
    # the lattice together with the same lists: identical plan
    pl2 = Plan(g.box_ptr, g.lattice, 2, T, p=1, extra_tag_cols=3, near=near)
    assert all(np.array_equal(a, b) for a, b in zip(pl.lists(), pl2.lists()))


def test_explicit_list_errors():
    from paper_2501_05528_amd.api import BlrError, Plan
    g = W.grid_geometry(2, 5, 3)
    near = chebyshev_lists(g.lattice, 1)
    ell = O.num_tag_columns(near, 3)
    T = W.tag_matrix(7, g.nboxes, ell)
    cases = []
    no_self = [list(n) for n in near]
    no_self[3].remove(3)
    cases.append((no_self, "BLR_ERR_INVALID_ARG", T))
    unsorted = [list(n) for n in near]
    unsorted[4] = unsorted[4][::-1]
    cases.append((unsorted, "BLR_ERR_INVALID_ARG", T))
    out_of_range = [list(n) for n in near]
    out_of_range[0] = out_of_range[0] + [g.nboxes]
    cases.append((out_of_range, "BLR_ERR_INVALID_ARG", T))
    asym = [list(n) for n in near]
    asym[0] = sorted(asym[0] + [24])     # 24 lists no 0
    cases.append((asym, "BLR_ERR_GEOMETRY", W.tag_matrix(7, g.nboxes, O.num_tag_columns(asym, 3))))
    everything = [list(range(g.nboxes)) for _ in range(g.nboxes)]
    cases.append((everything, "BLR_ERR_GEOMETRY", W.tag_matrix(7, g.nboxes, g.nboxes + 4)))
    for lists, name, Tc in cases:
        with pytest.raises(BlrError) as e:
            Plan(g.box_ptr, None, 2, Tc, p=1, extra_tag_cols=3, near=lists)
        assert e.value.name == name, (name, e.value)


def test_comparison_and_rank_entry_points_validate_on_the_host():
    """Alg. 1 / Alg. 3 / rank entry points: the block-nullification width equals the
    oracle's, and NULL outputs or operators are refused before any device work."""
    import ctypes
    from paper_2501_05528_amd.api import Plan
    L = _lib()
    g = W.grid_geometry(2, (5, 4), (3, 4))
    near = O.near_lists(g.lattice)
    T = W.tag_matrix(7, g.nboxes, O.num_tag_columns(near, 3))
    pl = Plan(g.box_ptr, g.lattice, 2, T, p=1, extra_tag_cols=3)
    s = ctypes.c_int64()
    assert L.blr_bn_min_columns(pl._h, ctypes.byref(s)) == 0
    assert s.value == O.bn_columns(g.box_ptr, near, 3) == 3 + 9 * 12
    assert L.blr_bn_min_columns(pl._h, None) == 1
    out = ctypes.c_void_p()
    k = ctypes.c_int32()
    dummy = ctypes.c_void_p(8)                # never dereferenced: the operator check fails first
    assert L.blr_basic_compress(pl._h, None, dummy, dummy, 0, None, ctypes.byref(out), None) == 1
    assert b"operator" in L.blr_last_error_message()
    assert L.blr_basic_compress(pl._h, None, dummy, dummy, 0, None, None, None) == 1
    assert L.blr_bn_compress(pl._h, None, s.value, dummy, dummy, 0, None, ctypes.byref(out), None) == 1
    assert out.value is None
    assert L.blr_tag_rank(pl._h, None, dummy, dummy, 1e-8, None, ctypes.byref(k), None) == 1
    assert L.blr_tag_rank(pl._h, None, dummy, dummy, 1e-8, None, None, None) == 1
