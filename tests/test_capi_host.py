"""Host-side checks of the C-ABI library that need no GPU.

* the library loads and exports every function declared in include/jfnk.h;
* the host mesh preprocessing (jfnk_inspect_mesh) reproduces the oracle's
  cell centroids and volumes (same geometric definitions, Section 2.3),
  and reports invalid meshes and options with the documented status codes;
* the bandwidth-reducing renumbering is a permutation and never worse than
  the input order.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import meshgen as mg
from oracle.geometry import mesh_geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jfnk.h")
LIB = os.path.join(ROOT, "paper_2502_17217_amd", "libjfnk.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:jfnk_status|const char\*)\s+(jfnk_\w+)\s*\(", text, re.M)))


def test_header_symbols_exported():
    assert os.path.exists(LIB), "libjfnk.so not built"
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


@pytest.fixture(scope="module")
def jfnk():
    from paper_2502_17217_amd import jfnk as j
    return j


def test_header_constants_match_binding(jfnk):
    """The enum values and flags the binding passes are the header's."""
    text = open(HEADER).read()
    assert int(re.search(r"#define JFNK_PC_Z32 (\d+)", text).group(1)) == jfnk.PC_Z32
    for name, val in re.findall(r"JFNK_PC_(NONE|JACOBI|AMG32|AMG64) = (\d+)", text):
        assert getattr(jfnk, "PC_" + name) == int(val), name
    assert jfnk._pc("amg32+z32") == jfnk.PC_AMG32 | jfnk.PC_Z32
    assert jfnk._pc("jacobi") == jfnk.PC_JACOBI
    with pytest.raises(ValueError):
        jfnk._pc("amg32+z16")


@pytest.mark.parametrize("kind", ["2d", "3d", "annulus"])
def test_inspect_geometry_matches_oracle(jfnk, kind):
    if kind == "2d":
        m = mg.box_mesh_2d(29, 17, 1.3, 0.9, jitter=0.25, seed=4)
    elif kind == "3d":
        m = mg.box_mesh_3d(11, 7, 5, 1.0, 0.8, 0.6, jitter=0.25, seed=5)
    else:
        m = mg.annulus_mesh_2d(6, 40, 0.5, 1.0)
    info, xc, vol = jfnk.inspect_mesh(m, mg.Material(), geometry=True)
    g = mesh_geometry(m)
    assert info["n_cells"] == m["n_cells"]
    assert info["n_internal_faces"] == m["n_internal"]
    assert np.abs(xc - g["xc"]).max() <= 1e-13 * np.abs(g["xc"]).max()
    assert np.abs(vol - g["V"]).max() <= 1e-12 * g["V"].max()


def test_cells_ordered_in_compact_tiles(jfnk):
    """Cells are renumbered into tiles of 256 that are compact blocks: on a
    60x8x5 box a tile's outside neighbours number about its surface (a
    brick of ~8x8x4 cells has 256), far below the 2x256 neighbours of a
    slab of the natural order, and within the LDS budget of the kernels."""
    m = mg.box_mesh_3d(60, 8, 5)
    info = jfnk.inspect_mesh(m, mg.Material())
    assert info["tiled"] == 1
    assert 0 < info["tile_halo_max"] <= 300
    # second ring and face lists of the single-pass kernel: a tile touches
    # at most 3 internal faces per cell plus its incoming faces; every
    # boundary face of the box belongs to exactly one tile
    assert 0 < info["tile_ring2_max"] <= 2 * info["tile_halo_max"]
    assert info["tile_faces_max"] <= 3 * 256 + info["tile_halo_max"]
    assert info["tile_faces_max"] <= info["tile_entries_max"]
    assert info["tile_halo_total"] > 0 and info["tile_ring2_total"] > 0
    assert info["fused"] == 1
    # stretched cells: tiles stay compact in cell counts, not in metres
    m = mg.box_mesh_3d(200, 20, 6, 10.0, 1.0, 1.0)
    info = jfnk.inspect_mesh(m, mg.Material())
    assert info["tiled"] == 1 and info["tile_halo_max"] <= 300


def test_invalid_mesh_reported(jfnk):
    m = mg.box_mesh_3d(3, 3, 3)
    bad = dict(m)
    nb = m["neighbour"].copy()
    nb[0] = m["n_cells"] + 5
    bad["neighbour"] = nb
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.inspect_mesh(bad, mg.Material())
    assert e.value.status == jfnk.E_MESH
    # inverted cell: swap two vertices of every face of one cell -> non-positive volume
    bad2 = dict(m)
    pts = m["points"].copy()
    pts[:, 0] *= -1.0
    bad2["points"] = pts
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.inspect_mesh(bad2, mg.Material())
    assert e.value.status == jfnk.E_MESH


def test_bad_material_and_patches(jfnk):
    m = mg.box_mesh_2d(4, 4)
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.inspect_mesh(m, mg.Material(nu=0.5))
    assert e.value.status == jfnk.E_ARG
    m2 = dict(m)
    m2["patches"] = m["patches"][:-1]      # a boundary face in no patch
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.inspect_mesh(m2, mg.Material())
    assert e.value.status == jfnk.E_ARG


def test_singular_least_squares_matrix(jfnk):
    m = mg.box_mesh_2d(5, 1)            # one cell thick: no y-direction neighbours
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.inspect_mesh(m, mg.Material())
    assert e.value.status == jfnk.E_MESH


def test_first_bad_face_reported(jfnk):
    """Face geometry is computed on parallel host threads in chunks of
    faces; the error names the lowest-numbered bad face, as one pass over
    the faces would, even when a later chunk also holds one."""
    m = mg.box_mesh_2d(100, 100)            # about 20k faces: several chunks
    assert m["n_faces"] > 3 * 4096
    bad = dict(m)
    fpts = m["face_pts"].copy()
    fptr = m["face_ptr"]
    for f in (9500, 2100):                  # zero-length faces (both ends on one point)
        fpts[fptr[f] + 1] = fpts[fptr[f]]
    bad["face_pts"] = fpts
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.inspect_mesh(bad, mg.Material())
    assert e.value.status == jfnk.E_MESH
    assert "face 2100 has zero area" in str(e.value)


def test_batch_reports_lowest_bad_mesh(jfnk):
    """A batch's meshes are prepared on parallel host threads; the error
    reported is the lowest-numbered invalid mesh's, before any device work."""
    good = mg.box_mesh_3d(4, 3, 3)
    bad = dict(good)
    nb = good["neighbour"].copy()
    nb[0] = good["n_cells"] + 5
    bad["neighbour"] = nb
    meshes = [good, good, bad, good, bad, good] * 3
    with pytest.raises(jfnk.JfnkError) as e:
        jfnk.create_batch(meshes, [mg.Material()] * len(meshes), stream=0)  # null stream: no GPU here
    assert e.value.status == jfnk.E_MESH
    assert "batch mesh 2:" in str(e.value)
