"""CPU tests of the C ABI library: it loads, exports every declared symbol,
and its host-side mesh preparation (validation, renumbering, partitions)
behaves.  No compute call runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth import mesh as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2404_08952_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    return binding


def test_exports_every_declared_symbol():
    b = _lib()
    hdr = open(os.path.join(ROOT, "include", "dolinc.h")).read()
    names = set(re.findall(r"\b(dolinc_[a-z_]+)\s*\(", hdr))
    lib = ctypes.CDLL(b.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(b.SIGNATURES) == names


def test_mesh_prepare_partitions_and_renumbering():
    b = _lib()
    mesh = M.periodic_3d(6, 5, 4, jitter=0.2, seed=1, kinds=M.mixed_kinds(6, 5, 4, 0.4, seed=2), perm_seed=3)
    for renumber in (0, 1, 2):
        for pc in (32, 256):
            perm, st = b.mesh_prepare(mesh, renumber=renumber, part_cells=pc)
            assert sorted(perm.tolist()) == list(range(mesh.n_cells))
            assert st["n_parts"] == -(-mesh.n_cells // pc)
            assert st["n_slots"] == 2 * mesh.n_faces
            assert mesh.n_faces <= st["n_entries"] <= 2 * mesh.n_faces
            if renumber == 0:
                assert np.array_equal(perm, np.arange(mesh.n_cells))


def test_locality_renumbering_reduces_seams():
    """The Hilbert order of a shuffled mesh cuts it into compact partitions:
    far fewer duplicated seam faces than the shuffled order.  (Reverse
    Cuthill-McKee keeps BFS level sets together, so its chunks are thin
    slices and it helps little here.)"""
    b = _lib()
    mesh = M.periodic_3d(16, jitter=0.2, seed=1, kinds=M.KUHN6, perm_seed=7)
    dup = {}
    for r in (0, 1, 2):
        _p, st = b.mesh_prepare(mesh, renumber=r, part_cells=256)
        dup[r] = st["n_entries"] / mesh.n_faces - 1.0
    assert dup[2] < 0.25 and dup[0] > 0.9 and dup[2] < dup[1] <= dup[0], dup


def test_mesh_validation_errors():
    b = _lib()
    mesh = M.periodic_2d(4, 4, split=1.0)
    bad = M.Mesh(mesh.dim, mesh.nodes, mesh.face_ptr, mesh.face_nodes, mesh.owner.copy(),
                 mesh.neighbour.copy(), mesh.shift, mesh.n_cells, mesh.lengths)
    bad.neighbour[3] = bad.owner[3]
    with pytest.raises(b.DolincError) as e:
        b.mesh_prepare(bad)
    assert e.value.status == b.EMESH
    bad.neighbour[3] = mesh.n_cells + 5
    with pytest.raises(b.DolincError) as e:
        b.mesh_prepare(bad)
    assert e.value.status == b.EMESH
    # a cell that lost faces is not closed
    keep = np.ones(mesh.n_faces, dtype=bool)
    c0 = mesh.owner[0]
    keep[(mesh.owner == c0) | (mesh.neighbour == c0)] = False
    idx = np.nonzero(keep)[0]
    fptr = np.arange(0, 2 * idx.size + 1, 2, dtype=np.int64)
    fn = mesh.face_nodes.reshape(-1, 2)[idx].reshape(-1)
    bad2 = M.Mesh(2, mesh.nodes, fptr, fn, mesh.owner[idx], mesh.neighbour[idx], mesh.shift[idx],
                  mesh.n_cells, mesh.lengths)
    with pytest.raises(b.DolincError) as e:
        b.mesh_prepare(bad2)
    assert e.value.status == b.EMESH
    with pytest.raises(b.DolincError) as e:
        b.mesh_prepare(mesh, part_cells=5000)
    assert e.value.status == b.EINVAL


def test_no_device_is_an_error_not_a_fallback():
    """Without a GPU the compute path fails loudly (EHIP) instead of running
    anything on the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    b = _lib()
    lib = b.load()
    mesh = M.periodic_2d(4, 4, split=1.0)
    d, keep = b.mesh_desc(mesh)
    h = ctypes.c_void_p()
    st = lib.dolinc_create(ctypes.byref(d), None, ctypes.byref(h))
    assert st == b.EHIP
    assert lib.dolinc_residual(ctypes.c_void_p(1), None, None, None) == b.ESTATE
    del keep


def test_mesh_prepare_with_boundary_faces():
    """Boundary faces (neighbour -1 with a patch) become auxiliary rows after
    the interior cells; a boundary face without a patch, or a two-cell face
    with one, is a mesh error."""
    from paper_2404_08952_amd import binding as B
    from synth import mesh as M
    m = M.bounded(M.periodic_3d(6, 4, 3, jitter=0.2, seed=7), 0)
    nb = int((m.neighbour < 0).sum())
    perm, st = B.mesh_prepare(m)
    assert st["n_rows"] == m.n_cells + nb and st["n_boundary_faces"] == nb
    assert np.array_equal(np.sort(perm), np.arange(m.n_cells))
    bad = M.Mesh(m.dim, m.nodes, m.face_ptr, m.face_nodes, m.owner, m.neighbour, m.shift, m.n_cells,
                 m.lengths, dict(m.info), np.where(m.patch >= 0, -1, m.patch).astype(np.int32))
    with pytest.raises(B.DolincError, match="patch"):
        B.mesh_prepare(bad)
    bad2 = M.Mesh(m.dim, m.nodes, m.face_ptr, m.face_nodes, m.owner, m.neighbour, m.shift, m.n_cells,
                  m.lengths, dict(m.info), np.where(m.patch >= 0, m.patch, 0).astype(np.int32))
    with pytest.raises(B.DolincError, match="patch"):
        B.mesh_prepare(bad2)
