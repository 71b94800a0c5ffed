"""The VTK writer (host side): structure arrays assembled from oracle cells are written as a
.vtu file, read back, and the polyhedron face stream is decoded sequentially and compared with
the cells it came from."""
import types

import numpy as np

from paper_1601_06429_amd import vtk
from paper_1601_06429_amd import workloads as wl


def _csr(cells):
    """CSR structure arrays (as vt_structure lays them out) from [(verts, faces)]."""
    vo, fo, lo = [0], [0], [0]
    verts, fnbr, lv = [], [], []
    for v, faces in cells:
        verts.append(v)
        vo.append(vo[-1] + len(v))
        for j, loop in faces:
            fnbr.append(j)
            lv.extend(loop.tolist())
            lo.append(lo[-1] + len(loop))
        fo.append(fo[-1] + len(faces))
    return types.SimpleNamespace(vert_off=np.array(vo), verts=np.concatenate(verts), face_off=np.array(fo),
                                 face_nbr=np.array(fnbr, np.int32), loop_off=np.array(lo),
                                 loop_vert=np.array(lv, np.int32))


def test_vtu_round_trip(oracle, tmp_path):
    p = wl.lattice("bcc", 4)
    rng = np.random.default_rng(4)
    p = np.mod(p + 0.01 * rng.standard_normal(p.shape), 1.0)
    q = [0, 3, 50, 101]
    cells = [oracle.structure(p, 0.0, 1.0, i) for i in q]
    st = _csr(cells)
    vol = np.array([1.0, 2.0, 3.0, 4.0])
    path = str(tmp_path / "cells.vtu")
    vtk.write_vtu(path, st, cell_data={"volume": vol, "id": np.array(q, np.int32)})
    r = vtk.read_vtu(path)
    np.testing.assert_array_equal(r["Points"], st.verts)
    np.testing.assert_array_equal(r["offsets"], st.vert_off[1:])
    np.testing.assert_array_equal(r["connectivity"], np.arange(len(st.verts)))
    assert np.all(r["types"] == vtk.VTK_POLYHEDRON)
    np.testing.assert_array_equal(r["volume"], vol)
    np.testing.assert_array_equal(r["id"], q)
    # decode the face stream cell by cell
    fs, fo = r["faces"], r["faceoffsets"]
    k = 0
    for c, (v, faces) in enumerate(cells):
        nf = fs[k]
        k += 1
        assert nf == len(faces)
        for j, loop in faces:
            m = fs[k]
            assert m == len(loop)
            np.testing.assert_array_equal(fs[k + 1:k + 1 + m], st.vert_off[c] + loop)
            k += 1 + m
        assert fo[c] == k
    assert k == len(fs)


def test_polyhedra_arrays_empty_cells():
    # a cell without structure (a failed cell) contributes a zero face count
    st = types.SimpleNamespace(vert_off=np.array([0, 4, 4]), face_off=np.array([0, 4, 4]),
                               loop_off=np.array([0, 3, 6, 9, 12]),
                               loop_vert=np.array([0, 1, 2, 0, 3, 1, 1, 3, 2, 2, 3, 0], np.int32))
    conn, offs, faces, foffs = vtk.polyhedra_arrays(st.vert_off, st.face_off, st.loop_off, st.loop_vert)
    assert faces.tolist() == [4, 3, 0, 1, 2, 3, 0, 3, 1, 3, 1, 3, 2, 3, 2, 3, 0, 0]
    assert foffs.tolist() == [17, 18]
    assert offs.tolist() == [4, 4]
