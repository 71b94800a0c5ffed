"""VTK output of the full cell structure (``Context.vt_structure``): an XML unstructured grid
(.vtu) of polyhedron cells, one per owned particle, with per-cell data arrays.

Layout of the file: the points are every cell's vertices, cell after cell (cells do not share
points); each cell lists its own points as connectivity and its faces in the ``faces`` /
``faceoffsets`` arrays (per cell: the face count, then per face the vertex count and the point
ids, counter-clockwise seen from outside).  Arrays are appended as raw little-endian binary
with 64-bit size headers.
"""
from __future__ import annotations

import numpy as np

VTK_POLYHEDRON = 42


def _host(a):
    if hasattr(a, "cpu"):
        a = a.cpu().numpy()
    return np.asarray(a)


def polyhedra_arrays(vert_off, face_off, loop_off, loop_vert):
    """The VTK cell arrays for CSR structure arrays (host or device): connectivity, offsets,
    faces and faceoffsets (int64)."""
    voff = _host(vert_off).astype(np.int64)
    foff = _host(face_off).astype(np.int64)
    loff = _host(loop_off).astype(np.int64)
    lv = _host(loop_vert).astype(np.int64)
    n = len(voff) - 1
    nf = int(foff[-1])
    nl = int(loff[nf]) if nf > 0 else 0
    connectivity = np.arange(int(voff[-1]), dtype=np.int64)
    offsets = voff[1:].copy()
    # the face stream of cell c: [F_c, len_f, ids of f ...] for its faces f in order.  Its
    # header sits at c + face_off[c] + loop_off[face_off[c]], face f's count at
    # c + 1 + f + loop_off[f], and loop entry l of face f at c + f + 2 + l.
    cell_of_face = np.repeat(np.arange(n, dtype=np.int64), np.diff(foff))
    face_of_loop = np.repeat(np.arange(nf, dtype=np.int64), np.diff(loff[: nf + 1]))
    faces = np.empty(n + nf + nl, dtype=np.int64)
    lstart = loff[np.minimum(foff, nf)] if nf > 0 else np.zeros(n + 1, np.int64)
    faces[np.arange(n) + foff[:-1] + lstart[:-1]] = np.diff(foff)
    f = np.arange(nf, dtype=np.int64)
    faces[cell_of_face + 1 + f + loff[:nf]] = np.diff(loff[: nf + 1])
    l = np.arange(nl, dtype=np.int64)
    c = cell_of_face[face_of_loop]
    faces[c + face_of_loop + 2 + l] = voff[c] + lv[:nl]
    faceoffsets = np.arange(1, n + 1) + foff[1:] + lstart[1:]
    return connectivity, offsets, faces, faceoffsets


def write_vtu(path, structure, cell_data=None):
    """Write a ``Structure`` (or any object with vert_off, verts, face_off, loop_off, loop_vert)
    as a .vtu file.  ``cell_data`` maps names to per-cell arrays (n or n x k)."""
    verts = _host(structure.verts).astype(np.float64).reshape(-1, 3)
    conn, offs, faces, foffs = polyhedra_arrays(structure.vert_off, structure.face_off, structure.loop_off,
                                                structure.loop_vert)
    n = len(offs)
    types = np.full(n, VTK_POLYHEDRON, dtype=np.uint8)
    blocks = []
    pos = [0]

    def add(arr):
        a = np.ascontiguousarray(arr)
        off = pos[0]
        blocks.append(a)
        pos[0] += 8 + a.nbytes
        return off

    def da(name, arr, vtype, ncomp=1):
        return ('<DataArray type="%s" Name="%s" NumberOfComponents="%d" format="appended" offset="%d"/>'
                % (vtype, name, ncomp, add(arr)))

    kinds = {np.dtype(np.float64): "Float64", np.dtype(np.float32): "Float32", np.dtype(np.int64): "Int64",
             np.dtype(np.int32): "Int32", np.dtype(np.uint8): "UInt8"}
    cd = []
    for name, arr in (cell_data or {}).items():
        a = _host(arr)
        if a.shape[0] != n:
            raise ValueError("cell data %r has %d rows, expected %d" % (name, a.shape[0], n))
        if a.dtype not in kinds:
            a = a.astype(np.float64)
        cd.append(da(name, a, kinds[a.dtype], 1 if a.ndim == 1 else a.shape[1]))
    head = [
        '<?xml version="1.0"?>',
        '<VTKFile type="UnstructuredGrid" version="1.0" byte_order="LittleEndian" header_type="UInt64">',
        "<UnstructuredGrid>",
        '<Piece NumberOfPoints="%d" NumberOfCells="%d">' % (len(verts), n),
        "<Points>", da("Points", verts, "Float64", 3), "</Points>",
        "<Cells>",
        da("connectivity", conn, "Int64"), da("offsets", offs, "Int64"), da("types", types, "UInt8"),
        da("faces", faces, "Int64"), da("faceoffsets", foffs, "Int64"),
        "</Cells>",
        "<CellData>", *cd, "</CellData>",
        "</Piece>",
        "</UnstructuredGrid>",
        '<AppendedData encoding="raw">',
    ]
    with open(path, "wb") as fh:
        fh.write(("\n".join(head) + "\n_").encode())
        for a in blocks:
            fh.write(np.uint64(a.nbytes).tobytes())
            fh.write(a.astype(a.dtype.newbyteorder("<"), copy=False).tobytes())
        fh.write(b"\n</AppendedData>\n</VTKFile>\n")


def read_vtu(path):
    """Read back a file written by ``write_vtu``: a dict of name -> numpy array."""
    import xml.etree.ElementTree as ET

    raw = open(path, "rb").read()
    mark = raw.index(b'<AppendedData encoding="raw">')
    start = raw.index(b"_", mark) + 1
    root = ET.fromstring(raw[:mark].decode() + "</VTKFile>")
    types = {"Float64": np.float64, "Float32": np.float32, "Int64": np.int64, "Int32": np.int32, "UInt8": np.uint8}
    out = {}
    for e in root.iter("DataArray"):
        off = start + int(e.get("offset"))
        nbytes = int(np.frombuffer(raw, np.uint64, 1, off)[0])
        a = np.frombuffer(raw, types[e.get("type")], nbytes // np.dtype(types[e.get("type")]).itemsize, off + 8)
        k = int(e.get("NumberOfComponents", "1"))
        out[e.get("Name")] = a.reshape(-1, k) if k > 1 else a
    return out
