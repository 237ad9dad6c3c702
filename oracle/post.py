"""Before and after the loop (Workflow and Key Features section): the voxel
surface of a thresholded design as an STL mesh, and the elements inside a
closed STL mesh (a design domain or an obstacle).

Test infrastructure only, like the rest of the oracle.

* surface: element e is solid when xPhys_e > threshold; every face shared by a
  solid element and a non-solid element or the outside of the grid is a square
  of side h split into two triangles; each triangle's vertex order is chosen so
  that its normal (v1 - v0) x (v2 - v0) points out of the solid element.
* STL image: the binary format (80-byte header, little-endian uint32 triangle
  count, per triangle 12 float32 -- normal, three vertices -- and a uint16
  attribute of 0).
* inside test: the generalised winding number of the mesh about the element
  centroid, sum over triangles of the solid angle they subtend divided by 4 pi
  (solid angle of a triangle by the formula of Van Oosterom and Strackee,
  IEEE Trans. Biomed. Eng. 30, 1983); it is +-1 inside a closed mesh (sign by
  orientation) and 0 outside, so |w| > 1/2 is "inside" for either orientation.
  This is a different construction from a ray-crossing count.
"""

from __future__ import annotations

import numpy as np

AXIS_STEPS = [(-1, 0), (1, 0), (-1, 1), (1, 1), (-1, 2), (1, 2)]  # (side, axis): -x, +x, -y, +y, -z, +z


def solid_elements(xphys, threshold=0.5):
    return np.asarray(xphys) > threshold


def boundary_faces(xphys, dims, threshold=0.5):
    """(element, side, axis) of every boundary face, elements in numbering order
    and faces per element in the order -x, +x, -y, +y, -z, +z."""
    nx, ny, nz = dims
    S = solid_elements(xphys, threshold).reshape(nz, ny, nx)  # [k, j, i]
    faces = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if not S[k, j, i]:
                    continue
                e = i + nx * (j + ny * k)
                for side, axis in AXIS_STEPS:
                    n = [i, j, k]
                    n[axis] += side
                    inside = 0 <= n[0] < nx and 0 <= n[1] < ny and 0 <= n[2] < nz
                    if not inside or not S[n[2], n[1], n[0]]:
                        faces.append((e, side, axis))
    return faces


def surface_triangles(xphys, dims, threshold=0.5, origin=(0.0, 0.0, 0.0), h=1.0):
    """(triangles (n, 3, 3), normals (n, 3)) in float64, two per boundary face."""
    nx, ny, _ = dims
    tris, normals = [], []
    for e, side, axis in boundary_faces(xphys, dims, threshold):
        ijk = np.array([e % nx, (e // nx) % ny, e // (nx * ny)], dtype=float)
        # the face lies in the plane coordinate[axis] = ijk[axis] (+1 for side +1)
        u, v = [a for a in range(3) if a != axis]
        base = ijk.copy()
        base[axis] += 1.0 if side > 0 else 0.0
        quad = []
        for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):  # a cycle around the square
            c = base.copy()
            c[u] += du
            c[v] += dv
            quad.append(np.asarray(origin, float) + h * c)
        nrm = np.zeros(3)
        nrm[axis] = float(side)
        for t in ((quad[0], quad[1], quad[2]), (quad[0], quad[2], quad[3])):
            a, b, c = t
            if np.dot(np.cross(b - a, c - a), nrm) < 0:  # orient outward
                t = (a, c, b)
            tris.append(np.array(t))
            normals.append(nrm.copy())
    return np.array(tris).reshape(-1, 3, 3), np.array(normals).reshape(-1, 3)


def stl_image(tris, normals, header=b""):
    """Bytes of a binary STL file."""
    n = len(tris)
    rec = np.zeros(n, dtype=[("normal", "<f4", 3), ("v", "<f4", (3, 3)), ("attr", "<u2")])
    rec["normal"] = np.asarray(normals, np.float32)
    rec["v"] = np.asarray(tris, np.float32)
    head = header[:80].ljust(80, b" ")
    return head + np.array([n], dtype="<u4").tobytes() + rec.tobytes()


def enclosed_volume(tris):
    """Divergence theorem: sum over triangles of v0 . (v1 x v2) / 6."""
    t = np.asarray(tris, float)
    return float(np.einsum("ij,ij->i", t[:, 0], np.cross(t[:, 1], t[:, 2])).sum() / 6.0)


def directed_edges(tris):
    """Directed edges (v_a -> v_b) of every triangle as rows of 6 coordinates."""
    t = np.asarray(tris, float)
    return np.concatenate([np.hstack([t[:, a], t[:, (a + 1) % 3]]) for a in range(3)])


def winding_number(tris, points):
    """Generalised winding number of the mesh about each point."""
    t = np.asarray(tris, float)
    w = np.zeros(len(points))
    for r, p in enumerate(np.asarray(points, float)):
        a, b, c = t[:, 0] - p, t[:, 1] - p, t[:, 2] - p
        la, lb, lc = (np.linalg.norm(x, axis=1) for x in (a, b, c))
        num = np.einsum("ij,ij->i", a, np.cross(b, c))
        den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc + np.einsum("ij,ij->i", a, c) * lb
               + np.einsum("ij,ij->i", b, c) * la)
        w[r] = (2.0 * np.arctan2(num, den)).sum() / (4.0 * np.pi)
    return w


def voxelize(tris, dims, origin=(0.0, 0.0, 0.0), h=1.0, code_inside=0, code_outside=1):
    """int8 element mask: code_inside where the centroid's winding number
    exceeds 1/2 in magnitude, else code_outside."""
    nx, ny, nz = dims
    e = np.arange(nx * ny * nz)
    cen = np.stack([e % nx, (e // nx) % ny, e // (nx * ny)], axis=1) + 0.5
    pts = np.asarray(origin, float) + h * cen
    w = winding_number(tris, pts)
    return np.where(np.abs(w) > 0.5, code_inside, code_outside).astype(np.int8)
