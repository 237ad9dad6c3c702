"""Pins of the oracle's surface export and voxelisation (oracle/post.py):
closed-surface invariants (every directed edge met once in each direction,
divergence-theorem volume = solid element count, area = face count), a face
count by a second formula, the STL byte layout read back with struct, and the
winding number against boxes and spheres."""

import struct

import numpy as np
import pytest

import synth
from oracle import post


def face_count_by_neighbours(x, dims, thr=0.5):
    """6 per solid element minus one per solid face-neighbour inside the grid."""
    nx, ny, nz = dims
    S = (np.asarray(x) > thr).reshape(nz, ny, nx)
    n = 6 * int(S.sum())
    n -= 2 * int((S[:, :, 1:] & S[:, :, :-1]).sum())
    n -= 2 * int((S[:, 1:, :] & S[:, :-1, :]).sum())
    n -= 2 * int((S[1:, :, :] & S[:-1, :, :]).sum())
    return n


def assert_closed(tris):
    e = post.directed_edges(tris)
    fwd = np.unique(e, axis=0, return_counts=True)
    rev = np.unique(np.hstack([e[:, 3:], e[:, :3]]), axis=0, return_counts=True)
    assert np.array_equal(fwd[0], rev[0]) and np.array_equal(fwd[1], rev[1])
    assert fwd[1].max() <= 2  # an edge shared by 4 faces may appear twice in each direction


def test_single_voxel_is_a_closed_unit_cube():
    tris, nrm = post.surface_triangles(np.array([1.0]), (1, 1, 1))
    assert tris.shape == (12, 3, 3)
    assert abs(post.enclosed_volume(tris) - 1.0) < 1e-15
    assert_closed(tris)
    # every normal points away from the cube's centre and equals the cross product's direction
    cen = tris.mean(axis=1) - 0.5
    assert np.all(np.einsum("ij,ij->i", cen, nrm) > 0)
    cr = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    np.testing.assert_allclose(cr, nrm, atol=0)


@pytest.mark.parametrize("seed,dims", [(0, (5, 4, 3)), (1, (7, 3, 6)), (2, (4, 4, 4))])
def test_random_voxel_surface_invariants(seed, dims):
    x = synth.random_voxels(seed, dims, 0.45)
    h, origin = 0.5, (1.0, -2.0, 0.25)
    tris, nrm = post.surface_triangles(x, dims, origin=origin, h=h)
    nsolid = int((x > 0.5).sum())
    assert abs(post.enclosed_volume(tris) - nsolid * h ** 3) < 1e-12
    assert len(tris) == 2 * face_count_by_neighbours(x, dims)
    area = 0.5 * np.linalg.norm(np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]), axis=1)
    np.testing.assert_allclose(area, 0.5 * h * h, rtol=0, atol=1e-15)
    assert_closed(tris)
    assert np.all(np.abs(nrm).sum(axis=1) == 1.0)


def test_stl_image_layout():
    x = synth.random_voxels(3, (3, 2, 2), 0.6)
    tris, nrm = post.surface_triangles(x, (3, 2, 2))
    img = post.stl_image(tris, nrm, b"abc")
    n = len(tris)
    assert len(img) == 84 + 50 * n and img[:3] == b"abc" and img[3:80] == b" " * 77
    assert struct.unpack_from("<I", img, 80)[0] == n
    for t in range(n):
        vals = struct.unpack_from("<12fH", img, 84 + 50 * t)
        assert vals[12] == 0
        np.testing.assert_array_equal(np.array(vals[:3]), nrm[t])
        np.testing.assert_array_equal(np.array(vals[3:12]).reshape(3, 3), tris[t])


def test_winding_number_of_box_and_sphere():
    box = synth.box_mesh([0.2, 0.1, 0.3], [2.7, 1.9, 1.4])
    pts = np.array([[1.0, 1.0, 1.0], [0.1, 1.0, 1.0], [3.0, 0.5, 0.5], [2.6, 1.8, 1.35]])
    np.testing.assert_allclose(post.winding_number(box, pts), [1, 0, 0, 1], atol=1e-12)
    # reversed orientation flips the sign only
    np.testing.assert_allclose(post.winding_number(box[:, ::-1], pts), [-1, 0, 0, -1], atol=1e-12)
    sph = synth.sphere_mesh([0.3, -0.2, 0.1], 2.0, 3)
    rng = np.random.default_rng(0)
    d = rng.normal(size=(40, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = np.concatenate([rng.uniform(0.0, 1.8, 20), rng.uniform(2.2, 4.0, 20)])
    w = post.winding_number(sph, np.array([0.3, -0.2, 0.1]) + d * r[:, None])
    np.testing.assert_allclose(w, np.where(r < 2.0, 1.0, 0.0), atol=1e-9)


def test_voxelize_box_and_round_trip():
    dims = (8, 6, 5)
    m = post.voxelize(synth.box_mesh([2.0, 1.0, 0.0], [6.0, 4.0, 3.0]), dims, code_inside=0, code_outside=1)
    e = np.arange(np.prod(dims))
    i, j, k = e % 8, (e // 8) % 6, e // 48
    ref = np.where((i >= 2) & (i < 6) & (j >= 1) & (j < 4) & (k < 3), 0, 1)
    np.testing.assert_array_equal(m, ref)
    # surface of a random voxel set, voxelised again: the same elements (cavities included)
    x = synth.random_voxels(4, (6, 5, 4), 0.5)
    tris, _ = post.surface_triangles(x, (6, 5, 4), origin=(0.5, 0.0, -1.0), h=0.75)
    back = post.voxelize(tris, (6, 5, 4), origin=(0.5, 0.0, -1.0), h=0.75, code_inside=2, code_outside=0)
    np.testing.assert_array_equal(back == 2, x > 0.5)


def test_threshold_is_strict():
    """Solid means xPhys strictly above the threshold: a value equal to it is not."""
    x = np.array([0.5, 0.5 + 1e-12, 0.4999])
    faces = post.boundary_faces(x, (3, 1, 1), 0.5)
    assert {f[0] for f in faces} == {1}
    assert len(faces) == 6
