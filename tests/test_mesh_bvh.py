"""The host-built triangle BVH (ms_build_mesh_bvh, no GPU needed): every
triangle lands in exactly one leaf whose box contains it, skip links close
each subtree, and a stackless traversal of a line -- descend on a box hit,
jump to skip otherwise -- reaches every triangle the line crosses (checked
against brute force over all triangles)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def msst():
    """The library loads without a GPU; these calls touch host memory only."""
    import paper_2011_03082_amd as M
    M.lib()
    return M


def build(msst, tris):
    n = tris.shape[0]
    nb = C.c_size_t()
    assert msst.lib().ms_mesh_bvh_size(n, C.byref(nb)) == 0
    nodes = np.zeros(nb.value, np.uint8)
    ts = np.zeros_like(tris)
    nn = C.c_int32()
    assert msst.lib().ms_build_mesh_bvh(tris.ctypes.data, n, nodes.ctypes.data, nb.value, ts.ctypes.data,
                                     C.byref(nn)) == 0
    raw = nodes[: nn.value * 32]
    return ts, raw.view(np.float32).reshape(-1, 8), raw.view(np.int32).reshape(-1, 8)


def crosses(tri, o, d):
    a, b, c = tri[0:3].astype(np.float64), tri[3:6].astype(np.float64), tri[6:9].astype(np.float64)
    e1, e2 = b - a, c - a
    p = np.cross(d, e2)
    det = e1 @ p
    if det == 0:
        return False
    s = o - a
    u = s @ p / det
    q = np.cross(s, e1)
    v = d @ q / det
    return 0 <= u <= 1 and v >= 0 and u + v <= 1


def test_leaves_partition_the_triangles(msst):
    tris = W.mesh_blob(1, 3)
    ts, f, i = build(msst, tris)
    np.testing.assert_array_equal(np.sort(ts.reshape(-1, 9), axis=0), np.sort(tris, axis=0))
    leaf, skip = i[:, 7], i[:, 3]
    covered = np.zeros(len(ts), int)
    for k in np.flatnonzero(leaf >= 0):
        first, cnt = leaf[k] >> 4, leaf[k] & 15
        assert 1 <= cnt <= 4 and skip[k] == k + 1
        covered[first:first + cnt] += 1
        v = ts[first:first + cnt].reshape(-1, 3)
        assert (v >= f[k, 0:3]).all() and (v <= f[k, 4:7]).all()
    assert (covered == 1).all()
    assert skip[0] == len(f)
    for k in np.flatnonzero(leaf < 0):  # children nest inside the parent's box and subtree
        assert k + 1 < skip[k] <= len(f)
        assert (f[k + 1, 0:3] >= f[k, 0:3]).all() and (f[k + 1, 4:7] <= f[k, 4:7]).all()


def test_stackless_traversal_reaches_every_crossed_triangle(msst):
    tris = W.mesh_blob(2, 3)
    ts, f, i = build(msst, tris)
    rng = np.random.default_rng(0)
    for _ in range(100):
        o = rng.uniform(-1.5, 1.5, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        want = {tuple(t) for t in ts if crosses(t, o, d)}
        got, k = set(), 0
        while k < len(f):
            with np.errstate(divide="ignore", invalid="ignore"):
                ta, tb = (f[k, 0:3] - o) / d, (f[k, 4:7] - o) / d
            hit = np.nanmax(np.minimum(ta, tb)) <= np.nanmin(np.maximum(ta, tb))
            if hit and i[k, 7] >= 0:
                first, cnt = i[k, 7] >> 4, i[k, 7] & 15
                got |= {tuple(t) for t in ts[first:first + cnt] if crosses(t, o, d)}
            k = k + 1 if (hit and i[k, 7] < 0) else i[k, 3]
        assert got == want
        assert len(want) % 2 == 0
