"""Pins of the oracle's cell tracking (Sec. 5) against library routines and
closed forms: connected components against scipy's labelling with face
connectivity, squared distances against scipy's exact Euclidean distance
transform, centres and backward links on spheres whose tracks are known, and
the joining of partial trajectories by tangent prolongation."""
import numpy as np
import pytest

scipy_ndimage = pytest.importorskip("scipy.ndimage")


def u_from_masks(orc, n, masks):
    """padded u with 1.0 on the given interior voxels (masks: (t, z, y, x) bool)"""
    u = np.zeros(orc.padded_shape(n))
    u[1:-1, 1:-1, 1:-1, 1:-1][masks] = 1.0
    return u


def spheres(n, tracks, radius):
    """(t, z, y, x) mask of balls |X - c_l| <= radius around integer centres"""
    n1, n2, n3, n4 = n
    z, y, x = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    m = np.zeros((n4, n3, n2, n1), dtype=bool)
    for tr in tracks:
        for l, c in enumerate(tr):
            if c is None:
                continue
            m[l] |= (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 <= radius * radius
    return m


@pytest.mark.parametrize("density", [0.3, 0.55, 0.7])
def test_labels_match_scipy_face_connectivity(orc, density):
    rng = np.random.default_rng(int(density * 100))
    n = (13, 11, 9, 3)
    u = rng.uniform(0.0, 1.0, size=orc.padded_shape(n))
    lab = orc.track_label(n, u, 1.0 - density)
    inner = u[1:-1, 1:-1, 1:-1, 1:-1] >= 1.0 - density
    assert np.array_equal(lab >= 0, inner)
    idx = np.arange(lab.size).reshape(lab.shape)
    st = scipy_ndimage.generate_binary_structure(3, 1)
    for l in range(n[3]):
        ref, k = scipy_ndimage.label(inner[l], structure=st)
        # same partition, each part named by its smallest index
        for c in range(1, k + 1):
            sel = ref == c
            names = np.unique(lab[l][sel])
            assert names.size == 1 and names[0] == idx[l][sel].min()


def test_dist2_matches_scipy_edt(orc):
    rng = np.random.default_rng(3)
    n = (12, 10, 9, 2)
    u = rng.uniform(0.0, 1.0, size=orc.padded_shape(n))
    u[1:-1, 2:7, 2:8, 3:9] = 1.0                  # a solid block, so distances exceed 1
    lab = orc.track_label(n, u, 0.35)
    d2 = orc.track_dist2(n, lab)
    for l in range(n[3]):
        mask = np.pad(lab[l] >= 0, 1)             # the outside of the image counts as outside
        edt = scipy_ndimage.distance_transform_edt(mask)[1:-1, 1:-1, 1:-1]
        assert np.array_equal(d2[l], np.rint(edt ** 2).astype(np.int32))


def test_centres_and_links_of_moving_spheres(orc):
    """Balls centred on voxels: each frame's cell centre is the ball centre; a
    ball moving 1 voxel per frame links by its centre (kind 1), one moving 4
    voxels (radius 3) by overlap (kind 2), one moving 9 voxels not at all."""
    n = (40, 16, 14, 4)
    slow = [(5 + l, 5, 5) for l in range(4)]
    fast = [(6 + 4 * l, 12, 9) for l in range(4)]
    jump = [(2 + 9 * l, 3, 10) if l < 4 else None for l in range(4)]
    res = orc.track(n, u_from_masks(orc, n, spheres(n, [slow, fast], 3.0) | spheres(n, [jump], 1.5)), 0.5, 0.0)
    cells = res["cells"]
    assert len(cells) == 12
    want = {}
    for name, tr in (("slow", slow), ("fast", fast), ("jump", jump)):
        for l, c in enumerate(tr):
            want[(l, c)] = name
    got = {}
    for c in cells:
        xyz = orc.voxel_xyz(n, c["centre"])
        key = (int(c["frame"]), xyz)
        assert key in want, key
        got[int(c["name"])] = (want[key], int(c["frame"]), int(c["kind"]), int(c["prev"]))
    for name, (who, f, kind, prev) in got.items():
        if f == 0:
            assert kind == 0 and prev == -1
            continue
        assert kind == {"slow": 1, "fast": 2, "jump": 0}[who], (who, f, kind)
        if prev >= 0:
            assert got[prev][0] == who and got[prev][1] == f - 1
    tracks = res["tracks"]
    assert sorted(len(t) for t in tracks) == [1, 1, 1, 1, 4, 4]


def test_join_by_prolongation(orc):
    """A ball moving 9 voxels per frame never overlaps itself: four partial
    trajectories of one cell each, joined into one when the radius covers the
    displacement (single cells prolong with zero velocity), not joined when it
    does not; a two-frame gap is never bridged."""
    n = (40, 8, 8, 4)
    jump = [(2 + 9 * l, 3, 3) for l in range(4)]
    u = u_from_masks(orc, n, spheres(n, [jump], 1.5))
    assert len(orc.track(n, u, 0.5, 8.9)["tracks"]) == 4
    t = orc.track(n, u, 0.5, 9.0)["tracks"]
    assert len(t) == 1 and len(t[0]) == 4
    gap = [c if l != 2 else None for l, c in enumerate(jump)]
    assert len(orc.track(n, u_from_masks(orc, n, spheres(n, [gap], 1.5)), 0.5, 40.0)["tracks"]) == 2
    # a trajectory of two cells prolongs with its displacement
    slow2 = [(2, 3, 3), (4, 3, 3), (13, 3, 3), (22, 3, 3)]
    # (its first two cells overlap and link; the forward prolongation of
    # 2 -> 4 is 6, which lies 7 before the third cell; the single fourth cell
    # lies 9 after the single third one)
    u2 = u_from_masks(orc, n, spheres(n, [slow2], 1.5))
    assert [len(x) for x in orc.track(n, u2, 0.5, 0.0)["tracks"]] == [2, 1, 1]
    assert [len(x) for x in orc.track(n, u2, 0.5, 7.0)["tracks"]] == [3, 1]
    assert [len(x) for x in orc.track(n, u2, 0.5, 9.0)["tracks"]] == [4]
