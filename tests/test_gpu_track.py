"""Cell tracking on the GPU (subsurf4d_track / subsurf4d_track_join) against
the oracle: labels, squared distances, cell records (centres and backward
links) bit-exact, and the joined trajectories the same."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as orc  # noqa: E402
import synth  # noqa: E402
from paper_2111_11866_amd import binding as B  # noqa: E402


def gpu_track(n, u, level, radius=None):
    cells, lab, d2 = B.track(n, torch.from_numpy(np.ascontiguousarray(u)).to("cuda"), level, join_radius=radius)
    torch.cuda.synchronize()
    return cells, lab.cpu().numpy(), d2.cpu().numpy()


def same_cells(got, ref):
    assert len(got) == len(ref), (len(got), len(ref))
    for f_got, f_ref in (("name", "name"), ("frame", "frame"), ("centre", "centre"), ("dist2", "d2"),
                         ("prev", "prev"), ("kind", "kind")):
        assert np.array_equal(got[f_got], ref[f_ref]), f_got


def chains(cells):
    """trajectories from the links: each cell no other cell links to ends one"""
    by = {int(c["name"]): c for c in cells}
    linked = {int(c["prev"]) for c in cells if c["prev"] >= 0}
    out = []
    for c in cells:
        if int(c["name"]) in linked:
            continue
        ch = [int(c["name"])]
        while by[ch[-1]]["prev"] >= 0:
            ch.append(int(by[ch[-1]]["prev"]))
        out.append(ch[::-1])
    return sorted(out, key=lambda ch: ch[0])


@pytest.mark.parametrize("n,level,seed", [((13, 11, 9, 3), 0.45, 1), ((1, 1, 1, 1), 0.5, 2), ((2, 1, 3, 2), 0.3, 3),
                                          ((40, 23, 12, 3), 0.62, 4), ((64, 7, 5, 4), 0.5, 5)])
def test_track_random_fields(n, level, seed):
    """Random fields: many small and some tortuous cells, ragged extents."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=orc.padded_shape(n))
    cells, lab, d2 = gpu_track(n, u, level)
    ref_lab = orc.track_label(n, u, level)
    assert np.array_equal(lab, ref_lab)
    ref_d2 = orc.track_dist2(n, ref_lab)
    assert np.array_equal(d2, ref_d2)
    same_cells(cells, orc.track_cells(n, ref_lab, ref_d2))


def test_track_percolating_labels():
    """At the percolation density the cells are large and branched: the
    union-find labels equal the oracle's flood fill."""
    n = (96, 80, 24, 2)
    rng = np.random.default_rng(9)
    u = rng.uniform(0.0, 1.0, size=orc.padded_shape(n))
    cells, lab, d2 = gpu_track(n, u, 0.69)
    assert np.array_equal(lab, orc.track_label(n, u, 0.69))


def test_track_config1_spheres_and_join():
    """The noisy spheres of the config-1 image thresholded at 0.5: three cells
    per frame, centres and links bit-exact; the joined trajectories (radius
    3) equal the oracle's and follow the three spheres."""
    img = synth.spheres_cfg1()
    n = img.n
    u = np.zeros(orc.padded_shape(n))
    u[1:-1, 1:-1, 1:-1, 1:-1] = img.image
    cells, lab, d2 = gpu_track(n, u, 0.5, radius=3.0)
    ref = orc.track(n, u, 0.5, 3.0)
    assert np.array_equal(lab, ref["label"]) and np.array_equal(d2, ref["d2"])
    plain, _, _ = gpu_track(n, u, 0.5)
    same_cells(plain, ref["cells"])
    assert chains(cells) == sorted(ref["tracks"], key=lambda ch: ch[0])
    big = [t for t in ref["tracks"] if len(t) == n[3]]
    assert len(big) >= 3


def test_track_capacity_and_empty():
    n = (9, 8, 7, 2)
    u = np.zeros(orc.padded_shape(n))
    cells, lab, d2 = gpu_track(n, u, 0.5)
    assert len(cells) == 0 and (lab == -1).all() and (d2 == 0).all()
    u[1:-1, 1:-1, 1:-1, 1:-1] = np.random.default_rng(2).uniform(size=orc.interior_shape(n))
    with pytest.raises(B.Subsurf4dError) as e:
        B.track(n, torch.from_numpy(u).to("cuda"), 0.5, capacity=3)
    assert e.value.status == B.EWORKSPACE


def test_track_nuclei_crop_against_oracle_and_edt():
    """A config-2-like crop (160 x 160 x 48 voxels, 4 frames, 120 Brownian
    nuclei) thresholded as the segmentation: labels equal the oracle's flood
    fill; distances equal scipy's exact Euclidean transform (pinned against
    the oracle's brute force in the CPU tests; the brute force is too slow
    here); the cell records equal the oracle's records built from those."""
    ndi = pytest.importorskip("scipy.ndimage")
    n = (160, 160, 48, 4)
    img = synth.nuclei_cfg2(n=n, n_nuclei=120, geom_seed=31, noise_seed=32)
    u = np.zeros(orc.padded_shape(n))
    u[1:-1, 1:-1, 1:-1, 1:-1] = img.image.astype(np.float64) / 255.0
    level = 0.35
    cells, lab, d2 = gpu_track(n, u, level)
    ref_lab = orc.track_label(n, u, level)
    assert np.array_equal(lab, ref_lab)
    ref_d2 = np.empty_like(d2)
    for l in range(n[3]):
        edt = ndi.distance_transform_edt(np.pad(ref_lab[l] >= 0, 1))[1:-1, 1:-1, 1:-1]
        ref_d2[l] = np.rint(edt ** 2).astype(np.int32)
    assert np.array_equal(d2, ref_d2)
    ref_cells = orc.track_cells(n, ref_lab, ref_d2)
    same_cells(cells, ref_cells)
    assert len(cells) > 100 and (cells["kind"][cells["frame"] > 0] > 0).mean() > 0.5


@pytest.mark.parametrize("entries", ["1", "2580", "12900"])   # 1, 2 and 10 rows per chunk
def test_track_overlap_row_chunks_same_records(monkeypatch, entries):
    """The overlap links computed in many row chunks of the (missed cell x
    cell) table (its size capped by SUBSURF4D_TRACK_TABLE) equal the
    one-chunk records and the oracle's."""
    n, level = (40, 23, 12, 3), 0.62
    u = np.random.default_rng(4).uniform(0.0, 1.0, size=orc.padded_shape(n))
    monkeypatch.delenv("SUBSURF4D_TRACK_TABLE", raising=False)
    one, _, _ = gpu_track(n, u, level)
    assert (one["kind"] == 2).sum() > 10          # the case has overlap links
    monkeypatch.setenv("SUBSURF4D_TRACK_TABLE", entries)
    many, lab, d2 = gpu_track(n, u, level)
    monkeypatch.delenv("SUBSURF4D_TRACK_TABLE", raising=False)
    assert np.array_equal(many, one)
    same_cells(many, orc.track_cells(n, lab, d2))
