"""Batched preparation of many windows (owner map, G, u0 and its rescale in one
sequence of launches) against the FP64 oracle, the single-job path, and
itself (alone vs in a mix)."""
from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as orc  # noqa: E402
import synth  # noqa: E402
from paper_2111_11866_amd import binding as B  # noqa: E402

PP = B.PrepareParams(image_scale=1.0 / 255.0)
SIZES = [(24, 30, 26, 3), (33, 25, 28, 5), (40, 40, 40, 5), (27, 35, 24, 9), (64, 24, 30, 4), (25, 25, 25, 3)]
BALL_R = 8.0


def H(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def orc_pp(p: B.PrepareParams):
    return orc.PrepareParams(K=p.K, delta=p.delta, vartheta=p.vartheta, lam=p.lam, ball_r=p.ball_r,
                             smooth_tau=p.smooth_tau, smooth_steps=p.smooth_steps,
                             smooth_omega=p.smooth_omega, smooth_tol=p.smooth_tol)


def windows(sizes, seed0=1000):
    return [synth.window_job(n, seed0 + q, seed0 + 100000 + q) for q, n in enumerate(sizes)]


def batched(imgs, pp=PP, v=1.0, R=0.0):
    jobs = [B.Job(im.n, im.image, im.centres, im.seeds, precision=B.MIXED, batch=True, shared_ws=False)
            for im in imgs]
    table = torch.empty(B.batch_table_bytes(len(jobs)), dtype=torch.uint8, device="cuda")
    rc, st = B.prepare_batched(jobs, pp, v, R, BALL_R, table)
    return rc, st, jobs


def oracle_prep(im, pp=PP, v=1.0, R=0.0):
    I0 = im.image.astype(np.float64) * pp.image_scale
    prep = orc.prepare(im.n, I0, im.centres, orc_pp(pp))
    u0 = orc.init_u(im.n, im.seeds, v, R)
    w = orc.rescale(im.n, u0, im.centres, BALL_R, prep["owner"])
    return prep, w


@pytest.fixture(scope="module")
def imgs():
    return windows(SIZES)


def test_batched_prepare_matches_oracle(imgs):
    rc, st, jobs = batched(imgs)
    assert rc == 0 and st == [0] * len(imgs)
    for im, j in zip(imgs, jobs):
        prep, w = oracle_prep(im)
        np.testing.assert_array_equal(H(j.owner), prep["owner"])
        assert np.abs(H(j.G) - prep["G"]).max() <= 1e-12
        # u0 and its rescale are exact decisions on exactly rounded values
        np.testing.assert_array_equal(H(j.u), w)


def test_batched_prepare_matches_single_job(imgs):
    rc, st, jobs = batched(imgs)
    assert rc == 0
    for im, j in zip(imgs, jobs):
        s = B.Job(im.n, im.image, im.centres, im.seeds, precision=B.MIXED)
        assert s.prepare(PP) == 0
        s.init(v=1.0, R=0.0, ball_r=BALL_R)
        np.testing.assert_array_equal(H(j.owner), H(s.owner))
        assert np.abs(H(j.G) - H(s.G)).max() <= 1e-13
        np.testing.assert_array_equal(H(j.u), H(s.u))


def test_batched_prepare_alone_equals_in_mix(imgs):
    _, _, mix = batched(imgs)
    for q in (0, 2, 5):
        _, _, alone = batched([imgs[q]])
        np.testing.assert_array_equal(H(alone[0].G), H(mix[q].G))
        np.testing.assert_array_equal(H(alone[0].u), H(mix[q].u))
        np.testing.assert_array_equal(H(alone[0].owner), H(mix[q].owner))


def test_batched_prepare_two_smoothing_steps_and_cutoff():
    """two heat steps per image and the R > 0 (scattered) initial function"""
    pp = replace(PP, smooth_steps=2)
    ims = windows([(26, 24, 25, 4), (30, 27, 24, 3)], seed0=2000)
    rc, st, jobs = batched(ims, pp=pp, v=1.0, R=6.0)
    assert rc == 0
    for im, j in zip(ims, jobs):
        prep, w = oracle_prep(im, pp=pp, v=1.0, R=6.0)
        np.testing.assert_array_equal(H(j.owner), prep["owner"])
        assert np.abs(H(j.G) - prep["G"]).max() <= 1e-12
        np.testing.assert_array_equal(H(j.u), w)


def test_batched_prepare_no_centres_and_f32_image():
    im = synth.window_job((28, 26, 24, 3), 3000, 103000)
    im32 = synth.Image4D(n=im.n, image=im.image.astype(np.float32), centres=im.centres[:0], seeds=im.seeds)
    rc, st, jobs = batched([im32])
    assert rc == 0
    prep, w = oracle_prep(synth.Image4D(n=im.n, image=im.image.astype(np.float64), centres=im.centres[:0],
                                        seeds=im.seeds))
    assert (H(jobs[0].owner) == -1).all()
    assert np.abs(H(jobs[0].G) - prep["G"]).max() <= 1e-12
    np.testing.assert_array_equal(H(jobs[0].u), w)


def test_batched_prepare_then_step(imgs):
    """the prepared jobs step like jobs prepared one by one"""
    sp = B.StepParams(precision=B.MIXED, refine_tol=1e-10, inner_sweeps=8)
    rc, st, jobs = batched(imgs)
    table = torch.empty(B.batch_table_bytes(len(jobs)), dtype=torch.uint8, device="cuda")
    rc, res = B.step_batched(jobs, sp, table)
    assert rc == 0 and all(r["status"] == 0 for r in res)
    for im, j in zip(imgs, jobs):
        s = B.Job(im.n, im.image, im.centres, im.seeds, precision=B.MIXED, batch=True)
        s.prepare(PP)
        s.init(v=1.0, R=0.0, ball_r=BALL_R)
        B.step_batched([s], sp, table)
        assert np.abs(H(j.u) - H(s.u)).max() <= 1e-10


def test_batched_prepare_bad_arguments(imgs):
    jobs = [B.Job(imgs[0].n, imgs[0].image, imgs[0].centres, imgs[0].seeds, precision=B.MIXED, batch=True,
                  shared_ws=False)]
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.Subsurf4dError):
        B.prepare_batched(jobs, PP, 1.0, 0.0, BALL_R, small)
    table = torch.empty(B.batch_table_bytes(1), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.Subsurf4dError):
        B.prepare_batched(jobs, replace(PP, lam=2.0), 1.0, 0.0, BALL_R, table)
    with pytest.raises(B.Subsurf4dError):
        B.prepare_batched(jobs, PP, 0.0, 0.0, BALL_R, table)
    for bad in (dict(delta=float("nan")), dict(vartheta=-1.0), dict(delta=float("inf")),
                dict(smooth_tau=float("inf")), dict(smooth_max_iter=2 ** 31 - 1)):
        with pytest.raises(B.Subsurf4dError):
            B.prepare_batched(jobs, replace(PP, **bad), 1.0, 0.0, BALL_R, table)


def test_prepare_grid_spacing_single_and_batched():
    """h = 0.5 enters the presmoothing (tau_s / h^2) and the face gradients of
    G (ball membership and u0 are in voxel units): the batched and the
    single-job preparation against the oracle."""
    h = 0.5
    ims = windows([(26, 24, 22, 3), (30, 25, 21, 4)], seed0=7000)
    jobs = [B.Job(im.n, im.image, im.centres, im.seeds, h=h, precision=B.MIXED, batch=True, shared_ws=False)
            for im in ims]
    table = torch.empty(B.batch_table_bytes(len(jobs)), dtype=torch.uint8, device="cuda")
    rc, st = B.prepare_batched(jobs, PP, 1.0, 0.0, BALL_R, table)
    assert rc == 0 and st == [0] * len(jobs)
    for im, j in zip(ims, jobs):
        I0 = im.image.astype(np.float64) * PP.image_scale
        prep = orc.prepare(im.n, I0, im.centres, replace(orc_pp(PP), h=h))
        np.testing.assert_array_equal(H(j.owner), prep["owner"])
        assert np.abs(H(j.G) - prep["G"]).max() <= 1e-12
        one = B.Job(im.n, im.image, im.centres, im.seeds, h=h, precision=B.FP64)
        assert one.prepare(PP) == 0
        np.testing.assert_array_equal(H(one.owner), prep["owner"])
        assert np.abs(H(one.G) - prep["G"]).max() <= 1e-12


@pytest.mark.parametrize("cap", [1, 3])
def test_batched_prepare_heat_solve_cut_by_max_iter(cap):
    """A heat solve stopped by its iteration limit returns that iterate with
    status NOT_CONVERGED: the batched form (which judges iterate k during the
    next pass and then puts back iterate k's red values) against the
    single-job form, which stops after iterate k itself."""
    pp = replace(PP, smooth_max_iter=cap)
    ims = windows([(26, 24, 25, 4), (31, 22, 24, 3)], seed0=8000)
    rc, st, jobs = batched(ims, pp=pp)
    assert rc == B.NOT_CONVERGED and st == [B.NOT_CONVERGED] * len(ims)
    _, _, full = batched(ims)
    for im, j, f in zip(ims, jobs, full):
        one = B.Job(im.n, im.image, im.centres, im.seeds, precision=B.FP64)
        assert one.prepare(pp) == B.NOT_CONVERGED
        assert np.abs(H(j.G) - H(one.G)).max() <= 1e-13
        # the limit did cut the solve short
        assert np.abs(H(j.G) - H(f.G)).max() > 1e-9


def test_prepare_wide_index_form_same_bits(monkeypatch):
    """The single-job preparation decodes cell indices with 32-bit multiplies
    on grids below 2^31 cells and with 64-bit divisions above; forcing the
    64-bit form on small grids (odd and even row lengths) gives the same G."""
    for n in [(33, 25, 28, 5), (24, 30, 26, 3)]:
        im = synth.window_job(n, 9100, 109100)
        a = B.Job(n, im.image, im.centres, im.seeds, precision=B.FP64)
        assert a.prepare(PP) == 0
        monkeypatch.setenv("SUBSURF4D_WIDE_INDEX", "1")
        b = B.Job(n, im.image, im.centres, im.seeds, precision=B.FP64)
        assert b.prepare(PP) == 0
        monkeypatch.delenv("SUBSURF4D_WIDE_INDEX")
        np.testing.assert_array_equal(H(a.G), H(b.G))
        np.testing.assert_array_equal(H(a.owner), H(b.owner))


def test_prepare_degenerate_shapes_single_and_batched():
    """Rows of one or two cells (one colour empty in a row, or a single cell
    of each), single planes and frames, a single cell: the colour-split heat
    solves and the face G of both forms against the oracle."""
    sizes = [(1, 5, 4, 3), (2, 3, 1, 2), (5, 1, 1, 4), (3, 2, 2, 1), (1, 1, 1, 1), (2, 2, 2, 2), (7, 1, 3, 1)]
    ims = [synth.window_job(n, 9300 + q, 109300 + q) for q, n in enumerate(sizes)]
    rc, st, jobs = batched(ims)
    assert rc == 0 and st == [0] * len(ims)
    for im, j in zip(ims, jobs):
        prep, _ = oracle_prep(im)
        np.testing.assert_array_equal(H(j.owner), prep["owner"])
        assert np.abs(H(j.G) - prep["G"]).max() <= 1e-12, im.n
        one = B.Job(im.n, im.image, im.centres, im.seeds, precision=B.FP64)
        assert one.prepare(PP) == 0
        assert np.abs(H(one.G) - prep["G"]).max() <= 1e-12, im.n
        assert np.abs(H(one.G) - H(j.G)).max() <= 1e-13, im.n
