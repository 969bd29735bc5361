"""Batched step over many uneven windows (mixed precision, graph-replayed
refinement passes) against the FP64 oracle, the single-job path, and itself
(alone vs in a mix, graph vs eager launches)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as orc  # noqa: E402
import synth  # noqa: E402
from paper_2111_11866_amd import binding as B  # noqa: E402

SP = B.StepParams(precision=B.MIXED, refine_tol=1e-10, inner_sweeps=8)
PP = B.PrepareParams(image_scale=1.0 / 255.0)


def H(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make_jobs(sizes, seed0=1000, prep_ws=None):
    jobs = []
    for q, n in enumerate(sizes):
        img = synth.window_job(n, seed0 + q, seed0 + 100000 + q)
        j = B.Job(n, img.image, img.centres, img.seeds, precision=B.MIXED, batch=True, shared_ws=prep_ws)
        j.prepare(PP)
        j.init(v=1.0, R=8.0, ball_r=SP.ball_r)
        j.img = img
        jobs.append(j)
    return jobs


SIZES = [(24, 30, 26, 3), (33, 25, 28, 5), (40, 40, 40, 5), (27, 35, 24, 9), (64, 24, 30, 4), (25, 25, 25, 3)]


@pytest.fixture(scope="module")
def batch():
    jobs = make_jobs(SIZES)
    u0 = [j.u.clone() for j in jobs]
    return jobs, u0


def run(jobs, sp=SP):
    table = torch.empty(B.batch_table_bytes(len(jobs)), dtype=torch.uint8, device="cuda")
    return B.step_batched(jobs, sp, table)


def test_batched_matches_oracle_and_single_job(batch):
    jobs, u0 = batch
    for j, u in zip(jobs, u0):
        j.u.copy_(u)
    rc, res = run(jobs)
    assert rc == 0
    for q, j in enumerate(jobs):
        assert res[q]["status"] == 0 and res[q]["rel_res"] <= 1e-10
        w = H(u0[q])
        G, owner = H(j.G), H(j.owner)
        ref = orc.step(j.n, G, w, j.img.centres, owner, orc.StepParams(tol=1e-14), orc.RB)
        got = H(j.u)
        err = np.abs(got - ref["u_resc"]).max() / max(np.abs(ref["u_resc"]).max(), 1e-300)
        assert err <= 1e-6, (q, err)
        # the single-job mixed path on the same input
        us = u0[q].clone()
        r1 = B.step(j.n, j.h, j.G, j.centres, j.nc, j.owner, us, SP, j.ws)
        assert r1["status"] == 0
        assert np.abs(H(us) - got).max() <= 1e-8


def test_batched_alone_equals_in_mix(batch):
    """Each window's result is bitwise the same alone and inside the batch."""
    jobs, u0 = batch
    for j, u in zip(jobs, u0):
        j.u.copy_(u)
    run(jobs)
    mixed = [H(j.u) for j in jobs]
    for q in (0, 3, 5):
        jobs[q].u.copy_(u0[q])
        rc, res = run([jobs[q]])
        assert np.array_equal(H(jobs[q].u), mixed[q]), q


def test_graph_replays_equal_eager(batch):
    """Refinement passes replayed from a captured graph give the same bits as
    the same kernels launched one by one (several replays per step)."""
    jobs, u0 = batch
    out = []
    for flags in (0, B.FLAG_NO_GRAPH, 0):
        for j, u in zip(jobs, u0):
            j.u.copy_(u)
        from dataclasses import replace
        rc, res = run(jobs, replace(SP, flags=flags))
        assert all(r["outer"] >= 2 for r in res)
        out.append([H(j.u) for j in jobs])
    for a, b, c in zip(*out):
        assert np.array_equal(a, b) and np.array_equal(a, c)


def test_sweep_shapes_give_the_same_bits(batch):
    """Both work shapes of the inner sweep (flat items, frame-marching
    columns) and the autotuner's choice give bitwise the same step."""
    from dataclasses import replace

    jobs, u0 = batch
    out = []
    for flags in (0, B.FLAG_SWEEP_FLAT, B.FLAG_SWEEP_MARCH, B.FLAG_SWEEP_MARCH | B.FLAG_NO_GRAPH):
        for j, u in zip(jobs, u0):
            j.u.copy_(u)
        rc, res = run(jobs, replace(SP, flags=flags))
        assert rc == 0
        out.append([H(j.u) for j in jobs])
    for per_job in zip(*out):
        for other in per_job[1:]:
            assert np.array_equal(per_job[0], other)
    with pytest.raises(B.Subsurf4dError):
        run(jobs, replace(SP, flags=B.FLAG_SWEEP_FLAT | B.FLAG_SWEEP_MARCH))
    with pytest.raises(B.Subsurf4dError):
        run(jobs, replace(SP, flags=64))


def test_batched_several_steps_stay_bounded(batch):
    jobs, u0 = batch
    for j, u in zip(jobs, u0):
        j.u.copy_(u)
    for s in range(5):
        rc, res = run(jobs)
        assert rc == 0
    for j in jobs:
        u = H(j.u)
        assert u.min() >= -1e-9 and u.max() <= 1 + 1e-9


def test_batched_tau_zero_and_not_converged():
    jobs = make_jobs([(26, 24, 25, 3), (30, 28, 24, 4)], seed0=5000)
    before = [H(j.u) for j in jobs]
    from dataclasses import replace
    rc, res = run(jobs, replace(SP, tau=0.0, rescale=False))
    assert rc == 0 and all(r["outer"] == 0 for r in res)
    for j, b in zip(jobs, before):
        assert np.array_equal(H(j.u), b)
    rc, res = run(jobs, replace(SP, refine_tol=1e-16, inner_sweeps=2, max_iter=4))
    assert rc == B.NOT_CONVERGED and all(r["status"] == B.NOT_CONVERGED for r in res)


def test_empty_batch():
    """No jobs: both batched calls return OK and enqueue nothing."""
    assert B.step_batched([], SP, None) == (0, [])
    assert B.prepare_batched([], PP, 1.0, 0.0, 8.0, None) == (0, [])


def raw_job(n, rng):
    """A batched job on random coefficients (G in [0.05, 1]) and a random
    level with zero Dirichlet ghosts, no balls (no rescale)."""
    from types import SimpleNamespace

    G = rng.uniform(0.05, 1.0, size=(4,) + B.padded_shape(n))
    w = np.zeros(B.padded_shape(n))
    w[1:-1, 1:-1, 1:-1, 1:-1] = rng.uniform(0.0, 1.0, size=tuple(reversed(n)))
    dev = lambda a: torch.from_numpy(a).to("cuda")  # noqa: E731
    bws = torch.empty(B.batch_workspace_bytes(n, 0), dtype=torch.uint8, device="cuda")
    return SimpleNamespace(n=n, h=1.0, G=dev(G), u=dev(w), owner=None, centres=None, nc=0, bws=bws), G, w


def test_batched_degenerate_windows_against_oracle():
    """Windows with one or two cells along some axes (rows of one slot, a
    single frame, a single cell) in one batch, each against the FP64 oracle
    converged to 1e-14."""
    from dataclasses import replace

    rng = np.random.default_rng(31)
    sizes = [(1, 1, 1, 1), (2, 1, 1, 1), (1, 3, 1, 2), (3, 2, 2, 1), (5, 1, 4, 2), (1, 1, 1, 7), (130, 1, 1, 1),
             (2, 2, 2, 2)]
    made = [raw_job(n, rng) for n in sizes]
    sp = replace(SP, rescale=False)
    rc, res = run([m[0] for m in made], sp)
    assert rc == 0
    for (j, G, w), r in zip(made, res):
        assert r["status"] == 0, (j.n, r)
        ref = orc.step(j.n, G, w, None, None, orc.StepParams(tol=1e-14, rescale=False), orc.RB)["u_resc"]
        err = np.abs(H(j.u) - ref).max()
        assert err <= 1e-8 * max(np.abs(ref).max(), 1e-300), (j.n, err)


def test_batched_window_at_the_size_limit():
    """A window of 200x200x200x2 (32.97 M padded cells, 98% of the 2^25
    limit of a batched job) next to a small one: every cell against the
    single-job FP64 step solved to 1e-12 (itself checked against the oracle),
    so the index decode and 32-bit offsets are exercised at their largest."""
    from dataclasses import replace

    rng = np.random.default_rng(37)
    big, small = (200, 200, 200, 2), (5, 4, 3, 3)
    assert np.prod([v + 2 for v in big]) <= 1 << 25
    assert B.batch_workspace_bytes(big, 0) > 0
    made = [raw_job(n, rng) for n in (big, small)]
    refs = []
    for j, G, w in made:
        u = torch.from_numpy(w).to("cuda")
        ws = B.alloc_workspace(j.n, 0, B.FP64)
        r = B.step(j.n, 1.0, j.G, None, 0, None, u,
                   B.StepParams(tol=1e-12, max_iter=100000, rescale=False), ws)
        assert r["status"] == 0
        refs.append(H(u))
        del ws, u
    rc, res = run([m[0] for m in made], replace(SP, rescale=False))
    assert rc == 0 and all(r["status"] == 0 for r in res)
    # refine_tol 1e-10 bounds ||r||_2 / ||b||_2; with ||A^-1||_inf <= 1 the
    # max error of 16 M cells is bounded by 1e-10 ||b||_2 ~ 2e-7 at worst
    for (j, _, _), ref in zip(made, refs):
        err = np.abs(H(j.u) - ref).max()
        assert err <= 1e-7 * np.abs(ref).max(), (j.n, err)


def test_batched_grid_spacing_and_dirichlet_data():
    """Jobs of different grid spacing (h = 0.37, 1, 2.5: tau/h^2 and the
    gradients scale per job) with non-zero Dirichlet data in their ghost
    layers, in one batch, each against the FP64 oracle converged to 1e-14."""
    from dataclasses import replace

    rng = np.random.default_rng(43)
    made = []
    for n, h in (((9, 7, 6, 5), 0.37), ((24, 20, 18, 3), 1.0), ((13, 11, 9, 4), 2.5)):
        j, G, _ = raw_job(n, rng)
        w = rng.uniform(0.0, 1.0, size=B.padded_shape(n))           # ghosts = u^D, not zero
        j.u = torch.from_numpy(w).to("cuda")
        j.h = h
        made.append((j, G, w, h))
    rc, res = run([m[0] for m in made], replace(SP, rescale=False))
    assert rc == 0
    for (j, G, w, h), r in zip(made, res):
        assert r["status"] == 0, (j.n, h, r)
        ref = orc.step(j.n, G, w, None, None, orc.StepParams(tol=1e-14, rescale=False, h=h), orc.RB)["u_resc"]
        got = H(j.u)
        err = np.abs(got - ref).max()
        assert err <= 1e-8 * np.abs(ref).max(), (j.n, h, err)
        # the ghost layer (Dirichlet data) is left as it was
        inner = (slice(1, -1),) * 4
        mask = np.ones(got.shape, bool)
        mask[inner] = False
        assert np.array_equal(got[mask], w[mask])


def test_batched_fp64_matches_oracle(batch):
    """Batched FP64 form: every window's FP64 red-black SOR with the stopping
    rule tested every m = 3 iterations equals the red-black oracle with the
    same rule (check_every = 3) to 1e-10, with the same iteration count; when
    a residual sits at the threshold and the counts split, the iterate at the
    GPU's count is compared instead."""
    from dataclasses import replace

    jobs, u0 = batch
    for j, u in zip(jobs, u0):
        j.u.copy_(u)
    sp = B.StepParams(precision=B.FP64, omega=1.35, tol=1e-9, inner_sweeps=3)
    rc, res = run(jobs, sp)
    assert rc == 0
    osp = orc.StepParams(omega=1.35, tol=1e-9, check_every=3)
    for q, j in enumerate(jobs):
        w, G, owner = H(u0[q]), H(j.G), H(j.owner)
        ref = orc.step(j.n, G, w, j.img.centres, owner, osp, orc.RB)
        k = res[q]["iterations"]
        assert res[q]["status"] == 0 and k % 3 == 0
        if k != ref["iterations"]:
            kmin = min(k, ref["iterations"])
            near = orc.step(j.n, G, w, j.img.centres, owner, osp, orc.RB, fixed_iters=kmin)
            assert abs(near["rel_res"] / osp.tol - 1) < 1e-6, (q, k, ref["iterations"], near["rel_res"])
            ref = orc.step(j.n, G, w, j.img.centres, owner, osp, orc.RB, fixed_iters=k)
        err = np.abs(H(j.u) - ref["u_resc"]).max()
        assert err <= 1e-10, (q, err)
    # the same batch again gives the same bits (kept graph executable, updated in place)
    first = [H(j.u) for j in jobs]
    for j, u in zip(jobs, u0):
        j.u.copy_(u)
    run(jobs[:3], replace(sp, tol=1e-6))          # a different batch in between
    for j, u in zip(jobs, u0):
        j.u.copy_(u)
    run(jobs, sp)
    for q, j in enumerate(jobs):
        assert np.array_equal(H(j.u), first[q]), q
