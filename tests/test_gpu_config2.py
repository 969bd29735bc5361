"""GPU parity at the full shape of the nuclei volume (512 x 512 x 96 voxels x
16 frames, ~2000 tracks), in the launch configuration the benchmark times.

The oracle cannot run the whole volume inside a test, so every check samples
cells and lets the oracle compute each one on a crop that holds everything the
sampled value depends on, with the GPU's own inputs around it (teacher
forcing).  Centres are shifted with the crop; the shift is exact in float32,
so ball decisions are the same as on the full grid.

- owner map and initial function: 1-cell crops, bit-exact;
- local rescaling: a crop holding the whole ball of a sampled centre, cells
  owned by that ball, bit-exact;
- coefficients and right-hand side of the step's system: 1-cell crops (the
  coefficients of a cell depend on u in its 3^4 neighbourhood and on G on its
  faces), 1e-13 relative;
- two red-black iterations: after k iterations a cell depends on the data
  within distance 2k, and a crop boundary held fixed disturbs its inside by at
  most one cell per half-sweep, so on a crop of radius 6 (aligned to the
  grid's colouring) the centre value is the full grid's; 1e-12 absolute;
- a converged step (tol 1e-8): every sampled residual row is bounded by the
  2-norm the stopping rule controls, |r_P| <= tol * ||b||.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as orc  # noqa: E402
import synth  # noqa: E402
from paper_2111_11866_amd import binding as B  # noqa: E402

DEV = "cuda"
N = (512, 512, 96, 16)
OMEGA = 1.8
R_CROP = 6


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def shifted(cs, o):
    """centres relative to a crop whose first interior cell is o = (x, y, z, t)"""
    out = cs.copy()
    out["x"] = cs["x"] - np.float32(o[0])
    out["y"] = cs["y"] - np.float32(o[1])
    out["z"] = cs["z"] - np.float32(o[2])
    out["frame"] = cs["frame"] - np.int32(o[3])
    return out


def crop_box(p, r):
    """interior ranges [lo, hi] of a crop of radius at least r around p, clipped to
    the grid, starting at an even coordinate sum so that the crop's red cells are
    the grid's red cells (colour = parity of the index sum)"""
    lo = [max(p[d] - r, 0) for d in range(4)]
    hi = [min(p[d] + r, N[d] - 1) for d in range(4)]
    if sum(lo) % 2:
        d = next(d for d in range(4) if lo[d] > 0)
        lo[d] -= 1
    return lo, hi


def padded_slices(lo, hi):
    """numpy slices (t, z, y, x) of the padded crop: interior [lo, hi] plus one ghost layer"""
    return tuple(slice(lo[d], hi[d] + 3) for d in (3, 2, 1, 0))


def pidx(p):
    """padded (t, z, y, x) index of interior cell p = (x, y, z, t)"""
    return (p[3] + 1, p[2] + 1, p[1] + 1, p[0] + 1)


def samples(img, rng):
    n1, n2, n3, n4 = N
    pts = [(0, 0, 0, 0), (n1 - 1, n2 - 1, n3 - 1, n4 - 1), (0, n2 - 1, 0, n4 - 1), (n1 - 1, 0, n3 - 1, 0),
           (0, 200, 40, 7), (n1 - 1, 300, 50, 8), (100, 0, 30, 3), (200, n2 - 1, 60, 12), (300, 100, 0, 5),
           (400, 400, n3 - 1, 9), (250, 250, 45, 0), (260, 240, 47, n4 - 1)]
    for q in rng.integers(0, len(img.seeds), 10):             # cells at seed points (non-trivial u)
        s = img.seeds[q]
        pts.append((int(round(float(s["x"]))), int(round(float(s["y"]))), int(round(float(s["z"]))),
                    int(s["frame"])))
    for _ in range(14):
        pts.append(tuple(int(rng.integers(0, N[d])) for d in range(4)))
    return pts


@pytest.fixture(scope="module")
def c2():
    img = synth.nuclei_cfg2()
    pp = B.PrepareParams(image_scale=1.0 / 255.0)
    sp = B.StepParams(omega=OMEGA)
    job = B.Job(N, img.image, img.centres, img.seeds, precision=B.FP64)
    assert job.prepare(pp) == 0
    B.init_u(N, 1.0, job.seeds, job.ns, 1.0, 8.0, job.u)
    u_raw = job.u.clone()
    B.rescale(N, 1.0, job.centres, job.nc, sp.ball_r, job.owner, job.u, job.ws)
    w0 = job.u.clone()
    torch.cuda.synchronize()
    pts = samples(img, np.random.default_rng(2024))
    return dict(img=img, pp=pp, sp=sp, job=job, u_raw=u_raw, w0=w0, pts=pts)


def gather(t, pts):
    """values of a padded device array at interior cells pts"""
    idx = [torch.tensor([pidx(p)[a] for p in pts], device=DEV) for a in range(4)]
    return H(t[idx[0], idx[1], idx[2], idx[3]])


def crop_np(t, lo, hi):
    return H(t[padded_slices(lo, hi)]).copy()


def test_owner_and_initial_function(c2):
    img, job, pts = c2["img"], c2["job"], c2["pts"]
    owner = H(job.owner)
    got_u = gather(c2["u_raw"], pts)
    for q, p in enumerate(pts):
        one = (1, 1, 1, 1)
        ref_o = orc.owner_map(one, shifted(img.centres, p), c2["pp"].ball_r)[0, 0, 0, 0]
        assert owner[p[3], p[2], p[1], p[0]] == ref_o, (p, owner[p[3], p[2], p[1], p[0]], ref_o)
        ref_u = orc.init_u(one, shifted(img.seeds, p), 1.0, 8.0)[1, 1, 1, 1]
        assert got_u[q] == ref_u, (p, got_u[q], ref_u)


def test_rescale_sampled_balls(c2):
    img, job, sp = c2["img"], c2["job"], c2["sp"]
    owner = H(job.owner)
    rng = np.random.default_rng(7)
    r = int(np.ceil(sp.ball_r)) + 1
    checked = 0
    for m in rng.choice(len(img.centres), 12, replace=False):
        c = img.centres[m]
        p = (int(np.floor(c["x"])), int(np.floor(c["y"])), int(np.floor(c["z"])), int(c["frame"]))
        lo = [max(p[d] - r, 0) for d in range(3)] + [p[3]]
        hi = [min(p[d] + r + 1, N[d] - 1) for d in range(3)] + [p[3]]
        nc = tuple(hi[d] - lo[d] + 1 for d in range(4))
        u_in = crop_np(c2["u_raw"], lo, hi)
        own = np.ascontiguousarray(owner[lo[3]:hi[3] + 1, lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1])
        ref = orc.rescale(nc, u_in, shifted(img.centres, lo), sp.ball_r, own)
        got = crop_np(c2["w0"], lo, hi)
        mask = np.zeros_like(ref, dtype=bool)
        mask[1:-1, 1:-1, 1:-1, 1:-1] = own == m
        assert mask.any()
        np.testing.assert_array_equal(got[mask], ref[mask], err_msg=f"ball {m}")
        checked += int(mask.sum())
    assert checked > 1000


def test_assembly_sampled_cells(c2):
    job, sp, pts = c2["job"], c2["sp"], c2["pts"]
    coef = torch.empty(B.interior_shape(N) + (8,), dtype=torch.float64, device=DEV)
    b = torch.empty(B.interior_shape(N), dtype=torch.float64, device=DEV)
    B.assemble(N, 1.0, job.G, c2["w0"], sp, coef, b)
    ti = torch.tensor([[p[3], p[2], p[1], p[0]] for p in pts], device=DEV)
    got_c = H(coef[ti[:, 0], ti[:, 1], ti[:, 2], ti[:, 3]])
    got_b = H(b[ti[:, 0], ti[:, 1], ti[:, 2], ti[:, 3]])
    del coef, b
    torch.cuda.empty_cache()
    for q, p in enumerate(pts):
        lo, hi = list(p), list(p)
        G_np = H(job.G[(slice(None),) + padded_slices(lo, hi)])
        w_np = crop_np(c2["w0"], lo, hi)
        ref_c, ref_b, _ = one_cell_system(G_np, w_np, p, sp)
        np.testing.assert_allclose(got_c[q], ref_c, rtol=1e-13, atol=0, err_msg=f"coef at {p}")
        np.testing.assert_allclose(got_b[q], ref_b, rtol=1e-13, atol=1e-300, err_msg=f"b at {p}")


def one_cell_system(Gc, wc, p, sp):
    """oracle coefficients (8) and right-hand side of cell p from its 3^4
    neighbourhood; Dirichlet terms enter b only where the neighbour is a ghost
    of the full grid"""
    ub = wc.copy()
    for d, ax in zip(range(4), (3, 2, 1, 0)):
        for idx, real in ((0, p[d] == 0), (2, p[d] == N[d] - 1)):
            if not real:
                s = [1, 1, 1, 1]
                s[ax] = idx
                ub[tuple(s)] = 0.0
    coef, b = orc.assemble((1, 1, 1, 1), np.ascontiguousarray(Gc), np.ascontiguousarray(wc), 1.0, sp.eps,
                           sp.tau, ub=ub)
    return coef[0, 0, 0, 0], b[0, 0, 0, 0], wc


def test_two_iterations_sampled_crops(c2):
    job, sp, pts = c2["job"], c2["sp"], c2["pts"]
    from dataclasses import replace

    u = c2["w0"].clone()
    r = B.step(N, 1.0, job.G, job.centres, job.nc, job.owner, u, replace(sp, fixed_iters=2, rescale=False), job.ws)
    assert r["iterations"] == 2
    got = gather(u, pts)
    del u
    for q, p in enumerate(pts):
        lo, hi = crop_box(p, R_CROP)
        nc = tuple(hi[d] - lo[d] + 1 for d in range(4))
        Gc = np.ascontiguousarray(H(job.G[(slice(None),) + padded_slices(lo, hi)]))
        wc = crop_np(c2["w0"], lo, hi)
        coef, b = orc.assemble(nc, Gc, wc, 1.0, sp.eps, sp.tau)
        uo, it, _, _ = orc.sor(nc, coef, b, wc, sp.omega, 0.0, 2, orc.RB)
        ref = uo[p[3] - lo[3] + 1, p[2] - lo[2] + 1, p[1] - lo[1] + 1, p[0] - lo[0] + 1]
        assert abs(got[q] - ref) <= 1e-12, (p, got[q], ref)


def test_converged_step_residual_rows(c2):
    job, sp, pts = c2["job"], c2["sp"], c2["pts"]
    from dataclasses import replace

    w0 = c2["w0"]
    # Dirichlet data of the segmentation function is zero: b = u^{resc;n-1} inside
    ghost = w0.clone()
    ghost[1:-1, 1:-1, 1:-1, 1:-1] = 0.0
    assert float(ghost.abs().max()) == 0.0
    del ghost
    bnorm = float(torch.linalg.vector_norm(w0[1:-1, 1:-1, 1:-1, 1:-1]))
    u = w0.clone()
    r = B.step(N, 1.0, job.G, job.centres, job.nc, job.owner, u, replace(sp, rescale=False), job.ws)
    assert r["status"] == 0 and r["rel_res"] <= sp.tol
    assert abs(r["bnorm"] - bnorm) <= 1e-12 * bnorm
    bound = sp.tol * bnorm * (1.0 + 1e-6)
    for p in pts:
        lo, hi = list(p), list(p)
        sl = padded_slices(lo, hi)
        Gc = H(job.G[(slice(None),) + sl])
        c, b, _ = one_cell_system(Gc, crop_np(w0, lo, hi), p, sp)
        un = crop_np(u, lo, hi)
        # neighbours in face order -x,+x,-y,+y,-z,+z,-t,+t; ghosts of the full grid carry u^D = 0
        nb = [un[1, 1, 1, 0], un[1, 1, 1, 2], un[1, 1, 0, 1], un[1, 1, 2, 1],
              un[1, 0, 1, 1], un[1, 2, 1, 1], un[0, 1, 1, 1], un[2, 1, 1, 1]]
        for f, (d, side) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1), (3, 0), (3, 1)]):
            if (side == 0 and p[d] == 0) or (side == 1 and p[d] == N[d] - 1):
                nb[f] = 0.0                     # the ghost term is already in b
        D = 1.0 + float(np.sum(c))
        res = b + float(np.dot(c, nb)) - D * un[1, 1, 1, 1]
        assert abs(res) <= bound, (p, res, bound)


def test_mixed_step_full_size(c2):
    """The mixed-precision step on the whole volume (FP32 sweeps on BF16
    coefficients, FP64 refinement to ||r||_2 <= 1e-10 ||b||_2) against the
    FP64 step converged to 1e-12 from the same level.  With ||A^-1||_inf <= 1
    (stability section) every cell's error is at most ||r||_inf <= ||r||_2, so
    both results lie within their tolerance times ||b||_2 of the exact
    solution, and of each other within the sum."""
    from dataclasses import replace

    job, sp = c2["job"], replace(c2["sp"], rescale=False)
    w0 = c2["w0"]
    ref = w0.clone()
    r64 = B.step(N, 1.0, job.G, job.centres, job.nc, job.owner, ref, replace(sp, tol=1e-12, max_iter=100000),
                 job.ws)
    assert r64["status"] == 0
    ws = B.alloc_workspace(N, job.nc, B.MIXED)
    u = w0.clone()
    mixed = replace(sp, precision=B.MIXED, refine_tol=1e-10, inner_sweeps=10, omega=1.5)
    r = B.step(N, 1.0, job.G, job.centres, job.nc, job.owner, u, mixed, ws)
    del ws
    assert r["status"] == 0 and r["rel_res"] <= 1e-10
    bnorm = r64["bnorm"]
    assert abs(r["bnorm"] - bnorm) <= 1e-12 * bnorm
    err = float((u - ref).abs().max())
    assert err <= (1e-10 + 1e-12) * bnorm * (1.0 + 1e-6), (err, bnorm)
    rel_l2 = float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(ref))
    print(f"mixed vs converged FP64 on the full volume: max-abs {err:.3e} (bound "
          f"{1.01e-10 * bnorm:.3e}), relative L2 {rel_l2:.3e}, {r['outer']} passes")
    del u, ref
